"""Seeded stream of steady-solve requests for the serving workload.

Each request draws (seed 5000 + k): a mesh kind (sphere shell or ramp
channel, p = 1/2), a cell count log-uniform in [n_min, n_max] met by scaling
the generator's resolution, a Mach number uniform in [0.2, 2.0], inviscid or
viscous flow (p = 1/2; Reynolds number uniform in [50, 500], Pr = 0.72).
Arrivals are a Poisson process (exponential inter-arrival times).  Only the
inputs are generated here; nothing of the method's arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .meshes import TetMesh, ramp_mesh, shell_mesh


@dataclass
class RequestSpec:
    index: int
    arrival_s: float
    kind: str          # "shell" | "ramp"
    target_cells: int
    mach: float
    viscous: bool
    reynolds: float
    seed: int

    def mesh(self) -> TetMesh:
        """The request's mesh, resolution scaled to about target_cells."""
        if self.kind == "shell":
            # 6 patches x n^2 x nr hexes x 6 tets, nr ~ 1.4 n (as the 202,752-tet shell)
            n = max(3, int(round((self.target_cells / (36 * 1.4)) ** (1.0 / 3.0))))
            nr = max(3, int(round(1.4 * n)))
            return shell_mesh(n, nr, grading=1.1, jitter=0.02, seed=self.seed)
        # ramp channel: hexes nx : ny : nz = 4 : 1.5 : 1 (as the 3,981,312-tet channel)
        nz = max(2, int(round((self.target_cells / (6 * 4 * 1.5)) ** (1.0 / 3.0))))
        return ramp_mesh(4 * nz, max(2, int(round(1.5 * nz))), nz, jitter=0.02, seed=self.seed, ramp_end=1.5,
                         height=2.0)

    def boundary_kinds(self) -> dict:
        """Boundary kind per tag (far field 0, slip wall 1, no-slip adiabatic 2,
        supersonic inflow 3, supersonic outflow 4)."""
        if self.kind == "shell":
            return {1: 2 if self.viscous else 1, 2: 0}
        inlet = 3 if self.mach > 1.0 else 0
        outlet = 4 if self.mach > 1.0 else 0
        return {1: inlet, 2: outlet, 3: 1, 4: 1, 5: 1, 6: 1}


def request_stream(n_requests: int = 64, rate_per_s: float = 0.5, seed: int = 5,
                   n_min: int = 50_000, n_max: int = 2_000_000) -> list[RequestSpec]:
    """The seeded request stream (arrival times in seconds from the start)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for k in range(n_requests):
        r = np.random.default_rng(5000 + k)
        kind = "shell" if r.uniform() < 0.5 else "ramp"
        cells = int(round(math.exp(r.uniform(math.log(n_min), math.log(n_max)))))
        mach = float(r.uniform(0.2, 2.0))
        viscous = bool(r.uniform() < 0.5)
        re = float(r.uniform(50.0, 500.0))
        out.append(RequestSpec(k, float(arrivals[k]), kind, cells, mach, viscous, re, 5000 + k))
    return out
