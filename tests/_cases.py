"""Shared test cases: one seeded input, built twice (oracle and HIP path)."""
from __future__ import annotations

import numpy as np

from inputs import cube_mesh, freestream_prim, perturbed_state, prim_to_cons, shell_mesh
from tests import _indep as I

# boundary kinds share their integer codes between the oracle and the C ABI
FAR, SLIP, NOSLIP, SUP_IN, SUP_OUT = 0, 1, 2, 3, 4


def flux_scale(mesh, prim):
    """max over cells of (sum of face areas) x |Euler flux of the free stream|:
    the scale residual parity is measured against."""
    q = prim_to_cons(prim)
    f = max(np.abs(I.euler_flux(q, d)).max() for d in np.eye(3))
    v = mesh.xyz[mesh.tets]
    area = np.zeros(len(v))
    for p in range(4):
        tri = np.delete(v, p, axis=1)
        area += 0.5 * np.linalg.norm(np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]), axis=1)
    return f * area.max()


def area_sums(mesh):
    """Sum of the four face areas of every tet (computed from the nodes)."""
    v = mesh.xyz[mesh.tets]
    area = np.zeros(len(v))
    for p in range(4):
        tri = np.delete(v, p, axis=1)
        area += 0.5 * np.linalg.norm(np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]), axis=1)
    return area


def grad_update_bound(mesh, Q, vol, rel=1e-12):
    """Per-cell bound of the compact gradient update of Eq. (derivative):
    it is (1/|Omega_i|) times a sum over the cell's faces of S_f times
    Gauss-point values of size |Q|, which carry the same relative rounding
    as the fluxes, so rel x max|Q| x (sum of face areas) / |Omega_i|."""
    return rel * np.abs(Q).max() * area_sums(mesh) / vol


def pair(oracle_mod, mesh, kinds, prim, **opts):
    from paper_2304_09485_amd import hgks
    o = oracle_mod.Oracle(mesh, kinds, prim, **{k: v for k, v in opts.items() if k != "precision"})
    s = hgks.Solver(mesh, kinds, prim, **opts)
    return o, s


CASES = {
    # name: (mesh builder, kinds, mach, options)
    "c1_weno": (lambda: cube_mesh(8), {t: FAR for t in range(1, 7)}, 0.3, {}),
    "cube_jit_weno_slip": (lambda: cube_mesh(5, jitter=0.15, seed=3), {t: SLIP for t in range(1, 7)}, 0.3, {}),
    "cube_jit_hweno": (lambda: cube_mesh(5, jitter=0.15, seed=4),
                       {1: SUP_IN, 2: SUP_OUT, 3: FAR, 4: FAR, 5: SLIP, 6: SLIP}, 0.4, {"scheme": 1}),
    "shell_weno": (lambda: shell_mesh(4, 4, grading=1.3, jitter=0.05, seed=2), {1: SLIP, 2: FAR}, 0.5, {}),
    "shell_hweno": (lambda: shell_mesh(4, 4, grading=1.3, jitter=0.05, seed=2), {1: SLIP, 2: FAR}, 0.5,
                    {"scheme": 1}),
    "shell_ns": (lambda: shell_mesh(4, 4, grading=1.3, jitter=0.05, seed=3), {1: NOSLIP, 2: FAR}, 0.25,
                 {"physics": 1, "mu": 0.25 / 118.0, "prandtl": 0.72}),
    "cube_linw": (lambda: cube_mesh(4, jitter=0.1, seed=5), {t: FAR for t in range(1, 7)}, 0.3, {"weights": 1}),
}


def state_for(n, mach, seed=1, amp=0.01):
    return perturbed_state(n, freestream_prim(mach), amp=amp, seed=seed)
