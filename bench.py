#!/usr/bin/env python3
"""Benchmark: implicit steps of the compact HWENO gas-kinetic scheme on one MI355X.

Workload (default): inviscid Mach 0.5 flow past a sphere, seeded jittered
cubed-sphere tetrahedral shell r in [0.5, 10] with 202,752 tets, slip wall on
the sphere and far field outside, compact HWENO reconstruction with gradients
updated from the gas distribution function, CFL 10, GMRES(10) x 3 restarts,
2 Jacobi sweeps, FP64.  One timed "step" is one implicit step: the base
residual, 32 FD Jacobian-vector products (each a full residual evaluation),
Jacobi sweeps, MGS Arnoldi, host Givens, the update and the gradient update.

Prints one JSON line: metric/value (Mcell-residual evaluations per second over
the timed steps), roofline of the dominant residual kernel (per-launch HIP
event timings recorded inside the timed region) and the CPU oracle baseline on
a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
PEAK_FP64_VALU = 78.6e12     # MI355X FP64 vector FLOP/s

# Algorithmic work per unit of the residual kernels (see the design notes):
#   flux kernel: FP64 operations of the gas-kinetic flux per Gauss point,
#   counted by running the flux function on the host with an operation-counting
#   scalar type (tools in csrc/flopcount.cpp); units per launch = 3 F
FLUX_FLOPS_PER_GP = {"euler": None, "euler_qg": None, "ns": None}
FLOPS_FILE = os.path.join(ROOT, "paper_2304_09485_amd", "flux_flops.json")


def algorithmic_units(kernel, N, F, Nb, scheme):
    """(bytes, flops) a launch of the kernel must move / compute at minimum."""
    if kernel == "recon":
        if scheme == 1:
            # operator 171 + P_m data 24 doubles, 4 neighbour ids, own Q and
            # gradients read once, 105 coefficients written, per cell
            b = N * (8 * (171 + 24) + 4 * 4 + 8 * (5 + 15) + 8 * 105 + 8)
        else:
            b = N * (8 * (144 + 72) + 4 * (16 + 24) + 1 + 8 * 5 + 8 * 105)
        return b, None
    if kernel == "side":
        # coefficients (105) of the side's cell, two cell states, 21 face
        # geometry values; 60 values written per side
        sides = 2 * F - Nb
        return sides * 8 * (105 + 10 + 21 + 60), None
    if kernel == "gather":
        return N * (4 * 4 + 5 * 8 * 4 + 5 * 8), None
    return None, None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=["c1", "c2"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path has no multi-GPU mode",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from inputs import freestream_prim, mesh_for_config, perturbed_state, uniform_state
    from paper_2304_09485_amd import hgks

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)

    if args.config == "c2":
        mesh = mesh_for_config("c2")
        mach, kinds, opts = 0.5, {1: hgks.SLIP_WALL, 2: hgks.FARFIELD}, dict(scheme=hgks.HWENO)
        workload = "sphere shell, inviscid Mach 0.5, compact HWENO, 202,752 tets, FP64 implicit steps"
    else:
        mesh = mesh_for_config("c1")
        mach, kinds, opts = 0.3, {t: hgks.FARFIELD for t in range(1, 7)}, dict(scheme=hgks.WENO)
        workload = "unit cube, Euler Mach 0.3, non-compact WENO, 3,072 tets, FP64 implicit steps"
    prim = freestream_prim(mach)
    t0 = time.time()
    s = hgks.Solver(mesh, kinds, prim, **opts)
    t_setup = time.time() - t0
    N, F = s.N, s.F
    Nb = len(mesh.bfaces)
    if args.config == "c2":
        Q0 = uniform_state(N, prim)
        s.set_state(Q0, np.zeros((15, N)))
    else:
        s.set_state(perturbed_state(N, prim, seed=1))

    for _ in range(args.warmup):
        s.implicit_step()
    torch.cuda.synchronize()
    s.kernel_times()  # enables per-launch event timing and resets it
    evals = 0
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = s.implicit_step()
        evals += info.n_resid_evals
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = s.kernel_times()
    n_launch = int(kt.pop("evaluations"))
    value = N * evals / elapsed / 1e6

    # roofline of the dominant kernel
    dom = max(kt, key=kt.get)
    scheme = opts.get("scheme", 0)
    flops_tab = {}
    if os.path.exists(FLOPS_FILE):
        with open(FLOPS_FILE) as f:
            flops_tab = json.load(f)
    roof = None
    avg_s = kt[dom] * 1e-3
    if dom == "flux" and flops_tab:
        key = "euler"
        per_gp = flops_tab[key]
        fl = per_gp * 3 * F
        ach = fl / avg_s / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP64_VALU / 1e12,
                "unit": "TFLOP/s", "frac": round(ach / (PEAK_FP64_VALU / 1e12), 4), "traffic": None,
                "avg_ms": round(kt[dom], 4), "launches": n_launch,
                "units_per_launch": f"{3 * F} Gauss points x {per_gp} FP64 flop"}
    else:
        b, _ = algorithmic_units(dom, N, F, Nb, scheme)
        if b is not None:
            ach = b / avg_s / 1e9
            roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None, "avg_ms": round(kt[dom], 4),
                    "launches": n_launch}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(mesh, kinds, prim, opts, args.cpu_seconds)

    out = {
        "metric": "Mcell-residual evals/s",
        "value": round(value, 3),
        "unit": "Mcell-residual/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "cells": N, "faces": F, "resid_evals_per_step": evals // args.steps,
                   "cfl": 10.0, "krylov_dim": 10, "restarts": 3, "jacobi_sweeps": 2},
        "roofline": roof,
        "kernel_ms": {k: round(v, 4) for k, v in kt.items()},
        "cpu_baseline": cpu,
        "res_first_last": [infos[0].res, infos[-1].res],
        "setup_s": round(t_setup, 2),
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(mesh, kinds, prim, opts, budget_s):
    """The oracle as it stands, timed on the host cores on a bounded sample:
    full residual evaluations of the same mesh and state, as many as fit the
    time budget (at least one)."""
    try:
        import oracle
    except Exception as e:  # pragma: no cover
        return {"error": str(e)}
    from inputs import uniform_state
    oracle.build(force=False)
    cores = min(os.cpu_count() or 1, 16)
    oracle.set_threads(cores)
    o = oracle.Oracle(mesh, kinds, prim, **{k: v for k, v in opts.items()})
    N = o.N
    Q = uniform_state(N, prim)
    G = np.zeros((15, N))
    n = 0
    t0 = time.perf_counter()
    while True:
        o.residual(Q, G=G, want_grad=opts.get("scheme", 0) == 1)
        n += 1
        if time.perf_counter() - t0 >= budget_s or n >= 50:
            break
    el = time.perf_counter() - t0
    return {"value": round(N * n / el / 1e6, 5), "unit": "Mcell-residual/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} full residual evaluation(s) of the same {N}-tet mesh and state, {el:.1f} s"}


if __name__ == "__main__":
    main()
