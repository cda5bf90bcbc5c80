#!/usr/bin/env python3
"""Benchmark: implicit steps of the implicit high-order gas-kinetic scheme on one MI355X.

Workload (default, --config c4): inviscid Mach 2 flow in a 3D channel (3 x 2 x 1)
with a 15-degree compression ramp (from x = 1 to 1.5, flat after it), 192 x 72 x
48 sheared hexahedra x 6 = 3,981,312 jittered tets, supersonic inflow and
outflow, slip walls, non-compact WENO
with nonlinear weights, CFL 10, GMRES(10) x 3 restarts on FD
Jacobian-vector products, 2 Jacobi sweeps, FP64.  From the uniform free
stream the plain update reaches a non-physical state in the first step (at
the corner of the ramp, the outlet and a side wall, even at CFL 1), so each
cell's update is limited to a 20 % change of density and pressure
(max_update 0.2, a runtime policy; steady states are unchanged).  One timed
"step" is one implicit step: the base residual, 32 FD Jacobian-vector
products (each a full residual evaluation), Jacobi sweeps, MGS Arnoldi, the
GMRES rotations and solve on the device, the (limited) update.

Other workloads: c1 (unit cube, 3,072 tets, Euler Mach 0.3, WENO), c2 (sphere
shell, 202,752 tets, Euler Mach 0.5, compact HWENO), c3 (boundary-layer
sphere shell, 995,328 tets, NS Mach 0.25 Re 118 Pr 0.72, WENO, update limit).

Prints one JSON line: metric/value (Mcell-residual evaluations per second over
the timed steps), the residual evaluation's roofline (method bytes of the
scheme per cell over the five residual kernels' per-launch HIP event times,
recorded inside the timed region on the context's stream), per-kernel rates,
secondary workloads, times to a 1e-8 drop, variants, and the CPU oracle
baseline on a bounded sample.
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

# FP64 operations of the gas-kinetic flux per Gauss point, counted by running
# the flux function on the host with an operation-counting scalar type
# (csrc/flopcount.cpp, run by the build); a flux launch covers 3 F points
FLOPS_FILE = os.path.join(ROOT, "paper_2304_09485_amd", "flux_flops.json")
# measured HBM traffic per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# calibrated against a plain copy), per workload, with the hash of the kernel
# sources the counters were taken with
TRAFFIC_FILES = {"c2": os.path.join(ROOT, "profiles", "hbm_traffic_c2_hweno.md"),
                 "c4": os.path.join(ROOT, "profiles", "hbm_traffic_c4_weno.md")}
KERNEL_SOURCES = ["hgks_kernels.hip", "side_kernel.h", "gks_flux.h", "hgks_device.h",
                  "hgks_kernels.h"]

# the workloads (boundary kinds: 0 far field, 1 slip wall, 2 no-slip
# adiabatic wall, 3 supersonic inflow, 4 supersonic outflow)
WORKLOADS = {
    "c1": dict(mach=0.3, kinds={t: 0 for t in range(1, 7)}, opts=dict(scheme=0), start="perturbed", ramp=None,
               desc="unit cube, Euler Mach 0.3, non-compact WENO, 3,072 tets, FP64 implicit steps"),
    "c2": dict(mach=0.5, kinds={1: 1, 2: 0}, opts=dict(scheme=1), start="uniform", ramp=None,
               desc="sphere shell, inviscid Mach 0.5, compact HWENO, 202,752 tets, FP64 implicit steps"),
    "c3": dict(mach=0.25, kinds={1: 2, 2: 0}, opts=dict(scheme=0, physics=1, mu=0.25 / 118.0, prandtl=0.72,
                                                       max_update=0.2),
               start="uniform", ramp=None,
               desc="boundary-layer sphere shell, NS Mach 0.25 Re 118 Pr 0.72, non-compact WENO, 995,328 tets, "
                    "FP64 implicit steps (update limit 0.2)"),
    "c4": dict(mach=2.0, kinds={1: 3, 2: 4, 3: 1, 4: 1, 5: 1, 6: 1}, opts=dict(scheme=0, max_update=0.2),
               start="uniform", ramp=None,
               desc="15-degree compression ramp in a 3 x 2 x 1 channel, Euler Mach 2, non-compact WENO, "
                    "3,981,312 tets, FP64 implicit steps (update limit 0.2)"),
}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2304_09485_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(workload, kernel):
    """HBM bytes per launch of the kernel on the workload as measured by the
    counters, or None if none were taken or the kernel sources changed since."""
    path = TRAFFIC_FILES.get(workload)
    if not path or not os.path.exists(path):
        return None
    want = kernel_source_hash()
    with open(path) as f:
        for line in f:
            p = line.split()
            # lines "traffic <kernel> <bytes per launch> <source hash>"
            if len(p) == 4 and p[0] == "traffic" and p[1] == kernel and p[3] == want:
                return int(float(p[2]))
    return None


SQ_FILES = {"c4": os.path.join(ROOT, "profiles", "sq_issue_c4_weno.md")}


def valu_for(workload, kernel):
    """FP64 rate, fraction of the FP64 vector peak and VALU-issuing share of
    the kernel from the SQ instruction counters (rocprofv3), or None if none
    were taken or the kernel sources changed since."""
    path = SQ_FILES.get(workload)
    if not path or not os.path.exists(path):
        return None
    want = kernel_source_hash()
    with open(path) as f:
        for line in f:
            p = line.split()
            # lines "valu <kernel> <FP64 TFLOP/s> <fraction of peak> <issue share> <source hash>"
            if len(p) == 6 and p[0] == "valu" and p[1] == kernel and p[5] == want:
                return {"fp64_TFLOP/s": float(p[2]), "fp64_frac": float(p[3]), "valu_issue_share": float(p[4]),
                        "source": "SQ counters"}
    return None


def method_bytes_per_cell(scheme, jv):
    """Bytes per cell one residual evaluation of the method must move at
    least (stored-operator design, FP64, a cell's data read once and its
    results written once): the state (and for an FD product the direction v),
    the residual written (and the base residual read by the FD epilogue), the
    stencil indices, the stored reconstruction operators, the cell geometry
    (centroid, 9 basis means, volume, 6 second moments), about two faces per
    cell (ids, normal, area, Gauss points), the time step; the compact scheme
    adds its frozen gradients and, on the base evaluation only, the gradient
    update written."""
    q = 40 + (40 if jv else 0)
    r = 40 + (40 if jv else 0)
    if scheme == 1:
        idx, ops, grad = 16, 1368 + 160, 120 + (0 if jv else 120)
    else:
        idx, ops, grad = 64, 1728, 0
    return q + r + idx + ops + 152 + 224 + 8 + grad


def step_method_bytes(scheme, N, evals_per_step):
    """Method bytes of one implicit step's residual evaluations (the base
    evaluation and evals_per_step - 1 FD products), per evaluation."""
    if evals_per_step <= 1:
        return N * method_bytes_per_cell(scheme, False)
    return N * (method_bytes_per_cell(scheme, False)
                + (evals_per_step - 1) * method_bytes_per_cell(scheme, True)) / evals_per_step


def algorithmic_bytes(kernel, N, F, Nb, scheme):
    """Bytes a launch of the kernel must move at least: every array it needs
    read once and every result written once (re-reads of a cell's data by its
    neighbours or its faces are not counted)."""
    NX = N + Nb
    sides = 2 * F - Nb
    if kernel == "recon":
        if scheme == 1:
            # CLS operator 9x19 + closed-form sub-stencil data 24 per cell, 4
            # neighbour ids, state and gradients (20 values per cell incl.
            # ghosts) read once, 105 coefficients written
            return N * (8 * (171 + 24) + 4 * 4 + 8 * 105) + NX * 8 * 20
        # WENO: LS operators 9x16 + 4x3x6, 16 + 24 stencil ids, sub-stencil mask
        return N * (8 * (144 + 72) + 4 * (16 + 24) + 1 + 8 * 105) + NX * 8 * 5
    if kernel == "side":
        # 105 coefficients, 6 second moments and h per cell; the state per
        # cell; per face normal, 2 x 9 Gauss-point offsets and the two cell
        # ids; 60 values written per reconstructed side
        return N * 8 * (105 + 7) + NX * 8 * 5 + F * (8 * 21 + 8) + sides * 8 * 60
    if kernel == "flux" and scheme == 2:
        # first-order KFVS: per face the two cell ids, normal, area, the
        # boundary kind of boundary faces, 5 values written; each cell's state
        # read once
        return F * (8 + 24 + 8 + 40) + Nb * 4 + N * 40
    if kernel == "lusgs_sweep":
        # one sweep over all colour classes: per cell 4 face ids, 4
        # neighbour ids, colour, order slot, diagonal, state, right-hand
        # side, its own and (once) its neighbours' unknowns, 5 values
        # written; per face normal, area and spectral radius
        return N * (16 + 16 + 4 + 4 + 8 + 40 + 40 + 40 + 40) + F * 40
    if kernel == "flux":
        # 60 side values per reconstructed side read; per face the two cell
        # ids, the two cells' time steps, 5 face-flux values written (the
        # base evaluation of the compact scheme, 1 launch in 33, also writes
        # 5 point-value sums: not counted)
        return sides * 8 * 60 + F * (8 + 8 * 2 + 8 * 5)
    if kernel == "gather":
        # per cell 4 face ids, 4 face fluxes (5 values) read, 5 values written
        return N * (4 * 4 + 4 * 5 * 8 + 5 * 8)
    if kernel == "ghost":
        return Nb * (8 * 5 * 2 + 8 * 3 + 8)
    return None


def flux_flops_per_launch(flops_tab, F, scheme, physics, evals_per_step):
    """FP64 operations of the gas-kinetic flux per launch, averaged over one
    implicit step: the base evaluation of the compact scheme also evaluates the
    point value Q_G of the gradient update, the FD products do not."""
    if not flops_tab:
        return None
    per = flops_tab["ns" if physics == 1 else "euler"]
    if scheme == 1 and physics == 0:
        per = (flops_tab["euler_qg"] + (evals_per_step - 1) * per) / evals_per_step
    return per * 3 * F


def _solver_for(hgks, name, mesh=None, **extra):
    """Context, mesh and free stream of a workload with its start state set."""
    from inputs import freestream_prim, mesh_for_config, perturbed_state, uniform_state
    w = WORKLOADS[name]
    mesh = mesh if mesh is not None else mesh_for_config(name)
    prim = freestream_prim(w["mach"])
    opts = dict(w["opts"])
    if w["ramp"]:
        opts.update(cfl_start=w["ramp"][0], cfl_growth=w["ramp"][1])
    opts.update(extra)
    t0 = time.time()
    s = hgks.Solver(mesh, w["kinds"], prim, **opts)
    t_setup = time.time() - t0
    if w["start"] == "perturbed":
        s.set_state(perturbed_state(s.N, prim, seed=1))
    else:
        s.set_state(uniform_state(s.N, prim), np.zeros((15, s.N)) if opts.get("scheme") == 1 else None)
    return s, mesh, prim, opts, t_setup


def _cfl_after(opts, steps):
    """CFL number after `steps` steps of the solve_steady ramp."""
    cfl = opts.get("cfl", 10.0)
    if not opts.get("cfl_start"):
        return cfl
    return min(cfl, opts["cfl_start"] * max(1.0, opts.get("cfl_growth", 1.5)) ** steps)


def measure_steps(torch, hgks, name, steps, warmup, mesh=None, chain=True):
    """Throughput of `steps` implicit steps after `warmup` (the warm-up runs
    the workload's CFL ramp through solve_steady), per-launch times of the
    residual kernels inside the timed region, the residual evaluation's
    roofline, and the isolated residual chain."""
    s, mesh, prim, opts, t_setup = _solver_for(hgks, name, mesh=mesh)
    N, F = s.N, s.F
    Nb = len(mesh.bfaces)
    scheme = opts.get("scheme", 0)
    physics = opts.get("physics", 0)
    if warmup > 0:
        if WORKLOADS[name]["ramp"]:
            s.solve_steady(drop=1e-30, max_steps=warmup)
        else:
            for _ in range(warmup):
                s.implicit_step()
    torch.cuda.synchronize()
    s.kernel_times()  # enables per-launch event timing and resets it
    evals = 0
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = s.implicit_step()
        evals += info.n_resid_evals
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = s.kernel_times()
    n_launch = int(kt.pop("evaluations"))
    evals_per_step = evals // steps
    flops_tab = {}
    if os.path.exists(FLOPS_FILE):
        with open(FLOPS_FILE) as f:
            flops_tab = json.load(f)
    kernels = {}
    for k, ms in kt.items():
        e = {"avg_ms": round(ms, 4)}
        b = algorithmic_bytes(k, N, F, Nb, scheme)
        if b is not None and ms > 0:
            # the bytes of the kernel's own inputs and outputs (intermediate
            # buffers of the five-kernel split included)
            e["buffer_bytes"] = int(b)
            e["buffer_GB/s"] = round(b / (ms * 1e-3) / 1e9, 1)
        tr = traffic_for(name, k)
        if tr is not None:
            e["traffic"] = tr
        sq = valu_for(name, k)
        if sq is not None:
            e["sq"] = sq
        if k == "flux":
            fl = flux_flops_per_launch(flops_tab, F, scheme, physics, evals_per_step)
            if fl is not None and ms > 0:
                e["flop"] = int(fl)
                e["TFLOP/s"] = round(fl / (ms * 1e-3) / 1e12, 2)
                e["valu_frac"] = round(fl / (ms * 1e-3) / PEAK_FP64_VALU, 4)
        kernels[k] = e
    # the residual evaluation as a whole: method bytes of the scheme per cell
    # over the summed per-launch times of its five kernels
    res_ms = sum(kt.values())
    mb = step_method_bytes(scheme, N, evals_per_step)
    traffic = None
    if all("traffic" in kernels.get(k, {}) for k in ("ghost", "recon", "side", "flux", "gather")):
        traffic = int(sum(kernels[k]["traffic"] for k in ("ghost", "recon", "side", "flux", "gather")))
    roof = {"kernel": "residual evaluation (ghost, recon, side, flux, gather kernels)", "bound": "hbm",
            "achieved": round(mb / (res_ms * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(mb / (res_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4), "traffic": traffic,
            "avg_ms": round(res_ms, 4), "launches": n_launch,
            "per_launch": f"{int(mb)} method bytes per evaluation ({mb / N:.0f} B/cell x {N} cells)"}
    if "flop" in kernels.get("flux", {}):
        roof["flux_fp64_frac"] = kernels["flux"]["valu_frac"]
    if "sq" in kernels.get("side", {}):
        # the side kernel's own method bytes are small: its binding roof is
        # the FP64 vector rate, measured by the instruction counters
        roof["side_fp64_frac"] = kernels["side"]["sq"]["fp64_frac"]
    out = {"value": round(N * evals / elapsed / 1e6, 3), "ms_per_step": round(1e3 * elapsed / steps, 3),
           "steps": steps, "warmup": warmup, "cells": N, "faces": F, "resid_evals_per_step": evals_per_step,
           "cfl": round(_cfl_after(opts, warmup), 3), "roofline": roof, "kernels": kernels,
           "res_first_last": [infos[0].res, infos[-1].res], "setup_s": round(t_setup, 2)}
    if chain:
        out["residual_chain"] = residual_chain(torch, s, N)
    s.close()
    return out, mesh, prim, opts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-secondary", action="store_true", help="skip the other workloads")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-1e-8 solves and the variants")
    ap.add_argument("--solve-steps", type=int, default=400, help="step cap of each time-to-1e-8 solve")
    ap.add_argument("--drop-steps", type=int, default=400,
                    help="step cap of the headline workload's own runs towards a 1e-8 drop")
    ap.add_argument("--serving", action="store_true",
                    help="run the served request stream instead of the implicit-step throughput")
    ap.add_argument("--requests", type=int, default=64, help="served requests")
    ap.add_argument("--rate", type=float, default=0.5, help="request arrival rate (1/s)")
    ap.add_argument("--max-cells", type=int, default=2_000_000, help="largest request (cells)")
    ap.add_argument("--max-steps", type=int, default=200, help="step cap of a served solve")
    ap.add_argument("--slots", type=int, default=8, help="concurrently admitted requests")
    ap.add_argument("--fp64-serving", action="store_true",
                    help="serve the plain FP64 form (default: FP32 inner / FP64 outer)")
    ap.add_argument("--variants-only", action="store_true",
                    help="only measure the first-order KFVS and LU-SGS variants on the 202,752-tet shell")
    ap.add_argument("--lusgs-steps", type=int, default=2000, help="step cap of the LU-SGS convergence run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path has no multi-GPU mode",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from inputs import mesh_for_config
    from paper_2304_09485_amd import hgks

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration(torch)
        return
    if args.serving:
        serving_bench(hgks, args)
        return
    if args.variants_only:
        mesh = mesh_for_config("c2")
        print(json.dumps({"variants": variants_bench(hgks, mesh, len(mesh.bfaces), args.lusgs_steps)}), flush=True)
        return

    name = args.config
    w = WORKLOADS[name]
    print(f"# {name}: {w['desc']}", file=sys.stderr, flush=True)
    head, mesh, prim, opts = measure_steps(torch, hgks, name, args.steps, args.warmup)
    print(f"# {name}: {head['value']} Mcell-residual/s, {head['ms_per_step']} ms per step", file=sys.stderr,
          flush=True)

    secondary = {}
    if not args.no_secondary:
        for other in ("c2", "c3"):
            if other == name:
                continue
            try:
                r, _, _, _ = measure_steps(torch, hgks, other, steps=5, warmup=2)
                r["workload"] = WORKLOADS[other]["desc"]
                secondary[other] = r
            except Exception as e:  # a workload that fails is reported, not fatal
                secondary[other] = {"error": str(e)}
            print(f"# secondary {other}: {secondary[other].get('value', secondary[other])}", file=sys.stderr,
                  flush=True)

    solves = None
    variants = None
    if not args.no_solve:
        c2mesh = mesh_for_config("c2") if name != "c2" else mesh
        from inputs import freestream_prim
        solves = time_to_drop(hgks, c2mesh, WORKLOADS["c2"]["kinds"], freestream_prim(WORKLOADS["c2"]["mach"]),
                              args.solve_steps)
        if name in ("c3", "c4"):
            solves += drop_runs(hgks, name, mesh, args.drop_steps)
        variants = variants_bench(hgks, c2mesh, len(c2mesh.bfaces), args.lusgs_steps)

    served = None
    if not args.no_solve:
        # the request stream's first 8 arrivals, meshes up to 200k cells, 120
        # steps at most: a short served run for the record (the full stream is
        # bench.py --serving)
        served = serve_stream(hgks, 8, args.rate, 200_000, 120, args.slots)
        served.pop("per_request", None)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(mesh, w["kinds"], prim, w["opts"], args.cpu_seconds)

    out = {
        "metric": "Mcell-residual evals/s",
        "value": head["value"],
        "unit": "Mcell-residual/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["desc"], "cells": head["cells"], "faces": head["faces"],
                   "resid_evals_per_step": head["resid_evals_per_step"], "cfl": head["cfl"],
                   "cfl_ramp": (f"from {w['ramp'][0]} x{w['ramp'][1]} per step over the warm-up steps, then held"
                                if w["ramp"] else None),
                   "max_update": w["opts"].get("max_update", 0.0),
                   "krylov_dim": 10, "restarts": 3, "jacobi_sweeps": 2},
        "roofline": head["roofline"],
        "kernels": head["kernels"],
        "residual_chain": head.get("residual_chain"),
        "secondary": secondary,
        "cpu_baseline": cpu,
        "time_to_1e-8": solves,
        "variants": variants,
        "serving_short": served,
        "res_first_last": head["res_first_last"],
        "setup_s": head["setup_s"],
    }
    print(json.dumps(out), flush=True)


def serving_bench(hgks, args):
    """The served request stream (--serving): prints its JSON line."""
    out = serve_stream(hgks, args.requests, args.rate, args.max_cells, args.max_steps, args.slots,
                       fp64=args.fp64_serving)
    print(json.dumps(out), flush=True)


def serve_stream(hgks, n_requests, rate, max_cells, max_steps, slots, fp64=False):
    """The served request stream: seeded requests (sphere shell or ramp
    channel, log-uniform cell counts, Mach 0.2-2, Euler or NS) arrive as a
    Poisson process and are submitted to the server as they arrive; each is
    solved from the free stream towards a 1e-8 residual drop (or the step
    cap) with the update limit of impulsive starts.  Reports time-to-steady
    percentiles (arrival to result), the fraction converged and throughput
    over the makespan.  Meshes are generated before the clock starts (the
    client side of a request)."""
    from inputs import freestream_prim
    from inputs.requests import request_stream
    specs = request_stream(n_requests, rate, seed=5, n_max=max_cells)
    meshes = [sp.mesh() for sp in specs]
    prec = hgks.FP64 if fp64 else hgks.FP32_INNER
    budget = 200 << 30  # leave headroom of the 288 GB for the runtime
    srv = hgks.Server(budget, slots)
    t0 = time.perf_counter()
    tickets = []
    for sp, m in zip(specs, meshes):
        delay = sp.arrival_s - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        # impulsive starts (supersonic ramps, no-slip walls): each cell's
        # update is limited to a 20 % change of density and pressure
        opts = dict(scheme=hgks.WENO, precision=prec, max_update=0.2)
        if sp.viscous:
            opts.update(physics=hgks.NS, mu=sp.mach / sp.reynolds, prandtl=0.72)
        tickets.append(srv.submit(m, sp.boundary_kinds(), freestream_prim(sp.mach), drop=1e-8,
                                  max_steps=max_steps, **opts))
        print(f"# submitted request {sp.index}: {sp.kind} {m.n_cells} cells Mach {sp.mach:.2f} "
              f"{'NS' if sp.viscous else 'Euler'} at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    # results in the order they finish; between them, a line per 500
    # implicit steps the server has completed over all requests
    res = [None] * len(tickets)
    pending = set(range(len(tickets)))
    next_report = 500
    while pending:
        for k in sorted(pending):
            r = srv.poll(tickets[k])
            if r is None:
                continue
            res[k] = r
            pending.discard(k)
            print(f"# request {specs[k].index}: status {r.status} steps {r.steps} "
                  f"drop {r.res_final / max(r.res0, 1e-300):.2e} queue {r.t_queue_ms:.0f} ms "
                  f"total {r.t_total_ms:.0f} ms", file=sys.stderr, flush=True)
        steps = srv.stats().steps_done
        if steps >= next_report:
            print(f"# {steps} implicit steps done, {len(pending)} requests pending at "
                  f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
            next_report = (steps // 500 + 1) * 500
        if pending:
            time.sleep(0.2)
    makespan = time.perf_counter() - t0
    srv.close()
    lat = np.array([r.t_total_ms for r in res]) * 1e-3
    conv = [r.status == 0 for r in res]
    cell_evals = sum(r.n_cells * r.n_resid_evals for r in res)
    kinds = {}
    for sp, r in zip(specs, res):
        key = f"{sp.kind}, {'NS' if sp.viscous else 'Euler'}, {'supersonic' if sp.mach > 1 else 'subsonic'}"
        k = kinds.setdefault(key, {"requests": 0, "converged": 0})
        k["requests"] += 1
        k["converged"] += int(r.status == 0)
    return {
        "metric": "p50/p99 solve latency (served stream)",
        "value": round(float(np.percentile(lat, 50)), 3),
        "unit": "s",
        "p99_s": round(float(np.percentile(lat, 99)), 3),
        "n_gpus": 1,
        "higher_is_better": False,
        "throughput": {"Mcell-residual/s": round(cell_evals / makespan / 1e6, 3),
                       "solves/s": round(len(res) / makespan, 4), "makespan_s": round(makespan, 2)},
        "requests": len(res), "converged": int(sum(conv)), "by_kind": kinds,
        "dtype": "f64" if fp64 else "f32 inner / f64 outer",
        "data": "synthetic",
        "config": {"workload": f"{len(res)} Poisson requests at {rate}/s, shell or ramp tet meshes of "
                               f"50k-{max_cells // 1000}k cells, Mach 0.2-2, Euler or NS, WENO, drop 1e-8, "
                               f"cap {max_steps} steps, update limit 0.2", "slots": slots},
        "per_request": [{"cells": r.n_cells, "status": r.status, "steps": r.steps,
                         "drop": r.res_final / max(r.res0, 1e-300), "t_total_s": round(r.t_total_ms * 1e-3, 3),
                         "t_queue_s": round(r.t_queue_ms * 1e-3, 3)} for r in res],
    }


def time_to_drop(hgks, mesh, kinds, prim, max_steps):
    """Wall time of solve_steady from a uniform free-stream start to a 1e-8
    drop of the density residual, per form, on the same mesh (context set-up
    reported apart).  A form that has not reached the drop after max_steps
    (the relaxed compact form: 1,600 steps, about 1,250 on the shell)
    reports the drop it reached."""
    from inputs import uniform_state
    forms = [("non-compact WENO, FP64", dict(scheme=hgks.WENO), max_steps),
             ("non-compact WENO, FP32 inner / FP64 outer", dict(scheme=hgks.WENO, precision=hgks.FP32_INNER),
              max_steps),
             ("non-compact WENO, linear weights, FP64", dict(scheme=hgks.WENO, weights=hgks.WEIGHTS_LINEAR),
              max_steps),
             ("non-compact WENO, linear weights, FP32 inner / FP64 outer",
              dict(scheme=hgks.WENO, weights=hgks.WEIGHTS_LINEAR, precision=hgks.FP32_INNER), max_steps),
             ("compact HWENO, FP64", dict(scheme=hgks.HWENO), max_steps),
             ("compact HWENO, gradient update relaxed (omega 0.8), FP64", dict(scheme=hgks.HWENO, grad_relax=0.8),
              max(max_steps, 1600))]
    out = []
    for name, opts, cap in forms:
        t0 = time.perf_counter()
        s = hgks.Solver(mesh, kinds, prim, **opts)
        t_setup = time.perf_counter() - t0
        s.set_state(uniform_state(s.N, prim), np.zeros((15, s.N)) if opts["scheme"] == hgks.HWENO else None)
        info = s.solve_steady(drop=1e-8, max_steps=cap)
        out.append({"form": name, "seconds": round(info.t_ms * 1e-3, 3), "steps": info.steps,
                    "converged": bool(info.converged), "drop": info.drop, "setup_s": round(t_setup, 2)})
        s.close()
        print(f"# time to 1e-8: {out[-1]}", file=sys.stderr, flush=True)
    return out


def drop_runs(hgks, name, mesh, max_steps):
    """The workload's own solve from the uniform free stream (with its
    options: update limit, CFL ramp) towards a 1e-8 drop, plain FP64 and FP32
    inner / FP64 outer, capped at max_steps: the drop reached, or the error
    that stopped it."""
    out = []
    for form, extra in (("FP64", {}), ("FP32 inner / FP64 outer", {"precision": hgks.FP32_INNER})):
        s, _, _, opts, t_setup = _solver_for(hgks, name, mesh=mesh, **extra)
        t0 = time.perf_counter()
        rec = {"form": f"{WORKLOADS[name]['desc'].split(', FP64')[0]}, {form}", "setup_s": round(t_setup, 2)}
        try:
            info = s.solve_steady(drop=1e-8, max_steps=max_steps)
            rec.update(seconds=round(info.t_ms * 1e-3, 3), steps=info.steps, converged=bool(info.converged),
                       drop=info.drop)
        except hgks.HgksError as e:
            rec.update(seconds=round(time.perf_counter() - t0, 3), converged=False, error=str(e))
        s.close()
        out.append(rec)
        print(f"# {name} towards 1e-8: {rec}", file=sys.stderr, flush=True)
    return out


def _rate(kernel, ms, N, F, Nb, scheme):
    b = algorithmic_bytes(kernel, N, F, Nb, scheme)
    return {"avg_ms": round(ms, 4), "bytes": int(b), "GB/s": round(b / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(b / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}


def variants_bench(hgks, mesh, Nb, lusgs_steps):
    """The first-order KFVS scheme on the supersonic sphere (Mach 3, the
    retest of Sec. 5), the LU-SGS comparison solver on the benchmark shell,
    and the hexahedral shell: per-step time, kernel rates, convergence."""
    from inputs import freestream_prim, uniform_state
    out = {}
    kinds = {1: hgks.SLIP_WALL, 2: hgks.FARFIELD}
    # KFVS, GMRES on FD products: kernel rate over 20 steps at CFL 10
    prim3 = freestream_prim(3.0)
    s = hgks.Solver(mesh, kinds, prim3, scheme=hgks.KFVS1, cfl=10.0)
    N, F = s.N, s.F
    s.set_state(uniform_state(N, prim3))
    s.implicit_step()
    s.kernel_times()
    t0 = time.perf_counter()
    for _ in range(20):
        s.implicit_step()
    ms_step = 1e3 * (time.perf_counter() - t0) / 20
    kt = s.kernel_times()
    s.close()
    ramp = []
    for cmax in (10.0, 200.0):
        s = hgks.Solver(mesh, kinds, prim3, scheme=hgks.KFVS1, cfl=cmax, cfl_start=min(5.0, cmax), cfl_growth=1.3)
        s.set_state(uniform_state(N, prim3))
        info = s.solve_steady(drop=1e-10, max_steps=400)
        ramp.append({"cfl": cmax, "cfl_start": min(5.0, cmax), "steps": info.steps, "drop": info.drop,
                     "converged": bool(info.converged), "seconds": round(info.t_ms * 1e-3, 3)})
        s.close()
    out["kfvs_mach3"] = {"ms_per_step": round(ms_step, 3), "flux_kfvs": _rate("flux", kt["flux"], N, F, Nb, 2),
                         "gather_ms": round(kt["gather"], 4), "time_to_1e-10": ramp}
    print(f"# KFVS Mach 3: {out['kfvs_mach3']}", file=sys.stderr, flush=True)
    # LU-SGS, non-compact WENO, Mach 0.5: step time and the drop after lusgs_steps steps
    prim = freestream_prim(0.5)
    s = hgks.Solver(mesh, kinds, prim, scheme=hgks.WENO, solver=hgks.SOLVER_LUSGS, cfl=10.0)
    s.set_state(uniform_state(N, prim))
    s.implicit_step()
    s.kernel_times()
    t0 = time.perf_counter()
    for _ in range(50):
        s.implicit_step()
    ms_step = 1e3 * (time.perf_counter() - t0) / 50
    kt = s.kernel_times()
    resid_ms = sum(v for k, v in kt.items() if k != "evaluations")
    s.close()
    s = hgks.Solver(mesh, kinds, prim, scheme=hgks.WENO, solver=hgks.SOLVER_LUSGS, cfl=10.0)
    s.set_state(uniform_state(N, prim))
    info = s.solve_steady(drop=1e-8, max_steps=lusgs_steps)
    s.close()
    out["lusgs_weno"] = {"ms_per_step": round(ms_step, 3), "residual_ms": round(resid_ms, 3),
                         "sweeps_and_update_ms": round(ms_step - resid_ms, 3), "steps": info.steps,
                         "drop": info.drop, "seconds": round(info.t_ms * 1e-3, 3),
                         "sweep_bytes": int(algorithmic_bytes("lusgs_sweep", N, F, Nb, 0))}
    print(f"# LU-SGS WENO: {out['lusgs_weno']}", file=sys.stderr, flush=True)
    # hexahedra: the benchmark shell's cubed-sphere layout without the
    # tetrahedral split (32 x 32 cells per patch, 22 layers, 135,168 hexes)
    from inputs import shell_mesh
    hm = shell_mesh(32, 22, grading=1.1, jitter=0.02, seed=2, hexahedra=True)
    hexres = {"cells": hm.n_cells}
    for name, sch in (("hweno", hgks.HWENO), ("weno", hgks.WENO)):
        s = hgks.Solver(hm, kinds, prim, scheme=sch)
        s.set_state(uniform_state(s.N, prim), np.zeros((15, s.N)) if sch == hgks.HWENO else None)
        s.implicit_step()
        s.kernel_times()
        t0 = time.perf_counter()
        ev = 0
        for _ in range(5):
            ev += s.implicit_step().n_resid_evals
        el = time.perf_counter() - t0
        kt = s.kernel_times()
        s.close()
        e = {"ms_per_step": round(1e3 * el / 5, 3), "Mcell_resid_per_s": round(hm.n_cells * ev / el / 1e6, 2),
             "kernel_ms": {k: round(v, 4) for k, v in kt.items() if k != "evaluations"}}
        # compact HWENO on FD products; non-compact WENO on the paper's
        # approximate-matrix operator
        opts = dict(scheme=sch) if sch == hgks.HWENO else dict(scheme=sch, jv_mode=hgks.JV_APPROX)
        s = hgks.Solver(hm, kinds, prim, **opts)
        s.set_state(uniform_state(s.N, prim), np.zeros((15, s.N)) if sch == hgks.HWENO else None)
        info = s.solve_steady(drop=1e-8, max_steps=500)
        s.close()
        e["time_to_1e-8"] = {"operator": "FD" if sch == hgks.HWENO else "approximate matrix", "steps": info.steps,
                             "drop": info.drop, "converged": bool(info.converged),
                             "seconds": round(info.t_ms * 1e-3, 3)}
        hexres[name] = e
    out["hex_shell_m05"] = hexres
    print(f"# hexahedra: {hexres}", file=sys.stderr, flush=True)
    return out


def copy_calibration(torch):
    """A plain device copy of known size (1 GiB read, 1 GiB written), three
    times: the HBM counters of these dispatches calibrate the counters of the
    residual kernels."""
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "copies": 3}), flush=True)


def residual_chain(torch, s, N, reps=25, warm=3):
    """The residual kernel chain on its own (state expansion, ghost cells,
    time steps, reconstruction, side values, flux, gather), outside any
    solve: each call is bracketed by HIP events on the stream it is queued
    on; the median over the timed calls gives the rate."""
    Q = torch.from_numpy(np.ascontiguousarray(s.get_state())).to("cuda")
    R = torch.empty_like(Q)
    st = torch.cuda.Stream()
    for _ in range(warm):
        s.residual_dev(Q, R, st.cuda_stream)
    st.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(st)
        s.residual_dev(Q, R, st.cuda_stream)
        b.record(st)
    st.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    med = float(np.median(ms))
    return {"median_ms": round(med, 4), "min_ms": round(ms[0], 4), "max_ms": round(ms[-1], 4), "calls": reps,
            "Mcell-residual/s": round(N / (med * 1e-3) / 1e6, 2)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(mesh, kinds, prim, opts, budget_s):
    """The oracle as it stands, timed on the host cores on a bounded sample of
    the same workload: face fluxes (reconstruction of both sides and the
    gas-kinetic flux at the Gauss points, the whole cost of a residual but
    the per-cell sum) of random batches of the mesh's faces, on the perturbed
    state, as many batches as fit the time budget; a full residual evaluates
    every face once, so cell-residuals per second = faces per second x N / F."""
    try:
        import oracle
    except Exception as e:  # pragma: no cover
        return {"error": str(e)}
    from inputs import perturbed_state
    oracle.build(force=False)
    cores = min(os.cpu_count() or 1, 16)
    oracle.set_threads(cores)
    o = oracle.Oracle(mesh, kinds, prim, **{k: v for k, v in opts.items()})
    N, F = o.N, o.F
    Q = perturbed_state(N, prim, amp=0.01, seed=1)
    G = np.zeros((15, N)) if opts.get("scheme", 0) == 1 else None
    dt = o.dt(Q)
    rng = np.random.default_rng(0)
    batch = min(F, 50_000)
    n = 0
    t0 = time.perf_counter()
    while True:
        o.face_fluxes(Q, rng.choice(F, size=batch, replace=False), G=G, dt=dt)
        n += batch
        if time.perf_counter() - t0 >= budget_s or n >= 20 * F:
            break
    el = time.perf_counter() - t0
    oracle.set_threads(1)
    b1 = min(F, 4_000)
    t1 = time.perf_counter()
    o.face_fluxes(Q, rng.choice(F, size=b1, replace=False), G=G, dt=dt)
    el1 = time.perf_counter() - t1
    oracle.set_threads(cores)
    return {"value": round(n / el * N / F / 1e6, 5), "unit": "Mcell-residual/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} face fluxes in random batches of {batch} of the {F} faces of the same {N}-cell mesh "
                      f"(perturbed state), {el:.1f} s; rate = faces/s x N/F",
            "single_thread": {"value": round(b1 / el1 * N / F / 1e6, 5), "cores": 1,
                              "sample": f"{b1} random face fluxes of the same mesh and state, {el1:.1f} s"},
            "host": {"nproc": os.cpu_count(), "cpu_model": cpu_model()}}


if __name__ == "__main__":
    main()
