"""Host logic of bench.py (CPU): the one-GPU guard, the algorithmic byte
counts the roofline uses, the traffic lookup keyed by the kernel sources, and
the forms and step caps of the time-to-1e-8 record."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_algorithmic_bytes():
    import bench
    N, F, Nb = 1000, 2100, 200
    sides = 2 * F - Nb
    # side: 112 doubles per cell, the state incl. ghosts, 21 geometry doubles
    # and 2 ids per face, 60 outputs per reconstructed side
    assert bench.algorithmic_bytes("side", N, F, Nb, 1) == N * 8 * 112 + (N + Nb) * 40 + F * 176 + sides * 480
    assert bench.algorithmic_bytes("flux", N, F, Nb, 1) == sides * 480 + F * 64
    assert bench.algorithmic_bytes("flux", N, F, Nb, 2) == F * 80 + Nb * 4 + N * 40
    assert bench.algorithmic_bytes("gather", N, F, Nb, 0) == N * 216
    assert bench.algorithmic_bytes("nonsense", N, F, Nb, 0) is None


def test_traffic_lookup_follows_the_sources_hash():
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 16
    seen = 0
    for wl, path in bench.TRAFFIC_FILES.items():
        if not os.path.exists(path):
            continue
        with open(path) as f:
            lines = [ln.split() for ln in f if ln.startswith("traffic ")]
        assert lines, f"no traffic lines in {path}"
        for p in lines:
            seen += 1
            if p[3] == h:
                assert bench.traffic_for(wl, p[1]) == int(float(p[2]))
            else:
                assert bench.traffic_for(wl, p[1]) is None
    assert seen > 0
    assert bench.traffic_for("no such workload", "side") is None


def test_method_bytes_follow_the_scheme_table():
    """Per-cell method bytes of one residual evaluation: about 2.26 KB for the
    non-compact scheme and 2.25 KB for the compact base evaluation, 80 B more
    (non-compact) or 40 B less (compact) as an FD product."""
    import bench
    assert bench.method_bytes_per_cell(0, False) == 2256
    assert bench.method_bytes_per_cell(0, True) == 2336
    assert bench.method_bytes_per_cell(1, False) == 2248
    assert bench.method_bytes_per_cell(1, True) == 2208
    # an implicit step of 33 evaluations: the base one and 32 FD products
    assert bench.step_method_bytes(0, 10, 33) == 10 * (2256 + 32 * 2336) / 33


def test_time_to_drop_forms_and_step_caps():
    """The time-to-1e-8 record runs every form on one mesh from the uniform
    stream, the compact forms with zero gradients, each with the common step
    cap except the relaxed compact form (1,600 steps at least), and reports
    each form's solve (a stand-in library records the calls)."""
    import types
    import numpy as np
    import bench
    from inputs import freestream_prim
    calls = []

    class Info:
        steps, converged, drop, t_ms = 7, 1, 5e-9, 12.0

    class Solver:
        def __init__(self, mesh, kinds, prim, **opts):
            self.N, self.opts = 10, opts

        def set_state(self, Q, G=None):
            calls.append(("state", Q.shape, None if G is None else (G.shape, float(np.abs(G).max()))))

        def solve_steady(self, drop, max_steps):
            calls.append(("solve", dict(self.opts), drop, max_steps))
            return Info()

        def close(self):
            pass

    lib = types.SimpleNamespace(WENO=0, HWENO=1, FP32_INNER=1, WEIGHTS_LINEAR=1, Solver=Solver)
    out = bench.time_to_drop(lib, None, {}, freestream_prim(0.5), 400)
    solves = [c for c in calls if c[0] == "solve"]
    states = [c for c in calls if c[0] == "state"]
    assert len(out) == len(solves) == len(states) == 6
    assert all(c[2] == 1e-8 for c in solves)
    for (_, opts, _, cap), (_, qshape, g) in zip(solves, states):
        assert qshape == (5, 10)
        assert (g is not None) == (opts["scheme"] == 1)
        if g is not None:
            assert g == ((15, 10), 0.0)
        assert cap == (1600 if opts.get("grad_relax", 1.0) < 1.0 else 400)
    assert [o["steps"] for o in out] == [7] * 6 and all(o["converged"] for o in out)
