"""Host logic of bench.py (CPU): the one-GPU guard, the algorithmic byte
counts the roofline uses, and the traffic lookup keyed by the kernel sources."""
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
    with open(bench.TRAFFIC_FILE) as f:
        lines = [ln.split() for ln in f if ln.startswith("traffic ")]
    assert lines, "no traffic lines"
    for p in lines:
        if p[3] == h:
            assert bench.traffic_for(p[1]) == int(float(p[2]))
        else:
            assert bench.traffic_for(p[1]) is None
