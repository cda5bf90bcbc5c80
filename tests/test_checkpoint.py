"""Checkpoint / resume of a steady solve through the C ABI.

A solve interrupted after k implicit steps, written to a file and resumed in a
fresh context, must continue bit for bit as the uninterrupted solve (the state,
the gradients of the compact scheme and the reference residual of res_rel are
all restored).  Files for another mesh or scheme, truncated and corrupted files
are refused and leave the state unchanged.
"""
import os

import numpy as np
import pytest

from inputs import cube_mesh, freestream_prim, perturbed_state, shell_mesh
from tests import _cases as C

pytestmark = pytest.mark.gpu


def _solver(hgks, scheme, mesh=None):
    m = mesh if mesh is not None else shell_mesh(4, 4, grading=1.3, jitter=0.05, seed=2)
    prim = freestream_prim(0.5)
    s = hgks.Solver(m, {1: C.SLIP, 2: C.FAR}, prim, scheme=scheme)
    G = np.random.default_rng(3).normal(scale=0.02, size=(15, s.N)) if scheme == 1 else None
    s.set_state(perturbed_state(s.N, prim, seed=4), G)
    return m, s


@pytest.mark.parametrize("scheme,hexa", [(0, False), (1, False), (1, True)])
def test_resume_is_bitwise(tmp_path, scheme, hexa):
    from paper_2304_09485_amd import hgks
    mesh = shell_mesh(4, 4, grading=1.3, jitter=0.05, seed=2, hexahedra=True) if hexa else None
    m, a = _solver(hgks, scheme, mesh=mesh)
    for _ in range(2):
        a.implicit_step()
    path = os.fspath(tmp_path / "solve.ckpt")
    a.checkpoint(path)
    ia = [a.implicit_step() for _ in range(2)]
    Qa, Ga = a.get_state(want_grad=True)

    _, b = _solver(hgks, scheme, mesh=m)
    b.restore(path)
    ib = [b.implicit_step() for _ in range(2)]
    Qb, Gb = b.get_state(want_grad=True)
    assert np.array_equal(Qa, Qb)
    assert np.array_equal(Ga, Gb)
    assert [i.res for i in ia] == [i.res for i in ib]
    assert [i.res_rel for i in ia] == [i.res_rel for i in ib]
    a.close()
    b.close()


def test_bad_files_are_refused(tmp_path):
    from paper_2304_09485_amd import hgks
    m, a = _solver(hgks, 1)
    path = os.fspath(tmp_path / "a.ckpt")
    a.checkpoint(path)
    Q0, G0 = a.get_state(want_grad=True)
    raw = open(path, "rb").read()

    def refused(data, solver):
        p = os.fspath(tmp_path / "bad.ckpt")
        with open(p, "wb") as f:
            f.write(data)
        with pytest.raises(hgks.HgksError) as e:
            solver.restore(p)
        assert e.value.status == -1
        return str(e.value)

    # corrupted payload byte, truncated file, trailing bytes, bad magic
    bad = bytearray(raw)
    bad[100] ^= 0x40
    assert "hash" in refused(bytes(bad), a)
    assert "truncated" in refused(raw[:-9], a)
    assert "trailing" in refused(raw + b"\0", a)
    assert "magic" in refused(b"XXXXXXXX" + raw[8:], a)
    Q1, G1 = a.get_state(want_grad=True)
    assert np.array_equal(Q0, Q1) and np.array_equal(G0, G1)

    # another scheme on the same mesh, another mesh
    _, w = _solver(hgks, 0, mesh=m)
    assert "scheme" in refused(raw, w)
    c = hgks.Solver(cube_mesh(3), {t: C.FAR for t in range(1, 7)}, freestream_prim(0.5), scheme=1)
    assert "mesh" in refused(raw, c)
    with pytest.raises(hgks.HgksError):
        a.restore(os.fspath(tmp_path / "missing.ckpt"))
    for s in (a, w, c):
        s.close()


def test_resumed_solve_continues_the_ramp_and_the_drop(tmp_path):
    """solve_steady with a CFL ramp, interrupted after 4 steps, written out and
    resumed in a fresh context for 5 more: the same state, step count and
    drop as 9 steps in one call (the restored reference residual and ramp
    position are used, not restarted)."""
    from paper_2304_09485_amd import hgks
    mesh = shell_mesh(4, 4, grading=1.3, jitter=0.05, seed=2)
    prim = freestream_prim(0.5)
    opts = dict(scheme=1, cfl=10.0, cfl_start=1.0, cfl_growth=1.5)

    def fresh():
        s = hgks.Solver(mesh, {1: C.SLIP, 2: C.FAR}, prim, **opts)
        s.set_state(perturbed_state(s.N, prim, seed=4), np.zeros((15, s.N)))
        return s

    a = fresh()
    ia = a.solve_steady(drop=1e-30, max_steps=9)
    Qa = a.get_state()
    b = fresh()
    b.solve_steady(drop=1e-30, max_steps=4)
    path = os.fspath(tmp_path / "ramp.ckpt")
    b.checkpoint(path)
    c = fresh()
    c.restore(path)
    ic = c.solve_steady(drop=1e-30, max_steps=5)
    Qc = c.get_state()
    assert np.array_equal(Qa, Qc)
    assert ia.res_final == ic.res_final
    assert ia.res0 == ic.res0 and ia.drop == ic.drop
    for s in (a, b, c):
        s.close()
