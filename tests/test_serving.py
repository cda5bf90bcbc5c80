"""Serving layer: continuous batching of steady solves.

CPU: the admission estimate and the failure path (a request whose context
cannot be created comes back with an error status, the server keeps going).
GPU: a request's result is bitwise the same alone and in a mix of concurrent
requests; a small HBM budget serialises admission.
"""
import os

import numpy as np
import pytest

from inputs import cube_mesh, freestream_prim, shell_mesh


def _lib_or_skip():
    from paper_2304_09485_amd import hgks
    if not os.path.exists(hgks.LIB_PATH):
        pytest.skip("libhgks.so not built")
    return hgks


def test_estimate_bytes_grows_with_size_and_options():
    hgks = _lib_or_skip()
    a = hgks.estimate_bytes(100_000, 2_000)
    b = hgks.estimate_bytes(200_000, 4_000)
    assert 1.9 * (a - (16 << 20)) < b - (16 << 20) < 2.1 * (a - (16 << 20))
    # per-cell cost of the plain FP64 WENO form: operators + work + Krylov basis
    per_cell = (b - a) / 100_000
    assert 3_000 < per_cell < 12_000
    assert hgks.estimate_bytes(100_000, 2_000, precision=1) > a
    assert hgks.estimate_bytes(100_000, 2_000, krylov_dim=20) > a


def test_server_reports_failed_requests_without_gpu():
    hgks = _lib_or_skip()
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: the failure path is exercised on CPU-only hosts")
    srv = hgks.Server(1 << 30, 2)
    m = cube_mesh(2)
    t1 = srv.submit(m, {k: hgks.FARFIELD for k in range(1, 7)}, freestream_prim(0.3), drop=1e-3, max_steps=3)
    t2 = srv.submit(m, {k: hgks.FARFIELD for k in range(1, 7)}, freestream_prim(0.4), drop=1e-3, max_steps=3)
    for t in (t1, t2):
        r = srv.wait(t)
        assert r.status == -6 and r.steps == 0
        assert r.t_total_ms >= r.t_queue_ms >= 0.0
    assert srv.stats().done == 2
    srv.close()


REQS = [
    (lambda: shell_mesh(4, 4, grading=1.3, jitter=0.05, seed=11), {1: 1, 2: 0}, 0.5, dict(scheme=1, max_update=0.2)),
    (lambda: cube_mesh(6, jitter=0.1, seed=12), {k: 0 for k in range(1, 7)}, 0.3, dict()),
    (lambda: shell_mesh(4, 3, grading=1.4, jitter=0.05, seed=13), {1: 2, 2: 0}, 0.25,
     dict(physics=1, mu=0.25 / 118.0, prandtl=0.72, precision=1)),
]


@pytest.mark.gpu
def test_same_result_alone_and_in_the_mix():
    hgks = _lib_or_skip()
    meshes = [r[0]() for r in REQS]
    solo = hgks.Server(8 << 30, 1)
    mk, kinds, mach, opts = REQS[0]
    ta = solo.submit(meshes[0], kinds, freestream_prim(mach), drop=1e-6, max_steps=8, **opts)
    ra = solo.wait(ta)
    qa = solo.state(ta)
    solo.close()
    assert ra.steps > 0 and ra.status in (0, -5)
    mix = hgks.Server(8 << 30, 3)
    tickets = []
    for k, (mk, kinds, mach, opts) in enumerate(REQS):
        tickets.append(mix.submit(meshes[k], kinds, freestream_prim(mach), drop=1e-6, max_steps=8, **opts))
    res = [mix.wait(t) for t in tickets]
    qm = mix.state(tickets[0])
    st = mix.stats()
    mix.close()
    print("solo", ra.steps, ra.res_final, "mix", [(r.steps, r.status, r.t_queue_ms, r.t_solve_ms) for r in res])
    assert st.done == 3
    # the server's progress count is the requests' implicit steps
    if all(r.status in (0, -5) for r in res):
        assert st.steps_done == sum(r.steps for r in res)
    assert res[0].steps == ra.steps
    assert np.array_equal(qa, qm)


@pytest.mark.gpu
def test_small_budget_serialises_admission():
    hgks = _lib_or_skip()
    m = cube_mesh(6, jitter=0.1, seed=12)
    kinds = {k: 0 for k in range(1, 7)}
    need = hgks.estimate_bytes(m.n_cells, len(m.bfaces))
    srv = hgks.Server(int(need * 1.5), 4)
    ts = [srv.submit(m, kinds, freestream_prim(0.3 + 0.05 * k), drop=1e-9, max_steps=3) for k in range(3)]
    rs = [srv.wait(t) for t in ts]
    srv.close()
    # each request is admitted only after the previous one finished
    for a, b in zip(rs, rs[1:]):
        assert b.t_queue_ms >= a.t_total_ms - 5.0


@pytest.mark.gpu
def test_first_order_and_lusgs_requests_match_standalone_solves():
    """Requests with the first-order KFVS scheme and with the LU-SGS solver,
    served together, end in the state a standalone context reaches with the
    same options from the free stream (the server runs the same library
    calls; its free-stream state is formed in C++, so the start may differ
    from numpy's in the last bit: 1e-9 relative)."""
    hgks = _lib_or_skip()
    from inputs import shell_mesh, uniform_state
    m = shell_mesh(4, 4, grading=1.3, jitter=0.05, seed=2)
    kinds = {1: hgks.SLIP_WALL, 2: hgks.FARFIELD}
    cases = [(freestream_prim(0.5), dict(scheme=hgks.KFVS1, cfl=1.0)),
             (freestream_prim(0.5), dict(scheme=hgks.WENO, solver=hgks.SOLVER_LUSGS, cfl=1.0))]
    srv = hgks.Server(8 << 30, 2)
    tickets = [srv.submit(m, kinds, prim, drop=1e-6, max_steps=20, **o) for prim, o in cases]
    res = [srv.wait(t) for t in tickets]
    states = [srv.state(t) for t in tickets]
    srv.close()
    for (prim, o), r, q in zip(cases, res, states):
        s = hgks.Solver(m, kinds, prim, **o)
        s.set_state(uniform_state(s.N, prim))
        info = s.solve_steady(drop=1e-6, max_steps=20)
        assert r.steps == info.steps
        np.testing.assert_allclose(q, s.get_state(), rtol=1e-9, atol=1e-12)
        s.close()
    with pytest.raises(ValueError):
        hgks.Server(1 << 30, 1).submit(cube_mesh(1, hexahedra=True), {1: 0}, freestream_prim(0.5))
