"""Pins of the oracle's LU-SGS solver (the LUSGS-WENO comparison solver of
Sec. 5: the approximate matrix of Eq. (deri-matrix) factorised as
(D + L) D^-1 (D + U), L and U split by a greedy colouring of the cells).

  * the colouring is proper (no two face neighbours share a colour, found by
    brute-force triangle matching), uses at most 5 colours, and is the greedy
    one (every smaller colour is taken by a lower-numbered neighbour);
  * the LU-SGS update equals a dense solve of (D + L) D^-1 (D + U) x = R with
    the blocks of A extracted column by column from the pinned A x product;
  * the LU-SGS implicit step is Q + that update, with one residual evaluation.
"""
import numpy as np
import pytest

from inputs import cube_mesh, freestream_prim, perturbed_state, shell_mesh

KINDS_MIXED = {1: 3, 2: 4, 3: 0, 4: 0, 5: 1, 6: 1}


def _neighbours(mesh):
    owner = {}
    nb = [set() for _ in range(len(mesh.tets))]
    for t, tet in enumerate(mesh.tets):
        for p in range(4):
            key = tuple(sorted(np.delete(tet, p)))
            if key in owner:
                nb[t].add(owner[key])
                nb[owner[key]].add(t)
            else:
                owner[key] = t
    return nb


@pytest.mark.parametrize("which", ["cube", "shell"])
def test_colouring_is_proper_and_greedy(oracle_lib, which):
    m = cube_mesh(3, jitter=0.15, seed=2) if which == "cube" else shell_mesh(3, 3, grading=1.3, jitter=0.05,
                                                                              seed=1)
    kinds = {t: 0 for t in range(1, 7)}
    o = oracle_lib.Oracle(m, kinds, freestream_prim(0.5))
    col, nc = o.colours()
    assert nc == col.max() + 1 <= 5
    for i, nbs in enumerate(_neighbours(m)):
        assert all(col[j] != col[i] for j in nbs)
        lower = {col[j] for j in nbs if j < i}
        assert set(range(col[i])) <= lower


def test_lusgs_equals_dense_factorised_solve(oracle_lib):
    m = cube_mesh(2, jitter=0.15, seed=5)
    prim = freestream_prim(0.5)
    o = oracle_lib.Oracle(m, KINDS_MIXED, prim, solver=1)
    N = o.N
    Q = perturbed_state(N, prim, amp=0.05, seed=2)
    dt = o.dt(Q)
    R = np.random.default_rng(3).normal(size=(5, N))
    # dense A from its products with unit vectors, variable-major index v*N+i
    n = 5 * N
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = o.amatvec(Q, dt, e.reshape(5, N)).ravel()
    col, _ = o.colours()
    cell = np.tile(np.arange(N), 5)
    ci, cj = col[cell][:, None], col[cell][None, :]
    same = cell[:, None] == cell[None, :]
    D = np.where(same, A, 0.0)
    L = np.where(~same & (cj < ci), A, 0.0)
    U = np.where(~same & (cj > ci), A, 0.0)
    assert np.allclose(A, D + L + U, rtol=0, atol=0)  # no block between cells of one colour
    M = (D + L) @ np.linalg.inv(D) @ (D + U)
    x = np.linalg.solve(M, R.ravel()).reshape(5, N)
    got = o.lusgs(Q, dt, R)
    np.testing.assert_allclose(got, x, rtol=0, atol=1e-12 * np.abs(x).max())


def test_lusgs_implicit_step(oracle_lib):
    m = cube_mesh(2, jitter=0.15, seed=5)
    prim = freestream_prim(0.5)
    o = oracle_lib.Oracle(m, KINDS_MIXED, prim, solver=1)
    Q = perturbed_state(o.N, prim, amp=0.05, seed=4)
    dt = o.dt(Q)
    want = Q + o.lusgs(Q, dt, o.residual(Q, dt=dt))
    st, info = o.implicit_step(Q)
    assert st == 0 and info.n_resid_evals == 1
    np.testing.assert_array_equal(Q, want)
