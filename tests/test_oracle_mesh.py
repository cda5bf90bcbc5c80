"""Pins of the oracle's geometry and stencils (paper Sec. 2 quadrature,
Sec. 3.1 stencil selection) against independent computations."""
import numpy as np
import pytest

from inputs import cube_mesh, freestream_prim, shell_mesh
from tests import _indep as I


@pytest.fixture(scope="module")
def jcube(oracle_lib):
    m = cube_mesh(4, jitter=0.15, seed=11)
    return m, oracle_lib.Oracle(m, {t: 0 for t in range(1, 7)}, freestream_prim(0.3))


def test_volumes_centroids_moments_vs_quadrature(jcube):
    m, o = jcube
    vol, cen, m2 = o.geometry()
    assert vol.sum() == pytest.approx(1.0, rel=1e-13)
    for i in range(0, m.n_cells, 37):
        pts, w = I.tet_quadrature(m.xyz[m.tets[i]], order=4)
        assert vol[i] == pytest.approx(w.sum(), rel=1e-12)
        c = (w[:, None] * pts).sum(0) / w.sum()
        np.testing.assert_allclose(cen[:, i], c, rtol=1e-12, atol=1e-14)
        d = pts - c
        M = np.einsum("p,pa,pb->ab", w, d, d) / w.sum()
        got = np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])
        np.testing.assert_allclose(m2[:, i], got, rtol=1e-10, atol=1e-16)


def test_face_closure_and_orientation(jcube):
    m, o = jcube
    L, R, S, n, gp = o.faces()
    vol, cen, _ = o.geometry()
    acc = np.zeros((3, o.N))
    np.add.at(acc.T, L, (n * S).T)
    inner = R >= 0
    np.add.at(acc.T, R[inner], -(n[:, inner] * S[inner]).T)
    assert np.abs(acc).max() <= 1e-15 * S.max() * 10
    # normals point from L to R (outward on boundary faces)
    fc = gp.reshape(3, 3, -1).mean(axis=0)
    assert (np.einsum("df,df->f", n, fc - cen[:, L]) > 0).all()
    assert (np.einsum("df,df->f", n[:, inner], cen[:, R[inner]] - fc[:, inner]) > 0).all()
    # interior faces are shared by exactly two cells, boundary count matches
    assert (~inner).sum() == len(m.bfaces)


def test_gauss_rule_exact_for_quadratics(jcube):
    m, o = jcube
    L, R, S, n, gp = o.faces()
    rng = np.random.default_rng(0)
    A = rng.normal(size=(3, 3))
    A = A + A.T
    b = rng.normal(size=3)
    q = lambda x: x @ A @ x + b @ x + 0.3  # noqa: E731
    # exact triangle average of a quadratic: mean of the edge midpoint values
    faces = {}
    for t in m.tets:
        for p in range(4):
            tri = tuple(sorted(np.delete(t, p)))
            faces[tri] = True
    cents = {tuple(np.round(m.xyz[list(k)].mean(0), 12)): k for k in faces}
    G = gp.reshape(3, 3, -1)
    for f in range(0, len(S), 17):
        c = G[:, :, f].mean(axis=0)
        key = cents[tuple(np.round(c, 12))]
        v = m.xyz[list(key)]
        mids = [(v[0] + v[1]) / 2, (v[1] + v[2]) / 2, (v[0] + v[2]) / 2]
        exact = np.mean([q(x) for x in mids])
        got = np.mean([q(G[g, :, f]) for g in range(3)])
        assert got == pytest.approx(exact, rel=1e-12, abs=1e-13)


def test_stencils(jcube):
    m, o = jcube
    N = o.N
    L, R, S, n, gp = o.faces()
    nbrs = [set() for _ in range(N)]
    for f in range(len(L)):
        if R[f] >= 0:
            nbrs[L[f]].add(R[f])
            nbrs[R[f]].add(L[f])
        else:
            nbrs[L[f]].add(N + (-R[f] - 1))
    for i in range(N):
        big = list(o.stencil(i, 0))
        assert big[0] == i and len(set(big)) == len(big)
        assert set(big[1:5]) == nbrs[i]
        two = set()
        for j in nbrs[i]:
            if j < N:
                two |= nbrs[j]
        assert set(big) == ({i} | nbrs[i] | two)
        for s in range(1, 5):
            sub = list(o.stencil(i, s))
            assert sub[0] == i and set(sub) <= set(big) and len(set(sub)) == len(sub)
            assert 4 <= len(sub) <= 7


def test_bad_mesh_rejected(oracle_lib):
    m = cube_mesh(2)
    t = m.tets.copy()
    t[0, [2, 3]] = t[0, [3, 2]]  # invert one tet
    m.tets = t
    with pytest.raises(ValueError):
        oracle_lib.Oracle(m, {k: 0 for k in range(1, 7)}, freestream_prim(0.3))


def test_shell_mesh_builds(oracle_lib):
    m = shell_mesh(4, 3, grading=1.2, jitter=0.02, seed=2)
    o = oracle_lib.Oracle(m, {1: oracle_lib.SLIP, 2: oracle_lib.FARFIELD}, freestream_prim(0.5))
    vol, _, _ = o.geometry()
    # faceted shell volume is below the sphere-shell volume but close to it
    exact = 4 / 3 * np.pi * (10 ** 3 - 0.5 ** 3)
    assert 0.9 * exact < vol.sum() < exact
