"""Pins of the oracle on hexahedral meshes (Sec. 3.1: six faces, the eight
non-compact sub-stencils {i, i_1 or i_6, two consecutive lateral neighbours},
the six compact sub-stencils {i, i_f}; reading A30 for the trilinear cells and
bilinear faces).

  * volumes, centroids and second moments against a 5-point-per-direction
    tensor Gauss rule on the trilinear map (written in the test);
  * closed cells (the outward face vector areas of every cell sum to zero),
    outward normals, and the face rule integrating quadratics exactly on a
    planar non-parallelogram face;
  * the eight sub-stencils of an interior cell of a regular grid span the
    eight octants;
  * linear data reproduced by every polynomial and by the nonlinear
    combination, quadratic data with linear weights (WENO and HWENO, the
    latter with either sub-stencil family);
  * the compact scheme with the eight S^WENO sub-stencils fits its P_m from
    cell averages alone (the non-compact P_m), with 8 weights;
  * free-stream preservation (WENO, HWENO, first-order KFVS) and
    conservation in a closed box;
  * the approximate matrix and two Jacobi sweeps against a direct assembly
    with a complex-step Euler Jacobian; LU-SGS against a dense factorised
    solve.
"""
import numpy as np
import pytest

from inputs import HexMesh, cube_mesh, freestream_prim, perturbed_state, shell_mesh, uniform_state
from tests import _indep as I
from tests.test_oracle_recon import GL, lin, lin_grad, quad, quad_grad

ALL_FAR = {t: 0 for t in range(1, 7)}


def jcube(n=4, seed=11):
    return cube_mesh(n, jitter=0.15, seed=seed, hexahedra=True)


def test_hex_geometry_vs_quadrature(oracle_lib):
    m = jcube()
    o = oracle_lib.Oracle(m, ALL_FAR, freestream_prim(0.3))
    vol, cen, m2 = o.geometry()
    for i in range(0, o.N, 5):
        pts, w = I.hex_quadrature(m.xyz[m.hexes[i]], order=5)
        V = w.sum()
        c = pts.T @ w / V
        d = pts - c
        M = np.einsum("p,pa,pb->ab", w, d, d) / V
        assert vol[i] == pytest.approx(V, rel=1e-13)
        np.testing.assert_allclose(cen[:, i], c, rtol=0, atol=1e-14)
        np.testing.assert_allclose(m2[:, i], [M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]],
                                   rtol=0, atol=1e-15)
    assert vol.sum() == pytest.approx(1.0, rel=1e-13)


def test_hex_faces_closed_and_outward(oracle_lib):
    m = shell_mesh(3, 3, grading=1.3, jitter=0.05, seed=1, hexahedra=True)
    o = oracle_lib.Oracle(m, {1: 1, 2: 0}, freestream_prim(0.3))
    L, R, S, n, gp = o.faces()
    vol, cen, _ = o.geometry()
    acc = np.zeros((3, o.N))
    np.add.at(acc.T, L, (S * n).T)
    np.add.at(acc.T, R[R >= 0], -(S * n)[:, R >= 0].T)
    assert np.abs(acc).max() <= 1e-12 * S.max()
    fc = gp.reshape(4, 3, -1).mean(axis=0)
    assert (np.einsum("df,df->f", n, fc - cen[:, L]) > 0).all()


def test_quad_face_rule_exact_for_quadratics(oracle_lib):
    """One hexahedron with planar trapezoid top and bottom faces: the face
    rule (4 points, weights from the area element) integrates a quadratic
    exactly (the degree of the triangle rule; the 2x2 rule times the bilinear
    area element is exact to degree 3 per reference direction)
    over the trapezoid; the reference integral uses a 6-point tensor rule on
    the same bilinear face with its own area element."""
    xyz = np.array([[0, 0, 0], [2, 0, 0], [1.5, 1, 0], [0.2, 1, 0],
                    [0, 0, 1], [2, 0, 1], [1.5, 1, 1], [0.2, 1, 1]], float)
    hexes = np.array([[0, 1, 2, 3, 4, 5, 6, 7]], np.int32)
    quads = np.array([[0, 3, 2, 1], [0, 1, 5, 4], [1, 2, 6, 5], [2, 3, 7, 6], [3, 0, 4, 7], [4, 5, 6, 7]], np.int32)
    m = HexMesh(xyz=xyz, hexes=hexes, bfaces=quads, btags=np.ones(6, np.int32))
    o = oracle_lib.Oracle(m, {1: 0}, freestream_prim(0.3))
    L, R, S, n, gp = o.faces()
    GP = gp.reshape(4, 3, -1)
    f = int(np.argmax(n[2]))  # the top face z = 1
    a, b, c, d = xyz[[4, 5, 6, 7]]
    cub = lambda x: 1 + x[:, 0] ** 2 - 2 * x[:, 0] * x[:, 1] + 0.5 * x[:, 1] ** 2 + x[:, 0]  # noqa
    g, wg = np.polynomial.legendre.leggauss(6)
    g, wg = 0.5 * (g + 1), 0.5 * wg
    U, W = [x.ravel() for x in np.meshgrid(g, g, indexing="ij")]
    WW = np.outer(wg, wg).ravel()
    x = ((1 - U) * (1 - W))[:, None] * a + (U * (1 - W))[:, None] * b + (U * W)[:, None] * c + ((1 - U) * W)[:, None] * d
    xu = (1 - W)[:, None] * (b - a) + W[:, None] * (c - d)
    xw = (1 - U)[:, None] * (d - a) + U[:, None] * (c - b)
    dA = np.linalg.norm(np.cross(xu, xw), axis=1)
    exact = (cub(x) * dA * WW).sum()
    assert S[f] == pytest.approx((dA * WW).sum(), rel=1e-14)
    # the weights are not returned: recover them from a linear function
    # (exact for any positive rule) and check the cubic with them
    P = GP[:, :, f]
    A = np.stack([np.ones(4), P[:, 0], P[:, 1], P[:, 0] * P[:, 1]])
    rhs = np.array([(v * dA * WW).sum() for v in (np.ones_like(U), x[:, 0], x[:, 1], x[:, 0] * x[:, 1])])
    w = np.linalg.solve(A, rhs)
    assert w.sum() == pytest.approx(S[f], rel=1e-14)
    assert (cub(P) * w).sum() == pytest.approx(exact, rel=1e-13)


def test_hex_sub_stencils_span_octants(oracle_lib):
    m = cube_mesh(3, hexahedra=True)
    o = oracle_lib.Oracle(m, ALL_FAR, freestream_prim(0.3))
    vol, cen, _ = o.geometry()
    i = int(np.argmin(np.linalg.norm(cen.T - 0.5, axis=1)))
    octs = set()
    for s in range(1, 9):
        st = o.stencil(i, s)
        assert len(st) == 4 and st[0] == i
        d = np.sign(np.round(cen[:, st[1:]] - cen[:, [i]], 12))
        assert (np.abs(d).sum(axis=0) == 1).all()  # three face neighbours
        octs.add(tuple(d.sum(axis=1).astype(int)))
    assert len(octs) == 8
    big = o.stencil(i, 0)
    assert len(big) == 25  # self, 6 face, 12 edge and 6 second face neighbours


def _interior_faces(o):
    L, R, S, n, gp = o.faces()
    ok = [f for f in range(len(L)) if R[f] >= 0 and all((o.stencil(c, 0) < o.N).all() for c in (L[f], R[f]))]
    return ok, gp.reshape(o.ng, 3, -1)


def _expected(o, f, fv, fg, P):
    fr = o.face_frame(f)
    out = np.zeros((o.ng, 4, 5))
    for g in range(o.ng):
        x = P[g][None, :]
        v = fv(x)[:, 0]
        G = fg(x)[:, :, 0]
        for d in range(4):
            q = v if d == 0 else G @ fr[d - 1]
            out[g, d] = [q[0], *(fr @ q[1:4]), q[4]]
    return out


@pytest.mark.parametrize("scheme,weights,data,subs", [(0, 0, "lin", 0), (1, 0, "lin", 0), (0, 1, "quad", 0),
                                                      (1, 1, "quad", 0), (1, 0, "lin", 1), (1, 1, "quad", 1)])
def test_hex_reproduction(oracle_lib, scheme, weights, data, subs):
    m = cube_mesh(7, jitter=0.15, seed=3, hexahedra=True)
    o = oracle_lib.Oracle(m, ALL_FAR, freestream_prim(0.3), scheme=scheme, weights=weights, compact_subs=subs)
    fv, fg = (lin, lin_grad) if data == "lin" else (quad, quad_grad)
    Q = I.cell_averages(m, fv, order=4)
    vol, cen, _ = o.geometry()
    G = fg(cen.T).reshape(15, -1)
    faces, GP = _interior_faces(o)
    assert len(faces) > 20
    for f in faces[::5]:
        exp = _expected(o, f, fv, fg, GP[:, :, f])
        for side in (0, 1):
            got, fb = o.side_values(Q, f, side, G=G)
            assert fb == 0
            np.testing.assert_allclose(got, exp, rtol=0, atol=1e-12)


@pytest.mark.parametrize("opts", [dict(scheme=0), dict(scheme=1), dict(scheme=1, compact_subs=1),
                                  dict(first_order=1)])
def test_hex_free_stream_preserved(oracle_lib, opts):
    m = shell_mesh(3, 3, grading=1.3, jitter=0.05, seed=2, hexahedra=True)
    prim = freestream_prim(0.6, direction=(1.0, 0.4, -0.3))
    o = oracle_lib.Oracle(m, {1: 0, 2: 0}, prim, **opts)
    R = o.residual(uniform_state(o.N, prim), G=np.zeros((15, o.N)))
    q = I.cons(prim[0], prim[1:4], prim[4])
    scale = max(np.abs(I.euler_flux(q, e)).max() for e in np.eye(3)) * o.faces()[2].max() * 6
    assert np.abs(R).max() <= 1e-13 * scale


@pytest.mark.parametrize("scheme,subs", [(0, 0), (1, 0), (1, 1)])
def test_hex_conservation_closed_box(oracle_lib, scheme, subs):
    m = jcube(4, seed=5)
    prim = freestream_prim(0.3)
    o = oracle_lib.Oracle(m, {t: oracle_lib.SLIP for t in range(1, 7)}, prim, scheme=scheme, compact_subs=subs)
    Q = perturbed_state(o.N, prim, amp=0.05, seed=3)
    G = np.random.default_rng(1).normal(scale=0.05, size=(15, o.N)) if scheme == 1 else None
    R = o.residual(Q, G=G)
    s = np.abs(R).sum(axis=1)
    assert abs(R[0].sum()) <= 1e-13 * s[0]
    assert abs(R[4].sum()) <= 1e-13 * s[4]


def test_hex_approximate_matrix_and_lusgs(oracle_lib):
    m = cube_mesh(2, jitter=0.1, seed=3, hexahedra=True)
    prim = freestream_prim(0.3)
    o = oracle_lib.Oracle(m, {t: oracle_lib.SUP_OUT for t in range(1, 7)}, prim)
    N = o.N
    Q = perturbed_state(N, prim, amp=0.05, seed=8)
    dt = o.dt(Q)
    vol = o.geometry()[0]
    L, R, S, n, gp = o.faces()

    def lam(a, b, nn):
        ra, Ua, pa = I.prim(Q[:, a])
        rb, Ub, pb = I.prim(Q[:, b])
        rho, U, p = (ra + rb) / 2, (Ua + Ub) / 2, (pa + pb) / 2
        return abs(U @ nn) + np.sqrt(1.4 * p / rho)
    D = vol / dt
    lam_f = np.array([lam(L[f], R[f] if R[f] >= 0 else L[f], n[:, f]) for f in range(len(L))])
    np.add.at(D, L, 0.5 * lam_f * S)
    np.add.at(D, R[R >= 0], 0.5 * lam_f[R >= 0] * S[R >= 0])
    np.testing.assert_allclose(o.diag(Q, dt), D, rtol=1e-13)

    def offdiag(x):
        out = np.zeros_like(x)
        for f in np.where(R >= 0)[0]:
            a, b = L[f], R[f]
            out[:, a] += 0.5 * S[f] * (I.euler_jn_cs(Q[:, b], n[:, f], x[:, b]) - lam_f[f] * x[:, b])
            out[:, b] += 0.5 * S[f] * (I.euler_jn_cs(Q[:, a], -n[:, f], x[:, a]) - lam_f[f] * x[:, a])
        return out
    y = np.random.default_rng(1).normal(size=(5, N))
    Ay = D * y + offdiag(y)
    np.testing.assert_allclose(o.amatvec(Q, dt, y), Ay, rtol=1e-12, atol=1e-14 * np.abs(Ay).max())
    r = np.random.default_rng(0).normal(size=(5, N))
    x = r / D
    for _ in range(2):
        x = (r - offdiag(x)) / D
    np.testing.assert_allclose(o.precond(Q, dt, r), x, rtol=1e-12, atol=1e-14 * np.abs(x).max())
    # LU-SGS: dense (D + L) D^-1 (D + U) on the colour split
    col, nc = o.colours()
    assert nc <= 7
    nn = 5 * N
    A = np.zeros((nn, nn))
    for k in range(nn):
        e = np.zeros(nn)
        e[k] = 1.0
        A[:, k] = o.amatvec(Q, dt, e.reshape(5, N)).ravel()
    cell = np.tile(np.arange(N), 5)
    ci, cj = col[cell][:, None], col[cell][None, :]
    same = cell[:, None] == cell[None, :]
    Dm = np.where(same, A, 0.0)
    Lm = np.where(~same & (cj < ci), A, 0.0)
    Um = np.where(~same & (cj > ci), A, 0.0)
    M = (Dm + Lm) @ np.linalg.inv(Dm) @ (Dm + Um)
    xs = np.linalg.solve(M, r.ravel()).reshape(5, N)
    np.testing.assert_allclose(o.lusgs(Q, dt, r), xs, rtol=0, atol=1e-12 * np.abs(xs).max())


def test_hex_compact_weno_sub_stencils_use_averages_only(oracle_lib):
    """With the eight S^WENO sub-stencils as the compact scheme's sub-stencils
    (the hexahedral sphere cases of Sec. 5), each P_m is fitted from the cell
    averages of its four cells alone: on linear data its gradient is the
    exact one whatever the supplied cell gradients are, there are 8 of them
    (gamma_0 = 1 - 8 x 0.025), and they are the non-compact scheme's P_m;
    with the faces' {i, i_f} sub-stencils the garbage gradients do enter."""
    m = cube_mesh(7, jitter=0.15, seed=4, hexahedra=True)
    prim = freestream_prim(0.3)
    Q = I.cell_averages(m, lin, order=4)
    G = np.random.default_rng(2).normal(scale=1.0, size=(15, len(m.hexes)))
    o1 = oracle_lib.Oracle(m, ALL_FAR, prim, scheme=1, compact_subs=1)
    o0 = oracle_lib.Oracle(m, ALL_FAR, prim, scheme=1, compact_subs=0)
    ow = oracle_lib.Oracle(m, ALL_FAR, prim, scheme=0)
    faces, _ = _interior_faces(ow)
    assert len(faces) > 5
    for f in faces[:12]:
        for side in (0, 1):
            d1 = o1.side_debug(Q, f, side, G=G)
            d0 = o0.side_debug(Q, f, side, G=G)
            dw = ow.side_debug(Q, f, side)
            Lc = d1["L"]
            fr = o1.face_frame(f)
            # exact gradient of each characteristic component of the linear data
            Gl = GL.copy()
            Gl[1:4] = fr @ GL[1:4]
            exact = Lc @ Gl  # (5, 3)
            assert (d1["M"] == 8).all() and (d0["M"] == 6).all()
            np.testing.assert_allclose(d1["b"], np.repeat(exact[:, None, :], 8, axis=1), rtol=0, atol=1e-12)
            np.testing.assert_allclose(d1["b"], dw["b"], rtol=0, atol=1e-13)
            assert np.abs(d0["b"][:, :6] - exact[:, None, :]).max() > 1e-3
