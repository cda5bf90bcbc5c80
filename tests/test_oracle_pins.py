"""Pins of the oracle's smoothness indicators, nonlinear weights,
characteristic projection, local time step and boundary ghosts against
arithmetic that does not come from the oracle.

* beta_0 and beta_m (Sec. 3.4): the oracle's own polynomials are
  differentiated by central differences (exact for quadratics) and the squares
  integrated by a Duffy-mapped Gauss rule on the cell, with the
  |Omega|^(2|l|/3 - 1) factors and every distinct multi-index once;
* the weights (Sec. 3.4): from those betas by the WENO-Z type formula with
  tau_Z = sum_m |beta_0 - beta_m| / M; on a contact discontinuity every
  sub-stencil that reaches across it gets a weight below 1e-2, and so does
  P0, while the sub-stencils on one side carry the weight;
* R* (Sec. 5): J_x(Q*) R* = R* diag(u - c, u, u, u, u + c) with the x-split
  Euler Jacobian taken by complex steps, at Q* = the mean of the two cell
  averages in the face frame;
* the local time step: on a regular tetrahedron of edge a its height is
  a sqrt(2/3), on a cube of edge a its width is a;
* the far-field ghost: the outgoing Riemann invariant from the interior, the
  incoming one from the free stream, entropy and tangential velocity from the
  upwind side, and both supersonic branches;
* wall ghost gradients: the gradient of the reflected field, taken by complex
  steps; and the compact residual with a slip wall on a mirror plane equals
  the residual of the mirrored full mesh;
* the residual's truncation error on a smooth field falls at second order on
  jittered meshes (the Euler limit of the flux).
"""
import numpy as np
import pytest

from inputs import TetMesh, HexMesh, cube_mesh, freestream_prim, prim_to_cons
from tests import _indep as I

FAR, SLIP, NOSLIP, SUP_IN, SUP_OUT = 0, 1, 2, 3, 4
GAMMA = 1.4


def smooth_field(x, amp=0.05):
    """A smooth conserved field with curvature in every variable."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    rho = 1.0 + amp * np.sin(2.1 * X + 0.3) * np.cos(1.7 * Y - 0.2) + amp * Z * Z
    u = 0.3 + amp * np.cos(1.3 * X + 2.0 * Z)
    v = amp * np.sin(1.9 * Y + 0.5 * X)
    w = -amp * np.cos(2.3 * Z - 0.4 * Y)
    p = 1.0 / GAMMA + amp * np.sin(1.1 * X + 1.2 * Y + 1.3 * Z)
    return np.stack([rho, rho * u, rho * v, rho * w, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v + w * w)])


def _tet_verts(mesh, i):
    return mesh.xyz[mesh.tets[i]]


def _p0_func(a, c, h, q0=0.0):
    """P0 of the scaled basis as a function of points (the mean subtraction
    does not matter for derivatives)."""
    def f(x):
        xi = (x - c) / h
        return (q0 + a[0] * xi[..., 0] + a[1] * xi[..., 1] + a[2] * xi[..., 2] + a[3] * xi[..., 0] ** 2
                + a[4] * xi[..., 1] ** 2 + a[5] * xi[..., 2] ** 2 + a[6] * xi[..., 0] * xi[..., 1]
                + a[7] * xi[..., 0] * xi[..., 2] + a[8] * xi[..., 1] * xi[..., 2])
    return f


def _beta_quadrature(f, verts, step):
    """sum over |l| = 1, 2 of |Omega|^(2|l|/3 - 1) int (d^l f)^2, derivatives
    by central differences of the polynomial f (exact for quadratics up to
    rounding), the integral by the Duffy rule."""
    pts, w = I.tet_quadrature(verts, order=4)
    vol = w.sum()
    E = np.eye(3) * step
    first = 0.0
    for d in range(3):
        g = (f(pts + E[d]) - f(pts - E[d])) / (2 * step)
        first += np.sum(w * g * g)
    second = 0.0
    for a in range(3):
        for b in range(a, 3):
            if a == b:
                g = (f(pts + E[a]) - 2 * f(pts) + f(pts - E[a])) / step ** 2
            else:
                g = (f(pts + E[a] + E[b]) - f(pts + E[a] - E[b]) - f(pts - E[a] + E[b])
                     + f(pts - E[a] - E[b])) / (4 * step * step)
            second += np.sum(w * g * g)
    return vol ** (2.0 / 3.0 - 1.0) * first + vol ** (4.0 / 3.0 - 1.0) * second


@pytest.fixture(scope="module")
def smooth_case(oracle_lib):
    mesh = cube_mesh(4, jitter=0.15, seed=11)
    kinds = {t: FAR for t in range(1, 7)}
    o = oracle_lib.Oracle(mesh, kinds, freestream_prim(0.3))
    Q = I.cell_averages(mesh, smooth_field)
    G = np.zeros((15, o.N))
    vol, cen, _ = o.geometry()
    ref = np.array([_tet_verts(mesh, i).mean(axis=0) for i in range(o.N)])
    assert np.allclose(cen.T, ref, atol=1e-14)  # oracle cells are the mesh's tets in order
    return mesh, o, Q, G


def _interior_sides(o, count):
    L, R, *_ = o.faces()
    out = []
    for f in range(len(L)):
        if R[f] >= 0:
            out.append((f, 0, int(L[f])))
            out.append((f, 1, int(R[f])))
        if len(out) >= count:
            break
    return out


@pytest.mark.parametrize("scheme", [0, 1])
def test_smoothness_indicators_vs_quadrature(oracle_lib, smooth_case, scheme):
    """beta_0 of P0 and beta_m of every P_m of Sec. 3.4 against quadrature of
    the differentiated polynomials, for every characteristic component."""
    mesh, o0, Q, G = smooth_case
    o = o0 if scheme == 0 else oracle_lib.Oracle(mesh, {t: FAR for t in range(1, 7)}, freestream_prim(0.3),
                                                 scheme=1)
    h, _ = o.cell_scales()
    vol, cen, _ = o.geometry()
    checked = 0
    for f, side, i in _interior_sides(o, 24):
        d = o.side_debug(Q, f, side, G=G)
        verts = _tet_verts(mesh, i)
        for c in range(5):
            p0 = _p0_func(d["a"][c], cen[:, i], h[i])
            scale = max(np.abs(d["a"][c]).max(), 1e-300) ** 2 / h[i] ** 2 * vol[i] ** (2.0 / 3.0)
            b0 = _beta_quadrature(p0, verts, 1e-3 * h[i])
            assert abs(d["beta"][c, 0] - b0) <= 1e-8 * scale, (f, side, c, d["beta"][c, 0], b0)
            for m in range(int(d["M"][c])):
                assert d["ok"][c, m]
                bm = d["b"][c, m]
                pm = lambda x, bm=bm: x @ bm  # noqa: E731
                ref = _beta_quadrature(pm, verts, 1e-3 * h[i])
                sc = max(bm @ bm, 1e-300) * vol[i] ** (2.0 / 3.0)
                assert abs(d["beta"][c, 1 + m] - ref) <= 1e-8 * sc, (f, side, c, m)
                checked += 1
    assert checked > 24 * 5 * 3


def _weights_from_betas(beta, M, gam, eps):
    b0, bm = beta[0], beta[1:1 + M]
    tz = np.sum(np.abs(b0 - bm)) / M
    g0 = 1.0 - gam * M
    wt = np.concatenate([[g0 * (1 + tz / (b0 + eps))], gam * (1 + tz / (bm + eps))])
    return wt / wt.sum(), tz


@pytest.mark.parametrize("scheme", [0, 1])
def test_weights_from_pinned_betas(oracle_lib, smooth_case, scheme):
    """The nonlinear weights of Sec. 3.4 from the quadrature-pinned betas; the
    data are chosen so that tau_Z / beta is of order one, where the 1/M in
    tau_Z changes the weights."""
    mesh, o0, Q, G = smooth_case
    o = o0 if scheme == 0 else oracle_lib.Oracle(mesh, {t: FAR for t in range(1, 7)}, freestream_prim(0.3),
                                                 scheme=1)
    sensitive = 0
    for f, side, _ in _interior_sides(o, 24):
        d = o.side_debug(Q, f, side, G=G)
        for c in range(5):
            M = int(d["M"][c])
            w, tz = _weights_from_betas(d["beta"][c], M, o.opts.gamma_lin, o.opts.weno_eps)
            assert abs(d["tau"][c] - tz) <= 1e-12 * max(tz, 1e-300) + 1e-300
            assert np.allclose(d["w"][c, :M + 1], w, rtol=1e-12, atol=1e-15), (f, side, c)
            assert abs(d["w"][c, :M + 1].sum() - 1.0) < 1e-14
            # the same with tau_Z summed without 1/M
            b0, bm = d["beta"][c, 0], d["beta"][c, 1:1 + M]
            tzM = np.sum(np.abs(b0 - bm))
            eps = o.opts.weno_eps
            wt = np.concatenate([[(1 - 0.025 * M) * (1 + tzM / (b0 + eps))], 0.025 * (1 + tzM / (bm + eps))])
            if np.abs(wt / wt.sum() - w).max() > 1e-3:
                sensitive += 1
    assert sensitive >= 10


def test_crossing_sub_stencils_get_no_weight(oracle_lib):
    """A contact discontinuity (density jump at uniform velocity and pressure)
    across the plane x = 0.52: on every face side whose cell has at least one
    sub-stencil entirely on its own side, P0 and every sub-stencil that reaches
    across the jump carry a weight below 1e-2 in the entropy component, the
    only one the jump projects onto, and the one-sided sub-stencils more than
    0.98 (with epsilon = 1e-5 the crossing weights scale as epsilon / tau_Z,
    a few 1e-3 for this jump)."""
    mesh = cube_mesh(6, jitter=0.1, seed=21)
    kinds = {t: FAR for t in range(1, 7)}
    prim = freestream_prim(0.3)
    o = oracle_lib.Oracle(mesh, kinds, prim)
    vol, cen, _ = o.geometry()
    N = o.N
    left = cen[0] < 0.52
    pr = np.repeat(prim[:, None], N, axis=1)
    pr[0] = np.where(left, 1.0, 0.5)
    Q = prim_to_cons(pr)
    L, R, *_ = o.faces()
    seen = 0
    for f in range(len(L)):
        for side in (0, 1):
            i = int(L[f]) if side == 0 else int(R[f])
            if i < 0:
                continue
            subs = [o.stencil(i, m) for m in range(1, 5)]
            big = o.stencil(i, 0)
            real = lambda s: s[s < N]  # noqa: E731
            cross = [bool(np.any(left[real(s)] != left[i])) for s in subs]
            if not any(cross) or all(cross) or not np.any(left[real(big)] != left[i]):
                continue
            d = o.side_debug(Q, f, side)
            w = d["w"][1]
            assert w[0] < 1e-2, (f, side, w)
            for m in range(4):
                if d["ok"][1, m] and cross[m]:
                    assert w[1 + m] < 1e-2, (f, side, m, w)
            assert sum(w[1 + m] for m in range(4) if not cross[m]) > 0.98
            seen += 1
            if seen >= 40:
                return
    assert seen >= 10


def test_right_eigenvectors_diagonalise_the_jacobian(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho = rng.uniform(0.3, 3.0)
        U = rng.normal(size=3)
        p = rng.uniform(0.2, 2.0)
        q = I.cons(rho, U, p)
        R = oracle_lib.right_eigenvectors(GAMMA, q)
        J = np.stack([I.euler_jn_cs(q, [1.0, 0.0, 0.0], e) for e in np.eye(5)], axis=1)
        c = np.sqrt(GAMMA * p / rho)
        lam = np.array([U[0] - c, U[0], U[0], U[0], U[0] + c])
        assert np.allclose(J @ R, R * lam[None, :], rtol=0, atol=1e-12 * np.abs(J).max() * np.abs(R).max())
        assert abs(np.linalg.det(R)) > 1e-6


def test_projection_uses_the_mean_of_the_two_cell_averages(oracle_lib, smooth_case):
    mesh, o, Q, G = smooth_case
    L, R, *_ = o.faces()
    for f, side, _ in _interior_sides(o, 10):
        d = o.side_debug(Q, f, side)
        fr = o.face_frame(f)
        qm = 0.5 * (Q[:, L[f]] + Q[:, R[f]])
        qloc = np.array([qm[0], *(fr @ qm[1:4]), qm[4]])
        Rref = oracle_lib.right_eigenvectors(GAMMA, qloc)
        assert np.allclose(d["R"], Rref, rtol=1e-14, atol=1e-14)
        assert np.allclose(d["L"] @ d["R"], np.eye(5), atol=1e-12)


def _single_tet(a=1.0):
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float) * (a / np.sqrt(8.0))
    tets = np.array([[0, 1, 2, 3]], np.int32)
    six = np.einsum("j,j->", np.cross(v[1] - v[0], v[2] - v[0]), v[3] - v[0])
    if six < 0:
        tets = np.array([[0, 1, 3, 2]], np.int32)
    bf = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]], np.int32)
    return TetMesh(xyz=v, tets=tets, bfaces=bf, btags=np.ones(4, np.int32))


def test_time_step_regular_tetrahedron_and_cube(oracle_lib):
    """Delta t = CFL h / (|U| + c + 2 nu / h) with h the height of a regular
    tetrahedron (a sqrt(2/3)) and the width of a cube (a)."""
    a = 0.37
    prim = np.array([1.3, 0.2, -0.1, 0.05, 0.9])
    q = prim_to_cons(prim)[:, None]
    spd = np.linalg.norm(prim[1:4])
    c = np.sqrt(GAMMA * prim[4] / prim[0])
    m = _single_tet(a)
    assert np.isclose(np.linalg.norm(m.xyz[0] - m.xyz[1]), a)
    o = oracle_lib.Oracle(m, {1: FAR}, freestream_prim(0.3), cfl=7.0)
    h = a * np.sqrt(2.0 / 3.0)
    assert np.isclose(o.dt(q)[0], 7.0 * h / (spd + c), rtol=1e-13)
    mu = 0.05
    o = oracle_lib.Oracle(m, {1: FAR}, freestream_prim(0.3), cfl=7.0, physics=1, mu=mu, prandtl=0.72)
    assert np.isclose(o.dt(q)[0], 7.0 * h / (spd + c + 2 * mu / prim[0] / h), rtol=1e-13)
    hm = cube_mesh(1, length=a, hexahedra=True)
    o = oracle_lib.Oracle(hm, {t: FAR for t in range(1, 7)}, freestream_prim(0.3), cfl=7.0)
    assert np.isclose(o.dt(q)[0], 7.0 * a / (spd + c), rtol=1e-13)


def _boundary_faces_of(o):
    L, R, S, n, gp = o.faces()
    return [f for f in range(len(L)) if R[f] < 0], n


def _riemann(q, nn):
    rho, U, p = I.prim(q)
    c = np.sqrt(GAMMA * p / rho)
    un = U @ nn
    return un + 2 * c / (GAMMA - 1), un - 2 * c / (GAMMA - 1), p / rho ** GAMMA, U - un * nn, un, c


@pytest.mark.parametrize("regime", ["subsonic", "sup_out", "sup_in"])
def test_farfield_ghost_characteristics(oracle_lib, regime):
    """Far-field ghost states against the characteristic theory of the Euler
    equations: the invariant leaving the domain comes from the interior, the
    one entering from the free stream; entropy and tangential velocity from
    the upwind side (both sides are reached); supersonic inflow takes the
    free stream, supersonic outflow the interior."""
    m = _single_tet(1.0)
    pinf = np.array([1.0, 0.4, 0.25, -0.1, 1.0 / GAMMA])
    o = oracle_lib.Oracle(m, {1: FAR}, pinf)
    qinf = prim_to_cons(pinf)
    faces, nrm = _boundary_faces_of(o)
    rng = np.random.default_rng(7)
    branches = set()
    uns = {"subsonic": (-0.7, -0.3, 0.0, 0.3, 0.7), "sup_out": (1.8,), "sup_in": (-1.9,)}[regime]
    for f in faces:
        n = nrm[:, f]
        for un in uns:
            U_t = rng.normal(scale=0.3, size=3)
            U_t -= (U_t @ n) * n
            pr = np.array([1.2, *(U_t + un * n), 0.8])
            qi = prim_to_cons(pr)
            kind, qg, _, _ = o.ghost(qi[:, None].copy(), f)
            assert kind == FAR
            if regime == "sup_in":
                assert np.allclose(qg, qinf, rtol=1e-14, atol=1e-14)
                continue
            if regime == "sup_out":
                assert np.allclose(qg, qi, rtol=1e-14, atol=1e-14)
                continue
            Jp_i, _, s_i, Ut_i, _, _ = _riemann(qi, n)
            _, Jm_inf, s_inf, Ut_inf, _, _ = _riemann(qinf, n)
            Jp_b, Jm_b, s_b, Ut_b, un_b, c_b = _riemann(qg, n)
            assert abs(un_b) < c_b
            assert np.isclose(Jp_b, Jp_i, rtol=1e-13)
            assert np.isclose(Jm_b, Jm_inf, rtol=1e-13)
            up_s, up_t = (s_i, Ut_i) if un_b >= 0 else (s_inf, Ut_inf)
            branches.add(bool(un_b >= 0))
            assert np.isclose(s_b, up_s, rtol=1e-13)
            assert np.allclose(Ut_b, up_t, rtol=1e-13, atol=1e-14)
    if regime == "subsonic":
        assert branches == {True, False}


@pytest.mark.parametrize("kind", [SLIP, NOSLIP])
def test_wall_ghost_gradient_is_the_reflected_field(oracle_lib, kind):
    """The ghost of a wall face is the owner's linear field reflected across
    the face plane, with the wall map applied to the momentum (slip: normal
    component reversed; no slip: all reversed).  Its state at the mirrored
    centroid and its gradient are taken by complex steps of that field."""
    mesh = cube_mesh(2, jitter=0.1, seed=9)
    o = oracle_lib.Oracle(mesh, {t: kind for t in range(1, 7)}, freestream_prim(0.3))
    N = o.N
    rng = np.random.default_rng(2)
    Q = prim_to_cons(freestream_prim(0.3))[:, None] * (1 + 0.05 * rng.uniform(-1, 1, size=(5, N)))
    G = rng.normal(scale=0.1, size=(15, N))
    vol, cen, _ = o.geometry()
    L, R, S, nrm, gp = o.faces()
    for f in [f for f in range(len(L)) if R[f] < 0][:12]:
        i = int(L[f])
        n = nrm[:, f]
        xf = gp[0:3, f]  # a point of the face plane
        Gi = G[:, i].reshape(5, 3)

        def ghost_field(x):
            xm = x - 2 * ((x - xf) @ n) * n            # reflected point
            q = Q[:, i] + Gi @ (xm - cen[:, i])       # owner's linear field there
            m = q[1:4]
            m = m - 2 * (m @ n) * n if kind == SLIP else -m
            return np.array([q[0], *m, q[4]])

        k, qg, gg, cg = o.ghost(Q, f, G=G)
        assert k == kind
        assert np.allclose(cg, cen[:, i] - 2 * ((cen[:, i] - xf) @ n) * n, atol=1e-14)
        assert np.allclose(qg, ghost_field(cg.astype(complex)).real, rtol=1e-14, atol=1e-14)
        hstep = 1e-30
        J = np.stack([ghost_field(cg + 1j * hstep * e).imag / hstep for e in np.eye(3)], axis=1)
        assert np.allclose(gg.reshape(5, 3), J, rtol=1e-13, atol=1e-14), (f, gg.reshape(5, 3), J)


def _mirror_full(mesh):
    """The half mesh x in [0, 1] and its mirror image across x = 0 as one mesh;
    cell i of the half has the mirror cell i + N."""
    xyz = mesh.xyz
    on = np.abs(xyz[:, 0]) < 1e-15
    assert on.sum() > 0
    off = np.where(~on)[0]
    new_id = np.arange(len(xyz))
    new_id[off] = len(xyz) + np.arange(len(off))
    mx = xyz[off] * np.array([-1.0, 1.0, 1.0])
    xyz_full = np.concatenate([xyz, mx])
    tm = new_id[mesh.tets][:, [0, 1, 3, 2]]          # mirrored, orientation restored
    tets = np.concatenate([mesh.tets, tm]).astype(np.int32)
    keep = mesh.btags != 1
    bf = np.concatenate([mesh.bfaces[keep], new_id[mesh.bfaces[keep]]]).astype(np.int32)
    bt = np.concatenate([mesh.btags[keep], mesh.btags[keep]]).astype(np.int32)
    return TetMesh(xyz=xyz_full, tets=tets, bfaces=bf, btags=bt)


def test_slip_wall_equals_mirror_image_compact(oracle_lib):
    """Compact HWENO residual and gradient update of a half cube with a slip
    wall on x = 0 against the full mesh made of the half and its mirror image
    with the mirrored state and gradients: the wall's ghost cell (state,
    gradients, centroid, moments) and its boundary flux must reproduce the
    mirror neighbour exactly."""
    half = cube_mesh(3, jitter=0.15, seed=13)
    full = _mirror_full(half)
    prim = freestream_prim(0.3, direction=(0.0, 1.0, 0.0))  # free stream parallel to the mirror plane
    kh = {1: SLIP, **{t: FAR for t in range(2, 7)}}
    kf = {t: FAR for t in range(1, 7)}
    oh = oracle_lib.Oracle(half, kh, prim, scheme=1)
    of = oracle_lib.Oracle(full, kf, prim, scheme=1)
    N = oh.N
    rng = np.random.default_rng(4)
    Qh = I.cell_averages(half, lambda x: smooth_field(x + np.array([0.2, 0.0, 0.0])))
    Gh = rng.normal(scale=0.05, size=(15, N))
    sv = np.array([1, -1, 1, 1, 1.0])                  # mirror of a conserved state
    sd = np.array([-1, 1, 1.0])                        # mirror of a derivative direction
    Qf = np.concatenate([Qh, Qh * sv[:, None]], axis=1)
    Gm = (Gh.reshape(5, 3, N) * sv[:, None, None] * sd[None, :, None]).reshape(15, N)
    Gf = np.concatenate([Gh, Gm], axis=1)
    dt_h = oh.dt(Qh)
    dt_f = np.concatenate([dt_h, dt_h])
    Rh, Gnh, _ = oh.residual(Qh, G=Gh, dt=dt_h, want_grad=True)
    Rf, Gnf, _ = of.residual(Qf, G=Gf, dt=dt_f, want_grad=True)
    scale = np.abs(Rh).max()
    assert np.abs(Rh - Rf[:, :N]).max() <= 1e-13 * scale, np.abs(Rh - Rf[:, :N]).max() / scale
    assert np.abs(Gnh - Gnf[:, :N]).max() <= 1e-13 * np.abs(Gnh).max()


def _div_flux(x, h=1e-30):
    """Divergence of the Euler flux of the smooth field, by complex steps."""
    out = 0.0
    for d in range(3):
        e = np.zeros(3)
        e[d] = 1.0
        q = smooth_field(x + 1j * h * e[None, :])
        rho = q[0]
        m = q[1:4]
        p = (GAMMA - 1) * (q[4] - 0.5 * np.sum(m * m, axis=0) / rho)
        ud = m[d] / rho
        F = np.stack([m[d], m[0] * ud, m[1] * ud, m[2] * ud, (q[4] + p) * ud])
        F[1 + d] += p
        out = out + F.imag / h
    return out


@pytest.mark.slow
def test_residual_truncation_order(oracle_lib):
    """|L(Q)/|Omega| + average of div F(Q)| over cells three hex layers from
    the boundary, WENO with nonlinear weights, in the Euler limit of the flux
    (flux interval -> 0): the observed order between n = 8, 16 and 24 is at
    least 1.8 on jittered meshes."""
    oracle_lib.set_threads(8)
    errs, hs = [], []
    for n in (8, 16, 24):
        mesh = cube_mesh(n, jitter=0.1, seed=30 + n)
        o = oracle_lib.Oracle(mesh, {t: FAR for t in range(1, 7)}, freestream_prim(0.3), cfl_flux=1e-7)
        Q = I.cell_averages(mesh, smooth_field, order=4)
        div = I.cell_averages(mesh, _div_flux, order=4)
        vol, cen, _ = o.geometry()
        R = o.residual(Q)
        inner = np.all((cen > 3.0 / n) & (cen < 1 - 3.0 / n), axis=0)
        err = np.abs(R[:, inner] / vol[inner] + div[:, inner])
        errs.append(np.mean(err))
        hs.append(1.0 / n)
    oracle_lib.set_threads(1)
    order = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert order >= 1.8, (errs, order)


@pytest.mark.parametrize("kind", [SLIP, NOSLIP, FAR, SUP_IN, SUP_OUT])
def test_boundary_right_state_and_derivatives(oracle_lib, kind):
    """The right side of a boundary Gauss point (local frame): for walls the
    value and the (n, t1, t2) derivatives of the reflected field with the
    wall map applied (complex steps of that field); for the far field the
    ghost state of the same interior state with zero derivatives; supersonic
    inflow the free stream, outflow a copy."""
    mesh = cube_mesh(2, jitter=0.1, seed=9)
    pinf = freestream_prim(0.4, direction=(0.3, 1.0, -0.2))
    o = oracle_lib.Oracle(mesh, {t: kind for t in range(1, 7)}, pinf)
    L, R, S, nrm, gp = o.faces()
    rng = np.random.default_rng(5)
    for f in [f for f in range(len(L)) if R[f] < 0][:8]:
        fr = o.face_frame(f)  # rows n, t1, t2
        Wl = I.cons(1.1, rng.normal(scale=0.3, size=3), 0.75)
        dWl = rng.normal(scale=0.1, size=(3, 5))

        def left_field(y):
            # the left state as a linear field of the local coordinates y (n, t1, t2)
            return Wl + y @ dWl

        def right_field(y):
            ym = y * np.array([-1.0, 1.0, 1.0])  # reflection across the face plane
            q = left_field(ym)
            m = q[1:4] * (np.array([-1.0, 1.0, 1.0]) if kind == SLIP else -1.0)
            return np.array([q[0], *m, q[4]])

        k, Wr, dWr = o.boundary_right(f, Wl, dWl)
        assert k == kind
        if kind in (SLIP, NOSLIP):
            assert np.allclose(Wr, right_field(np.zeros(3, complex)).real, rtol=1e-15, atol=1e-15)
            J = np.stack([right_field(1j * 1e-30 * e).imag / 1e-30 for e in np.eye(3)])
            assert np.allclose(dWr, J, rtol=1e-14, atol=1e-15)
        elif kind == FAR:
            qg_glob = np.array([Wl[0], *(fr.T @ Wl[1:4]), Wl[4]])
            Q = np.repeat(qg_glob[:, None], o.N, axis=1)
            _, qg, _, _ = o.ghost(Q, f)
            assert np.allclose(Wr, [qg[0], *(fr @ qg[1:4]), qg[4]], rtol=1e-13, atol=1e-14)
            assert np.all(dWr == 0.0)
        elif kind == SUP_IN:
            qinf = prim_to_cons(pinf)
            assert np.allclose(Wr, [qinf[0], *(fr @ qinf[1:4]), qinf[4]], rtol=1e-14, atol=1e-15)
            assert np.all(dWr == 0.0)
        else:
            assert np.array_equal(Wr, Wl) and np.array_equal(dWr, dWl)
