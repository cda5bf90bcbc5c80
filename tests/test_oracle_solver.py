"""Pins of the oracle's residual assembly and implicit solver (paper Sec. 2
Eq. (finite); Sec. 4 Eq. (impsystem), (frechet), (deri-matrix), (precond),
Algorithm 1)."""
import numpy as np
import pytest

from inputs import cube_mesh, freestream_prim, perturbed_state, prim_to_cons, shell_mesh, uniform_state
from tests import _indep as I

ALL_FAR = {t: 0 for t in range(1, 7)}


def flux_scale(o, prim):
    L, R, S, n, gp = o.faces()
    q = prim_to_cons(prim)
    f = max(np.abs(I.euler_flux(q, d)).max() for d in np.eye(3))
    per = np.zeros(o.N)
    np.add.at(per, L, S)
    np.add.at(per, R[R >= 0], S[R >= 0])
    return f * per.max()


@pytest.mark.parametrize("scheme", [0, 1])
def test_free_stream_preserved(oracle_lib, scheme):
    prim = freestream_prim(0.6, direction=(1.0, 0.4, -0.3))
    for m, kinds in [(cube_mesh(4, jitter=0.2, seed=1), ALL_FAR),
                     (shell_mesh(3, 3, grading=1.3, jitter=0.05, seed=2), {1: 0, 2: 0})]:
        o = oracle_lib.Oracle(m, kinds, prim, scheme=scheme)
        Q = uniform_state(o.N, prim)
        R, Gn, fb = o.residual(Q, G=np.zeros((15, o.N)), want_grad=True)
        assert fb == 0
        assert np.abs(R).max() <= 1e-13 * flux_scale(o, prim)
        if scheme == 1:  # gradient update of a uniform state is zero
            assert np.abs(Gn).max() <= 1e-12


@pytest.mark.parametrize("scheme", [0, 1])
def test_conservation_closed_box(oracle_lib, scheme):
    """All slip walls: interior fluxes cancel pairwise and the mirrored wall
    state carries no mass or energy through the wall, so sum_i L_rho and
    sum_i L_E vanish to round-off."""
    m = cube_mesh(4, jitter=0.2, seed=5)
    prim = freestream_prim(0.3)
    o = oracle_lib.Oracle(m, {t: oracle_lib.SLIP for t in range(1, 7)}, prim, scheme=scheme)
    Q = perturbed_state(o.N, prim, amp=0.05, seed=3)
    G = np.random.default_rng(1).normal(scale=0.05, size=(15, o.N)) if scheme == 1 else None
    R = o.residual(Q, G=G)
    s = np.abs(R).sum(axis=1)
    assert abs(R[0].sum()) <= 1e-13 * s[0]
    assert abs(R[4].sum()) <= 1e-13 * s[4]


def _richardson_dir(o, Q, dt, v, G=None):
    def d(h):
        return (o.residual(Q + h * v, G=G, dt=dt) - o.residual(Q - h * v, G=G, dt=dt)) / (2 * h)
    h = 1e-5
    return (4 * d(h / 2) - d(h)) / 3


@pytest.mark.parametrize("scheme", [0, 1])
def test_fd_jv_matches_derivative(oracle_lib, scheme):
    # The reference derivative must not straddle a kink: slip walls instead of
    # the far field (whose Riemann-invariant branch switches where u.n changes
    # sign) and C = 0 in the collision time (|p_l - p_r| has a kink at p_l = p_r).
    # A gentle state (Mach 0.05 in a closed box, CFL 1) keeps the flux free of
    # large cancellations that would swamp the comparison in round-off.
    m = cube_mesh(2, jitter=0.1, seed=2)
    prim = freestream_prim(0.05)
    o = oracle_lib.Oracle(m, {t: oracle_lib.SLIP for t in range(1, 7)}, prim, scheme=scheme, weights=1,
                          tau_C=0.0, cfl=1.0)
    Q = perturbed_state(o.N, prim, seed=4)
    G = np.random.default_rng(2).normal(scale=0.02, size=(15, o.N)) if scheme == 1 else None
    dt = o.dt(Q)
    b = o.residual(Q, G=G, dt=dt)
    v = np.random.default_rng(7).normal(size=(5, o.N))
    vol = o.geometry()[0]
    ref = vol / dt * v - _richardson_dir(o, Q, dt, v, G=G)
    scale = np.abs(ref).max()

    def err(sig):
        Av, s = o.jv(Q, dt, b, v, sigma=sig, G=G)
        assert s > 0
        return np.abs(Av - ref).max() / scale
    # forward difference: error O(sigma) (+ O(eps/sigma) round-off)
    e6, e7 = err(1e-6), err(1e-7)
    assert 7.0 < e6 / e7 < 13.0, (e6, e7)
    assert err(0.0) <= 1e-5  # automatic sigma, reading A22


def test_jacobi_preconditioner(oracle_lib):
    """D and two Jacobi sweeps of Eq. (precond) against a direct assembly of
    Eq. (deri-matrix) (supersonic-outflow boundaries make the ghost equal the
    owner, so |lambda| on a boundary face is that of the owner)."""
    m = cube_mesh(2, jitter=0.1, seed=3)
    prim = freestream_prim(0.3)
    o = oracle_lib.Oracle(m, {t: oracle_lib.SUP_OUT for t in range(1, 7)}, prim)
    Q = perturbed_state(o.N, prim, amp=0.05, seed=8)
    dt = o.dt(Q)
    vol = o.geometry()[0]
    L, R, S, n, gp = o.faces()
    N = o.N

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
    r = np.random.default_rng(0).normal(size=(5, N))
    x = r / D
    for _ in range(2):
        x = (r - offdiag(x)) / D
    np.testing.assert_allclose(o.precond(Q, dt, r), x, rtol=1e-12, atol=1e-14 * np.abs(x).max())
    # the approximate matrix itself (the GMRES operator of the paper's solver)
    y = np.random.default_rng(1).normal(size=(5, N))
    Ay = D * y + offdiag(y)
    np.testing.assert_allclose(o.amatvec(Q, dt, y), Ay, rtol=1e-12, atol=1e-14 * np.abs(Ay).max())


def test_gmres_on_the_approximate_matrix_equals_dense_solve(oracle_lib):
    """With the paper's operator (Eq. (deri-matrix)) GMRES is a linear solve:
    at full Krylov dimension one restart reproduces a dense solve of
    A dQ = L(Q^n), A assembled column by column from an independent
    complex-step Euler Jacobian, and evaluates the residual once."""
    m = cube_mesh(1, jitter=0.1, seed=4)
    prim = freestream_prim(0.3)
    kinds = {t: oracle_lib.SUP_OUT for t in range(1, 7)}
    o = oracle_lib.Oracle(m, kinds, prim, jv_mode=1, krylov_dim=30, restarts=1)
    Q = perturbed_state(o.N, prim, amp=0.05, seed=3)
    dt = o.dt(Q)
    b = o.residual(Q, dt=dt)
    vol = o.geometry()[0]
    L, R, S, n, gp = o.faces()
    N = o.N

    def lam(a, c, nn):
        ra, Ua, pa = I.prim(Q[:, a])
        rb, Ub, pb = I.prim(Q[:, c])
        rho, U, p = (ra + rb) / 2, (Ua + Ub) / 2, (pa + pb) / 2
        return abs(U @ nn) + np.sqrt(1.4 * p / rho)
    lam_f = np.array([lam(L[f], R[f] if R[f] >= 0 else L[f], n[:, f]) for f in range(len(L))])
    D = vol / dt
    np.add.at(D, L, 0.5 * lam_f * S)
    np.add.at(D, R[R >= 0], 0.5 * lam_f[R >= 0] * S[R >= 0])
    A = np.zeros((5 * N, 5 * N))
    for k in range(5 * N):
        e = np.zeros((5, N))
        e.flat[k] = 1.0
        out = D * e
        for f in np.where(R >= 0)[0]:
            a, c = L[f], R[f]
            out[:, a] += 0.5 * S[f] * (I.euler_jn_cs(Q[:, c], n[:, f], e[:, c]) - lam_f[f] * e[:, c])
            out[:, c] += 0.5 * S[f] * (I.euler_jn_cs(Q[:, a], -n[:, f], e[:, a]) - lam_f[f] * e[:, a])
        A[:, k] = out.ravel()
    ref = np.linalg.solve(A, b.ravel())
    Q1 = Q.copy()
    st, info = o.implicit_step(Q1)
    assert st == 0 and info.n_resid_evals == 1 and info.gmres_rel < 1e-10
    np.testing.assert_allclose((Q1 - Q).ravel(), ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_gmres_full_dimension_equals_dense_solve(oracle_lib):
    m = cube_mesh(1)
    prim = freestream_prim(0.3)
    o = oracle_lib.Oracle(m, ALL_FAR, prim, weights=1, krylov_dim=30, restarts=1)
    Q = perturbed_state(o.N, prim, seed=2)
    dt = o.dt(Q)
    b = o.residual(Q, dt=dt)
    n = 5 * o.N
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = o.jv(Q, dt, b, e.reshape(5, -1))[0].ravel()
    ref = np.linalg.solve(A, b.ravel())
    Q1 = Q.copy()
    st, info = o.implicit_step(Q1)
    assert st == 0 and info.n_resid_evals <= 31 and info.gmres_rel < 1e-12
    # the FD operator is linear only up to O(sigma |L''|) ~ 1e-6 relative
    # (sigma ~ 1.6e-8, |L''|/|L'| ~ 1e2), amplified by cond(A) ~ 3e3 at most
    np.testing.assert_allclose((Q1 - Q).ravel(), ref, rtol=0, atol=5e-5 * np.abs(ref).max())


def test_explicit_limit(oracle_lib):
    m = cube_mesh(2, jitter=0.1, seed=1)
    prim = freestream_prim(0.3)
    o = oracle_lib.Oracle(m, ALL_FAR, prim, cfl=1e-6)
    Q = perturbed_state(o.N, prim, seed=6)
    dt = o.dt(Q)
    b = o.residual(Q, dt=dt)
    vol = o.geometry()[0]
    Q1 = Q.copy()
    st, info = o.implicit_step(Q1)
    exp = dt / vol * b
    np.testing.assert_allclose(Q1 - Q, exp, rtol=0, atol=1e-4 * np.abs(exp).max())


@pytest.mark.slow
def test_config1_ten_steps_converge(oracle_lib):
    from inputs import mesh_for_config
    m = mesh_for_config("c1")
    prim = freestream_prim(0.3)
    o = oracle_lib.Oracle(m, ALL_FAR, prim)
    oracle_lib.set_threads(8)
    Q = perturbed_state(o.N, prim, seed=1)
    res = []
    for _ in range(10):
        st, info = o.implicit_step(Q)
        assert st == 0 and info.n_resid_evals == 33 and info.n_fallbacks == 0
        res.append(info.res)
    oracle_lib.set_threads(1)
    # at CFL 10 the preconditioned FD-Jv operator is indefinite and GMRES(10)
    # gains little per step; the density residual still falls several-fold
    assert res[-1] < 0.2 * res[0], res
    assert all(np.isfinite(res))


def test_gmres_breakdown_single_tet_is_exact(oracle_lib):
    """One tetrahedron: all four faces are boundary faces, whose off-diagonal
    blocks of Eq. (deri-matrix) are dropped, so A = D I with the scalar
    diagonal D = |Omega|/dt + sum_f lam_f S_f / 2, recomputed here from the
    face data (supersonic-inflow boundaries: the ghost is the free stream, and
    lam_f comes from the mean of the owner's and the free stream's primitive
    variables).  The Jacobi-preconditioned Arnoldi process therefore loses
    its second direction to rounding right after the first column (happy
    breakdown), and the step must be Q + L(Q)/D."""
    from tests.test_edge_cases import tiny_mesh
    m = tiny_mesh(1)
    prim = freestream_prim(0.3)
    kinds = {t: oracle_lib.SUP_IN for t in range(1, 7)}
    o = oracle_lib.Oracle(m, kinds, prim, jv_mode=1, cfl=1.0)
    Q = perturbed_state(o.N, prim, amp=0.01, seed=5)
    dt = o.dt(Q)
    b = o.residual(Q, dt=dt)
    vol = o.geometry()[0]
    L, R, S, n, gp = o.faces()
    assert o.N == 1 and (R < 0).all()
    ra, Ua, pa = I.prim(Q[:, 0])
    rb, Ub, pb = I.prim(prim_to_cons(prim))
    r, U, p = (ra + rb) / 2, (Ua + Ub) / 2, (pa + pb) / 2
    lam_f = np.array([abs(U @ n[:, f]) + np.sqrt(1.4 * p / r) for f in range(len(L))])
    D = vol[0] / dt[0] + 0.5 * (lam_f * S).sum()
    Q1 = Q.copy()
    st, info = o.implicit_step(Q1)
    assert st == 0 and info.n_resid_evals == 1 and info.gmres_rel < 1e-14
    assert np.abs(b).max() > 1e-4  # the inflow makes a residual of size
    ref = b / D
    np.testing.assert_allclose(Q1 - Q, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("scheme", [0, 1])
def test_sampled_residual_equals_full(oracle_lib, scheme):
    """The residual of a sample of cells (used at sizes where the full oracle
    residual is too slow) is the same as those cells' entries of the full
    residual, gradient update included."""
    from inputs import freestream_prim, perturbed_state, shell_mesh
    m = shell_mesh(4, 4, grading=1.3, jitter=0.05, seed=2)
    o = oracle_lib.Oracle(m, {1: 1, 2: 0}, freestream_prim(0.5), scheme=scheme)
    Q = perturbed_state(o.N, freestream_prim(0.5), seed=3)
    G = np.random.default_rng(1).normal(scale=0.01, size=(15, o.N))
    R, Gn, _ = o.residual(Q, G=G, want_grad=True)
    cells = np.random.default_rng(2).choice(o.N, 50, replace=False)
    Rs, Gs = o.residual_cells(Q, cells, G=G, want_grad=True)
    assert np.array_equal(Rs, R[:, cells]) and np.array_equal(Gs, Gn[:, cells])


def test_update_limit(oracle_lib):
    """max_update = theta: the step's change of every cell is the unlimited
    change times a power of two 2^-k (k <= 20), the largest for which density
    and pressure move by at most theta of their old values (a Mach 2 ramp at
    CFL 10 from the uniform stream, where the unlimited step changes some
    cells by far more than theta); with theta large nothing is scaled."""
    from inputs import ramp_mesh
    m = ramp_mesh(16, 6, 4, jitter=0.02, seed=4)
    kinds = {1: 3, 2: 4, 3: 1, 4: 1, 5: 1, 6: 1}
    prim = freestream_prim(2.0)
    Q0 = uniform_state(m.n_cells, prim)
    full = Q0.copy()
    ofull = oracle_lib.Oracle(m, kinds, prim, cfl=10.0, jv_mode=1)
    ofull.implicit_step(full)
    lim = Q0.copy()
    st, info = oracle_lib.Oracle(m, kinds, prim, cfl=10.0, jv_mode=1, max_update=0.2).implicit_step(lim)
    assert st == 0 and info.n_limited > 0
    d_full, d_lim = full - Q0, lim - Q0

    def pres(q):
        return 0.4 * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0])
    p0 = pres(Q0)
    scaled = 0
    for i in range(m.n_cells):
        k = np.argmax(np.abs(d_full[:, i]))
        a = d_lim[k, i] / d_full[k, i] if d_full[k, i] != 0 else 1.0
        e = np.round(-np.log2(a))
        assert 0 <= e <= 20 and abs(a - 2.0 ** -e) <= 1e-12 * a
        a = 2.0 ** -e
        np.testing.assert_allclose(d_lim[:, i], a * d_full[:, i], rtol=0, atol=1e-14 * np.abs(Q0[:, i]).max())
        ok = lambda al: (abs(al * d_full[0, i]) <= 0.2 * Q0[0, i]  # noqa: E731
                         and abs(pres(Q0[:, [i]] + al * d_full[:, [i]])[0] - p0[i]) <= 0.2 * p0[i])
        if e < 20:
            assert ok(a)
        if e > 0:
            assert not ok(2 * a)
            scaled += 1
    assert scaled == info.n_limited
    big = Q0.copy()
    oracle_lib.Oracle(m, kinds, prim, cfl=10.0, jv_mode=1, max_update=1e6).implicit_step(big)
    assert np.array_equal(big, full)


def test_relaxed_gradient_update(oracle_lib):
    """grad_relax = omega (compact scheme): the step's state update does not
    depend on omega (the gradient update is formed from the base residual at
    the old state), and the gradients after the step are G + omega (G_1 - G),
    G_1 being the gradients after the paper's step (omega = 1) from the same
    (Q, G); omega = 1 is the default."""
    m = cube_mesh(3, jitter=0.05, seed=5)
    prim = freestream_prim(0.3)
    Q0 = perturbed_state(m.n_cells, prim, amp=0.02, seed=6)
    _, G0, _ = oracle_lib.Oracle(m, ALL_FAR, prim, scheme=1).residual(Q0, np.zeros((15, m.n_cells)), want_grad=True)
    out = {}
    for w in (None, 1.0, 0.3):
        Q, G = Q0.copy(), G0.copy()
        kw = {} if w is None else {"grad_relax": w}
        st, _ = oracle_lib.Oracle(m, ALL_FAR, prim, scheme=1, **kw).implicit_step(Q, G)
        assert st == 0
        out[w] = (Q, G)
    assert np.array_equal(out[None][0], out[1.0][0]) and np.array_equal(out[None][1], out[1.0][1])
    assert np.array_equal(out[0.3][0], out[1.0][0])
    G1 = out[1.0][1]
    assert np.abs(G1 - G0).max() > 1e-3 * np.abs(G0).max()
    np.testing.assert_allclose(out[0.3][1], G0 + 0.3 * (G1 - G0), rtol=0, atol=1e-14 * np.abs(G1).max())
