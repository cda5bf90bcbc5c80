"""Pins of the oracle's kinetic layer (paper Sec. 2, Eq. (flux) and the moment
systems below it; Sec. 5 collision time) against independent numerics.

Each pin is chosen so that a plausible slip (dropped term, wrong sign, a
transposed operand, a wrong half-space limit) fails one of them:
  * Maxwellian moments vs direct quadrature (half and full space);
  * the 5x5 slope systems vs a numpy solve of a quadrature-built matrix;
  * zero slopes: flux = time-weighted mix of Euler(Q0) and the KFVS flux,
    both evaluated by quadrature (exact for any tau);
  * continuous data: flux = Euler - tau <u psi (a.u + A)> + dt/2 <u psi A>,
    evaluated by quadrature, and the same equals the Chapman-Enskog
    Navier-Stokes flux with mu = tau p, Pr = 1 (textbook closed form);
  * Prandtl fix in the dt -> 0 limit: heat flux scaled by 1/Pr;
  * point value Q_G at t^n equals the state for continuous data;
  * mirror antisymmetry and invariance under rotating (t1, t2) about n.
"""
import numpy as np
import pytest
from scipy import integrate

from tests import _indep as I

GAM = 1.4
K = I.KDOF


class VQuad:
    """Tensor quadrature for E[f(u, v, w, s)] under the normalised Maxwellian,
    s = xi^2 (for K = 2, xi^2 is exponential with rate lam)."""

    def __init__(self, U, V, W, lam, half=0):
        if half == 0:
            x, wx = np.polynomial.hermite.hermgauss(24)
            u, wu = U + x / np.sqrt(lam), wx / np.sqrt(np.pi)
        else:
            lo, hi = (0.0, max(U, 0) + 14 / np.sqrt(lam)) if half > 0 else (min(U, 0) - 14 / np.sqrt(lam), 0.0)
            g, wg = np.polynomial.legendre.leggauss(160)
            u = 0.5 * (hi - lo) * (g + 1) + lo
            wu = 0.5 * (hi - lo) * wg * np.sqrt(lam / np.pi) * np.exp(-lam * (u - U) ** 2)
        x, wx = np.polynomial.hermite.hermgauss(24)
        v, wv = V + x / np.sqrt(lam), wx / np.sqrt(np.pi)
        w, ww = W + x / np.sqrt(lam), wx / np.sqrt(np.pi)
        sx, sw = np.polynomial.laguerre.laggauss(12)
        s, ws = sx / lam, sw
        UU, VV, WW, SS = np.meshgrid(u, v, w, s, indexing="ij")
        self.u, self.v, self.w, self.s = UU.ravel(), VV.ravel(), WW.ravel(), SS.ravel()
        self.wt = (wu[:, None, None, None] * wv[None, :, None, None] * ww[None, None, :, None]
                   * ws[None, None, None, :]).ravel()
        self.psi = np.stack([np.ones_like(self.u), self.u, self.v, self.w,
                             0.5 * (self.u ** 2 + self.v ** 2 + self.w ** 2 + self.s)])

    def E(self, f):
        return (self.psi * (self.wt * f)).sum(axis=1)

    def poly(self, a):
        return a @ self.psi


def lam_of(W):
    rho, U, p = I.prim(W)
    return rho, U, p, rho / (2 * p)


@pytest.fixture(scope="module")
def orc(oracle_lib):
    from inputs import cube_mesh, freestream_prim
    m = cube_mesh(1)
    return lambda **kw: oracle_lib.Oracle(m, {t: 0 for t in range(1, 7)}, freestream_prim(0.5), **kw)


@pytest.mark.parametrize("half", [-1, 0, 1])
@pytest.mark.parametrize("U,lam", [(0.3, 0.7), (-1.2, 2.5), (2.0, 0.4)])
def test_moments_vs_quadrature(oracle_lib, half, U, lam):
    for a in range(7):
        f = lambda u: u ** a * np.sqrt(lam / np.pi) * np.exp(-lam * (u - U) ** 2)  # noqa: E731
        lo, hi = {1: (0, np.inf), -1: (-np.inf, 0), 0: (-np.inf, np.inf)}[half]
        ref = integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-13, limit=200)[0]
        got = oracle_lib.moment(U, 0.1, -0.2, lam, K, half, a, 0, 0, 0)
        assert got == pytest.approx(ref, rel=1e-11, abs=1e-13)
    # v, w and xi moments
    q = VQuad(U, 0.1, -0.2, lam)
    for (b, c, d) in [(1, 0, 0), (2, 0, 0), (3, 1, 0), (0, 2, 1), (1, 1, 2), (0, 0, 1)]:
        ref = np.sum(q.wt * q.v ** b * q.w ** c * q.s ** d)
        got = oracle_lib.moment(U, 0.1, -0.2, lam, K, 0, 0, b, c, d)
        assert got == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("seed", range(4))
def test_slope_solve_vs_quadrature(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    U, V, W = rng.uniform(-1, 1, 3)
    lam = rng.uniform(0.3, 3)
    rhs = rng.normal(size=5)
    M = I.maxwellian_moment_matrix(U, V, W, lam)
    ref = np.linalg.solve(M, rhs)
    got = oracle_lib.slope_solve(U, V, W, lam, K, rhs)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    # <a psi> reproduces the right-hand side
    q = VQuad(U, V, W, lam)
    np.testing.assert_allclose(q.E(q.poly(got)), rhs, rtol=1e-10, atol=1e-12)


def test_euler_jacobian_vs_complex_step(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(5):
        Q = I.cons(rng.uniform(0.5, 2), rng.uniform(-1, 1, 3), rng.uniform(0.3, 2))
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        x = rng.normal(size=5)
        np.testing.assert_allclose(oracle_lib.euler_jn(GAM, Q, n, x), I.euler_jn_cs(Q, n, x), rtol=1e-12,
                                   atol=1e-13)


def _time_integrals(dt, tau):
    x = dt / tau
    e, em1 = np.exp(-x), -np.expm1(-x)
    return (dt - tau * em1, tau * em1)


def test_zero_slope_flux_is_euler_kfvs_mix(orc):
    """Zero slopes: f = (1 - e^{-t/tau}) g0 + e^{-t/tau} (g_l H + g_r (1 - H)),
    time-averaged; Q0 from half-space moments (all by quadrature)."""
    o = orc(tau_eps=0.37, tau_C=1.0)
    Wl = I.cons(1.2, [0.4, 0.1, -0.3], 0.9)
    Wr = I.cons(0.8, [-0.2, 0.3, 0.2], 0.6)
    z = np.zeros((3, 5))
    dt = 0.013
    rl, Ul, pl, ll = lam_of(Wl)
    rr, Ur, pr, lr = lam_of(Wr)
    ql, qr = VQuad(*Ul, ll, +1), VQuad(*Ur, lr, -1)
    Q0 = rl * ql.E(1.0) + rr * qr.E(1.0)
    kfvs = rl * ql.E(ql.u) + rr * qr.E(qr.u)
    tau = (0.37 + abs(pl - pr) / (pl + pr)) * dt
    T1, T4 = _time_integrals(dt, tau)
    ref = (T1 * I.euler_flux(Q0, [1, 0, 0]) + T4 * kfvs) / dt
    got = o.gks_point(Wl, z, Wr, z, dt)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12)


def _continuous_reference(W, dW, tau, dt):
    """Flux and point value of Eq. (flux) for l = r, by quadrature:
    F = rho [<u psi> - tau <u psi (a.u + A)> + dt/2 <u psi A>]."""
    rho, U, p, lam = lam_of(W)
    M = I.maxwellian_moment_matrix(*U, lam)
    q = VQuad(*U, lam)
    vel = [q.u, q.v, q.w]
    a = [np.linalg.solve(M, dW[d] / rho) for d in range(3)]
    au = sum(q.poly(a[d]) * vel[d] for d in range(3))
    A = np.linalg.solve(M, -q.E(au))
    Ap = q.poly(A)
    F = rho * (q.E(q.u) - tau * q.E(q.u * (au + Ap)) + 0.5 * dt * q.E(q.u * Ap))
    # point value of Eq. (point) at t^n (local t = 0): f = g [1 - tau (a.u + A)]
    QG = rho * (q.E(1.0) - tau * q.E(au + Ap))
    return F, QG


def _ns_closed_form(W, dW, mu, dt, Pr=1.0):
    """Euler flux minus the Chapman-Enskog viscous flux of BGK with K internal
    degrees of freedom (stress with bulk term 2/(K+3), heat flux mu/Pr dh)."""
    rho, U, p = I.prim(W)
    dr = np.array([dW[d][0] for d in range(3)])
    dU = np.array([[(dW[d][1 + k] - U[k] * dW[d][0]) / rho for k in range(3)] for d in range(3)])  # dU[d][k]
    dp = np.array([(GAM - 1) * (dW[d][4] - U @ dW[d][1:4] + 0.5 * U @ U * dW[d][0]) for d in range(3)])
    div = np.trace(dU)
    sig = mu * (dU + dU.T - 2.0 / (K + 3) * div * np.eye(3))  # sig[d][k]
    dh = GAM / (GAM - 1) * (dp[0] / rho - p * dr[0] / rho ** 2)
    Fv = np.array([0.0, *sig[0], sig[0] @ U + mu / Pr * dh])
    Qt = -sum(I.euler_jn_cs(W, np.eye(3)[d], dW[d]) for d in range(3))
    return I.euler_flux(W, [1, 0, 0]) - Fv + 0.5 * dt * I.euler_jn_cs(W, [1, 0, 0], Qt), Qt


@pytest.mark.parametrize("seed", range(3))
def test_continuous_flux_vs_quadrature_and_navier_stokes(orc, seed):
    rng = np.random.default_rng(10 + seed)
    W = I.cons(rng.uniform(0.7, 1.3), rng.uniform(-0.6, 0.6, 3), rng.uniform(0.5, 1.2))
    dW = rng.normal(scale=0.3, size=(3, 5))
    dt = 0.02
    o = orc(tau_eps=0.1, tau_C=1.0)
    tau = 0.1 * dt
    F, QG = o.gks_point(W, dW, W, dW, dt, want_qg=True)
    Fq, QGq = _continuous_reference(W, dW, tau, dt)
    np.testing.assert_allclose(F, Fq, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(QG, QGq, rtol=1e-9, atol=1e-11)
    Fns, Qt = _ns_closed_form(W, dW, tau * I.prim(W)[2], dt)
    np.testing.assert_allclose(F, Fns, rtol=1e-9, atol=1e-11)
    # Eq. (point) for continuous data at t^n: the compatibility condition
    # <psi (a.u + A)> = 0 makes the point value the state itself
    np.testing.assert_allclose(QG, W, rtol=1e-9, atol=1e-11)


def test_euler_limit(orc):
    """epsilon = C = 0 (tau = 0): continuous data gives F_E + dt/2 J_n Q_t."""
    o = orc(tau_eps=0.0, tau_C=0.0)
    W = I.cons(1.1, [0.3, -0.2, 0.1], 0.8)
    dW = np.random.default_rng(4).normal(scale=0.2, size=(3, 5))
    F = o.gks_point(W, dW, W, dW, 0.01)
    ref, _ = _ns_closed_form(W, dW, 0.0, 0.01)
    np.testing.assert_allclose(F, ref, rtol=1e-11, atol=1e-13)


def test_prandtl_fix_small_dt(orc):
    mu, Pr = 0.05, 0.72
    o = orc(physics=1, mu=mu, prandtl=Pr, tau_C=1.0)
    W = I.cons(1.0, [0.5, 0.2, -0.1], 0.7)
    dW = np.random.default_rng(5).normal(scale=0.2, size=(3, 5))
    dt = 1e-9
    F = o.gks_point(W, dW, W, dW, dt)
    ref, _ = _ns_closed_form(W, dW, mu, 0.0, Pr=Pr)
    np.testing.assert_allclose(F, ref, rtol=1e-7, atol=1e-9)


def _mirror(W):
    return W * np.array([1, -1, 1, 1, 1])


def test_mirror_antisymmetry(orc):
    o = orc(tau_eps=0.1, tau_C=1.0)
    rng = np.random.default_rng(6)
    Wl = I.cons(1.2, [0.4, 0.1, -0.3], 0.9)
    Wr = I.cons(0.9, [0.1, 0.2, 0.2], 0.7)
    dl, dr = rng.normal(scale=0.3, size=(2, 3, 5))
    Mv = np.array([1, -1, 1, 1, 1])
    F = o.gks_point(Wl, dl, Wr, dr, 0.02)
    mir = lambda d: np.stack([-Mv * d[0], Mv * d[1], Mv * d[2]])  # noqa: E731
    F2 = o.gks_point(_mirror(Wr), mir(dr), _mirror(Wl), mir(dl), 0.02)
    np.testing.assert_allclose(F2, -Mv * F, rtol=1e-11, atol=1e-13)


def test_tangent_rotation_invariance(orc):
    o = orc(tau_eps=0.1, tau_C=1.0)
    rng = np.random.default_rng(7)
    Wl = I.cons(1.2, [0.4, 0.1, -0.3], 0.9)
    Wr = I.cons(0.9, [0.1, 0.2, 0.2], 0.7)
    dl, dr = rng.normal(scale=0.3, size=(2, 3, 5))
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])

    def rot_state(W):
        W = W.copy()
        W[2:4] = R @ W[2:4]
        return W

    def rot_der(d):
        d = np.array([rot_state(x) for x in d])
        d[1:3] = np.tensordot(R, d[1:3], axes=1)
        return d
    F = o.gks_point(Wl, dl, Wr, dr, 0.02)
    F2 = o.gks_point(rot_state(Wl), rot_der(dl), rot_state(Wr), rot_der(dr), 0.02)
    np.testing.assert_allclose(F2, rot_state(F), rtol=1e-11, atol=1e-13)


# ---------------------------------------------------------------------------
# first-order KFVS flux (the Mach 3 sphere retest of Sec. 5): free transport of
# the two half-space Maxwellians of the cell averages
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(3))
def test_kfvs_point_vs_quadrature(orc, seed):
    """F = rho_l <u psi>_{u>0} + rho_r <u psi>_{u<0} and the half-space
    density moments, against the tensor quadrature of the two half spaces."""
    rng = np.random.default_rng(40 + seed)
    Wl = I.cons(rng.uniform(0.5, 2), rng.uniform(-1.5, 1.5, 3), rng.uniform(0.3, 2))
    Wr = I.cons(rng.uniform(0.5, 2), rng.uniform(-1.5, 1.5, 3), rng.uniform(0.3, 2))
    rl, Ul, pl, ll = lam_of(Wl)
    rr, Ur, pr, lr = lam_of(Wr)
    ql, qr = VQuad(*Ul, ll, +1), VQuad(*Ur, lr, -1)
    F, QG = orc(first_order=1).kfvs_point(Wl, Wr, want_qg=True)
    np.testing.assert_allclose(F, rl * ql.E(ql.u) + rr * qr.E(qr.u), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(QG, rl * ql.E(1.0) + rr * qr.E(1.0), rtol=1e-11, atol=1e-13)


def test_kfvs_special_cases(orc):
    """Equal states: the two half spaces add up to the full Maxwellian, so the
    flux is the Euler flux and the density moments the state itself.  A
    Mach 8 stream moving away from the right state: the left state's u<0 tail
    and the right state's u<0 half are below 1e-19 of the flux, so the flux
    is the Euler flux of the left state."""
    o = orc(first_order=1)
    rng = np.random.default_rng(47)
    for _ in range(4):
        W = I.cons(rng.uniform(0.5, 2), rng.uniform(-1, 1, 3), rng.uniform(0.3, 2))
        F, QG = o.kfvs_point(W, W, want_qg=True)
        np.testing.assert_allclose(F, I.euler_flux(W, [1, 0, 0]), rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(QG, W, rtol=1e-13, atol=1e-14)
    c = np.sqrt(GAM * 1.0 / 1.2)
    Wl = I.cons(1.2, [8.0 * c, 0.3, -0.2], 1.0)
    Wr = I.cons(0.7, [9.0, 0.1, 0.0], 0.5)  # sound speed 1: the right state streams right at Mach 9
    np.testing.assert_allclose(o.kfvs_point(Wl, Wr), I.euler_flux(Wl, [1, 0, 0]), rtol=1e-14, atol=0)


def test_kfvs_is_free_transport_limit(orc):
    """Zero slopes and tau >> dt: the collision-free limit of the gas-kinetic
    flux of Eq. (flux) is the KFVS flux."""
    Wl = I.cons(1.1, [0.4, -0.3, 0.2], 0.8)
    Wr = I.cons(0.9, [-0.1, 0.2, 0.5], 1.1)
    z = np.zeros((3, 5))
    got = orc(tau_eps=1e12, tau_C=0.0).gks_point(Wl, z, Wr, z, 1e-3)
    np.testing.assert_allclose(got, orc(first_order=1).kfvs_point(Wl, Wr), rtol=1e-10, atol=1e-13)


def _faces_brute(mesh):
    """Faces of a tet mesh by matching sorted node triples: (owner, neighbour
    or -1, unit normal out of the owner, area)."""
    xyz, tets = mesh.xyz, mesh.tets
    seen, out = {}, []
    for t, tet in enumerate(tets):
        for p in range(4):
            tri = np.delete(tet, p)
            key = tuple(sorted(tri))
            if key in seen:
                out[seen[key]][1] = t
                continue
            a, b, c = xyz[tri]
            nv = np.cross(b - a, c - a)
            if nv @ (xyz[tet[p]] - a) > 0:
                nv = -nv
            seen[key] = len(out)
            out.append([t, -1, nv / np.linalg.norm(nv), 0.5 * np.linalg.norm(nv)])
    return out


@pytest.mark.parametrize("mach", [0.5, 3.0])
def test_kfvs_residual_brute_force(oracle_lib, mach):
    """First-order residual of a jittered cube, supersonic inflow on every
    boundary (right state = free stream): faces, normals and areas found by
    brute force, a tangent frame of the test's own choosing, the flux from
    the pinned point function; L_i = -sum of outward face fluxes times area."""
    from inputs import cube_mesh, freestream_prim, perturbed_state
    m = cube_mesh(2, jitter=0.15, seed=5)
    prim = freestream_prim(mach)
    o = oracle_lib.Oracle(m, {t: oracle_lib.SUP_IN for t in range(1, 7)}, prim, first_order=1)
    Q = perturbed_state(o.N, prim, amp=0.05, seed=6)
    qinf = I.cons(prim[0], prim[1:4], prim[4])
    R = np.zeros((5, o.N))
    for L, Rn, n, S in _faces_brute(m):
        t1 = np.cross(n, [0.6, 0.0, 0.8]) if abs(n @ [0.6, 0.0, 0.8]) < 0.9 else np.cross(n, [0.0, 1.0, 0.0])
        t1 /= np.linalg.norm(t1)
        t2 = np.cross(n, t1)
        Rot = np.array([n, t1, t2])
        loc = lambda q: np.concatenate([[q[0]], Rot @ q[1:4], [q[4]]])  # noqa: E731
        qr = Q[:, Rn] if Rn >= 0 else qinf
        Fl = o.kfvs_point(loc(Q[:, L]), loc(qr))
        Fg = np.concatenate([[Fl[0]], Rot.T @ Fl[1:4], [Fl[4]]])
        R[:, L] -= S * Fg
        if Rn >= 0:
            R[:, Rn] += S * Fg
    got = o.residual(Q)
    np.testing.assert_allclose(got, R, rtol=0, atol=1e-13 * np.abs(R).max())


def test_kfvs_free_stream_preserved(oracle_lib):
    """A uniform free stream with far-field boundaries is a steady state of
    the first-order residual (closed cells: the face normals times areas sum
    to zero, and equal states give the Euler flux)."""
    from inputs import cube_mesh, freestream_prim
    m = cube_mesh(3, jitter=0.15, seed=8)
    prim = freestream_prim(0.7, direction=(1.0, 0.4, -0.3))
    o = oracle_lib.Oracle(m, {t: oracle_lib.FARFIELD for t in range(1, 7)}, prim, first_order=1)
    q = I.cons(prim[0], prim[1:4], prim[4])
    Q = np.repeat(q[:, None], o.N, axis=1)
    assert np.abs(o.residual(Q)).max() < 1e-14


@pytest.mark.parametrize("seed", range(2))
def test_discontinuous_flux_with_slopes_vs_quadrature(orc, seed):
    """Different left and right states, each with its own slopes in the three
    local directions: the time average of Eq. (flux) with every velocity
    moment taken by quadrature and the time integral by a Gauss rule in t.
    The slopes a^{l,r} solve <a psi> = dW / rho, the equilibrium slopes come
    from the kinetic-weighted derivative of Q0 (both half spaces, reading A6),
    and A^{l,r}, A-bar from the compatibility condition <a.u + A> = 0, all by
    quadrature."""
    rng = np.random.default_rng(40 + seed)
    Wl = I.cons(rng.uniform(0.8, 1.3), rng.uniform(-0.5, 0.5, 3), rng.uniform(0.6, 1.1))
    Wr = I.cons(rng.uniform(0.6, 1.1), rng.uniform(-0.5, 0.5, 3), rng.uniform(0.5, 1.0))
    dWl = rng.normal(scale=0.3, size=(3, 5))
    dWr = rng.normal(scale=0.3, size=(3, 5))
    dt = 0.015
    eps_t, C_t = 0.1, 1.0
    o = orc(tau_eps=eps_t, tau_C=C_t)
    got = o.gks_point(Wl, dWl, Wr, dWr, dt)

    def side(W, dW, half):
        rho, U, p, lam = lam_of(W)
        M = I.maxwellian_moment_matrix(*U, lam)
        full = VQuad(*U, lam)
        a = [np.linalg.solve(M, dW[d] / rho) for d in range(3)]
        A = np.linalg.solve(M, -full.E(sum(full.poly(a[d]) * [full.u, full.v, full.w][d] for d in range(3))))
        return rho, p, a, A, VQuad(*U, lam, half)

    rl, pl, al, Al, hl = side(Wl, dWl, +1)
    rr, pr, ar, Ar, hr = side(Wr, dWr, -1)
    Q0 = rl * hl.E(1.0) + rr * hr.E(1.0)
    r0, U0, p0 = I.prim(Q0)
    lam0 = r0 / (2 * p0)
    M0 = I.maxwellian_moment_matrix(*U0, lam0)
    q0 = VQuad(*U0, lam0)
    ab = [np.linalg.solve(M0, (rl * hl.E(hl.poly(al[d])) + rr * hr.E(hr.poly(ar[d]))) / r0) for d in range(3)]
    vel0 = [q0.u, q0.v, q0.w]
    abu = sum(q0.poly(ab[d]) * vel0[d] for d in range(3))
    Ab = np.linalg.solve(M0, -q0.E(abu))
    alu = sum(hl.poly(al[d]) * [hl.u, hl.v, hl.w][d] for d in range(3))
    aru = sum(hr.poly(ar[d]) * [hr.u, hr.v, hr.w][d] for d in range(3))
    # the velocity moments of u psi times each term of Eq. (flux)
    E_g0, E_g0a, E_g0A = q0.E(q0.u), q0.E(q0.u * abu), q0.E(q0.u * q0.poly(Ab))
    E_l, E_la, E_lA = hl.E(hl.u), hl.E(hl.u * alu), hl.E(hl.u * hl.poly(Al))
    E_r, E_ra, E_rA = hr.E(hr.u), hr.E(hr.u * aru), hr.E(hr.u * hr.poly(Ar))
    tau = (eps_t + C_t * abs(pl - pr) / (pl + pr)) * dt
    tg, wg = np.polynomial.legendre.leggauss(60)
    ref = np.zeros(5)
    for t, w in zip(0.5 * dt * (tg + 1), 0.5 * dt * wg):
        e = np.exp(-t / tau)
        f = r0 * ((1 - e) * E_g0 + ((t + tau) * e - tau) * E_g0a + (t - tau + tau * e) * E_g0A)
        f += e * rl * (E_l - (t + tau) * E_la - tau * E_lA)
        f += e * rr * (E_r - (t + tau) * E_ra - tau * E_rA)
        ref += w * f
    ref /= dt
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-11)


def _receding_pair(x, rng, mirror=True):
    """Two states that both stream away from the face, the normal speed being
    x thermal speeds (x = sqrt(lam) |U|): the left one towards -n, the right
    one towards +n (a mirror pair is the slip-wall case)."""
    rl, pl = rng.uniform(0.2, 1.5), rng.uniform(0.01, 1.0)
    Ul = -x / np.sqrt(rl / (2 * pl))
    Wl = I.cons(rl, [Ul, *rng.normal(size=2)], pl)
    if mirror:
        Wr = Wl * np.array([1, -1, 1, 1, 1])
    else:
        rr, pr = rng.uniform(0.2, 1.5), rng.uniform(0.01, 1.0)
        Wr = I.cons(rr, [x / np.sqrt(rr / (2 * pr)), *rng.normal(size=2)], pr)
    return Wl, Wr


@pytest.mark.parametrize("physics", [0, 1])
def test_vacuum_interface(orc, physics):
    """Reading A34: where the half-space tails that reach the face carry less
    than 2^-40 of the adjacent densities (checked here by quadrature of the
    two tails, independently of the oracle's erfc), the face is vacuum and
    its flux and point value are zero.  Just above that fraction the flux is
    still of the size of the tails (zero slopes: below 1e-9 of the stream's
    momentum flux), so the rule does not cut off anything the residual sums
    would resolve."""
    o = orc(physics=1, mu=0.006, prandtl=0.72) if physics else orc()
    rng = np.random.default_rng(71 + physics)
    z = np.zeros((3, 5))
    for x, mirror in [(8.0, True), (9.0, False), (6.5, True)]:
        Wl, Wr = _receding_pair(x, rng, mirror)
        rl, Ul, pl, ll = lam_of(Wl)
        rr, Ur, pr, lr = lam_of(Wr)
        tail = rl * VQuad(*Ul, ll, +1).E(1.0)[0] + rr * VQuad(*Ur, lr, -1).E(1.0)[0]
        assert tail < 2.0 ** -40 * (rl + rr)
        d = rng.normal(size=(2, 3, 5))
        F, QG = o.gks_point(Wl, d[0], Wr, d[1], 0.05, want_qg=True)
        assert np.all(F == 0.0) and np.all(QG == 0.0)
    if not physics:
        # x = 4.8: tail fraction about 1e-11, above the cut
        Wl, Wr = _receding_pair(4.8, rng, True)
        rl, Ul, pl, ll = lam_of(Wl)
        tail = 2 * rl * VQuad(*Ul, ll, +1).E(1.0)[0]
        assert 2.0 ** -40 * 2 * rl < tail < 1e-9 * 2 * rl
        F = o.gks_point(Wl, z, Wr, z, 0.05)
        assert np.all(np.isfinite(F)) and np.abs(F).max() < 1e-9 * rl * (Ul @ Ul + pl / rl)
