"""Pins of the oracle's reconstruction (paper Sec. 3.2-3.4, Eq. (polys),
(compact-big-1/2), (weno); characteristic projection of Sec. 5).

* linear data: P0, every P_m and the nonlinear combination reproduce it
  (values and derivatives at the Gauss points), for WENO and HWENO;
* quadratic data with linear weights: Eq. (weno) collapses to P0, which
  reproduces quadratics (HWENO given the exact averaged gradients);
* smooth data: point values converge at third order on jittered meshes;
* rigid rotation of mesh and state (linear weights) rotates the residual.
"""
import numpy as np
import pytest

from inputs import cube_mesh, freestream_prim, prim_to_cons
from tests import _indep as I

Q0 = prim_to_cons(freestream_prim(0.3))
GL = np.array([[0.05, -0.03, 0.02], [0.02, 0.04, -0.01], [-0.03, 0.01, 0.03],
               [0.01, -0.02, 0.04], [0.06, 0.02, -0.05]])
HQ = np.random.default_rng(5).normal(scale=0.02, size=(5, 3, 3))
HQ = HQ + HQ.transpose(0, 2, 1)


def lin(x):
    d = x - 0.5
    return Q0[:, None] + GL @ d.T


def lin_grad(x):
    return np.repeat(GL[:, :, None], len(x), axis=2)


def quad(x):
    d = x - 0.5
    return lin(x) + np.einsum("vab,pa,pb->vp", HQ, d, d)


def quad_grad(x):
    d = x - 0.5
    return GL[:, :, None] + 2 * np.einsum("vab,pb->vap", HQ, d)


def local_expected(o, f, f_val, f_grad, gp):
    fr = o.face_frame(f)  # rows n, t1, t2
    out = np.zeros((3, 4, 5))
    for g in range(3):
        x = gp[g][None, :]
        v = f_val(x)[:, 0]
        G = f_grad(x)[:, :, 0]  # (5, 3)
        for d in range(4):
            q = v if d == 0 else G @ fr[d - 1]
            out[g, d] = [q[0], *(fr @ q[1:4]), q[4]]
    return out


def interior_faces(o, scheme):
    L, R, S, n, gp = o.faces()
    N = o.N
    ok = []
    for f in range(len(L)):
        if R[f] < 0:
            continue
        cells = [L[f], R[f]]
        if all((o.stencil(c, 0) < N).all() for c in cells):
            ok.append(f)
    return ok, gp


@pytest.mark.parametrize("scheme,weights", [(0, 0), (1, 0)])
def test_linear_data_reproduced(oracle_lib, scheme, weights):
    m = cube_mesh(5, jitter=0.15, seed=3)
    o = oracle_lib.Oracle(m, {t: 0 for t in range(1, 7)}, freestream_prim(0.3), scheme=scheme,
                          weights=weights)
    Q = I.cell_averages(m, lin, order=3)
    vol, cen, _ = o.geometry()
    G = lin_grad(cen.T).reshape(15, -1)
    faces, gp = interior_faces(o, scheme)
    assert len(faces) > 50
    GP = gp.reshape(3, 3, -1)
    for f in faces[::7]:
        exp = local_expected(o, f, lin, lin_grad, GP[:, :, f])
        for side in (0, 1):
            got, fb = o.side_values(Q, f, side, G=G)
            assert fb == 0
            np.testing.assert_allclose(got, exp, rtol=0, atol=1e-12)


@pytest.mark.parametrize("scheme", [0, 1])
def test_quadratic_data_linear_weights(oracle_lib, scheme):
    m = cube_mesh(5, jitter=0.15, seed=4)
    o = oracle_lib.Oracle(m, {t: 0 for t in range(1, 7)}, freestream_prim(0.3), scheme=scheme, weights=1)
    Q = I.cell_averages(m, quad, order=3)
    # cell-averaged gradient of a quadratic is its gradient at the centroid
    vol, cen, _ = o.geometry()
    G = quad_grad(cen.T).reshape(15, -1)
    faces, gp = interior_faces(o, scheme)
    GP = gp.reshape(3, 3, -1)
    for f in faces[::7]:
        exp = local_expected(o, f, quad, quad_grad, GP[:, :, f])
        for side in (0, 1):
            got, _ = o.side_values(Q, f, side, G=G)
            np.testing.assert_allclose(got, exp, rtol=0, atol=1e-12)


def smooth(x):
    s = np.stack([np.sin(2 * np.pi * x[:, 0] + 0.3) * np.cos(2 * np.pi * x[:, 1]),
                  np.cos(2 * np.pi * x[:, 1] - 0.2) * np.sin(2 * np.pi * x[:, 2] + 0.1),
                  np.sin(2 * np.pi * (x[:, 0] + x[:, 2])),
                  np.cos(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 2]),
                  np.sin(2 * np.pi * (x[:, 0] - x[:, 1]))])
    return Q0[:, None] + 0.02 * s


@pytest.mark.slow
def test_third_order_point_values(oracle_lib):
    errs = []
    for n in (6, 12, 24):
        m = cube_mesh(n, jitter=0.1, seed=n)
        o = oracle_lib.Oracle(m, {t: 0 for t in range(1, 7)}, freestream_prim(0.3))
        Q = I.cell_averages(m, smooth, order=3)
        L, R, S, nrm, gp = o.faces()
        GP = gp.reshape(3, 3, -1)
        fc = GP.mean(axis=0)
        cand = np.where((R >= 0) & np.all((fc > 0.35) & (fc < 0.65), axis=0))[0]
        cand = cand[np.linspace(0, len(cand) - 1, 120).astype(int)]
        e = 0.0
        for f in cand:
            fr = o.face_frame(f)
            got, _ = o.side_values(Q, f, 0)
            ex = smooth(GP[:, :, f])
            for g in range(3):
                q = ex[:, g]
                e = max(e, np.abs(got[g, 0] - np.array([q[0], *(fr @ q[1:4]), q[4]])).max())
        errs.append(e)
    rates = [np.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert rates[-1] > 2.5, (errs, rates)


def test_residual_rotation_covariance(oracle_lib):
    th = np.array([0.3, -0.5, 0.8])
    Kx = np.array([[0, -th[2], th[1]], [th[2], 0, -th[0]], [-th[1], th[0], 0]])
    from scipy.linalg import expm
    Rm = expm(Kx)
    m = cube_mesh(3, jitter=0.15, seed=9)
    prim = freestream_prim(0.4)
    Q = I.cell_averages(m, smooth, order=3)
    o = oracle_lib.Oracle(m, {t: 0 for t in range(1, 7)}, prim, weights=1)
    R = o.residual(Q)
    m2 = cube_mesh(3, jitter=0.15, seed=9)
    m2.xyz = m.xyz @ Rm.T
    prim2 = prim.copy()
    prim2[1:4] = Rm @ prim[1:4]
    Q2 = Q.copy()
    Q2[1:4] = Rm @ Q[1:4]
    o2 = oracle_lib.Oracle(m2, {t: 0 for t in range(1, 7)}, prim2, weights=1)
    R2 = o2.residual(Q2)
    Rexp = R.copy()
    Rexp[1:4] = Rm @ R[1:4]
    scale = np.abs(R).max()
    np.testing.assert_allclose(R2, Rexp, rtol=0, atol=1e-11 * scale)
