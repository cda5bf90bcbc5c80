"""Independent numerics used to pin the oracle (not derived from its code).

Velocity-space integrals are done by Gauss-Hermite quadrature, cell averages by
a Duffy-mapped tensor Gauss rule, derivatives by complex steps, and the Euler
and Chapman-Enskog Navier-Stokes fluxes are written from their textbook closed
forms.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4
KDOF = (5 - 3 * GAMMA) / (GAMMA - 1)  # internal degrees of freedom, 2 at gamma = 1.4


def prim(Q, gamma=GAMMA):
    rho = Q[0]
    U = np.array(Q[1:4]) / rho
    p = (gamma - 1) * (Q[4] - 0.5 * rho * U @ U)
    return rho, U, p


def cons(rho, U, p, gamma=GAMMA):
    U = np.asarray(U, dtype=float)
    return np.array([rho, *(rho * U), p / (gamma - 1) + 0.5 * rho * U @ U])


def euler_flux(Q, n, gamma=GAMMA):
    Q = np.asarray(Q)
    rho = Q[0]
    U = Q[1:4] / rho
    p = (gamma - 1) * (Q[4] - 0.5 * (Q[1:4] @ Q[1:4]) / rho)
    un = U @ np.asarray(n)
    return np.array([rho * un, *(Q[1:4] * un + p * np.asarray(n)), (Q[4] + p) * un])


def euler_jn_cs(Q, n, x, gamma=GAMMA, h=1e-30):
    """J_n(Q) x by a complex step."""
    Qc = np.asarray(Q, dtype=complex) + 1j * h * np.asarray(x)
    rho = Qc[0]
    m = Qc[1:4]
    p = (gamma - 1) * (Qc[4] - 0.5 * (m @ m) / rho)
    un = (m @ np.asarray(n)) / rho
    F = np.array([rho * un, *(m * un + p * np.asarray(n)), (Qc[4] + p) * un])
    return F.imag / h


# --- velocity space quadrature -------------------------------------------------
_GH_X, _GH_W = np.polynomial.hermite.hermgauss(40)


def _axis_nodes(U, lam):
    return U + _GH_X / np.sqrt(lam), _GH_W / np.sqrt(np.pi)


def maxwellian_moment_matrix(U, V, W, lam, K=KDOF):
    """M_kj = <psi_k psi_j> (normalised by rho) by tensor Gauss-Hermite
    quadrature in (u, v, w) and in K internal directions (K = 2)."""
    assert abs(K - 2.0) < 1e-12
    u, wu = _axis_nodes(U, lam)
    v, wv = _axis_nodes(V, lam)
    w, ww = _axis_nodes(W, lam)
    x1, w1 = _axis_nodes(0.0, lam)
    x2, w2 = _axis_nodes(0.0, lam)
    # reduce xi^2 = x1^2 + x2^2: tabulate its moments <xi^0>, <xi^2>, <xi^4>
    X1, X2 = np.meshgrid(x1, x2, indexing="ij")
    WX = np.outer(w1, w2)
    xi2 = X1 ** 2 + X2 ** 2
    mxi = [np.sum(WX * xi2 ** k) for k in range(3)]
    Uq, Vq, Wq = np.meshgrid(u, v, w, indexing="ij")
    Wt = wu[:, None, None] * wv[None, :, None] * ww[None, None, :]
    c2 = Uq ** 2 + Vq ** 2 + Wq ** 2
    # psi with xi^2 kept symbolic: psi_4 = (c2 + xi2)/2
    base = [np.ones_like(Uq), Uq, Vq, Wq]
    M = np.zeros((5, 5))
    for k in range(5):
        for j in range(5):
            if k < 4 and j < 4:
                M[k, j] = np.sum(Wt * base[k] * base[j])
            elif k < 4 or j < 4:
                b = base[k] if k < 4 else base[j]
                M[k, j] = 0.5 * (np.sum(Wt * b * c2) + np.sum(Wt * b) * mxi[1])
            else:
                M[k, j] = 0.25 * (np.sum(Wt * c2 * c2) + 2 * np.sum(Wt * c2) * mxi[1] + mxi[2])
    return M


def tet_quadrature(verts, order=6):
    """Collapsed (Duffy) tensor Gauss rule on a tetrahedron: points (P, 3),
    weights (P,) summing to the volume."""
    g, wg = np.polynomial.legendre.leggauss(order)
    g = 0.5 * (g + 1)
    wg = 0.5 * wg
    A, B, C = np.meshgrid(g, g, g, indexing="ij")
    WA, WB, WC = np.meshgrid(wg, wg, wg, indexing="ij")
    a, b, c = A.ravel(), B.ravel(), C.ravel()
    w = (WA * WB * WC).ravel() * (1 - a) ** 2 * (1 - b)
    # reference tet coordinates
    r1 = a
    r2 = b * (1 - a)
    r3 = c * (1 - a) * (1 - b)
    v0, v1, v2, v3 = [np.asarray(x) for x in verts]
    J = np.stack([v1 - v0, v2 - v0, v3 - v0], axis=1)
    pts = v0 + np.stack([r1, r2, r3], axis=1) @ J.T
    vol = abs(np.linalg.det(J))
    return pts, w * vol


# trilinear map of a hexahedron from the unit cube; corners in ring order
# (0-3 bottom counter-clockwise, 4-7 above them)
_HEX_REF = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float)


def hex_quadrature(verts, order=5):
    """Tensor Gauss rule on the trilinear image of the unit cube: points
    (P, 3), weights (P,) summing to the volume (exact for the volume, centroid
    and second moments from order 3 on)."""
    g, wg = np.polynomial.legendre.leggauss(order)
    g = 0.5 * (g + 1)
    wg = 0.5 * wg
    r, s, t = [x.ravel() for x in np.meshgrid(g, g, g, indexing="ij")]
    w = np.einsum("i,j,k->ijk", wg, wg, wg).ravel()
    v = np.asarray(verts, float)
    c = _HEX_REF
    fr = np.where(c[:, 0][None] == 1, r[:, None], 1 - r[:, None])
    fs = np.where(c[:, 1][None] == 1, s[:, None], 1 - s[:, None])
    ft = np.where(c[:, 2][None] == 1, t[:, None], 1 - t[:, None])
    sr, ss, st = 2 * c[:, 0] - 1, 2 * c[:, 1] - 1, 2 * c[:, 2] - 1
    pts = (fr * fs * ft) @ v
    dr = (sr[None] * fs * ft) @ v
    ds = (fr * ss[None] * ft) @ v
    dt = (fr * fs * st[None]) @ v
    J = np.einsum("pi,pi->p", np.cross(dr, ds), dt)
    return pts, w * J


def cell_averages(mesh, func, order=6):
    """Quadrature cell averages of func(points (P,3)) -> (5, P) for every tet
    (vectorised Duffy rule, exact for polynomials of degree <= 2*order-3), or
    every hexahedron (tensor Gauss rule on its trilinear map)."""
    if mesh.tets.shape[1] == 8:
        out = np.zeros((5, len(mesh.tets)))
        for i, h in enumerate(mesh.tets):
            pts, w = hex_quadrature(mesh.xyz[h], order=max(order, 3))
            out[:, i] = func(pts) @ w / w.sum()
        return out
    g, wg = np.polynomial.legendre.leggauss(order)
    g = 0.5 * (g + 1)
    wg = 0.5 * wg
    A, B, C = [x.ravel() for x in np.meshgrid(g, g, g, indexing="ij")]
    WA, WB, WC = [x.ravel() for x in np.meshgrid(wg, wg, wg, indexing="ij")]
    w = WA * WB * WC * (1 - A) ** 2 * (1 - B)
    r = np.stack([A, B * (1 - A), C * (1 - A) * (1 - B)], axis=1)  # (q, 3)
    v = mesh.xyz[mesh.tets]  # (N, 4, 3)
    J = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)  # (N, 3, 3)
    pts = v[:, None, 0, :] + np.einsum("nij,qj->nqi", J, r)  # (N, q, 3)
    vals = func(pts.reshape(-1, 3)).reshape(5, len(v), len(w))
    return (vals * w[None, None, :]).sum(axis=2) / w.sum()
