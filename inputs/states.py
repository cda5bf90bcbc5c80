"""Seeded initial states (conserved variables, variable-major [5][N])."""
from __future__ import annotations

import numpy as np


def freestream_prim(mach: float, gamma: float = 1.4, direction=(1.0, 0.0, 0.0)) -> np.ndarray:
    """(rho, U, V, W, p) = (1, Ma * direction, 1/gamma): unit sound speed."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    u = mach * d
    return np.array([1.0, u[0], u[1], u[2], 1.0 / gamma])


def prim_to_cons(prim: np.ndarray, gamma: float = 1.4) -> np.ndarray:
    """Primitive (rho,U,V,W,p) -> conserved (rho, rho U, rho V, rho W, rho E).
    Works on (5,) or (5, N)."""
    prim = np.asarray(prim, dtype=np.float64)
    rho, u, v, w, p = prim
    return np.stack([rho, rho * u, rho * v, rho * w,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])


def uniform_state(n: int, prim: np.ndarray, gamma: float = 1.4) -> np.ndarray:
    q = prim_to_cons(prim, gamma)
    return np.ascontiguousarray(np.repeat(q[:, None], n, axis=1))


def perturbed_state(n: int, prim: np.ndarray, gamma: float = 1.4, amp: float = 0.01,
                    seed: int = 1) -> np.ndarray:
    """Free stream with a seeded uniform-random perturbation: rho and p are
    multiplied by (1 + amp r), each velocity component gets amp |U_inf| r added,
    r ~ U[-1, 1] independently per cell and variable."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(-1.0, 1.0, size=(5, n))
    speed = float(np.linalg.norm(prim[1:4]))
    pr = np.empty((5, n))
    pr[0] = prim[0] * (1.0 + amp * r[0])
    for k in range(1, 4):
        pr[k] = prim[k] + amp * speed * r[k]
    pr[4] = prim[4] * (1.0 + amp * r[4])
    return np.ascontiguousarray(prim_to_cons(pr, gamma))
