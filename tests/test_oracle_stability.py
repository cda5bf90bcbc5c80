"""Linear stability of the spatial scheme at a uniform stream (reading A36).

The residual of a uniform stream is zero, and its linearisation there is the
operator whose eigenvalues decide whether pseudo-time marching can settle: an
eigenvalue with positive real part is a mode that grows (or, under backward
Euler at large steps, alternates from step to step without decaying).  The
Jacobian here is formed by brute-force central differences of the oracle's
residual (independent of any linearisation in the oracle), scaled by the cell
volumes.  On a far-field cube every eigenvalue must lie in the left half
plane; with the quadratic P0 fit in the cells on the cube's edges the largest
real part was +67 per unit time (the spectrum reaching down to -124),
localised at those cells, while the first-order KFVS scheme was stable; with
the linear fit there it is -0.85 (the spectrum reaching down to -32).

The Navier-Stokes form at a cell Reynolds number of about 50 (mu = 0.002)
with Pr = 0.72 had a growing mode (+0.51) while Pr = 1 had none: the
Prandtl correction then rescaled the energy flux's whole heat-flux moment of
the time-averaged distribution, numerical transport included.  With the
correction taken as the Fourier flux of the interface temperature gradient
(reading A19) the largest real part is -0.72.
"""
import numpy as np
import pytest

from inputs import cube_mesh, freestream_prim, uniform_state


def _spectrum(oracle_lib, **opts):
    prim = freestream_prim(0.3)
    o = oracle_lib.Oracle(cube_mesh(3), {t: 0 for t in range(1, 7)}, prim, **opts)
    Q0 = uniform_state(o.N, prim)
    dt = o.dt(Q0)
    vol, _, _ = o.geometry()
    n = 5 * o.N
    J = np.zeros((n, n))
    h = 1e-6
    for k in range(n):
        v, c = divmod(k, o.N)
        sc = max(1.0, abs(Q0[v, c]))
        Qp, Qm = Q0.copy(), Q0.copy()
        Qp[v, c] += h * sc
        Qm[v, c] -= h * sc
        J[:, k] = ((o.residual(Qp, dt=dt) - o.residual(Qm, dt=dt)) / (2 * h * sc)).ravel()
    return np.linalg.eigvals(np.tile(1.0 / vol, 5)[:, None] * J)


@pytest.mark.parametrize("opts", [{}, {"physics": 1, "mu": 0.002, "prandtl": 0.72}], ids=["euler", "ns"])
def test_uniform_stream_linearisation_is_stable(oracle_lib, opts):
    oracle_lib.set_threads(8)
    try:
        ev = _spectrum(oracle_lib, **opts)
    finally:
        oracle_lib.set_threads(1)
    print(f"largest real part {ev.real.max():.3f}, smallest {ev.real.min():.3f}")
    # a non-trivial spectrum, and no growing mode
    assert ev.real.min() < -10.0
    assert ev.real.max() < 0.0
