"""The device gas-kinetic flux function, instantiated on the host, against the
oracle's flux at random states (CPU; the same template runs in k_flux)."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "_build", "libhgks_hostcheck.so")


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(LIB):
        pytest.skip("host-check library not built")
    L = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    L.hgks_hostcheck_flux.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp, ctypes.c_int32, ctypes.c_int32, vp, vp]
    L.hgks_hostcheck_flux_f32.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp, ctypes.c_int32, vp]
    return L


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _states(rng):
    from tests import _indep as I
    Wl = I.cons(rng.uniform(0.6, 1.4), rng.uniform(-1.5, 1.5, 3), rng.uniform(0.4, 1.5))
    Wr = I.cons(rng.uniform(0.6, 1.4), rng.uniform(-1.5, 1.5, 3), rng.uniform(0.4, 1.5))
    dl, dr = rng.normal(scale=0.5, size=(2, 3, 5))
    return Wl, dl, Wr, dr


@pytest.mark.parametrize("physics,qg", [(0, 0), (0, 1), (1, 0)])
def test_device_flux_matches_oracle(oracle_lib, hc, physics, qg):
    from inputs import cube_mesh, freestream_prim
    kw = dict(physics=1, mu=0.01, prandtl=0.72) if physics else {}
    o = oracle_lib.Oracle(cube_mesh(1), {t: 0 for t in range(1, 7)}, freestream_prim(0.5), **kw)
    par = np.array([1.4, 2.0, 0.1, 1.0, kw.get("mu", 0.0), kw.get("prandtl", 1.0)])
    rng = np.random.default_rng(physics * 10 + qg)
    for _ in range(200):
        Wl, dl, Wr, dr = _states(rng)
        dt = rng.uniform(1e-3, 0.5)
        F = np.zeros(5)
        Q = np.zeros(5)
        hc.hgks_hostcheck_flux(_p(Wl), _p(dl), _p(Wr), _p(dr), dt, _p(par), physics, qg, _p(F), _p(Q))
        Fo, Qo = o.gks_point(Wl, dl, Wr, dr, dt, want_qg=True)
        scale = np.abs(Fo).max() + 1.0
        np.testing.assert_allclose(F, Fo, rtol=0, atol=1e-13 * scale)
        if qg:
            np.testing.assert_allclose(Q, Qo, rtol=0, atol=1e-13 * (np.abs(Qo).max() + 1.0))


def test_device_flux_fp32(oracle_lib, hc):
    from inputs import cube_mesh, freestream_prim
    o = oracle_lib.Oracle(cube_mesh(1), {t: 0 for t in range(1, 7)}, freestream_prim(0.5))
    par = np.array([1.4, 2.0, 0.1, 1.0, 0.0, 1.0])
    rng = np.random.default_rng(3)
    worst = 0.0
    for _ in range(200):
        Wl, dl, Wr, dr = _states(rng)
        dt = rng.uniform(1e-3, 0.5)
        F = np.zeros(5)
        hc.hgks_hostcheck_flux_f32(_p(Wl), _p(dl), _p(Wr), _p(dr), dt, _p(par), 0, _p(F))
        Fo = o.gks_point(Wl, dl, Wr, dr, dt)
        worst = max(worst, np.abs(F - Fo).max() / (np.abs(Fo).max() + 1.0))
    # FP32 evaluation of the same formula: a few hundred ulps of cancellation
    assert worst < 2e-5, worst


def test_device_kfvs_matches_oracle(oracle_lib, hc):
    """The first-order KFVS flux of the device code against the oracle's."""
    from inputs import cube_mesh, freestream_prim
    hc.hgks_hostcheck_kfvs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_void_p]
    o = oracle_lib.Oracle(cube_mesh(1), {t: 0 for t in range(1, 7)}, freestream_prim(0.5), first_order=1)
    rng = np.random.default_rng(11)
    for _ in range(200):
        Wl, _, Wr, _ = _states(rng)
        F = np.zeros(5)
        hc.hgks_hostcheck_kfvs(_p(Wl), _p(Wr), 1.4, 2.0, _p(F))
        Fo = o.kfvs_point(Wl, Wr)
        np.testing.assert_allclose(F, Fo, rtol=0, atol=1e-14 * (np.abs(Fo).max() + 1.0))


@pytest.mark.parametrize("physics", [0, 1])
def test_device_flux_vacuum_interface(oracle_lib, hc, physics):
    """Two states streaming away from the face at 6.5-9 thermal speeds (a
    slip wall behind an expansion, the case that produced a NaN in the FP32
    flux: the interface density underflows): the device flux is zero in both
    precisions, as the oracle's.  At 4.8 thermal speeds (interface density
    about 1e-11 of the sides') both precisions are finite and FP64 matches
    the oracle."""
    from inputs import cube_mesh, freestream_prim
    kw = dict(physics=1, mu=0.006, prandtl=0.72) if physics else {}
    o = oracle_lib.Oracle(cube_mesh(1), {t: 0 for t in range(1, 7)}, freestream_prim(0.5), **kw)
    par = np.array([1.4, 2.0, 0.1, 1.0, kw.get("mu", 0.0), kw.get("prandtl", 1.0)])
    rng = np.random.default_rng(5 + physics)
    for x in (4.8, 6.5, 8.0, 9.0):
        for _ in range(20):
            rl, pl = rng.uniform(0.2, 1.5), rng.uniform(0.01, 1.0)
            Wl = np.array([rl, -rl * x * np.sqrt(2 * pl / rl), *(rl * rng.normal(size=2)), 0.0])
            Wl[4] = pl / 0.4 + 0.5 * (Wl[1:4] @ Wl[1:4]) / rl
            Wr = Wl * np.array([1, -1, 1, 1, 1])
            dl, dr = rng.normal(size=(2, 3, 5))
            F, Q, F32 = np.zeros(5), np.zeros(5), np.zeros(5)
            hc.hgks_hostcheck_flux(_p(Wl), _p(dl), _p(Wr), _p(dr), 0.05, _p(par), physics, 0, _p(F), _p(Q))
            hc.hgks_hostcheck_flux_f32(_p(Wl), _p(dl), _p(Wr), _p(dr), 0.05, _p(par), physics, _p(F32))
            Fo = o.gks_point(Wl, dl, Wr, dr, 0.05)
            assert np.all(np.isfinite(F32))
            if x > 6:
                assert np.all(F == 0.0) and np.all(F32 == 0.0) and np.all(Fo == 0.0)
            else:
                # Navier-Stokes: tau = mu / p0 is far above dt at this nearly
                # empty interface, and the time integrals of Eq. (flux) cancel
                tol = 1e-12 if physics else 1e-13
                np.testing.assert_allclose(F, Fo, rtol=0, atol=tol * (np.abs(Fo).max() + 1.0))
