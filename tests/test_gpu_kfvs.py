"""The first-order KFVS scheme (HGKS_KFVS1: the flux of the cell averages that
the Mach 3 sphere case of Sec. 5 is retested with) through the C ABI against
the oracle.

Tolerances, as for the high-order path: the residual is one flux evaluation
per face in FP64 on both sides, so 1e-12 x flux scale; Jv at step sigma
2 x 1e-12 x flux scale / sigma; implicit steps with the approximate matrix
are a linear solve that differs only in reduction order, 1e-10 relative;
with FD products, each step is compared from the same start state against
the oracle's own spread under a 1e-13 change of that state."""
import numpy as np
import pytest

from inputs import cube_mesh, freestream_prim, mesh_for_config, perturbed_state, shell_mesh
from tests import _cases as C

pytestmark = pytest.mark.gpu

KCASES = {
    "cube_mixed_m04": (lambda: cube_mesh(5, jitter=0.15, seed=4),
                       {1: C.SUP_IN, 2: C.SUP_OUT, 3: C.FAR, 4: C.FAR, 5: C.SLIP, 6: C.SLIP}, 0.4),
    "shell_m3": (lambda: shell_mesh(4, 4, grading=1.3, jitter=0.05, seed=2), {1: C.SLIP, 2: C.FAR}, 3.0),
    "cube_noslip_m02": (lambda: cube_mesh(3, jitter=0.1, seed=7), {t: C.NOSLIP for t in range(1, 7)}, 0.2),
}


def _pair(oracle_lib, case, **opts):
    from paper_2304_09485_amd import hgks
    mk, kinds, mach = KCASES[case]
    m = mk()
    prim = freestream_prim(mach)
    o = oracle_lib.Oracle(m, kinds, prim, first_order=1, **opts)
    s = hgks.Solver(m, kinds, prim, scheme=hgks.KFVS1, **opts)
    return m, prim, o, s


@pytest.mark.parametrize("case", list(KCASES))
def test_kfvs_residual_parity(oracle_lib, case):
    m, prim, o, s = _pair(oracle_lib, case)
    Q = perturbed_state(o.N, prim, amp=0.05, seed=2)
    err = np.abs(s.residual(Q) - o.residual(Q)).max() / C.flux_scale(m, prim)
    print(f"{case}: max|dR|/flux_scale = {err:.3e}")
    assert err <= 1e-12
    s.close()


def test_kfvs_residual_full_size(oracle_lib):
    """The 202,752-tet sphere shell at Mach 3 (slip wall, far field)."""
    from paper_2304_09485_amd import hgks
    m = mesh_for_config("c2")
    prim = freestream_prim(3.0)
    kinds = {1: C.SLIP, 2: C.FAR}
    o = oracle_lib.Oracle(m, kinds, prim, first_order=1)
    s = hgks.Solver(m, kinds, prim, scheme=hgks.KFVS1)
    Q = perturbed_state(o.N, prim, amp=0.05, seed=3)
    oracle_lib.set_threads(16)
    try:
        Ro = o.residual(Q)
    finally:
        oracle_lib.set_threads(1)
    err = np.abs(s.residual(Q) - Ro).max() / C.flux_scale(m, prim)
    print(f"c2 mesh, Mach 3 KFVS: max|dR|/flux_scale = {err:.3e}")
    assert err <= 1e-12
    s.close()


@pytest.mark.parametrize("case", ["shell_m3", "cube_mixed_m04"])
def test_kfvs_jv_parity(oracle_lib, case):
    m, prim, o, s = _pair(oracle_lib, case)
    Q = perturbed_state(o.N, prim, seed=4)
    s.set_state(Q)
    dt = o.dt(Q)
    b = o.residual(Q, dt=dt)
    v = np.random.default_rng(11).normal(size=(5, o.N))
    fs = C.flux_scale(m, prim)
    for sigma in (1e-6, 0.0):
        Avg, sg = s.jv(v, sigma)
        Avo, so = o.jv(Q, dt, b, v, sigma=sigma)
        assert sg == pytest.approx(so, rel=1e-12)
        tol = 2e-12 * fs / so + 1e-12 * np.abs(Avo).max()
        err = np.abs(Avg - Avo).max()
        print(f"{case} sigma={so:.3e}: max|dAv| = {err:.3e} (tol {tol:.3e})")
        assert err <= tol
    s.close()


def test_kfvs_implicit_steps_approximate_matrix(oracle_lib):
    m, prim, o, s = _pair(oracle_lib, "shell_m3", jv_mode=1)
    s.set_state(perturbed_state(o.N, prim, amp=0.05, seed=1))
    for k in range(5):
        Qo = s.get_state()
        st, io = o.implicit_step(Qo)
        ig = s.implicit_step()
        assert st == 0 and ig.n_resid_evals == io.n_resid_evals == 1
        err = np.abs(s.get_state() - Qo).max() / np.abs(Qo).max()
        print(f"approximate matrix step {k + 1}: res gpu {ig.res:.6e} orc {io.res:.6e} err {err:.3e}")
        assert ig.res == pytest.approx(io.res, rel=1e-10)
        assert err <= 1e-10
    s.close()


def test_kfvs_implicit_steps_fd(oracle_lib):
    m, prim, o, s = _pair(oracle_lib, "shell_m3", fd_sigma=1e-4)
    s.set_state(perturbed_state(o.N, prim, amp=0.05, seed=1))
    rng = np.random.default_rng(12)
    for k in range(5):
        Qs = s.get_state()
        Qo = Qs.copy()
        st, io = o.implicit_step(Qo)
        Qp = Qs * (1.0 + 1e-13 * rng.uniform(-1.0, 1.0, Qs.shape))
        o.implicit_step(Qp)
        ig = s.implicit_step()
        assert st == 0 and ig.n_resid_evals == io.n_resid_evals == 33
        scale = np.abs(Qo).max()
        err = np.abs(s.get_state() - Qo).max() / scale
        spread = np.abs(Qp - Qo).max() / scale
        print(f"FD step {k + 1}: res gpu {ig.res:.6e} orc {io.res:.6e} err {err:.3e} spread {spread:.3e}")
        assert ig.res == pytest.approx(io.res, rel=1e-9)
        assert err <= max(1e-9, 20.0 * spread)
    s.close()


def test_kfvs_rejects_navier_stokes():
    from paper_2304_09485_amd import hgks
    with pytest.raises(hgks.HgksError) as e:
        hgks.Solver(cube_mesh(1), {t: C.FAR for t in range(1, 7)}, freestream_prim(0.3), scheme=hgks.KFVS1,
                    physics=hgks.NS, mu=0.01, prandtl=0.72)
    assert e.value.status == -1
