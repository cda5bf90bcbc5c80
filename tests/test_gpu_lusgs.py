"""LU-SGS implicit steps (HGKS_SOLVER_LUSGS: the LUSGS-WENO comparison solver
of Sec. 5) through the C ABI against the oracle.  An LU-SGS step is one
residual evaluation and two sweeps of plain FP64 arithmetic, with no FD
product, so each GPU step is compared with the oracle's step from the same
state at 1e-11 relative (round-off of the residual, amplified by the
factorised solve at CFL 10)."""
import numpy as np
import pytest

from inputs import freestream_prim, mesh_for_config, perturbed_state
from tests import _cases as C
from tests.test_gpu_kfvs import KCASES

pytestmark = pytest.mark.gpu


def _steps(oracle_lib, m, kinds, prim, nsteps, seed, **opts):
    from paper_2304_09485_amd import hgks
    oopts = {k: v for k, v in opts.items() if k != "scheme" or v != hgks.KFVS1}
    if opts.get("scheme") == hgks.KFVS1:
        oopts["first_order"] = 1
    o = oracle_lib.Oracle(m, kinds, prim, solver=1, **oopts)
    s = hgks.Solver(m, kinds, prim, solver=hgks.SOLVER_LUSGS, **opts)
    hw = opts.get("scheme") == hgks.HWENO
    G0 = np.random.default_rng(seed).normal(scale=0.02, size=(15, o.N)) if hw else None
    s.set_state(perturbed_state(o.N, prim, amp=0.05, seed=seed), G0)
    for k in range(nsteps):
        Qo, Go = s.get_state(want_grad=True)
        st, io = o.implicit_step(Qo, Go if hw else None)
        ig = s.implicit_step()
        assert st == 0 and ig.n_resid_evals == io.n_resid_evals == 1
        Qg, Gg = s.get_state(want_grad=True)
        err = np.abs(Qg - Qo).max() / np.abs(Qo).max()
        print(f"step {k + 1}: res gpu {ig.res:.6e} orc {io.res:.6e} one-step err {err:.3e}")
        assert ig.res == pytest.approx(io.res, rel=1e-11)
        assert err <= 1e-11
        if hw:
            np.testing.assert_allclose(Gg, Go, rtol=0, atol=1e-11 * np.abs(Go).max())
    s.close()


@pytest.mark.parametrize("case", ["shell_weno", "cube_jit_hweno", "c1_weno"])
def test_lusgs_steps(oracle_lib, case):
    mk, kinds, mach, opts = C.CASES[case]
    _steps(oracle_lib, mk(), kinds, freestream_prim(mach), 4, 3, **opts)


def test_lusgs_steps_kfvs_mach3(oracle_lib):
    from paper_2304_09485_amd import hgks
    mk, kinds, mach = KCASES["shell_m3"]
    _steps(oracle_lib, mk(), kinds, freestream_prim(mach), 4, 5, scheme=hgks.KFVS1)


def test_lusgs_step_full_size(oracle_lib):
    """The 202,752-tet sphere shell: first-order KFVS at Mach 3 keeps the
    oracle's residual cheap, so the LU-SGS sweeps over all colour classes
    are compared at full size."""
    from paper_2304_09485_amd import hgks
    m = mesh_for_config("c2")
    oracle_lib.set_threads(16)
    try:
        _steps(oracle_lib, m, {1: C.SLIP, 2: C.FAR}, freestream_prim(3.0), 2, 7, scheme=hgks.KFVS1)
    finally:
        oracle_lib.set_threads(1)
