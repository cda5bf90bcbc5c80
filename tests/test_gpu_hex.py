"""Hexahedral meshes through the C ABI (hgks_load_hex_mesh) against the oracle.

Tolerances as for tetrahedra (see test_gpu_parity.py): residual 1e-12 x flux
scale (the largest cell surface times the free stream's Euler flux); Jv
2 x 1e-12 x flux scale / sigma; implicit steps with the approximate matrix or
LU-SGS, each from the same state, 1e-10 relative."""
import numpy as np
import pytest

from inputs import cube_mesh, freestream_prim, perturbed_state, shell_mesh
from tests import _cases as C

pytestmark = pytest.mark.gpu

HCASES = {
    "hcube_mixed": (lambda: cube_mesh(5, jitter=0.15, seed=4, hexahedra=True),
                    {1: C.SUP_IN, 2: C.SUP_OUT, 3: C.FAR, 4: C.FAR, 5: C.SLIP, 6: C.SLIP}, 0.4),
    "hshell": (lambda: shell_mesh(4, 4, grading=1.3, jitter=0.05, seed=2, hexahedra=True), {1: C.SLIP, 2: C.FAR}, 0.5),
    "hcube_noslip": (lambda: cube_mesh(3, jitter=0.1, seed=7, hexahedra=True), {t: C.NOSLIP for t in range(1, 7)}, 0.2),
}
# "hweno_w": the compact scheme with the eight S^WENO sub-stencils (the
# hexahedral sphere cases of Sec. 5)
SCHEMES = {"weno": dict(scheme=0), "hweno": dict(scheme=1), "hweno_w": dict(scheme=1, compact_subs=1),
           "kfvs": dict(scheme=2)}


def _area_sums(o):
    L, R, S, n, gp = o.faces()
    area = np.zeros(o.N)
    np.add.at(area, L, S)
    np.add.at(area, R[R >= 0], S[R >= 0])
    return area


def _flux_scale(o, prim):
    """largest cell surface (from the oracle's faces) x the free stream's Euler flux"""
    from inputs import prim_to_cons
    from tests import _indep as I
    return max(np.abs(I.euler_flux(prim_to_cons(prim), d)).max() for d in np.eye(3)) * _area_sums(o).max()


def _pair(oracle_lib, case, scheme, **opts):
    from paper_2304_09485_amd import hgks
    mk, kinds, mach = HCASES[case]
    m = mk()
    prim = freestream_prim(mach)
    so = dict(SCHEMES[scheme], **opts)
    oo = dict(so)
    if oo.get("scheme") == 2:
        oo.pop("scheme")
        oo["first_order"] = 1
    o = oracle_lib.Oracle(m, kinds, prim, **oo)
    s = hgks.Solver(m, kinds, prim, **so)
    return m, prim, o, s


@pytest.mark.parametrize("scheme", list(SCHEMES))
@pytest.mark.parametrize("case", list(HCASES))
def test_hex_residual_parity(oracle_lib, case, scheme):
    m, prim, o, s = _pair(oracle_lib, case, scheme)
    assert s.N == o.N and s.F == o.F
    Q = perturbed_state(o.N, prim, amp=0.03, seed=2)
    hw = scheme.startswith("hweno")
    G = np.random.default_rng(7).normal(scale=0.05, size=(15, o.N)) if hw else None
    Ro = o.residual(Q, G=G, want_grad=hw)
    Rg = s.residual(Q, G=G, want_grad=hw)
    if hw:
        Ro, Gno, _ = Ro
        Rg, Gng = Rg
    fs = _flux_scale(o, prim)
    err = np.abs(Rg - Ro).max() / fs
    print(f"{case} {scheme}: max|dR|/flux_scale = {err:.3e}")
    assert err <= 1e-12
    if hw:
        # the gradient update of Eq. (derivative): face sums of S_f times
        # Gauss-point values of size |Q| with the flux's relative rounding,
        # divided by the volume
        bound = 1e-12 * np.abs(Q).max() * _area_sums(o) / o.geometry()[0]
        gerr = np.abs(Gng - Gno).max(axis=0)
        print(f"{case} {scheme}: gradient-update error / bound = {(gerr / bound).max():.3e}")
        assert np.all(gerr <= bound)
    s.close()


@pytest.mark.parametrize("scheme", ["weno", "hweno", "hweno_w"])
def test_hex_jv_parity(oracle_lib, scheme):
    m, prim, o, s = _pair(oracle_lib, "hshell", scheme)
    Q = perturbed_state(o.N, prim, seed=4)
    G = np.random.default_rng(9).normal(scale=0.05, size=(15, o.N)) if scheme.startswith("hweno") else None
    s.set_state(Q, G)
    dt = o.dt(Q)
    np.testing.assert_allclose(s.time_step(Q), dt, rtol=1e-13)
    b = o.residual(Q, G=G, dt=dt)
    v = np.random.default_rng(11).normal(size=(5, o.N))
    fs = _flux_scale(o, prim)
    Avg, sg = s.jv(v, 1e-6)
    Avo, so = o.jv(Q, dt, b, v, sigma=1e-6, G=G)
    tol = 2e-12 * fs / so + 1e-12 * np.abs(Avo).max()
    err = np.abs(Avg - Avo).max()
    print(f"hex {scheme} Jv: max|dAv| = {err:.3e} (tol {tol:.3e})")
    assert err <= tol
    s.close()


@pytest.mark.parametrize("scheme,solver", [("weno", "approx"), ("hweno", "approx"), ("hweno_w", "approx"),
                                           ("weno", "lusgs"), ("kfvs", "lusgs")])
def test_hex_implicit_steps(oracle_lib, scheme, solver):
    from paper_2304_09485_amd import hgks
    opts = dict(jv_mode=1) if solver == "approx" else dict(solver=1)
    m, prim, o, s = _pair(oracle_lib, "hshell", scheme, **opts)
    hw = scheme.startswith("hweno")
    G0 = np.random.default_rng(3).normal(scale=0.02, size=(15, o.N)) if hw else None
    s.set_state(perturbed_state(o.N, prim, amp=0.05, seed=1), G0)
    for k in range(4):
        Qo, Go = s.get_state(want_grad=True)
        st, io = o.implicit_step(Qo, Go if hw else None)
        ig = s.implicit_step()
        assert st == 0 and ig.n_resid_evals == io.n_resid_evals == 1
        Qg, Gg = s.get_state(want_grad=True)
        err = np.abs(Qg - Qo).max() / np.abs(Qo).max()
        print(f"hex {scheme} {solver} step {k + 1}: res gpu {ig.res:.6e} orc {io.res:.6e} err {err:.3e}")
        assert ig.res == pytest.approx(io.res, rel=1e-10)
        assert err <= 1e-10
        if hw:
            np.testing.assert_allclose(Gg, Go, rtol=0, atol=1e-10 * np.abs(Go).max())
    s.close()


def test_hex_fp32_inner_step(oracle_lib):
    """The FP32-inner form on hexahedra: one implicit step runs and lands
    within the FD-rounding distance of the FP64 step (linear weights)."""
    from paper_2304_09485_amd import hgks
    mk, kinds, mach = HCASES["hshell"]
    m = mk()
    prim = freestream_prim(mach)
    Q0 = perturbed_state(m.n_cells, prim, amp=0.02, seed=5)
    out = []
    for prec in (hgks.FP64, hgks.FP32_INNER):
        s = hgks.Solver(m, kinds, prim, weights=1, precision=prec)
        s.set_state(Q0)
        info = s.implicit_step()
        assert np.isfinite(info.res)
        out.append(s.get_state())
        s.close()
    d = np.abs(out[1] - out[0]).max() / np.abs(out[0] - Q0).max()
    print(f"FP32-inner vs FP64 update: {d:.3e} of the update")
    assert d < 1e-2


def test_hex_full_size(oracle_lib):
    """A 135,168-hex sphere shell (the benchmark shell's cubed-sphere layout
    without the tetrahedral split, 32 x 32 per patch, 22 layers): residual of
    the non-compact scheme, the compact scheme with the eight S^WENO
    sub-stencils (with its gradient update) and the first-order scheme at
    Mach 0.5."""
    from paper_2304_09485_amd import hgks
    m = shell_mesh(32, 22, grading=1.1, jitter=0.02, seed=2, hexahedra=True)
    prim = freestream_prim(0.5)
    kinds = {1: C.SLIP, 2: C.FAR}
    Q = perturbed_state(m.n_cells, prim, amp=0.03, seed=3)
    oracle_lib.set_threads(16)
    try:
        G = np.random.default_rng(4).normal(scale=0.02, size=(15, m.n_cells))
        for name in ("weno", "hweno_w", "kfvs"):
            so = SCHEMES[name]
            oo = {"first_order": 1} if name == "kfvs" else so
            o = oracle_lib.Oracle(m, kinds, prim, **oo)
            s = hgks.Solver(m, kinds, prim, **so)
            hw = name == "hweno_w"
            Ro = o.residual(Q, G=G, want_grad=hw)
            Rg = s.residual(Q, G=G if hw else None, want_grad=hw)
            if hw:
                Ro, Gno, _ = Ro
                Rg, Gng = Rg
                bound = 1e-12 * np.abs(Q).max() * _area_sums(o) / o.geometry()[0]
                assert np.all(np.abs(Gng - Gno).max(axis=0) <= bound)
            fs = _flux_scale(o, prim)
            err = np.abs(Rg - Ro).max() / fs
            print(f"hex shell {m.n_cells} cells, {name}: max|dR|/flux_scale = {err:.3e}")
            assert err <= 1e-12
            s.close()
    finally:
        oracle_lib.set_threads(1)


@pytest.mark.parametrize("scheme", list(SCHEMES))
def test_hex_repeat_and_free_stream(oracle_lib, scheme):
    """Repeated evaluations are bitwise equal and a uniform free stream stays
    a steady state on a jittered hexahedral shell: every accumulator of the
    4-point quadrilateral path is cleared per evaluation."""
    from inputs import uniform_state
    from paper_2304_09485_amd import hgks
    mk, _, mach = HCASES["hshell"]
    m, prim = mk(), freestream_prim(mach)
    far = {1: C.FAR, 2: C.FAR}  # a uniform stream is steady only with far field on every boundary
    o = oracle_lib.Oracle(m, far, prim)
    s = hgks.Solver(m, far, prim, **SCHEMES[scheme])
    Q = perturbed_state(o.N, prim, amp=0.03, seed=9)
    U = uniform_state(o.N, prim)
    G = np.zeros((15, o.N)) if scheme.startswith("hweno") else None
    r0 = s.residual(Q, G)
    for _ in range(3):
        assert np.abs(s.residual(U, G)).max() <= 1e-13 * _flux_scale(o, prim)
        assert np.array_equal(s.residual(Q, G), r0)
    s.close()
