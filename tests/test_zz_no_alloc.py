"""The allocation-free residual entry point (hgks_residual_dev_static) through
the C ABI: bitwise the same as hgks_residual_dev on two calls in a row, the
second on a smaller mesh, for the non-compact and compact schemes; a mesh
whose work space exceeds the static buffer is refused before anything runs."""
import sys

import numpy as np
import pytest

from inputs import cube_mesh, freestream_prim, perturbed_state, shell_mesh

FAR, SLIP = 0, 1


def _pair(torch, hgks, mesh, kinds, mach, seed, **opts):
    s = hgks.Solver(mesh, kinds, freestream_prim(mach), **opts)
    Q = perturbed_state(s.N, freestream_prim(mach), seed=seed)
    if opts.get("scheme") == hgks.HWENO:
        G = np.random.default_rng(seed).normal(scale=0.01, size=(15, s.N))
        s.set_state(Q, G)
    Qd = torch.from_numpy(Q).to("cuda")
    return s, Qd


@pytest.mark.gpu
@pytest.mark.parametrize("scheme", [0, 1])
def test_static_residual_matches_residual_dev(scheme):
    import torch
    from paper_2304_09485_amd import hgks
    opts = {"scheme": scheme}
    big = (shell_mesh(6, 8, grading=1.2, jitter=0.05, seed=3), {1: SLIP, 2: FAR}, 0.5)
    small = (cube_mesh(4, jitter=0.1, seed=5), {t: FAR for t in range(1, 7)}, 0.3)
    sizes = []
    for k, (mesh, kinds, mach) in enumerate((big, small)):
        print(f"static residual: scheme {scheme} call {k} cells {mesh.n_cells}", flush=True)
        sys.stdout.flush()
        s, Qd = _pair(torch, hgks, mesh, kinds, mach, seed=7 + k, **opts)
        sizes.append(s.N)
        assert 0 < s.residual_static_bytes() <= 64 << 20
        R1 = torch.empty_like(Qd)
        R2 = torch.full_like(Qd, float("nan"))
        s.residual_dev(Qd, R1)
        s.residual_dev_static(Qd, R2)
        torch.cuda.synchronize()
        a, b = R1.cpu().numpy(), R2.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), np.abs(a - b).max()
        s.close()
    assert sizes[1] < sizes[0]


@pytest.mark.gpu
def test_static_residual_refuses_large_mesh():
    import torch
    from paper_2304_09485_amd import hgks
    mesh = cube_mesh(16)  # 24,576 tets: more work space than the static buffer holds
    s = hgks.Solver(mesh, {t: FAR for t in range(1, 7)}, freestream_prim(0.3))
    assert s.residual_static_bytes() > 64 << 20
    Q = torch.from_numpy(perturbed_state(s.N, freestream_prim(0.3), seed=1)).to("cuda")
    R = torch.empty_like(Q)
    with pytest.raises(hgks.HgksError, match="static device buffer"):
        s.residual_dev_static(Q, R)
    s.close()
