"""Edge cases through the C ABI: the smallest meshes (one and two tets, whose
stencils are rank deficient and fall back as reading A17 states), sizes that
leave ragged last blocks in every kernel, and the error paths of mesh loading,
options and boundary tags."""
import numpy as np
import pytest

from inputs import TetMesh, cube_mesh, freestream_prim, perturbed_state
from tests import _cases as C

pytestmark = pytest.mark.gpu


def tiny_mesh(n_tets):
    """One tet, or two sharing a face; all boundary faces far field (tag 1)."""
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], float)
    tets = np.array([[0, 1, 2, 3], [1, 2, 3, 4]][:n_tets], np.int32)
    for t in tets:
        a, b, c, d = xyz[t]
        if np.linalg.det(np.array([b - a, c - a, d - a])) < 0:
            t[[2, 3]] = t[[3, 2]]
    count = {}
    for t in tets:
        for p in range(4):
            k = tuple(sorted(np.delete(t, p)))
            count[k] = count.get(k, 0) + 1
    bf = np.array([k for k, c in count.items() if c == 1], np.int32)
    return TetMesh(xyz=xyz, tets=tets, bfaces=bf, btags=np.ones(len(bf), np.int32))


@pytest.mark.parametrize("mesh", ["one_tet", "two_tets", "cube1", "cube3"])
@pytest.mark.parametrize("scheme", [0, 1])
def test_small_and_ragged_meshes(oracle_lib, mesh, scheme):
    """1, 2, 6 and 162 tets: residual parity at 1e-12 x flux scale (the
    block sizes 64/128/256 leave a partial last block in every kernel)."""
    from paper_2304_09485_amd import hgks
    m = {"one_tet": lambda: tiny_mesh(1), "two_tets": lambda: tiny_mesh(2),
         "cube1": lambda: cube_mesh(1, jitter=0.1, seed=2), "cube3": lambda: cube_mesh(3, jitter=0.1, seed=2)}[mesh]()
    prim = freestream_prim(0.3)
    kinds = {t: C.FAR for t in range(1, 7)}
    o = oracle_lib.Oracle(m, kinds, prim, scheme=scheme)
    s = hgks.Solver(m, kinds, prim, scheme=scheme)
    Q = perturbed_state(o.N, prim, amp=0.02, seed=3)
    G = np.random.default_rng(4).normal(scale=0.05, size=(15, o.N)) if scheme == 1 else None
    Ro = o.residual(Q, G=G)
    Rg = s.residual(Q, G)
    assert np.abs(Rg - Ro).max() <= 1e-12 * C.flux_scale(m, prim)
    # one implicit step runs end to end on the degenerate stencils
    s.set_state(Q, G)
    info = s.implicit_step()
    assert np.isfinite(info.res)
    s.close()


def _expect(status, fn):
    from paper_2304_09485_amd import hgks
    with pytest.raises(hgks.HgksError) as e:
        fn()
    assert e.value.status == status, str(e.value)


def test_mesh_errors():
    from paper_2304_09485_amd import hgks
    prim = freestream_prim(0.3)
    far = {t: C.FAR for t in range(1, 7)}
    EINVAL, EMESH = -1, -3
    good = cube_mesh(2)
    # no cells
    empty = TetMesh(xyz=good.xyz, tets=np.zeros((0, 4), np.int32), bfaces=good.bfaces[:0], btags=good.btags[:0])
    _expect(EINVAL, lambda: hgks.Solver(empty, far, prim))
    # a degenerate (zero-volume) tet
    deg = tiny_mesh(1)
    deg.xyz = deg.xyz.copy()
    deg.xyz[3] = [0.5, 0.5, 0.0]
    _expect(EMESH, lambda: hgks.Solver(deg, far, prim))
    # a boundary triangle missing from the boundary list
    miss = TetMesh(xyz=good.xyz, tets=good.tets, bfaces=good.bfaces[1:], btags=good.btags[1:])
    _expect(EMESH, lambda: hgks.Solver(miss, far, prim))
    # a triangle shared by three tets (non-manifold)
    t2 = tiny_mesh(2)
    xyz = np.vstack([t2.xyz, [[0.3, 0.3, -1.0]]])
    tets = np.vstack([t2.tets, [[1, 2, 3, 5]]]).astype(np.int32)
    a, b, c, d = xyz[tets[2]]
    if np.linalg.det(np.array([b - a, c - a, d - a])) < 0:
        tets[2, [2, 3]] = tets[2, [3, 2]]
    nm = TetMesh(xyz=xyz, tets=tets, bfaces=t2.bfaces, btags=t2.btags)
    _expect(EMESH, lambda: hgks.Solver(nm, far, prim))
    # a boundary tag outside 0..255
    badtag = TetMesh(xyz=good.xyz, tets=good.tets, bfaces=good.bfaces, btags=good.btags.copy())
    badtag.btags[0] = 300
    _expect(EMESH, lambda: hgks.Solver(badtag, far, prim))


@pytest.mark.parametrize("opts", [dict(cfl=0.0), dict(gamma=1.0), dict(krylov_dim=33), dict(restarts=0),
                                  dict(physics=1, mu=0.0), dict(jv_mode=2), dict(scheme=3), dict(precision=3)])
def test_invalid_options(opts):
    from paper_2304_09485_amd import hgks
    _expect(-1, lambda: hgks.Solver(cube_mesh(1), {t: C.FAR for t in range(1, 7)}, freestream_prim(0.3), **opts))


def test_invalid_boundary_kind():
    from paper_2304_09485_amd import hgks
    _expect(-1, lambda: hgks.Solver(cube_mesh(1), {1: 7}, freestream_prim(0.3)))


def test_hex_mesh_errors():
    from paper_2304_09485_amd import hgks
    from inputs import HexMesh
    prim = freestream_prim(0.3)
    far = {t: C.FAR for t in range(1, 7)}
    good = cube_mesh(2, hexahedra=True)
    # top and bottom rings swapped: a left-handed (inverted) hexahedron
    inv = good.hexes.copy()
    inv[0] = inv[0][[4, 5, 6, 7, 0, 1, 2, 3]]
    _expect(-3, lambda: hgks.Solver(HexMesh(xyz=good.xyz, hexes=inv, bfaces=good.bfaces, btags=good.btags), far, prim))
    # a boundary quadrilateral missing from the boundary list
    miss = HexMesh(xyz=good.xyz, hexes=good.hexes, bfaces=good.bfaces[1:], btags=good.btags[1:])
    _expect(-3, lambda: hgks.Solver(miss, far, prim))
    # node id out of range
    bad = good.hexes.copy()
    bad[1, 3] = len(good.xyz) + 5
    _expect(-3, lambda: hgks.Solver(HexMesh(xyz=good.xyz, hexes=bad, bfaces=good.bfaces, btags=good.btags), far, prim))


@pytest.mark.parametrize("n_tets", [1, 2])
def test_gmres_breakdown_matches_oracle(oracle_lib, n_tets):
    """5 or 10 unknowns and a Krylov dimension of 10: the Arnoldi process
    exhausts the space (happy breakdown) inside the first cycle.  The step
    with the approximate matrix (a linear solve) equals the oracle's, whose
    loop stops at the breakdown, at 1e-10."""
    from paper_2304_09485_amd import hgks
    m = tiny_mesh(n_tets)
    prim = freestream_prim(0.3)
    kinds = {t: C.FAR for t in range(1, 7)}
    o = oracle_lib.Oracle(m, kinds, prim, jv_mode=1, cfl=1.0)
    s = hgks.Solver(m, kinds, prim, jv_mode=hgks.JV_APPROX, cfl=1.0)
    Q = perturbed_state(o.N, prim, amp=0.01, seed=5)
    s.set_state(Q)
    Qo = Q.copy()
    st, io = o.implicit_step(Qo)
    ig = s.implicit_step()
    assert st == 0 and np.isfinite(ig.res)
    assert io.gmres_rel < 1e-20  # the oracle's cycle ended in an exact solve
    np.testing.assert_allclose(s.get_state(), Qo, rtol=1e-10, atol=1e-12)
    s.close()
