"""Seeded synthetic tetrahedral meshes shaped like the paper's test cases.

The paper's own meshes (cavity, sphere, ONERA M6) are not available, so these
generators stand in for them: a unit cube, a cubed-sphere shell around a sphere
of diameter 1 (optionally boundary-layer graded), and a 3D channel with a 15
degree compression ramp.  Every hexahedron is cut into 6 tetrahedra by the
Kuhn (Freudenthal) split along its index-space main diagonal, which keeps the
triangulation conforming as long as neighbouring hexes agree on the direction
of their shared indices (all generators below index along the global axes).

Outputs are raw arrays only: node coordinates, tet connectivity (positively
oriented), boundary triangles and an integer tag per boundary triangle.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# corner id inside a hex with local index (a, b, c) in {0,1}^3 is a + 2b + 4c
_STEP = (1, 2, 4)
_KUHN = [(0, _STEP[p[0]], _STEP[p[0]] + _STEP[p[1]], 7) for p in itertools.permutations(range(3))]


@dataclass
class TetMesh:
    xyz: np.ndarray            # (n_nodes, 3) float64
    tets: np.ndarray           # (n_tets, 4) int32, positive orientation
    bfaces: np.ndarray         # (n_bfaces, 3) int32
    btags: np.ndarray          # (n_bfaces,) int32
    name: str = ""
    tag_names: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.tets.shape[0])

    def arrays(self):
        return (np.ascontiguousarray(self.xyz, dtype=np.float64),
                np.ascontiguousarray(self.tets, dtype=np.int32),
                np.ascontiguousarray(self.bfaces, dtype=np.int32),
                np.ascontiguousarray(self.btags, dtype=np.int32))


@dataclass
class HexMesh:
    xyz: np.ndarray            # (n_nodes, 3) float64
    hexes: np.ndarray          # (n_hex, 8) int32: 0-3 bottom counter-clockwise seen from above, 4-7 above them
    bfaces: np.ndarray         # (n_bfaces, 4) int32 boundary quadrilaterals
    btags: np.ndarray          # (n_bfaces,) int32
    name: str = ""
    tag_names: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.hexes.shape[0])

    @property
    def tets(self):
        """cell connectivity under the name the tetrahedral meshes use"""
        return self.hexes

    def arrays(self):
        return (np.ascontiguousarray(self.xyz, dtype=np.float64),
                np.ascontiguousarray(self.hexes, dtype=np.int32),
                np.ascontiguousarray(self.bfaces, dtype=np.int32),
                np.ascontiguousarray(self.btags, dtype=np.int32))


# hex corner order: lattice (a + 2b + 4c) -> bottom ring, then top ring
_LAT_TO_RING = [0, 1, 3, 2, 4, 5, 7, 6]
_QUADS = [(0, 3, 2, 1), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7), (4, 5, 6, 7)]


def _finish_hex(xyz, hexes_lat, tag_rules, lat, name, tag_names) -> HexMesh:
    """Lattice-ordered hexes -> ring order, flipped where the trilinear map is
    left-handed; boundary quadrilaterals tagged by lattice rules."""
    h = hexes_lat[:, _LAT_TO_RING].copy()
    x = xyz[h]
    jac = np.einsum("ij,ij->i", np.cross(x[:, 1] - x[:, 0], x[:, 3] - x[:, 0]), x[:, 4] - x[:, 0])
    flip = jac < 0
    h[flip] = h[flip][:, [4, 5, 6, 7, 0, 1, 2, 3]]
    quads = np.concatenate([h[:, list(q)] for q in _QUADS])
    s = np.sort(quads, axis=1).astype(np.int64)
    n = len(xyz)
    keys = ((s[:, 0] * n + s[:, 1]) * n + s[:, 2]) * n + s[:, 3]
    _, first, cnt = np.unique(keys, return_index=True, return_counts=True)
    if cnt.max() > 2:
        raise RuntimeError("non-manifold hexahedral mesh")
    bf = quads[first[cnt == 1]]
    tags = _tag_by_lattice(bf, lat, tag_rules)
    return HexMesh(xyz=np.ascontiguousarray(xyz, dtype=np.float64), hexes=np.ascontiguousarray(h, dtype=np.int32),
                   bfaces=np.ascontiguousarray(bf, dtype=np.int32), btags=np.ascontiguousarray(tags, dtype=np.int32),
                   name=name, tag_names=tag_names)


def _hexes_to_tets(hexes: np.ndarray) -> np.ndarray:
    """hexes: (H, 8) node ids with corner order a + 2b + 4c -> (6H, 4) tets."""
    t = np.stack([hexes[:, list(k)] for k in _KUHN], axis=1)
    return t.reshape(-1, 4).astype(np.int64)


def _signed_vol6(xyz, tets):
    a = xyz[tets[:, 0]]
    return np.einsum("ij,ij->i", np.cross(xyz[tets[:, 1]] - a, xyz[tets[:, 2]] - a),
                     xyz[tets[:, 3]] - a)


def _orient(xyz, tets):
    v = _signed_vol6(xyz, tets)
    neg = v < 0
    t = tets[neg].copy()
    tets[neg, 2] = t[:, 3]
    tets[neg, 3] = t[:, 2]
    return tets


def _face_keys(tri: np.ndarray, n_nodes: int) -> np.ndarray:
    s = np.sort(tri, axis=1).astype(np.int64)
    return (s[:, 0] * n_nodes + s[:, 1]) * n_nodes + s[:, 2]


def _boundary_faces(tets: np.ndarray, n_nodes: int) -> np.ndarray:
    faces = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]],
                            tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    keys = _face_keys(faces, n_nodes)
    uniq, first, cnt = np.unique(keys, return_index=True, return_counts=True)
    if cnt.max() > 2:
        raise RuntimeError("non-manifold triangulation")
    return faces[first[cnt == 1]]


def _min_edge_per_node(xyz, tets):
    h = np.full(len(xyz), np.inf)
    for a, b in itertools.combinations(range(4), 2):
        ln = np.linalg.norm(xyz[tets[:, a]] - xyz[tets[:, b]], axis=1)
        np.minimum.at(h, tets[:, a], ln)
        np.minimum.at(h, tets[:, b], ln)
    return h


def _finish(xyz, tets, bf, tags, name, tag_names) -> TetMesh:
    tets = _orient(xyz, tets)
    if (_signed_vol6(xyz, tets) <= 0).any():
        raise RuntimeError("degenerate tetrahedron after jitter")
    return TetMesh(xyz=np.ascontiguousarray(xyz, dtype=np.float64),
                   tets=np.ascontiguousarray(tets, dtype=np.int32),
                   bfaces=np.ascontiguousarray(bf, dtype=np.int32),
                   btags=np.ascontiguousarray(tags, dtype=np.int32),
                   name=name, tag_names=tag_names)


def _tag_by_lattice(bf, lat, rules):
    """rules: list of (tag, axis, value); a face gets the first tag whose
    lattice coordinate `axis` equals `value` on all three nodes."""
    tags = np.zeros(len(bf), dtype=np.int32)
    for tag, axis, value in rules:
        on = np.all(lat[bf, axis] == value, axis=1) & (tags == 0)
        tags[on] = tag
    if (tags == 0).any():
        raise RuntimeError("untagged boundary face")
    return tags


def cube_mesh(n: int, jitter: float = 0.0, seed: int = 0, length: float = 1.0, hexahedra: bool = False):
    """Unit cube, n^3 hexes x 6 Kuhn tets (or the n^3 hexahedra themselves).
    Tags: 1 x-, 2 x+, 3 y-, 4 y+, 5 z-, 6 z+."""
    r = np.arange(n + 1)
    I, J, K = np.meshgrid(r, r, r, indexing="ij")
    lat = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    xyz = lat.astype(np.float64) * (length / n)
    nid = lambda i, j, k: (i * (n + 1) + j) * (n + 1) + k  # noqa: E731
    c = np.arange(n)
    hi, hj, hk = [a.ravel() for a in np.meshgrid(c, c, c, indexing="ij")]
    hexes = np.stack([nid(hi + (q & 1), hj + ((q >> 1) & 1), hk + ((q >> 2) & 1)) for q in range(8)], axis=1)
    tets = _hexes_to_tets(hexes)
    if jitter > 0:
        rng = np.random.default_rng(seed)
        h = _min_edge_per_node(xyz, tets)
        interior = np.all((lat > 0) & (lat < n), axis=1)
        d = rng.uniform(-jitter, jitter, size=xyz.shape) * h[:, None]
        xyz = xyz + d * interior[:, None]
    rules = [(1, 0, 0), (2, 0, n), (3, 1, 0), (4, 1, n), (5, 2, 0), (6, 2, n)]
    names = {1: "x-", 2: "x+", 3: "y-", 4: "y+", 5: "z-", 6: "z+"}
    if hexahedra:
        return _finish_hex(xyz, hexes, rules, lat, f"hexcube{n}", names)
    bf = _boundary_faces(tets, len(xyz))
    tags = _tag_by_lattice(bf, lat, rules)
    return _finish(xyz, tets, bf, tags, f"cube{n}", names)


def _solve_grading(first: float, total: float, nr: int) -> float:
    lo, hi = 1.0 + 1e-12, 4.0
    for _ in range(200):
        g = 0.5 * (lo + hi)
        s = first * (g ** nr - 1.0) / (g - 1.0)
        lo, hi = (g, hi) if s < total else (lo, g)
    return 0.5 * (lo + hi)


def shell_mesh(n: int, nr: int, r0: float = 0.5, r1: float = 10.0, grading: float | None = 1.1,
               first: float | None = None, jitter: float = 0.0, seed: int = 0,
               bl_layers: int = 0, hexahedra: bool = False):
    """Cubed-sphere shell between spheres of radius r0 and r1 (tetrahedra, or
    with hexahedra=True the hexahedra they are cut from).

    6 patches of n x n cells per layer, nr geometrically graded radial layers
    (either `grading` is the ratio, or `first` is the first-layer height and the
    ratio is solved for).  Interior nodes are jittered by U[-jitter, jitter]
    times the local minimum edge length per coordinate; in the first
    `bl_layers` layers the jitter is tangential only.
    Tags: 1 inner sphere, 2 outer sphere.
    """
    if first is not None:
        grading = _solve_grading(first, r1 - r0, nr)
    g = float(grading)
    h0 = (r1 - r0) * (g - 1.0) / (g ** nr - 1.0) if g != 1.0 else (r1 - r0) / nr
    radii = np.array([r0 + (h0 * (g ** k - 1.0) / (g - 1.0) if g != 1.0 else h0 * k) for k in range(nr + 1)])
    radii[-1] = r1
    # surface lattice of the cube [0, n]^3
    smap = -np.ones((n + 1,) * 3, dtype=np.int64)
    r = np.arange(n + 1)
    I, J, K = np.meshgrid(r, r, r, indexing="ij")
    on = (np.minimum(np.minimum(I, J), K) == 0) | (np.maximum(np.maximum(I, J), K) == n)
    surf = np.stack([I[on], J[on], K[on]], axis=1)
    smap[surf[:, 0], surf[:, 1], surf[:, 2]] = np.arange(len(surf))
    t = np.tan(0.25 * math.pi * (2.0 * surf / n - 1.0))
    t[surf == 0] = -1.0
    t[surf == n] = 1.0
    dirs = t / np.linalg.norm(t, axis=1, keepdims=True)
    ns = len(surf)
    xyz = (dirs[:, None, :] * radii[None, :, None]).reshape(-1, 3)
    lev = np.tile(np.arange(nr + 1), ns)
    sid = np.repeat(np.arange(ns), nr + 1)
    hexes = []
    c = np.arange(n)
    ck = np.arange(nr)
    ia, ib, kk = [a.ravel() for a in np.meshgrid(c, c, ck, indexing="ij")]
    for ax in range(3):
        fa = [a for a in range(3) if a != ax]
        for side in (0, n):
            cols = []
            for q in range(8):
                a, b, cc = q & 1, (q >> 1) & 1, (q >> 2) & 1
                L = [None, None, None]
                L[ax] = np.full_like(ia, side)
                L[fa[0]] = ia + a
                L[fa[1]] = ib + b
                s = smap[L[0], L[1], L[2]]
                cols.append(s * (nr + 1) + kk + cc)
            hexes.append(np.stack(cols, axis=1))
    hexes = np.concatenate(hexes)
    tets = _hexes_to_tets(hexes)
    if jitter > 0:
        rng = np.random.default_rng(seed)
        h = _min_edge_per_node(xyz, tets)
        d = rng.uniform(-jitter, jitter, size=xyz.shape) * h[:, None]
        interior = (lev > 0) & (lev < nr)
        radial = dirs[sid]
        bl = lev <= bl_layers
        d[bl] -= np.sum(d[bl] * radial[bl], axis=1, keepdims=True) * radial[bl]
        xyz = xyz + d * interior[:, None]
    lat = lev[:, None]
    if hexahedra:
        return _finish_hex(xyz, hexes, [(1, 0, 0), (2, 0, nr)], lat, f"hexshell{n}x{nr}",
                           {1: "sphere", 2: "farfield"})
    bf = _boundary_faces(tets, len(xyz))
    tags = _tag_by_lattice(bf, lat, [(1, 0, 0), (2, 0, nr)])
    return _finish(xyz, tets, bf, tags, f"shell{n}x{nr}", {1: "sphere", 2: "farfield"})


def ramp_mesh(nx: int, ny: int, nz: int, angle_deg: float = 15.0, length: float = 3.0,
              ramp_start: float = 1.0, jitter: float = 0.0, seed: int = 0, ramp_end: float | None = None,
              height: float = 1.0) -> TetMesh:
    """Channel x in [0, length], z in [0, 1], y from the floor to `height`, with
    sheared hexes.  The floor rises at `angle_deg` from x = ramp_start to
    x = ramp_end (None: to the outlet) and is flat after it.  Interior nodes
    are jittered.  Tags: 1 inlet (x=0), 2 outlet (x=length), 3 bottom/ramp,
    4 top, 5 z=0 side, 6 z=1 side.

    A floor that rises to the outlet of a unit-height channel closes it to
    0.46 of its inlet area at x = 3, below the sonic area of any supersonic
    inflow from Mach 1 to 2 (0.59 at Mach 2): such a channel has no started
    steady flow.  A ramp of finite length (the floor 0.13 up after half a
    unit) in a channel of height 2 keeps the Mach 2 stream started."""
    i, j, k = [a.ravel() for a in np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")]
    lat = np.stack([i, j, k], axis=1)
    x = length * i / nx
    run = np.maximum(0.0, x - ramp_start)
    if ramp_end is not None:
        run = np.minimum(run, ramp_end - ramp_start)
    yb = run * math.tan(math.radians(angle_deg))
    y = yb + (height - yb) * j / ny
    z = k / nz
    xyz = np.stack([x, y, z], axis=1)
    nid = lambda a, b, c: (a * (ny + 1) + b) * (nz + 1) + c  # noqa: E731
    hi, hj, hk = [a.ravel() for a in np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")]
    hexes = np.stack([nid(hi + (q & 1), hj + ((q >> 1) & 1), hk + ((q >> 2) & 1)) for q in range(8)], axis=1)
    tets = _hexes_to_tets(hexes)
    if jitter > 0:
        rng = np.random.default_rng(seed)
        h = _min_edge_per_node(xyz, tets)
        interior = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)
        d = rng.uniform(-jitter, jitter, size=xyz.shape) * h[:, None]
        xyz = xyz + d * interior[:, None]
    bf = _boundary_faces(tets, len(xyz))
    tags = _tag_by_lattice(bf, lat, [(1, 0, 0), (2, 0, nx), (3, 1, 0), (4, 1, ny), (5, 2, 0), (6, 2, nz)])
    return _finish(xyz, tets, bf, tags, f"ramp{nx}x{ny}x{nz}",
                   {1: "inlet", 2: "outlet", 3: "ramp", 4: "top", 5: "side-", 6: "side+"})


def mesh_for_config(name: str) -> TetMesh:
    """The synthetic meshes of the five workloads (sizes in cells)."""
    name = name.lower()
    if name == "c1":   # 3,072 tets
        return cube_mesh(8)
    if name == "c2":   # 202,752 tets
        return shell_mesh(16, 22, grading=1.1, jitter=0.02, seed=2)
    if name == "c3":   # 995,328 tets
        return shell_mesh(24, 48, first=1e-3, jitter=0.02, seed=3, bl_layers=10)
    if name == "c4":   # 3,981,312 tets
        return ramp_mesh(192, 72, 48, jitter=0.02, seed=4, ramp_end=1.5, height=2.0)
    raise KeyError(name)
