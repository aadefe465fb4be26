"""Macro grid, uniform Bey refinement and canonical numbering (paper Section 2.1, eq. (2.2), Fig. 2).

Part of the CPU oracle: test infrastructure only (tests, smoke check, CPU baseline).

The macro grid is the unit cube split into 2x2x2 sub-cubes of side 1/2, each cut
into 6 tetrahedra along its (1,1,1) diagonal (48 macro tetrahedra; the paper's
Sections 4-6 use a 48-tet macro grid of the unit cube).  Each refinement splits
every tetrahedron into 8 by Bey's rule: the 4 corner children plus the 4 children
of the inner octahedron cut along the diagonal joining the midpoints of edges
(x0,x2) and (x1,x3), with the children's vertices listed in the order Bey gives.

Nothing here assumes the refined grid is a lattice.  ``canonical_ids`` afterwards
*recovers* a canonical number for every vertex and element from the coordinates:
node p = X + (n+1)(Y + (n+1) Z) for lattice coordinates X,Y,Z of the vertex, and
element e = s + 6 (cx + n (cy + n cz)) where (cx,cy,cz) is the lowest corner of
the element and s in 0..5 numbers the axis order of its three unit steps
(0: x,y,z  1: x,z,y  2: y,x,z  3: y,z,x  4: z,x,y  5: z,y,x).  It fails loudly if
an element is not such a "Kuhn" simplex.  Ids are what the GPU library uses;
the oracle derives them independently from geometry.
"""

from __future__ import annotations

from dataclasses import dataclass
from itertools import permutations
from typing import List

import numpy as np

PERMS = list(permutations(range(3)))          # s -> axis order, lexicographic
_PERM_CODE = {p[0] * 9 + p[1] * 3 + p[2]: s for s, p in enumerate(PERMS)}

# Bey's children of [x0, x1, x2, x3] in terms of the 4 vertices (0..3) and the
# 6 edge midpoints, named by the vertex pair.
_BEY_CHILDREN = [
    ("0", "01", "02", "03"),
    ("01", "1", "12", "13"),
    ("02", "12", "2", "23"),
    ("03", "13", "23", "3"),
    ("01", "02", "03", "13"),
    ("01", "02", "12", "13"),
    ("02", "03", "13", "23"),
    ("02", "12", "13", "23"),
]
_EDGES = ["01", "02", "03", "12", "13", "23"]


@dataclass
class Level:
    """One level of the nested tetrahedral hierarchy."""
    level: int
    coords: np.ndarray      # (Nv, 3) vertex coordinates
    tets: np.ndarray        # (T, 4) vertex indices, in Bey order
    parent: np.ndarray      # (T,) index of the parent tet on level-1 (-1 on level 0)
    node_id: np.ndarray     # (Nv,) canonical node id
    elem_id: np.ndarray     # (T,) canonical element id

    @property
    def n(self) -> int:
        return 2 ** (self.level + 1)


def macro_mesh():
    """48 macro tetrahedra: 2x2x2 cubes of side 1/2, 6 tets per cube along (1,1,1)."""
    pts = np.array([[x, y, z] for z in range(3) for y in range(3) for x in range(3)],
                   dtype=np.float64) * 0.5
    index = {tuple(int(v) for v in (2 * p)): i for i, p in enumerate(pts)}
    tets = []
    for cz in range(2):
        for cy in range(2):
            for cx in range(2):
                for perm in PERMS:
                    v = [cx, cy, cz]
                    verts = [index[tuple(v)]]
                    for ax in perm:
                        v = list(v)
                        v[ax] += 1
                        verts.append(index[tuple(v)])
                    tets.append(verts)
    return pts, np.array(tets, dtype=np.int64)


def bey_refine(coords: np.ndarray, tets: np.ndarray):
    """One uniform refinement step: 8 children per tet, shared edge midpoints merged.

    Returns (new_coords, children (8T, 4), parent (8T,)).  Child k of tet t is
    row 8 t + k.
    """
    nv = coords.shape[0]
    T = tets.shape[0]
    a_idx = {"0": 0, "1": 1, "2": 2, "3": 3}
    ends = np.stack([np.stack([tets[:, a_idx[e[0]]], tets[:, a_idx[e[1]]]], axis=1)
                     for e in _EDGES], axis=1)              # (T, 6, 2)
    lo = ends.min(axis=2)
    hi = ends.max(axis=2)
    key = lo.astype(np.int64) * nv + hi
    uniq, inv = np.unique(key.ravel(), return_inverse=True)
    u_lo, u_hi = uniq // nv, uniq % nv
    mids = 0.5 * (coords[u_lo] + coords[u_hi])
    new_coords = np.vstack([coords, mids])
    mid = (nv + inv).reshape(T, 6)
    name = {"0": tets[:, 0], "1": tets[:, 1], "2": tets[:, 2], "3": tets[:, 3]}
    for j, e in enumerate(_EDGES):
        name[e] = mid[:, j]
    children = np.stack([np.stack([name[v] for v in ch], axis=1) for ch in _BEY_CHILDREN],
                        axis=1)                             # (T, 8, 4)
    parent = np.repeat(np.arange(T), 8)
    return new_coords, children.reshape(8 * T, 4), parent


def canonical_ids(coords: np.ndarray, tets: np.ndarray, level: int):
    """Recover canonical node and element ids from coordinates (see module docstring)."""
    n = 2 ** (level + 1)
    X = np.rint(coords * n).astype(np.int64)
    if not np.allclose(X / n, coords, atol=1e-12, rtol=0):
        raise ValueError("vertex not on the level lattice")
    node_id = X[:, 0] + (n + 1) * (X[:, 1] + (n + 1) * X[:, 2])
    V = X[tets]                                            # (T, 4, 3)
    order = np.argsort(V.sum(axis=2), axis=1, kind="stable")
    Vs = np.take_along_axis(V, order[:, :, None], axis=1)
    steps = np.diff(Vs, axis=1)                            # (T, 3, 3)
    if not (np.all((steps == 0) | (steps == 1)) and np.all(steps.sum(axis=2) == 1)):
        raise ValueError("element is not a Kuhn simplex of the level lattice")
    axes = steps.argmax(axis=2)                            # (T, 3)
    code = axes[:, 0] * 9 + axes[:, 1] * 3 + axes[:, 2]
    lut = np.full(27, -1, dtype=np.int64)
    for k, v in _PERM_CODE.items():
        lut[k] = v
    s = lut[code]
    if np.any(s < 0):
        raise ValueError("repeated step axis")
    c = Vs[:, 0, :]
    elem_id = s + 6 * (c[:, 0] + n * (c[:, 1] + n * c[:, 2]))
    return node_id, elem_id.astype(np.int64)


def hierarchy(L: int) -> List[Level]:
    """Levels 0..L of the uniformly refined 48-tet macro grid (eq. (2.2))."""
    coords, tets = macro_mesh()
    parent = -np.ones(tets.shape[0], dtype=np.int64)
    levels = []
    for lev in range(L + 1):
        if lev > 0:
            coords, tets, parent = bey_refine(coords, tets)
        nid, eid = canonical_ids(coords, tets, lev)
        levels.append(Level(lev, coords, tets, parent, nid, eid))
    return levels


def centroids(level: Level) -> np.ndarray:
    """Element centroids in the level's own (Bey) element order."""
    return level.coords[level.tets].mean(axis=1)


def centroids_canonical(level: Level) -> np.ndarray:
    """Element centroids ordered by canonical element id."""
    c = centroids(level)
    out = np.empty_like(c)
    out[level.elem_id] = c
    return out


def ancestor(levels: List[Level], coarse: int, fine: int) -> np.ndarray:
    """For each tet of level ``fine`` (Bey order), the index of its ancestor on level ``coarse``."""
    a = np.arange(levels[fine].tets.shape[0])
    for lev in range(fine, coarse, -1):
        a = levels[lev].parent[a]
    return a


def free_node_mask(level: Level) -> np.ndarray:
    """True for vertices strictly inside the unit cube (homogeneous Dirichlet elsewhere)."""
    c = level.coords
    return np.all((c > 1e-12) & (c < 1.0 - 1e-12), axis=1)
