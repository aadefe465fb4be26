"""Canonical numbering of the refined Kuhn lattice (host-side index arithmetic).

Level l of the 48-tet macro grid has n = 2^(l+1) cells per axis, nodes
p = x + (n+1)(y + (n+1) z) and elements e = s + 6 (cx + n (cy + n cz)), s the
axis order (0 xyz, 1 xzy, 2 yxz, 3 yzx, 4 zxy, 5 zyx) of the element's path
from its lowest corner (paper Section 2.1, eq. (2.2)).  These helpers produce
the points at which callers sample coefficient and forcing fields.
"""

from __future__ import annotations

import numpy as np

AXIS_ORDERS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def cells(level: int) -> int:
    return 2 ** (level + 1)


def num_nodes(level: int) -> int:
    return (cells(level) + 1) ** 3


def num_elements(level: int) -> int:
    return 6 * cells(level) ** 3


def element_centroids(level: int, chunk=None) -> np.ndarray:
    """(6 n^3, 3) centroids by element id: lowest corner + (3/4, 1/2, 1/4) h along (a1, a2, a3)."""
    n = cells(level)
    h = 1.0 / n
    off = np.zeros((6, 3))
    for s, (a1, a2, a3) in enumerate(AXIS_ORDERS):
        off[s, a1] += 0.75
        off[s, a2] += 0.5
        off[s, a3] += 0.25
    c = np.arange(n, dtype=np.float64)
    cz, cy, cx = np.meshgrid(c, c, c, indexing="ij")
    base = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)      # cell id order
    pts = (base[:, None, :] + off[None, :, :]) * h                      # (n^3, 6, 3)
    return pts.reshape(-1, 3)


def node_coords(level: int) -> np.ndarray:
    n = cells(level)
    c = np.arange(n + 1, dtype=np.float64) / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def interior_mask(level: int) -> np.ndarray:
    n = cells(level)
    i = np.arange(n + 1)
    inner = (i > 0) & (i < n)
    return (inner[None, None, :] & inner[None, :, None] & inner[:, None, None]).ravel()
