"""Sample points of the refined unit-cube lattice, for evaluating the seeded fields.

Level l has n = 2^(l+1) cells per axis and six tetrahedra per cell; element
e = s + 6 (cx + n (cy + n cz)) is the simplex whose path from the cell's lowest
corner steps along the axes in order s (0 xyz, 1 xzy, 2 yxz, 3 yzx, 4 zxy, 5 zyx).
Its centroid is the lowest corner plus (3/4, 1/2, 1/4) h along its first, second
and third axis.  Used to generate inputs only.
"""

from __future__ import annotations

import numpy as np

_ORDERS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def element_centroids(level: int) -> np.ndarray:
    """(6 n^3, 3) element centroids by element id."""
    n = 2 ** (level + 1)
    off = np.zeros((6, 3))
    for s, axes in enumerate(_ORDERS):
        for k, a in enumerate(axes):
            off[s, a] = (3 - k) / 4.0
    c = np.arange(n, dtype=np.float64)
    cz, cy, cx = np.meshgrid(c, c, c, indexing="ij")
    base = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    return ((base[:, None, :] + off[None, :, :]) / n).reshape(-1, 3)


def element_centroids_torch(level: int, start: int, stop: int, device):
    """Centroids of elements start..stop-1 (element-id order) as a torch tensor on device."""
    import torch
    n = 2 ** (level + 1)
    off = torch.zeros((6, 3), dtype=torch.float64, device=device)
    for s, axes in enumerate(_ORDERS):
        for k, a in enumerate(axes):
            off[s, a] = (3 - k) / 4.0
    e = torch.arange(start, stop, dtype=torch.int64, device=device)
    s = e % 6
    cell = e // 6
    cx = cell % n
    cy = (cell // n) % n
    cz = cell // (n * n)
    base = torch.stack([cx, cy, cz], dim=1).to(torch.float64)
    return (base + off[s]) / n
