"""Grid transfers (paper Section 2.1, eq. (2.4)).

Part of the CPU oracle: test infrastructure only (tests, smoke check, CPU baseline).

Linear interpolation P_l^{l+1} between the nested P1 spaces: entry (i, j) is the
value of coarse hat function phi_j at fine vertex i.  It is evaluated by point
location: every fine vertex lies in (the closure of) the coarse tetrahedron whose
refinement created it, and there phi_j equals the barycentric coordinate of the
vertex with respect to that tetrahedron (barycentric coordinates from the
inverse of the 4x4 barycentric matrix).  Restriction is the transpose.

Matrices are indexed by canonical node ids, per component (block diagonal over
components for the vector case, as in eq. (B.2)).
"""

from __future__ import annotations

from typing import List

import numpy as np
import scipy.sparse as sp

from .mesh import Level


def prolongation(coarse: Level, fine: Level) -> sp.csr_matrix:
    """Scalar P_l^{l+1} over all nodes: shape ((n_f+1)^3, (n_c+1)^3)."""
    T = coarse.tets.shape[0]
    C4 = coarse.coords[coarse.tets]                         # (T, 4, 3)
    M = np.ones((T, 4, 4))
    M[:, 1:, :] = C4.transpose(0, 2, 1)
    Minv = np.linalg.inv(M)
    # fine tets are grouped by parent: rows 8t..8t+7 are the children of coarse tet t
    ch = fine.tets.reshape(T, 8 * 4)                        # (T, 32) fine vertex indices
    X = fine.coords[ch]                                     # (T, 32, 3)
    Xh = np.concatenate([np.ones((T, 32, 1)), X], axis=2)   # (T, 32, 4)
    lam = np.einsum("tij,tkj->tki", Minv, Xh)               # (T, 32, 4): lambda_i(x_k)
    if lam.min() < -1e-12:
        raise ValueError("a child vertex lies outside its parent")
    rows = np.repeat(fine.node_id[ch], 4, axis=1).reshape(T, 32, 4)
    cols = np.broadcast_to(coarse.node_id[coarse.tets][:, None, :], (T, 32, 4))
    vals = lam
    keep = np.abs(vals) > 1e-14
    r, c, v = rows[keep], cols[keep], vals[keep]
    # each (row, col) pair is evaluated once per containing coarse element; the
    # values must agree (continuity of the hat functions) -- keep one of them.
    nf = (fine.n + 1) ** 3
    nc = (coarse.n + 1) ** 3
    key = r.astype(np.int64) * nc + c
    order = np.argsort(key, kind="stable")
    key, v = key[order], v[order]
    first = np.ones(key.size, dtype=bool)
    first[1:] = key[1:] != key[:-1]
    grp = np.cumsum(first) - 1
    vmin = np.full(first.sum(), np.inf)
    vmax = np.full(first.sum(), -np.inf)
    np.minimum.at(vmin, grp, v)
    np.maximum.at(vmax, grp, v)
    if np.max(vmax - vmin) > 1e-13:
        raise ValueError("interpolation weights disagree between elements")
    uk = key[first]
    P = sp.csr_matrix((v[first], (uk // nc, uk % nc)), shape=(nf, nc))
    return P


def block_diag_components(P: sp.spmatrix, ncomp: int) -> sp.csr_matrix:
    """Block-diagonal interpolation, one copy per velocity component (eq. (B.2))."""
    if ncomp == 1:
        return P.tocsr()
    return sp.block_diag([P] * ncomp, format="csr")


def prolongations(levels: List[Level], ncomp: int) -> List[sp.csr_matrix]:
    """P[l] maps level l to level l+1 (all nodes, all components)."""
    return [block_diag_components(prolongation(levels[l], levels[l + 1]), ncomp)
            for l in range(len(levels) - 1)]


def composite(Ps: List[sp.csr_matrix], coarse: int, fine: int) -> sp.csr_matrix:
    """Pi = P_{fine-1}^{fine} ... P_{coarse}^{coarse+1} (identity when coarse == fine)."""
    if coarse == fine:
        n = Ps[fine - 1].shape[0] if fine > 0 else Ps[0].shape[1]
        return sp.identity(n, format="csr")
    Pi = Ps[coarse]
    for l in range(coarse + 1, fine):
        Pi = Ps[l] @ Pi
    return Pi.tocsr()
