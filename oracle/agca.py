"""Flags, DCA / GCA / AGCA coarse operators and local Galerkin blocks (paper Section 2.2-2.3).

Part of the CPU oracle: test infrastructure only (tests, smoke check, CPU baseline).

* DCA (eq. (2.5)): re-discretise on level l with the coefficient evaluated there
  (one value per coarse element, ``nu_levels[l]``).
* GCA (eqs. (2.6)-(2.7)): A_l = Pi_l^T A_L Pi_l with Pi_l the composite linear
  interpolation from level l to the finest level L.
* AGCA (eq. (2.9)): on level l < L, DCA element matrices on unflagged coarse
  elements plus the Galerkin product of the fine operator restricted to the fine
  elements lying inside flagged coarse elements; the finest level is unchanged.
  Because interpolation is linear on each coarse element and coarse hat
  functions vanish outside their support, the sum of the element-wise blocks
  (2.7) over a set of coarse elements equals Pi_l^T A_L(mask) Pi_l where the mask
  keeps the fine elements under that set; the oracle forms that global product.

Flag (element-wise viscosity-variation test): a coarse element m on level l < L
is flagged when the maximum of the finest-level coefficient over its finest
descendants exceeds tau times the minimum (strict, in FP64).  The paper's own
test (eq. (2.8)) is a gradient test at macro-element granularity: the
coefficient is interpolated into the P1 space of the finest level, the norm of
its (element-wise constant) gradient is taken on every finest element, and a
macro element (level 0) is Galerkin-coarsened on all coarse levels when the
largest norm inside it exceeds the tolerance; ``macro_gradient_max`` computes
those maxima and mode FLAG_MACRO takes the 48 macro flags from the caller.

Local block layout: a block belongs to one coarse element; its rows and columns
are ordered (component c, vertex a) -> 4 c + a, with the element's vertices in
increasing order of their lattice-coordinate sum (the path order of a Kuhn
simplex: lowest corner first).
"""

from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np
import scipy.sparse as sp

from .fem import assemble, element_dofs, element_geometry, element_matrices
from .mesh import Level, ancestor
from .transfer import composite

FLAG_RATIO, FLAG_MACRO, FLAG_NONE, FLAG_ALL = 0, 1, 2, 3


def macro_gradient_max(levels: List[Level], eta_nodes: np.ndarray) -> np.ndarray:
    """max over the finest elements d inside each macro element M of ||grad eta_h|_d||
    (eq. (2.8)); eta_h is the P1 function with nodal values ``eta_nodes`` (by canonical
    node id of the finest level).  Returned by canonical id of level 0 (48 values)."""
    L = len(levels) - 1
    fine = levels[L]
    g, _ = element_geometry(fine.coords[fine.tets])            # (T, 4, 3), Bey order
    vals = eta_nodes[fine.node_id[fine.tets]]                  # (T, 4)
    grad = np.einsum("tb,tbd->td", vals, g)
    norm = np.sqrt((grad ** 2).sum(axis=1))
    anc = ancestor(levels, 0, L)                               # Bey index on level 0
    out = np.zeros(levels[0].tets.shape[0])
    np.maximum.at(out, anc, norm)
    canon = np.empty_like(out)
    canon[levels[0].elem_id] = out
    return canon


def macro_descendant_flags(levels: List[Level], macro_flags: np.ndarray, l: int) -> np.ndarray:
    """Flag per canonical id of level l: the flag of the element's macro ancestor."""
    anc = ancestor(levels, 0, l)                               # Bey index on level 0
    out = np.zeros(levels[l].tets.shape[0], dtype=bool)
    out[levels[l].elem_id] = np.asarray(macro_flags, dtype=bool)[levels[0].elem_id[anc]]
    return out


def descendant_minmax(levels: List[Level], nu_fine: np.ndarray, l: int):
    """Min and max of the finest coefficient over the finest descendants of each level-l element.

    Returned arrays are indexed by canonical element id of level l.
    """
    L = len(levels) - 1
    anc = ancestor(levels, l, L)                           # Bey index on level l
    vals = nu_fine[levels[L].elem_id]
    T = levels[l].tets.shape[0]
    mn = np.full(T, np.inf)
    mx = np.full(T, -np.inf)
    np.minimum.at(mn, anc, vals)
    np.maximum.at(mx, anc, vals)
    out_mn = np.empty(T)
    out_mx = np.empty(T)
    out_mn[levels[l].elem_id] = mn
    out_mx[levels[l].elem_id] = mx
    return out_mn, out_mx


def flags(levels: List[Level], nu_fine: np.ndarray, l: int, tau: float = 10.0,
          mode: int = FLAG_RATIO, macro_flags: Optional[np.ndarray] = None) -> np.ndarray:
    """Boolean flag per canonical element id of level l (l < L)."""
    T = levels[l].tets.shape[0]
    if mode == FLAG_NONE:
        return np.zeros(T, dtype=bool)
    if mode == FLAG_ALL:
        return np.ones(T, dtype=bool)
    if mode == FLAG_MACRO:
        return macro_descendant_flags(levels, macro_flags, l)
    if mode != FLAG_RATIO:
        raise ValueError(mode)
    mn, mx = descendant_minmax(levels, nu_fine, l)
    return mx > tau * mn


def fine_mask_under(levels: List[Level], flag_l: np.ndarray, l: int) -> np.ndarray:
    """Canonical-id mask of finest elements whose level-l ancestor is flagged."""
    L = len(levels) - 1
    anc = ancestor(levels, l, L)
    anc_canon = levels[l].elem_id[anc]                     # per fine tet (Bey order)
    mask = np.zeros(levels[L].tets.shape[0], dtype=bool)
    mask[levels[L].elem_id] = flag_l[anc_canon]
    return mask


def agca_operators(levels: List[Level], Ps: List[sp.csr_matrix], nu_levels: List[np.ndarray],
                   ncomp: int, tau: float = 10.0, mode: int = FLAG_RATIO,
                   macro_flags: Optional[np.ndarray] = None) -> Dict:
    """Full (Neumann) AGCA operators on every level, plus the flags.

    ``nu_levels[l]`` is the coefficient by canonical element id on level l;
    ``nu_levels[L]`` is the finest one, also used for flagging and for GCA.
    """
    L = len(levels) - 1
    nu_fine = nu_levels[L]
    ops: List[Optional[sp.csr_matrix]] = [None] * (L + 1)
    fl: List[np.ndarray] = [None] * (L + 1)
    ops[L] = assemble(levels[L], nu_fine, ncomp)
    fl[L] = np.zeros(levels[L].tets.shape[0], dtype=bool)
    for l in range(L - 1, -1, -1):
        f = flags(levels, nu_fine, l, tau, mode, macro_flags)
        fl[l] = f
        A = assemble(levels[l], nu_levels[l], ncomp, elem_mask=~f)
        if f.any():
            Pi = composite(Ps, l, L)
            Af = assemble(levels[L], nu_fine, ncomp, elem_mask=fine_mask_under(levels, f, l))
            A = (A + (Pi.T @ Af @ Pi)).tocsr()
        ops[l] = A
    return {"ops": ops, "flags": fl}


def gca_operator(levels, Ps, nu_fine, ncomp, l):
    """Pure Galerkin operator Pi_l^T A_L Pi_l (eq. (2.6), textbook form)."""
    L = len(levels) - 1
    Pi = composite(Ps, l, L)
    return (Pi.T @ assemble(levels[L], nu_fine, ncomp) @ Pi).tocsr()


def path_order(level: Level) -> np.ndarray:
    """(T, 4) vertex indices of each element (Bey order) sorted into path order."""
    X = np.rint(level.coords * level.n).astype(np.int64)
    s = X[level.tets].sum(axis=2)
    order = np.argsort(s, axis=1, kind="stable")
    return np.take_along_axis(level.tets, order, axis=1)


def local_gca_blocks(levels: List[Level], Ps: List[sp.csr_matrix], nu_fine: np.ndarray,
                     ncomp: int, l: int, elems: np.ndarray) -> np.ndarray:
    """Local Galerkin blocks (eq. (2.7)) of the level-l elements with canonical ids ``elems``.

    block(m) = sum over finest descendants d of Pi_d^T A_d Pi_d with Pi_d the rows
    of the composite interpolation belonging to d's vertices and the columns of
    m's vertices.  Returns (len(elems), 4 ncomp, 4 ncomp) in the block layout.
    """
    L = len(levels) - 1
    nnc = (levels[l].n + 1) ** 3
    Pi = composite(Ps, l, L).tocsc() if l < L else None
    inv = np.empty(levels[l].tets.shape[0], dtype=np.int64)
    inv[levels[l].elem_id] = np.arange(levels[l].tets.shape[0])
    pv = path_order(levels[l])                             # (Tc, 4) Bey-indexed rows
    anc = ancestor(levels, l, L)
    want = np.zeros(levels[l].tets.shape[0], dtype=bool)
    want[inv[elems]] = True
    fine_sel = np.nonzero(want[anc])[0]
    Ke = element_matrices(levels[L], nu_fine, ncomp)[fine_sel]      # (F, m, m)
    fd = element_dofs(levels[L], ncomp)[fine_sel]                    # (F, m)
    cnodes = levels[l].node_id[pv[anc[fine_sel]]]                    # (F, 4)
    cd = np.concatenate([c * nnc + cnodes for c in range(ncomp)], axis=1)  # (F, m)
    m = 4 * ncomp
    rr = np.repeat(fd, m, axis=1)                          # (F, m*m): fine dof a
    cc = np.tile(cd, (1, m))                               # coarse dof j
    Pd = np.asarray(Pi[rr.ravel(), cc.ravel()]).reshape(-1, m, m)    # Pd[a, j]
    prod = np.einsum("fai,fab,fbj->fij", Pd, Ke, Pd)
    out = np.zeros((levels[l].tets.shape[0], m, m))
    np.add.at(out, anc[fine_sel], prod)
    return out[inv[elems]]


def unit_element_matrix_path(h: float, ncomp: int, perm) -> np.ndarray:
    """Element matrix with nu = 1 of the Kuhn simplex with step order ``perm`` and side h.

    Used by tests to state the closed form of a Galerkin block (mean coefficient
    times the unit element matrix); computed with the generic formulas.
    """
    from .fem import scalar_element_matrices, vector_element_matrices
    v = np.zeros(3)
    pts = [v.copy()]
    for ax in perm:
        v[ax] += h
        pts.append(v.copy())
    c4 = np.array(pts)[None]
    if ncomp == 1:
        return scalar_element_matrices(c4, np.ones(1))[0]
    return vector_element_matrices(c4, np.ones(1))[0]
