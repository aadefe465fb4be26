"""Element-by-element oracle for checks at sizes where global matrices are out of reach.

Test infrastructure (only tests/ use it).  Instead of refining the whole macro
grid, single elements are found by descending the refinement tree: at every
step the one tetrahedron that contains a given point is split by Bey's rule
(eq. (2.2)) and the child containing the point is kept.  Canonical ids come from
``mesh.canonical_ids`` (recovered from coordinates), element matrices from
``fem`` (eq. (2.3) / (3.5)), and Galerkin blocks are formed as in eq. (2.7)
recursed to the finest level: the finest-level matrix of all descendants of
one coarse element, multiplied on both sides by the values of the coarse
element's hat functions at the fine vertices.

Operator rows at a node need every element around it; those are found by
locating points just off the node in many directions and are checked to be
complete (their solid angles at the node sum to 4 pi).  The Stokes rows (divergence,
its transpose, the 1/nu pressure mass) integrate over the support of one pressure hat:
the coarse star around the pressure node, each coarse element split into its children.
"""

from __future__ import annotations

from typing import List, Tuple

import numpy as np

from . import fem, mesh

_TOL = 1e-12


def _bary(c4: np.ndarray, p: np.ndarray) -> np.ndarray:
    M = np.ones((4, 4))
    M[1:, :] = c4.T
    return np.linalg.solve(M, np.concatenate([[1.0], p]))


def _contains(c4: np.ndarray, p: np.ndarray) -> bool:
    return bool(np.all(_bary(c4, p) >= -_TOL))


def locate(level: int, p) -> Tuple[np.ndarray, np.ndarray, int]:
    """The level-``level`` element containing point p: (vertex coordinates (4, 3) in Bey
    order, canonical node ids (4,), canonical element id)."""
    p = np.asarray(p, dtype=np.float64)
    coords, tets = mesh.macro_mesh()
    cand = [t for t in range(tets.shape[0]) if _contains(coords[tets[t]], p)]
    if not cand:
        raise ValueError("point outside the unit cube")
    c4 = coords[tets[cand[0]]]
    for _ in range(level):
        cc, ch, _ = mesh.bey_refine(c4, np.arange(4)[None, :])
        nxt = [k for k in range(8) if _contains(cc[ch[k]], p)]
        c4 = cc[ch[nxt[0]]]
    nid, eid = mesh.canonical_ids(c4, np.arange(4)[None, :], level)
    return c4, nid, int(eid[0])


def _solid_angle(c4: np.ndarray, a: int) -> float:
    """Solid angle of the tetrahedron at its vertex a (Van Oosterom and Strackee)."""
    o = c4[a]
    r = [c4[b] - o for b in range(4) if b != a]
    l = [np.linalg.norm(v) for v in r]
    num = abs(np.dot(r[0], np.cross(r[1], r[2])))
    den = (l[0] * l[1] * l[2] + np.dot(r[0], r[1]) * l[2] + np.dot(r[0], r[2]) * l[1]
           + np.dot(r[1], r[2]) * l[0])
    return 2.0 * np.arctan2(num, den)


def elements_around(level: int, node_xyz, seed: int = 0, directions: int = 200):
    """All level elements having the interior node at node_xyz as a vertex:
    list of (coords4, node ids, element id, local index of the node)."""
    x = np.asarray(node_xyz, dtype=np.float64)
    h = 1.0 / 2 ** (level + 1)
    rng = np.random.default_rng(seed)
    found = {}
    for _ in range(4):            # more directions until the star is complete
        d = rng.standard_normal((directions, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        for v in d:
            c4, nid, eid = locate(level, x + 1e-3 * h * v)
            if eid not in found:
                a = int(np.argmin(np.linalg.norm(c4 - x, axis=1)))
                if np.linalg.norm(c4[a] - x) > 1e-12:
                    continue
                found[eid] = (c4, nid, eid, a)
        total = sum(_solid_angle(e[0], e[3]) for e in found.values())
        if abs(total - 4.0 * np.pi) <= 1e-9:
            return list(found.values())
    raise RuntimeError("incomplete element star around the node")


def _elem_matrix(c4: np.ndarray, nu: float, ncomp: int) -> np.ndarray:
    if ncomp == 1:
        return fem.scalar_element_matrices(c4[None], np.array([nu]))[0]
    return fem.vector_element_matrices(c4[None], np.array([nu]))[0]


def apply_at_node(level: int, node_xyz, nu_by_id: np.ndarray, ncomp: int, u_full: np.ndarray,
                  seed: int = 0) -> np.ndarray:
    """(A u) at one interior node, all components (u_full: [ncomp][(n+1)^3] with boundary
    values taken as zero)."""
    n = 2 ** (level + 1)
    nn = (n + 1) ** 3
    free = _free_mask(level)
    out = np.zeros(ncomp)
    for c4, nid, eid, a in elements_around(level, node_xyz, seed):
        K = _elem_matrix(c4, nu_by_id[eid], ncomp)
        ue = np.concatenate([np.where(free(nid), u_full[c * nn + nid], 0.0) for c in range(ncomp)])
        y = K @ ue
        for c in range(ncomp):
            out[c] += y[4 * c + a]
    return out


def load_at_node(level: int, node_xyz, f_by_id: np.ndarray, ncomp: int, seed: int = 0) -> np.ndarray:
    """b at one interior node: sum over the elements around it of |e| f_e / 4 (f_by_id:
    (ncomp, elements) per-element forcing by canonical id)."""
    out = np.zeros(ncomp)
    f = np.asarray(f_by_id).reshape(ncomp, -1)
    for c4, _, eid, _ in elements_around(level, node_xyz, seed):
        _, vol = fem.element_geometry(c4[None])
        out += vol[0] * f[:, eid] / 4.0
    return out


def _free_mask(level: int):
    n = 2 ** (level + 1)

    def free(nid):
        x = nid % (n + 1)
        y = (nid // (n + 1)) % (n + 1)
        z = nid // (n + 1) ** 2
        return (x > 0) & (y > 0) & (z > 0) & (x < n) & (y < n) & (z < n)
    return free


def grad_at_point(level: int, p, nu_by_id: np.ndarray, ncomp: int, u_full: np.ndarray,
                  w_full: np.ndarray) -> Tuple[int, float]:
    """(element id, -w_e^T A_e u_e) for the level element containing p."""
    n = 2 ** (level + 1)
    nn = (n + 1) ** 3
    c4, nid, eid = locate(level, p)
    K = _elem_matrix(c4, nu_by_id[eid], ncomp)
    ue = np.concatenate([u_full[c * nn + nid] for c in range(ncomp)])
    we = np.concatenate([w_full[c * nn + nid] for c in range(ncomp)])
    return eid, float(-we @ K @ ue)


def descendants(coarse: int, fine: int, p) -> Tuple[np.ndarray, np.ndarray, int, np.ndarray]:
    """The level-``coarse`` element containing p and all its level-``fine`` descendants:
    (coarse coords4, fine coordinates (Nv, 3), fine tets (T, 4), coarse element id,
    fine element ids (T,))."""
    c4, _, eid = locate(coarse, p)
    coords, tets = c4.copy(), np.arange(4)[None, :]
    for _ in range(fine - coarse):
        coords, tets, _ = mesh.bey_refine(coords, tets)
    _, fids = mesh.canonical_ids(coords, tets, fine)
    return c4, coords, tets, eid, fids


def flag_at_point(coarse: int, fine: int, p, nu_fine_by_id: np.ndarray, tau: float = 10.0):
    """(coarse element id, flag) with the ratio test over the finest descendants."""
    _, _, _, eid, fids = descendants(coarse, fine, p)
    v = nu_fine_by_id[fids]
    return eid, bool(v.max() > tau * v.min())


def block_at_point(coarse: int, fine: int, p, nu_fine_by_id: np.ndarray, ncomp: int):
    """(coarse element id, Galerkin block (4 ncomp)^2) of the coarse element containing p:
    sum over its finest descendants d of Pi_d^T A_d Pi_d, Pi_d the coarse hat values at
    d's vertices.  Local index 4 c + a, a the coarse vertex in path order (the order of
    increasing coordinate sum)."""
    c4, coords, tets, eid, fids = descendants(coarse, fine, p)
    c4 = c4[np.argsort(c4.sum(axis=1), kind="stable")]     # path order: coordinate sum increases
    M = np.ones((4, 4))
    M[1:, :] = c4.T
    lam = np.linalg.solve(M, np.vstack([np.ones(coords.shape[0]), coords.T]))   # (4, Nv)
    c4f = coords[tets]
    nu = nu_fine_by_id[fids]
    K = (fem.scalar_element_matrices(c4f, nu) if ncomp == 1
         else fem.vector_element_matrices(c4f, nu))                              # (T, m, m)
    Pi1 = lam[:, tets].transpose(1, 2, 0)                                        # (T, 4 fine, 4 coarse)
    m = 4 * ncomp
    Pi = np.zeros((tets.shape[0], m, m))
    for c in range(ncomp):
        Pi[:, 4 * c:4 * c + 4, 4 * c:4 * c + 4] = Pi1
    B = np.einsum("tia,tij,tjb->ab", Pi, K, Pi)
    return eid, B


def coarse_apply_at_node(level: int, fine: int, node_xyz, nu_level_by_id: np.ndarray,
                         nu_fine_by_id: np.ndarray, ncomp: int, u_full: np.ndarray,
                         tau: float = 10.0, seed: int = 0, macro_flags=None) -> np.ndarray:
    """(A_l u) at one interior node of a coarse level (eq. (2.9)): the Galerkin block of
    every flagged element around the node, the DCA element matrix with the level's own
    coefficient for the others.  Flags: the ratio test, or with ``macro_flags`` (48
    values by level-0 element id) the flag of the macro element holding the element."""
    n = 2 ** (level + 1)
    nn = (n + 1) ** 3
    free = _free_mask(level)
    x = np.asarray(node_xyz, dtype=np.float64)
    out = np.zeros(ncomp)
    for c4, nid, eid, a in elements_around(level, x, seed):
        cen = c4.mean(axis=0)
        if macro_flags is None:
            _, flagged = flag_at_point(level, fine, cen, nu_fine_by_id, tau)
        else:
            flagged = bool(macro_flags[locate(0, cen)[2]])
        if flagged:
            _, K = block_at_point(level, fine, cen, nu_fine_by_id, ncomp)
            order = np.argsort(c4.sum(axis=1), kind="stable")
            nid = nid[order]
            a = int(np.nonzero(order == a)[0][0])
        else:
            K = _elem_matrix(c4, nu_level_by_id[eid], ncomp)
        ue = np.concatenate([np.where(free(nid), u_full[c * nn + nid], 0.0) for c in range(ncomp)])
        y = K @ ue
        for c in range(ncomp):
            out[c] += y[4 * c + a]
    return out


# ---------------------------------------------------------------------------
# Generalized Stokes pieces (Section 3.1, the P1-iso-P2 / P1 pair of eqs. (3.3)-(3.5)):
# velocity P1 on level ``fine``, pressure P1 on level ``fine - 1``.  B_kj is minus the
# integral of psi_k div Phi_j with psi_k the pressure hat of node k; psi_k is linear on
# every velocity element d, so that integral over d is |d| (div Phi_j)|_d times the mean
# of psi_k at d's four vertices.
# ---------------------------------------------------------------------------

def _values_at(level: int, x, values_by_node: np.ndarray) -> float:
    """Value at the point x of the level-``level`` P1 function with the given nodal values
    (barycentric interpolation in an element containing x; every containing element
    gives the same value, the function being continuous)."""
    c4, nid, _ = locate(level, x)
    return float(_bary(c4, np.asarray(x, dtype=np.float64)) @ values_by_node[nid])


def _node_ids(coords: np.ndarray, level: int) -> np.ndarray:
    n = 2 ** (level + 1)
    q = np.rint(np.asarray(coords) * n).astype(np.int64)
    return q[..., 0] + (n + 1) * (q[..., 1] + (n + 1) * q[..., 2])


def pressure_support(fine: int, node_xyz, seed: int = 0):
    """The level-``fine`` elements in the support of the pressure hat psi_k of the interior
    level-(fine-1) node at node_xyz: list of (coords4, node ids (4,), element id, psi_k at
    the four vertices).  The support is the star of coarse elements around the node,
    each split into its eight Bey children."""
    x = np.asarray(node_xyz, dtype=np.float64)
    coarse = fine - 1
    out = []
    for c4, _, _, _ in elements_around(coarse, x, seed):
        cc4, coords, tets, _, fids = descendants(coarse, fine, c4.mean(axis=0))
        k = int(np.argmin(np.linalg.norm(cc4 - x, axis=1)))
        for t in range(tets.shape[0]):
            f4 = coords[tets[t]]
            psi = np.array([_bary(cc4, v)[k] for v in f4])
            out.append((f4, _node_ids(f4, fine), int(fids[t]), psi))
    return out


def div_at_pressure_node(fine: int, node_xyz, u_full: np.ndarray, seed: int = 0) -> float:
    """(B u)_k at an interior pressure node: minus the sum over the velocity elements d in
    the support of psi_k of |d| div(u)|_d times the mean of psi_k over d (u_full:
    [3][(n+1)^3], boundary velocity values taken as zero)."""
    n = 2 ** (fine + 1)
    nn = (n + 1) ** 3
    free = _free_mask(fine)
    out = 0.0
    for f4, nid, _, psi in pressure_support(fine, node_xyz, seed):
        g, vol = fem.element_geometry(f4[None])
        div = 0.0
        for c in range(3):
            div += float(g[0, :, c] @ np.where(free(nid), u_full[c * nn + nid], 0.0))
        out -= vol[0] * div * psi.mean()
    return out


def mass_at_pressure_node(fine: int, node_xyz, nu_fine_by_id: np.ndarray, seed: int = 0) -> float:
    """The 1/nu-weighted lumped pressure mass m_k = sum over the velocity elements d in the
    support of psi_k of |d| / nu_d times psi_k at d's centroid (the mean at its vertices)."""
    out = 0.0
    for f4, _, eid, psi in pressure_support(fine, node_xyz, seed):
        _, vol = fem.element_geometry(f4[None])
        out += vol[0] / float(nu_fine_by_id[eid]) * psi.mean()
    return out


def grad_at_velocity_node(fine: int, node_xyz, p_coarse: np.ndarray, seed: int = 0) -> np.ndarray:
    """(B^T p) at an interior velocity node j, components c = 0..2: minus the sum over the
    level-``fine`` elements d around j of |d| (d lambda_j / d x_c)|_d times the mean over d
    of the pressure p_h (the level fine-1 P1 function with nodal values p_coarse),
    evaluated at d's vertices by interpolation on the pressure level."""
    out = np.zeros(3)
    for c4, _, _, a in elements_around(fine, node_xyz, seed):
        g, vol = fem.element_geometry(c4[None])
        ph = np.mean([_values_at(fine - 1, v, p_coarse) for v in c4])
        out -= vol[0] * g[0, a, :] * ph
    return out
