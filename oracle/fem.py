"""P1 finite elements: element matrices and global sparse assembly (paper eqs. (2.3), (2.5), (3.5)).

Part of the CPU oracle: test infrastructure only (tests, smoke check, CPU baseline).

Element matrices come from the inverse of the 4x4 barycentric matrix
[[1 1 1 1], [x_0 .. x_3]] (rows 1..3 of the inverse's columns are the constant
gradients of the barycentric coordinates) and the volume |det| / 6.

* scalar diffusion:  [A_e]_ab = nu_e |e| grad(l_a) . grad(l_b)
* vector viscous block, from  int 2 nu eps(u) : eps(v)  (eq. (3.5)); for the
  trial function l_b e_d and the test function l_a e_c:
      [A_e]_(c,a),(d,b) = nu_e |e| ( delta_cd grad(l_a).grad(l_b) + d_d l_a  d_c l_b )

The coefficient is one value per element (P0): for P1 stiffness only the element
integral of nu enters, so a per-element value is exact for any quadrature that
integrates it (Remark 3).

Global vectors use the GPU library's layout: ``ncomp`` blocks of (n+1)^3
values, one per canonical node id (component-major).  Assembly gives the full
(Neumann) matrix over all nodes; ``restrict_free`` takes the principal
submatrix on nodes strictly inside the cube (homogeneous Dirichlet data,
eq. (3.1) with g = 0).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import Level, free_node_mask


def element_geometry(coords4: np.ndarray):
    """Gradients (T, 4, 3) of the barycentric coordinates and volumes (T,)."""
    T = coords4.shape[0]
    M = np.ones((T, 4, 4))
    M[:, 1:, :] = coords4.transpose(0, 2, 1)
    Minv = np.linalg.inv(M)
    grads = Minv[:, :, 1:]
    vol = np.abs(np.linalg.det(M)) / 6.0
    return grads, vol


def scalar_element_matrices(coords4: np.ndarray, nu: np.ndarray) -> np.ndarray:
    g, vol = element_geometry(coords4)
    return (nu * vol)[:, None, None] * np.einsum("tad,tbd->tab", g, g)


def vector_element_matrices(coords4: np.ndarray, nu: np.ndarray) -> np.ndarray:
    """(T, 12, 12) with local index 4*c + a (component c, vertex a)."""
    g, vol = element_geometry(coords4)
    T = g.shape[0]
    gg = np.einsum("tad,tbd->tab", g, g)                    # grad l_a . grad l_b
    K = np.zeros((T, 3, 4, 3, 4))
    for c in range(3):
        K[:, c, :, c, :] += gg
        for d in range(3):
            # d_d l_a * d_c l_b
            K[:, c, :, d, :] += g[:, :, d][:, :, None] * g[:, :, c][:, None, :]
    return (nu * vol)[:, None, None] * K.reshape(T, 12, 12)


def element_matrices(level: Level, nu_canon: np.ndarray, ncomp: int) -> np.ndarray:
    """Element matrices in the level's Bey element order; nu given by canonical id."""
    nu = nu_canon[level.elem_id]
    c4 = level.coords[level.tets]
    if ncomp == 1:
        return scalar_element_matrices(c4, nu)
    return vector_element_matrices(c4, nu)


def element_dofs(level: Level, ncomp: int) -> np.ndarray:
    """(T, 4*ncomp) global dof of each local dof (local index 4*c + a)."""
    nn = (level.n + 1) ** 3
    nid = level.node_id[level.tets]                         # (T, 4)
    return np.concatenate([c * nn + nid for c in range(ncomp)], axis=1)


def assemble(level: Level, nu_canon: np.ndarray, ncomp: int, elem_mask=None) -> sp.csr_matrix:
    """Full Neumann matrix sum_e I_e A_e I_e^T (eq. (2.3)) over all nodes.

    ``elem_mask`` (canonical-id boolean array) keeps only the selected elements;
    this is how the oracle builds masked operators.
    """
    Ke = element_matrices(level, nu_canon, ncomp)
    dofs = element_dofs(level, ncomp)
    if elem_mask is not None:
        keep = elem_mask[level.elem_id]
        Ke, dofs = Ke[keep], dofs[keep]
    m = dofs.shape[1]
    rows = np.repeat(dofs, m, axis=1).ravel()
    cols = np.tile(dofs, (1, m)).ravel()
    N = ncomp * (level.n + 1) ** 3
    A = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(N, N)).tocsr()
    A.sum_duplicates()
    return A


def free_dofs(level: Level, ncomp: int) -> np.ndarray:
    """Sorted global dof indices of the free (interior) nodes, all components."""
    nn = (level.n + 1) ** 3
    free_nodes = np.zeros(nn, dtype=bool)
    free_nodes[level.node_id[free_node_mask(level)]] = True
    idx = np.nonzero(free_nodes)[0]
    return np.concatenate([c * nn + idx for c in range(ncomp)])


def restrict_free(A: sp.spmatrix, free: np.ndarray) -> sp.csr_matrix:
    return A.tocsr()[free][:, free].tocsr()


def load_vector(level: Level, f_canon: np.ndarray, ncomp: int) -> np.ndarray:
    """b_i = int f phi_i for a per-element constant f: each vertex gets f_e |e| / 4.

    ``f_canon`` is (T,) for ncomp = 1 or (T, ncomp), indexed by canonical element id.
    Boundary entries are set to zero.
    """
    nn = (level.n + 1) ** 3
    _, vol = element_geometry(level.coords[level.tets])
    f = np.asarray(f_canon).reshape(f_canon.shape[0], -1)[level.elem_id]
    b = np.zeros(ncomp * nn)
    nid = level.node_id[level.tets]
    for c in range(ncomp):
        w = np.repeat(f[:, c] * vol / 4.0, 4)
        np.add.at(b, c * nn + nid.ravel(), w)
    free_nodes = np.zeros(nn, dtype=bool)
    free_nodes[level.node_id[free_node_mask(level)]] = True
    for c in range(ncomp):
        b[c * nn:(c + 1) * nn][~free_nodes] = 0.0
    return b
