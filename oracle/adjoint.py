"""Adjoint gradient of J = 1/2 ||u - u_obs||^2 with respect to log nu per finest element.

Part of the CPU oracle: test infrastructure only (tests, smoke check, CPU baseline).

Not part of the paper (an extension of the method): with A(nu) u = f and A
symmetric, the Lagrangian J + lambda^T (A u - f) gives A lambda = -(u - u_obs).
Each element matrix is linear in its own coefficient, dA_e/dnu_e = A_e / nu_e,
so with w = A^{-1} (u - u_obs):

    dJ / dlog nu_e = nu_e lambda_e^T (dA_e/dnu_e) u_e = - w_e^T A_e u_e.

J is summed over free DoFs only (boundary values are zero on both u and u_obs).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fem


def grad_log_nu(level, nu_canon: np.ndarray, ncomp: int, u_full: np.ndarray,
                w_full: np.ndarray) -> np.ndarray:
    """g_e = -w_e^T A_e u_e for every element, by canonical id (u, w full nodal vectors)."""
    Ke = fem.element_matrices(level, nu_canon, ncomp)
    dofs = fem.element_dofs(level, ncomp)
    ue = u_full[dofs]
    we = w_full[dofs]
    g = -np.einsum("ta,tab,tb->t", we, Ke, ue)
    out = np.empty_like(g)
    out[level.elem_id] = g
    return out


def solve_free(A_free, b_free):
    """Direct sparse solve used as the exact forward/adjoint solve at small sizes."""
    return spla.splu(A_free.tocsc()).solve(b_free)
