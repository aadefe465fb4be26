"""Rounding floor of the relative residual (the stopping test of eq. (4.3) in FP64).

Part of the CPU oracle: test infrastructure only (tests, smoke check, CPU baseline).

With u = 2^-53 the unit roundoff of FP64, replacing every entry x_j of an iterate by a
value within relative u of it (one more rounding) changes b - A x by at most
u (sum_e |A_e| |x_e|) entrywise, where A_e are the element matrices of eq. (2.3) /
(3.5) and |.| is taken entry by entry; forming b - A x element by element commits
errors of the same order.  The floor of the relative residual of x is therefore

    rho(x) = u || |b| + sum_e |A_e| |x_e| ||_2 / ||b||_2,

both norms over the free dofs: a solver cannot certify relative residuals much below
rho for an FP64 iterate near x.
"""

from __future__ import annotations

import numpy as np

from . import fem
from .mesh import Level

U = 2.0 ** -53


def abs_element_product(level: Level, nu_canon: np.ndarray, ncomp: int, x: np.ndarray) -> np.ndarray:
    """sum_e |A_e| |x_e| on every dof of a full level vector (x given on all dofs)."""
    Ke = np.abs(fem.element_matrices(level, nu_canon, ncomp))
    dofs = fem.element_dofs(level, ncomp)
    out = np.zeros(x.size)
    np.add.at(out, dofs.ravel(), np.einsum("tab,tb->ta", Ke, np.abs(x[dofs])).ravel())
    return out


def residual_floor(level: Level, nu_canon: np.ndarray, ncomp: int, b: np.ndarray,
                   x: np.ndarray) -> float:
    """rho(x) for full level vectors b and x (boundary entries of x count as zero)."""
    free = fem.free_dofs(level, ncomp)
    xz = np.zeros(x.size)
    xz[free] = x[free]
    s = np.abs(b[free]) + abs_element_product(level, nu_canon, ncomp, xz)[free]
    bn = np.linalg.norm(b[free])
    return float(U * np.linalg.norm(s) / bn) if bn > 0 else 0.0
