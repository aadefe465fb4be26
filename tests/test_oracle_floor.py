"""Pins of the oracle's rounding floor (oracle/floor.py) against facts it must obey."""

import numpy as np
import pytest

from oracle import fem, floor, mesh
from workloads import Sinkers


def _lattice(level, v):
    n = level.n
    return v.reshape(n + 1, n + 1, n + 1)       # index [z, y, x]


def test_unit_scalar_coefficient_is_the_seven_point_stencil():
    """nu = 1, scalar: every element matrix is (h/6) times a path Laplacian with
    nonnegative off-path zeros, the six tets around an axis edge add up without
    cancellation, so sum_e |A_e| |x_e| = h (6 |x_i| + sum of |x| at the 6 axis
    neighbours) at interior nodes (the textbook operator of App. A.1)."""
    L = 2
    lv = mesh.hierarchy(L)[L]
    n = lv.n
    h = 1.0 / n
    rng = np.random.default_rng(0)
    x = rng.standard_normal((n + 1) ** 3)
    s = floor.abs_element_product(lv, np.ones(lv.tets.shape[0]), 1, x)
    ax = np.abs(_lattice(lv, x))
    ref = 6.0 * ax[1:-1, 1:-1, 1:-1]
    for axis in range(3):
        for sh in (-1, 1):
            ref = ref + np.roll(ax, sh, axis=axis)[1:-1, 1:-1, 1:-1]
    assert np.allclose(_lattice(lv, s)[1:-1, 1:-1, 1:-1], h * ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("ncomp", [1, 3])
def test_bounds_and_unit_vectors(ncomp):
    """|A x| <= sum_e |A_e||x_e| entrywise; a perturbation |d_j| <= u |x_j| moves A x by at
    most u sum_e |A_e||x_e|; for x = e_j the j-th entry equals the (positive) diagonal
    A_jj and every other entry is at least |A_ij|."""
    L = 2
    levels = mesh.hierarchy(L)
    lv = levels[L]
    field = Sinkers(3, 2, radius=0.2, width=0.05, contrast=1e6)
    nu = field.nu(mesh.centroids_canonical(lv))
    A = fem.assemble(lv, nu, ncomp)
    N = ncomp * (lv.n + 1) ** 3
    rng = np.random.default_rng(1)
    x = rng.standard_normal(N)
    s = floor.abs_element_product(lv, nu, ncomp, x)
    assert np.all(np.abs(A @ x) <= s * (1 + 1e-12))
    d = floor.U * x * rng.uniform(-1, 1, N)
    assert np.all(np.abs(A @ d) <= floor.U * s * (1 + 1e-12))
    Ad = A.toarray()
    for j in rng.choice(N, 5, replace=False):
        e = np.zeros(N)
        e[j] = 1.0
        sj = floor.abs_element_product(lv, nu, ncomp, e)
        assert abs(sj[j] - Ad[j, j]) <= 1e-13 * Ad[j, j]
        assert np.all(sj >= np.abs(Ad[:, j]) * (1 - 1e-12))


def test_floor_definition():
    """rho = u || |b| + S |x| || / ||b|| over free dofs; boundary entries of x are ignored
    and rho scales like 1/||b|| for fixed x."""
    L = 2
    lv = mesh.hierarchy(L)[L]
    rng = np.random.default_rng(2)
    nu = np.exp(rng.uniform(-3, 3, lv.tets.shape[0]))
    free = fem.free_dofs(lv, 3)
    N = 3 * (lv.n + 1) ** 3
    x = np.zeros(N)
    x[free] = rng.standard_normal(free.size)
    b = np.zeros(N)
    b[free] = rng.standard_normal(free.size)
    rho = floor.residual_floor(lv, nu, 3, b, x)
    s = np.abs(b[free]) + floor.abs_element_product(lv, nu, 3, x)[free]
    assert rho == pytest.approx(floor.U * np.linalg.norm(s) / np.linalg.norm(b[free]), rel=1e-14)
    xb = x.copy()
    xb[np.setdiff1d(np.arange(N), free)] = 5.0
    assert floor.residual_floor(lv, nu, 3, b, xb) == pytest.approx(rho, rel=1e-14)
    b2 = 1e-3 * b
    rho2 = floor.residual_floor(lv, nu, 3, b2, x)
    s2 = np.abs(b2[free]) + floor.abs_element_product(lv, nu, 3, x)[free]
    assert rho2 == pytest.approx(floor.U * np.linalg.norm(s2) / np.linalg.norm(b2[free]), rel=1e-14)
    assert rho2 > 100 * rho
