"""Pins of the oracle's Chebyshev smoother (paper Section 4: Chebyshev polynomial
smoother) and of its eigenvalue estimate.

* With b = 0 the smoother maps an eigenvector v of D^-1 A (eigenvalue lam) to
  p_m(lam) v, where p_m(lam) = T_m((theta - lam) / delta) / T_m(theta / delta) is the
  shifted and scaled Chebyshev polynomial of degree m on [lmin, lmax] (closed form).
* The estimate is the largest Ritz value of the Lanczos process for the pencil
  (A, D): a lower bound of the largest generalized eigenvalue, within 2% of it after
  20 steps on a high-contrast level, and exact once the Krylov space is the whole
  space (brute force on a small pencil).
"""

from types import SimpleNamespace

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem, mesh, mg
from workloads import Sinkers


def _operator(L=2, ncomp=3):
    levels = mesh.hierarchy(L)
    rng = np.random.default_rng(5)
    nu = np.exp(rng.uniform(-3, 3, levels[L].tets.shape[0]))
    free = fem.free_dofs(levels[L], ncomp)
    A = fem.restrict_free(fem.assemble(levels[L], nu, ncomp), free)
    return levels, A, free


def _largest_generalized(A, D):
    """Largest eigenvalue of A v = lam D v by ARPACK on D^-1/2 A D^-1/2 (to rounding)."""
    s = 1.0 / np.sqrt(D)
    S = sp.diags(s) @ A @ sp.diags(s)
    return float(spla.eigsh(S, k=1, which="LA", tol=1e-14, return_eigenvectors=False)[0])


def _cheb_T(m, x):
    x = np.asarray(x, dtype=float)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1
    out[inside] = np.cos(m * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** m * np.cosh(m * np.arccosh(np.abs(xo)))
    return out


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_error_propagation_is_the_scaled_chebyshev_polynomial(degree):
    levels, A, free = _operator()
    D = A.diagonal().copy()
    lam, V = sla.eigh(A.toarray(), np.diag(D))        # A v = lam D v
    lmax_true = lam[-1]
    H = SimpleNamespace(A={1: A}, D={1: D}, lam={1: lmax_true / mg.CHEB_BOOST})
    lmax = lmax_true
    lmin = lmax / mg.CHEB_RATIO
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    for j in (0, 3, len(lam) // 2, len(lam) - 1):
        v = V[:, j]
        out = mg.chebyshev(H, 1, np.zeros_like(v), v.copy(), degree)
        p = _cheb_T(degree, (theta - lam[j]) / delta) / _cheb_T(degree, theta / delta)
        assert np.allclose(out, p * v, rtol=0, atol=1e-10 * np.abs(v).max()), (degree, j)


def test_eigenvalue_estimate_bounds():
    levels, A, free = _operator(L=3)
    D = A.diagonal().copy()
    x0 = mg.alternating_start(levels[3], 3, free)
    est = mg.lambda_max_estimate(A, D, x0)
    lam = _largest_generalized(A, D)
    assert est <= lam * (1 + 1e-12)
    assert est >= 0.98 * lam


def test_eigenvalue_estimate_exact_on_small_pencil():
    # 12 unknowns < 20 steps: the process exhausts the space and breaks down, and
    # its largest Ritz value is the largest generalized eigenvalue
    rng = np.random.default_rng(3)
    G = rng.standard_normal((12, 12))
    A = G @ G.T + 12 * np.eye(12)
    D = np.diag(A).copy()
    lam = sla.eigh(A, np.diag(D), eigvals_only=True)[-1]
    est = mg.lambda_max_estimate(A, D, rng.standard_normal(12))
    assert abs(est - lam) <= 1e-10 * lam
    # fewer steps than unknowns: a strict lower bound
    est3 = mg.lambda_max_estimate(A, D, rng.standard_normal(12), steps=3)
    assert est3 < lam


def test_eigenvalue_estimate_high_contrast_sinkers():
    # sharp 1e6 viscosity jumps: the top eigenvectors of D^-1 A concentrate at the
    # interfaces, where 20 Lanczos steps still come within 2% (20 plain power steps
    # lose over 10% on such levels)
    L = 3
    levels = mesh.hierarchy(L)
    field = Sinkers(4, 2, radius=0.15, width=2.0 / 2 ** (L + 1), contrast=1e6)
    nu = field.nu(mesh.centroids_canonical(levels[L]))
    free = fem.free_dofs(levels[L], 3)
    A = fem.restrict_free(fem.assemble(levels[L], nu, 3), free)
    D = A.diagonal().copy()
    lam = _largest_generalized(A, D)
    est = mg.lambda_max_estimate(A, D, mg.alternating_start(levels[L], 3, free))
    assert lam * 0.98 <= est <= lam * (1 + 1e-12)


def test_chebyshev_vcycle_pcg_converges_faster_than_jacobi():
    L = 3
    levels = mesh.hierarchy(L)
    field = Sinkers(4, 2, radius=0.15, width=2.0 / 2 ** (L + 1), contrast=1e6)
    nu = [field.nu(mesh.centroids_canonical(lv)) for lv in levels]
    f = np.asarray(field.force(mesh.centroids_canonical(levels[L]), 3))
    its = {}
    for sm in ("jacobi", "chebyshev"):
        H = mg.build(L, nu, 3, levels=levels, smoother=sm)
        b = fem.load_vector(levels[L], f, 3)[H.free[L]]
        r = mg.pcg(H.A[L], b, lambda rr: mg.vcycle(H, rr), 1e-8, maxit=2000)
        assert r.converged
        its[sm] = r.iterations
    assert its["chebyshev"] < its["jacobi"], its
