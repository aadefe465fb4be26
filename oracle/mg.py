"""Multigrid V-cycle and Krylov solvers on assembled free-DoF matrices.

Part of the CPU oracle: test infrastructure only (tests, smoke check, CPU baseline).

V-cycle (paper Section 4: one V-cycle approximates the inverse of the viscous
block): damped Jacobi smoothing with the diagonal of the level operator,
omega = 2/3, nu1 pre- and nu2 post-sweeps, restriction = P^T, interpolation = P
(Section 2.1), zero initial guess on every coarser level, and a dense direct
solve on level 0.  The SOR-CG coarse solver of the paper is replaced by a direct
solve (level 0 has one free node).

Smoothers: damped Jacobi (the benchmark's) or the Chebyshev polynomial smoother
of Section 4 (degree nu1 / nu2): the Chebyshev iteration for D^-1 A on the
interval [lambda_max / 10, lambda_max] with lambda_max = 1.1 times an estimate
of the largest eigenvalue of D^-1 A.  The paper gives no estimation procedure;
the estimate here is the largest Ritz value after 20 steps of the Lanczos process
for the pencil (A, D) (D^-1 A is self-adjoint in the D inner product), started
from the alternating vector (-1)^(X+Y+Z) on the free nodes.  A Ritz value is a
lower bound of the largest eigenvalue; plain power steps converge far more slowly
where the top eigenvectors concentrate at sharp viscosity jumps.

Solvers, all starting from x0 = 0 and stopping when ||b - A x||_2 <= tol ||b||_2
(eq. (4.3) with the benchmark's tolerance):
  stationary MG, PCG, flexible CG (FCG(1)), iterative refinement, FGMRES(m),
  MINRES.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import agca as _agca
from . import fem, mesh, transfer


@dataclass
class Hierarchy:
    levels: list
    ncomp: int
    ops_full: List[sp.csr_matrix]            # Neumann operators, all nodes
    A: List[sp.csr_matrix]                   # free-DoF operators
    P: List[sp.csr_matrix]                   # free-DoF interpolation, level l -> l+1
    P_full: List[sp.csr_matrix]              # all-node interpolation
    free: List[np.ndarray]                   # free dof indices per level
    flags: List[np.ndarray]
    nu_levels: List[np.ndarray]
    omega: float = 2.0 / 3.0
    nu1: int = 2
    nu2: int = 2
    coarse_chol: object = None
    D: List[np.ndarray] = field(default_factory=list)
    smoother: str = "jacobi"
    lam: List[float] = field(default_factory=list)   # Chebyshev: eigenvalue estimates per level

    @property
    def L(self) -> int:
        return len(self.levels) - 1


CHEB_RATIO = 10.0   # lambda_min = lambda_max / CHEB_RATIO
CHEB_BOOST = 1.1    # lambda_max = CHEB_BOOST * estimate
LANCZOS_STEPS = 20
LANCZOS_BREAKDOWN = 1e-12   # beta_k <= this * |alpha_k| ends the process


def alternating_start(level, ncomp: int, free: np.ndarray) -> np.ndarray:
    """(-1)^(X+Y+Z) at every free dof (X, Y, Z the node's lattice coordinates)."""
    nn = (level.n + 1) ** 3
    X = np.rint(level.coords * level.n).astype(np.int64)
    sign = np.empty(nn)
    sign[level.node_id] = np.where(X.sum(axis=1) % 2 == 0, 1.0, -1.0)
    return np.tile(sign, ncomp)[free]


def lambda_max_estimate(A, D: np.ndarray, x0: np.ndarray, steps: int = LANCZOS_STEPS) -> float:
    """Largest Ritz value of D^-1 A after ``steps`` Lanczos steps in the D inner product
    <x, y>_D = x.Dy (Lanczos 1950): with v_0 = x0 / ||x0||_D,
        alpha_k = v_k.A v_k,  w = D^-1 A v_k - alpha_k v_k - beta_{k-1} v_{k-1},
        beta_k = ||w||_D,     v_{k+1} = w / beta_k,
    and the estimate is the largest eigenvalue of the symmetric tridiagonal matrix with
    diagonal alpha and off-diagonal beta.  The process stops early when beta_k vanishes
    (the Krylov space is invariant; its Ritz values are then eigenvalues)."""
    v = x0 / np.sqrt(x0 @ (D * x0))
    v_prev = np.zeros_like(v)
    alpha, beta = [], []
    b = 0.0
    for _ in range(steps):
        y = A @ v
        a = float(v @ y)
        w = y / D - a * v - b * v_prev
        alpha.append(a)
        b = float(np.sqrt(w @ (D * w)))
        if not b > LANCZOS_BREAKDOWN * abs(a):
            break
        beta.append(b)
        v_prev, v = v, w / b
    m = len(alpha)
    return float(sla.eigvalsh_tridiagonal(np.array(alpha), np.array(beta[:m - 1]),
                                          select="i", select_range=(m - 1, m - 1))[0])


def build(L: int, nu_levels: List[np.ndarray], ncomp: int, tau: float = 10.0,
          mode: int = _agca.FLAG_RATIO, levels=None, smoother: str = "jacobi",
          macro_flags: Optional[np.ndarray] = None) -> Hierarchy:
    """Assemble the AGCA hierarchy for coefficients ``nu_levels`` (canonical ids per level)."""
    if levels is None:
        levels = mesh.hierarchy(L)
    Pf = transfer.prolongations(levels, ncomp)
    res = _agca.agca_operators(levels, Pf, nu_levels, ncomp, tau, mode, macro_flags)
    free = [fem.free_dofs(lv, ncomp) for lv in levels]
    A = [fem.restrict_free(op, fr) for op, fr in zip(res["ops"], free)]
    P = [Pf[l][free[l + 1]][:, free[l]].tocsr() for l in range(L)]
    H = Hierarchy(levels, ncomp, res["ops"], A, P, Pf, free, res["flags"], nu_levels)
    H.D = [a.diagonal().copy() for a in A]
    A0 = A[0].toarray()
    H.coarse_chol = sla.cho_factor(A0)
    H.smoother = smoother
    if smoother == "chebyshev":
        H.lam = [0.0] + [lambda_max_estimate(A[l], H.D[l], alternating_start(levels[l], ncomp, free[l]))
                         for l in range(1, L + 1)]
    elif smoother != "jacobi":
        raise ValueError(smoother)
    return H


def full_to_free(H: Hierarchy, l: int, x: np.ndarray) -> np.ndarray:
    return x[H.free[l]]


def free_to_full(H: Hierarchy, l: int, xf: np.ndarray) -> np.ndarray:
    n = H.ncomp * (H.levels[l].n + 1) ** 3
    x = np.zeros(n)
    x[H.free[l]] = xf
    return x


def jacobi(H: Hierarchy, l: int, b: np.ndarray, x: np.ndarray, sweeps: int) -> np.ndarray:
    A, D = H.A[l], H.D[l]
    for _ in range(sweeps):
        x = x + H.omega * (b - A @ x) / D
    return x


def chebyshev(H: Hierarchy, l: int, b: np.ndarray, x: np.ndarray, degree: int) -> np.ndarray:
    """degree steps of the Chebyshev iteration for D^-1 A on [lmax / CHEB_RATIO, lmax]
    (three-term recurrence of the shifted and scaled Chebyshev polynomials)."""
    A, D = H.A[l], H.D[l]
    lmax = CHEB_BOOST * H.lam[l]
    lmin = lmax / CHEB_RATIO
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = (b - A @ x) / D / theta
    x = x + d
    for _ in range(1, degree):
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (b - A @ x) / D
        x = x + d
        rho = rho_new
    return x


def smooth(H: Hierarchy, l: int, b: np.ndarray, x: np.ndarray, sweeps: int) -> np.ndarray:
    if H.smoother == "chebyshev":
        return chebyshev(H, l, b, x, sweeps) if sweeps > 0 else x
    return jacobi(H, l, b, x, sweeps)


def vcycle(H: Hierarchy, b: np.ndarray, l: Optional[int] = None, x: Optional[np.ndarray] = None):
    """One V-cycle on level l for A_l x = b (free-DoF vectors)."""
    if l is None:
        l = H.L
    if x is None:
        x = np.zeros_like(b)
    if l == 0:
        return sla.cho_solve(H.coarse_chol, b)
    x = smooth(H, l, b, x, H.nu1)
    r = b - H.A[l] @ x
    rc = H.P[l - 1].T @ r
    ec = vcycle(H, rc, l - 1, None)
    x = x + H.P[l - 1] @ ec
    x = smooth(H, l, b, x, H.nu2)
    return x


@dataclass
class SolveResult:
    x: np.ndarray
    iterations: int
    history: List[float]
    converged: bool


def _rel(r, bn):
    return float(np.linalg.norm(r) / bn)


def stationary(H: Hierarchy, b: np.ndarray, tol: float, maxit: int = 200) -> SolveResult:
    """x <- x + V(b - A x) until the relative residual is below tol."""
    A = H.A[H.L]
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    hist = [_rel(r, bn)]
    for it in range(1, maxit + 1):
        x = x + vcycle(H, r)
        r = b - A @ x
        hist.append(_rel(r, bn))
        if hist[-1] <= tol:
            return SolveResult(x, it, hist, True)
    return SolveResult(x, maxit, hist, False)


def pcg(A, b, M: Callable, tol: float, maxit: int = 500) -> SolveResult:
    """Preconditioned conjugate gradients (M a symmetric positive definite preconditioner)."""
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = r @ z
    hist = [_rel(r, bn)]
    for it in range(1, maxit + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        hist.append(_rel(r, bn))
        if hist[-1] <= tol:
            return SolveResult(x, it, hist, True)
        z = M(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return SolveResult(x, maxit, hist, False)


def fcg(A, b, M: Callable, tol: float, maxit: int = 500) -> SolveResult:
    """Flexible CG with one-term orthogonalisation (FCG(1), Notay):
    beta = z_k . (r_k - r_{k-1}) / (z_{k-1} . r_{k-1})  (Polak-Ribiere form)."""
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = r @ z
    hist = [_rel(r, bn)]
    for it in range(1, maxit + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r_old = r.copy()
        r -= alpha * q
        hist.append(_rel(r, bn))
        if hist[-1] <= tol:
            return SolveResult(x, it, hist, True)
        z = M(r)
        beta = (z @ (r - r_old)) / rz
        rz = r @ z
        p = z + beta * p
    return SolveResult(x, maxit, hist, False)


def iterative_refinement(A, b, M: Callable, tol: float, maxit: int = 500) -> SolveResult:
    """x <- x + M(b - A x)."""
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    hist = [_rel(r, bn)]
    for it in range(1, maxit + 1):
        x = x + M(r)
        r = b - A @ x
        hist.append(_rel(r, bn))
        if hist[-1] <= tol:
            return SolveResult(x, it, hist, True)
    return SolveResult(x, maxit, hist, False)


def fgmres(A, b, M: Callable, tol: float, restart: int = 30, maxit: int = 500) -> SolveResult:
    """Right-preconditioned flexible GMRES(m) with modified Gram-Schmidt."""
    bn = np.linalg.norm(b)
    n = b.size
    x = np.zeros(n)
    r = b.copy()
    hist = [_rel(r, bn)]
    it = 0
    while it < maxit:
        beta = np.linalg.norm(r)
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        Hm = np.zeros((restart + 1, restart))
        V[0] = r / beta
        g = np.zeros(restart + 1)
        g[0] = beta
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        k_done = 0
        for k in range(restart):
            Z[k] = M(V[k])
            w = A @ Z[k]
            for i in range(k + 1):
                Hm[i, k] = w @ V[i]
                w = w - Hm[i, k] * V[i]
            Hm[k + 1, k] = np.linalg.norm(w)
            if Hm[k + 1, k] > 0:
                V[k + 1] = w / Hm[k + 1, k]
            for i in range(k):
                t = cs[i] * Hm[i, k] + sn[i] * Hm[i + 1, k]
                Hm[i + 1, k] = -sn[i] * Hm[i, k] + cs[i] * Hm[i + 1, k]
                Hm[i, k] = t
            d = np.hypot(Hm[k, k], Hm[k + 1, k])
            cs[k], sn[k] = Hm[k, k] / d, Hm[k + 1, k] / d
            Hm[k, k] = d
            Hm[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            it += 1
            k_done = k + 1
            hist.append(abs(g[k + 1]) / bn)
            if hist[-1] <= tol or it >= maxit:
                break
        y = sla.solve_triangular(Hm[:k_done, :k_done], g[:k_done])
        x = x + Z[:k_done].T @ y
        r = b - A @ x
        hist[-1] = _rel(r, bn)
        if hist[-1] <= tol:
            return SolveResult(x, it, hist, True)
    return SolveResult(x, it, hist, False)


def minres(A, b, M: Callable, tol: float, maxit: int = 500) -> SolveResult:
    """MINRES (Paige and Saunders, SIAM J. Numer. Anal. 12, 1975) for a symmetric,
    possibly indefinite or singular but consistent A, with a symmetric positive definite
    preconditioner M (z = M(r)), in its plainest form: the Lanczos process and, at every
    step, an explicit least-squares solve of the small tridiagonal system.

    Write M = C C^T.  MINRES for C^T A C y = C^T b, x = C y, builds the Lanczos vectors
    q_j of C^T A C; this routine keeps w_j = C^-T q_j (residual space) and u_j = C q_j =
    M w_j (solution space), so C itself is never needed:
        beta_1 = sqrt(b . M b),  w_1 = b / beta_1,  u_1 = M b / beta_1,
        v = A u_j - beta_j w_(j-1),  alpha_j = u_j . v,  v -= alpha_j w_j,
        beta_(j+1) = sqrt(v . M v),  w_(j+1) = v / beta_(j+1),  u_(j+1) = M v / beta_(j+1).
    Then A U_k = W_(k+1) T_k with T_k the (k+1) x k tridiagonal matrix (alpha on the
    diagonal, beta_(j+1) below and above it), and the iterate x_k = U_k t with
    t = argmin ||beta_1 e_1 - T_k t||_2 minimises the M-norm of b - A x over the
    preconditioned Krylov space.  The stopping test is eq. (4.3) on the true residual
    b - A x_k, recomputed from x_k at every step (its 2-norm need not decrease
    monotonically).  A step with beta_(j+1) = 0 has reached an invariant space, where
    x_k solves the system."""
    n = b.size
    bn = np.linalg.norm(b)
    x = np.zeros(n)
    hist = [1.0]
    mb = M(b)
    beta1 = float(np.sqrt(b @ mb))
    if beta1 == 0.0:
        return SolveResult(x, 0, hist, True)
    U = np.zeros((n, 16))
    alphas: List[float] = []
    betas: List[float] = [beta1]           # betas[j] = beta_(j+1)
    w_prev = np.zeros(n)
    w = b / beta1
    u = mb / beta1
    for k in range(1, maxit + 1):
        if k > U.shape[1]:
            U = np.concatenate([U, np.zeros_like(U)], axis=1)
        U[:, k - 1] = u
        v = A @ u - (betas[k - 1] * w_prev if k > 1 else 0.0)
        a = float(u @ v)
        v = v - a * w
        mv = M(v)
        bnext = float(np.sqrt(max(v @ mv, 0.0)))
        alphas.append(a)
        betas.append(bnext)
        T = np.zeros((k + 1, k))
        for j in range(k):
            T[j, j] = alphas[j]
            T[j + 1, j] = betas[j + 1]
            if j > 0:
                T[j - 1, j] = betas[j]
        rhs = np.zeros(k + 1)
        rhs[0] = beta1
        t = np.linalg.lstsq(T, rhs, rcond=None)[0]
        x = U[:, :k] @ t
        rel = _rel(b - A @ x, bn)
        hist.append(rel)
        if rel <= tol or bnext == 0.0:
            return SolveResult(x, k, hist, rel <= tol)
        w_prev, w, u = w, v / bnext, mv / bnext
    return SolveResult(x, maxit, hist, False)
