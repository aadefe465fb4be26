"""Generalized Stokes pieces (paper Section 3.1, eqs. (3.1)-(3.5)), FP64 CPU oracle.

Test infrastructure.  Velocity: P1 per component on level L (P1-iso-P2); pressure:
P1 on level L-1, every node of that level a degree of freedom (no pressure boundary
condition).  Readings taken here:

* B_kj = - integral of psi_k div Phi_j, the sign that makes the saddle-point matrix
  K = [[A, B^T], [B, 0]] symmetric ((3.2) and (3.4) differ in sign).
* psi_k is linear on every level-L element d, so the integral over d is
  |d| (div Phi_j)|_d times the mean of psi_k over d, which is the mean of its values
  at d's vertices.  Those values come from the level L-1 -> L interpolation P of
  eq. (2.4): B = -P^T B_L with (B_L)_{v,(j,c)} = sum over d containing v and j of
  |d|/4 * d lambda_j / d x_c.
* The pressure block of the preconditioner is the lumped mass weighted by 1/nu,
  m_k = sum_d |d| / nu_d * psi_k(centroid of d) = (P^T m_L)_k with
  m_L(v) = sum over d containing v of |d| / (4 nu_d).
* The pressure is fixed up to a constant (B^T 1 = 0 on free velocities); solutions
  are reported with zero mean pressure (plain average over the pressure nodes).
* The diag(A)-BFBT Schur approximation of eq. (4.2):
  S~^-1 = Z^-1 (B W^-1 A W^-1 B^T) Z^-1 with W = diag(A) and Z = B W^-1 B^T, both
  taken on the free velocity dofs.  Z has the constant pressure in its kernel; the
  paper solves with Z by an algebraic multigrid cycle, which this build does not
  have: here "Z^-1 r" means a fixed number k of Jacobi-preconditioned CG steps on
  Z y = r from y = 0 (a step whose direction has zero Z-energy, as for r = 0, has
  step size zero).  A fixed k keeps the map deterministic; it is not linear in r,
  so it serves inside FGMRES only.
* Preconditioners: block diagonal, diag(V-cycle of A, diag(m)^-1), and the upper
  block-triangular one of eq. (4.1).  With S~ an approximation of the positive
  B A^-1 B^T, the inverse of [[A, B^T], [0, -S~]] is
  [[A~^-1, A~^-1 B^T S~^-1], [0, -S~^-1]]: (4.1) as printed has +S~^-1 in the
  pressure block, which with exact blocks would not make K Q^-1 = [[I, 0], [B A^-1, I]]
  (two GMRES steps); the sign is read so that it does.  Here S~ = diag(m).
"""

from __future__ import annotations

from typing import Callable

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, mg, transfer
from .mesh import Level


def fine_div_matrix(fine: Level) -> sp.csr_matrix:
    """B_L over all nodes: rows fine nodes v, columns velocity dofs c * nn + j."""
    nn = (fine.n + 1) ** 3
    g, vol = fem.element_geometry(fine.coords[fine.tets])       # (T, 4, 3), (T,)
    nid = fine.node_id[fine.tets]                               # (T, 4)
    rows, cols, vals = [], [], []
    for a in range(4):          # vertex v of d (row)
        for b in range(4):      # vertex j of d (column)
            for c in range(3):
                rows.append(nid[:, a])
                cols.append(c * nn + nid[:, b])
                vals.append(vol / 4.0 * g[:, b, c])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nn, 3 * nn))


def div_matrix(coarse: Level, fine: Level) -> sp.csr_matrix:
    """B over all pressure nodes (level L-1) and all velocity dofs (level L)."""
    P = transfer.prolongation(coarse, fine)                     # (fine nodes, coarse nodes)
    return (-(P.T @ fine_div_matrix(fine))).tocsr()


def lumped_mass(coarse: Level, fine: Level, nu_fine_canon: np.ndarray) -> np.ndarray:
    """m_k = sum_d |d| / nu_d psi_k(centroid of d), over all pressure nodes."""
    nn = (fine.n + 1) ** 3
    _, vol = fem.element_geometry(fine.coords[fine.tets])
    nu = nu_fine_canon[fine.elem_id]
    mL = np.zeros(nn)
    np.add.at(mL, fine.node_id[fine.tets].ravel(), np.repeat(vol / (4.0 * nu), 4))
    P = transfer.prolongation(coarse, fine)
    return P.T @ mL


class StokesSystem:
    """K = [[A, B^T], [B, 0]] on free velocity dofs and all pressure nodes."""

    def __init__(self, H: mg.Hierarchy):
        L = H.L
        self.H = H
        coarse, fine = H.levels[L - 1], H.levels[L]
        self.free_u = H.free[L]
        self.nu_ = self.free_u.size
        self.np_ = (coarse.n + 1) ** 3
        self.nn_fine = (fine.n + 1) ** 3
        B = div_matrix(coarse, fine)[:, self.free_u]
        self.B = B.tocsr()
        self.A = H.A[L]
        self.K = sp.bmat([[self.A, self.B.T], [self.B, None]]).tocsr()
        self.m = lumped_mass(coarse, fine, H.nu_levels[L])

    def split(self, x):
        return x[:self.nu_], x[self.nu_:]

    def precond(self, kind: str = "diagonal", a_inv: Callable = None,
                s_inv: Callable = None) -> Callable:
        """diag(V-cycle, lumped 1/nu mass inverse), or the upper block-triangular
        [[A~^-1, A~^-1 B^T S~^-1], [0, -S~^-1]]; a_inv / s_inv replace the V-cycle and
        the mass inverse (the exact inverses make K Q^-1 unipotent)."""
        H = self.H
        a_inv = a_inv or (lambda ru: mg.vcycle(H, ru))
        s_inv = s_inv or (lambda rp: rp / self.m)

        def M(r):
            ru, rp = self.split(r)
            if kind == "diagonal":
                return np.concatenate([a_inv(ru), s_inv(rp)])
            if kind != "triangular":
                raise ValueError(kind)
            q = s_inv(rp)
            return np.concatenate([a_inv(ru + self.B.T @ q), -q])
        return M

    def z_operator(self) -> sp.csr_matrix:
        """Z = B W^-1 B^T over all pressure nodes, W = diag(A) on free velocity dofs."""
        w = self.A.diagonal()
        return (self.B @ sp.diags(1.0 / w) @ self.B.T).tocsr()

    def z_solve(self, iters: int, Z: sp.csr_matrix = None) -> Callable:
        """r -> k steps of Jacobi-preconditioned CG on Z y = r from y = 0."""
        Z = self.z_operator() if Z is None else Z
        dz = Z.diagonal()

        def solve(r):
            y = np.zeros_like(r)
            res = r.copy()
            z = res / dz
            p = z.copy()
            rz = res @ z
            for k in range(iters):
                q = Z @ p
                pq = p @ q
                alpha = rz / pq if pq != 0.0 else 0.0
                y += alpha * p
                res -= alpha * q
                if k == iters - 1:
                    break
                z = res / dz
                rz_new = res @ z
                p = z + (rz_new / rz if rz != 0.0 else 0.0) * p
                rz = rz_new
            return y
        return solve

    def bfbt(self, iters: int = 0, z_solve: Callable = None) -> Callable:
        """S~^-1 of eq. (4.2): Z^-1 B W^-1 A W^-1 B^T Z^-1, with Z^-1 the fixed-step
        Jacobi-CG solve (or a given z_solve, e.g. an exact one)."""
        w = self.A.diagonal()
        zs = z_solve or self.z_solve(iters)

        def s_inv(rp):
            y1 = zs(rp)
            t = self.A @ ((self.B.T @ y1) / w)
            return zs(self.B @ (t / w))
        return s_inv

    def direct(self, b: np.ndarray) -> np.ndarray:
        """Exact solution with zero mean pressure: the first pressure unknown is fixed at
        zero (the constant pressure spans the kernel), the rest solved by sparse LU, and
        the mean removed afterwards."""
        n = self.K.shape[0]
        keep = np.ones(n, dtype=bool)
        keep[self.nu_] = False
        Kr = self.K[keep][:, keep].tocsc()
        x = np.zeros(n)
        x[keep] = spla.splu(Kr).solve(b[keep])
        return self.zero_mean(x)

    def zero_mean(self, x: np.ndarray) -> np.ndarray:
        x = x.copy()
        x[self.nu_:] -= x[self.nu_:].mean()
        return x

    def solve(self, b: np.ndarray, solver: str, tol: float, restart: int = 30,
              maxit: int = 500, precond: str = "diagonal", schur: str = "mass",
              schur_iters: int = 20) -> mg.SolveResult:
        if schur == "mass":
            M = self.precond(precond)
        elif schur == "bfbt":
            if solver != "fgmres":
                raise ValueError("the BFBT approximation is not a fixed linear map: FGMRES only")
            M = self.precond(precond, s_inv=self.bfbt(schur_iters))
        else:
            raise ValueError(schur)
        if solver == "fgmres":
            res = mg.fgmres(self.K, b, M, tol, restart=restart, maxit=maxit)
        elif solver == "minres":
            res = mg.minres(self.K, b, M, tol, maxit=maxit)
        else:
            raise ValueError(solver)
        res.x = self.zero_mean(res.x)
        return res
