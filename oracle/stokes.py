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
  paper solves with Z by an algebraic multigrid cycle inside CG.  Here "Z^-1 r" is a
  fixed number k of CG steps on Z y = r from y = 0 (a step whose direction has zero
  Z-energy, as for r = 0, has step size zero), preconditioned either by Jacobi
  (z_solve) or by one V-cycle of a geometric multigrid for Z (ZHierarchy, below).
  A fixed k keeps the map deterministic; it is not linear in r, so it serves inside
  FGMRES only.
* The velocity block's approximate inverse is one V-cycle (Section 4); k V-cycles of
  a stationary iteration from zero are an option (velocity_cycles).
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

    def velocity_cycles(self, k: int) -> Callable:
        """A~^-1 as k V-cycles of a stationary iteration from zero: x = V r, then
        x += V (r - A x) (k = 1: the single V-cycle of Section 4)."""
        H = self.H

        def a_inv(ru):
            x = mg.vcycle(H, ru)
            for _ in range(k - 1):
                x = x + mg.vcycle(H, ru - self.A @ x)
            return x
        return a_inv

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

    def z_hierarchy(self, omega: float = 2.0 / 3.0, sweeps: int = 2) -> "ZHierarchy":
        return ZHierarchy(self, omega, sweeps)

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
              schur_iters: int = 20, velocity_cycles: int = 1) -> mg.SolveResult:
        a_inv = self.velocity_cycles(velocity_cycles) if velocity_cycles > 1 else None
        if schur == "mass":
            M = self.precond(precond, a_inv=a_inv)
        elif schur in ("bfbt", "bfbt_mg"):
            if solver != "fgmres":
                raise ValueError("the BFBT approximation is not a fixed linear map: FGMRES only")
            zs = self.z_hierarchy().z_solve(schur_iters) if schur == "bfbt_mg" else None
            M = self.precond(precond, a_inv=a_inv, s_inv=self.bfbt(schur_iters, z_solve=zs))
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


# Offsets of the pressure-space stencils of Z: every coupling of Z = B W^-1 B^T goes
# through a velocity node j that both pressure hats' supports reach, and B couples a
# pressure node k with the fine nodes within one Kuhn edge of the fine node 2k, so
# Z couples k with k + o for o a sum of two Kuhn-lattice edges (offsets in {0,1}^3 or
# {0,-1}^3): the 65 offsets in [-2,2]^3 with max(o, 0) - min(o, 0) <= 2.  Galerkin
# coarsening with the linear interpolation keeps that set.
Z_OFFSETS = [(dx, dy, dz) for dz in range(-2, 3) for dy in range(-2, 3) for dx in range(-2, 3)
             if max(dx, dy, dz, 0) - min(dx, dy, dz, 0) <= 2]


class ZHierarchy:
    """Geometric multigrid for the BFBT operator Z = B W^-1 B^T of eq. (4.2) (test
    infrastructure).  The paper solves with Z by an algebraic multigrid cycle inside
    CG; this is the geometric counterpart on the pressure lattice: levels L-1 (the
    pressure space, every node a dof) down to 0, linear interpolation P over all nodes
    (eq. (2.4), no boundary condition), Galerkin coarse operators Z_l = P^T Z_{l+1} P
    (the constant pressure stays in every Z_l's kernel), damped Jacobi V(sweeps,
    sweeps) with omega = 2/3 and zero initial guesses, and on level 0 (27 nodes) the
    solution of minimal norm, from the bordered system [[Z_0, 1], [1^T, 0]].  Z^-1 r
    (r of zero sum, as every B v is) is then approximated by `iters` steps of CG on
    Z y = r from y = 0 preconditioned by one V-cycle."""

    def __init__(self, S: StokesSystem, omega: float = 2.0 / 3.0, sweeps: int = 2):
        levels = S.H.levels
        Lp = S.H.L - 1
        self.levels = levels[:Lp + 1]
        self.omega, self.sweeps = omega, sweeps
        self.P = [transfer.prolongation(levels[l], levels[l + 1]) for l in range(Lp)]
        Z = [None] * (Lp + 1)
        Z[Lp] = S.z_operator()
        for l in range(Lp - 1, -1, -1):
            Z[l] = (self.P[l].T @ Z[l + 1] @ self.P[l]).tocsr()
        self.Z = Z
        self.D = [z.diagonal().copy() for z in Z]
        Z0 = Z[0].toarray()
        n0 = Z0.shape[0]
        Bord = np.zeros((n0 + 1, n0 + 1))
        Bord[:n0, :n0] = Z0
        Bord[:n0, n0] = 1.0
        Bord[n0, :n0] = 1.0
        self.coarse_inv = np.linalg.inv(Bord)[:n0, :n0]

    @property
    def top(self) -> int:
        return len(self.Z) - 1

    def vcycle(self, r: np.ndarray, l: int = None) -> np.ndarray:
        if l is None:
            l = self.top
        if l == 0:
            return self.coarse_inv @ r
        Z, D = self.Z[l], self.D[l]
        y = np.zeros_like(r)
        for _ in range(self.sweeps):
            y = y + self.omega * (r - Z @ y) / D
        rc = self.P[l - 1].T @ (r - Z @ y)
        y = y + self.P[l - 1] @ self.vcycle(rc, l - 1)
        for _ in range(self.sweeps):
            y = y + self.omega * (r - Z @ y) / D
        return y

    def z_solve(self, iters: int) -> Callable:
        """r -> `iters` steps of V-cycle-preconditioned CG on Z y = r from y = 0 (a step
        whose direction has zero Z-energy has step size zero)."""
        Z = self.Z[self.top]

        def solve(r):
            y = np.zeros_like(r)
            res = r.copy()
            z = self.vcycle(res)
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
                z = self.vcycle(res)
                rz_new = res @ z
                p = z + (rz_new / rz if rz != 0.0 else 0.0) * p
                rz = rz_new
            return y
        return solve

    def stencil(self, l: int) -> np.ndarray:
        """(65, nodes) entries of Z_l by offset (Z_OFFSETS order) and node: the row of
        node k at column k + o, 0 where k + o lies outside the lattice."""
        n = self.levels[l].n
        n1 = n + 1
        N = n1 ** 3
        Zc = self.Z[l].tocoo()
        r, c = Zc.row, Zc.col
        o = np.stack([c % n1 - r % n1, (c // n1) % n1 - (r // n1) % n1, c // (n1 * n1) - r // (n1 * n1)], 1)
        idx = {off: i for i, off in enumerate(Z_OFFSETS)}
        out = np.zeros((len(Z_OFFSETS), N))
        for (ox, oy, oz), row, v in zip(o, r, Zc.data):
            key = (int(ox), int(oy), int(oz))
            if key not in idx:
                if abs(v) > 0:
                    raise ValueError(f"Z couples offset {key}, outside the stencil")
                continue
            out[idx[key], row] += v
        return out


def stencil_apply(st: np.ndarray, n: int, x: np.ndarray) -> np.ndarray:
    """y_k = sum over the 65 offsets o of st[o, k] x_{k+o}, on the (n+1)^3 lattice (terms
    whose k + o leaves the lattice are dropped: their entries are zero)."""
    n1 = n + 1
    X = x.reshape(n1, n1, n1)                       # [z, y, x]
    y = np.zeros((n1, n1, n1))
    for i, (dx, dy, dz) in enumerate(Z_OFFSETS):
        S = st[i].reshape(n1, n1, n1)
        src = X[max(dz, 0):n1 + min(dz, 0), max(dy, 0):n1 + min(dy, 0), max(dx, 0):n1 + min(dx, 0)]
        y[max(-dz, 0):n1 + min(-dz, 0), max(-dy, 0):n1 + min(-dy, 0), max(-dx, 0):n1 + min(-dx, 0)] += \
            S[max(-dz, 0):n1 + min(-dz, 0), max(-dy, 0):n1 + min(-dy, 0), max(-dx, 0):n1 + min(-dx, 0)] * src
    return y.reshape(-1)
