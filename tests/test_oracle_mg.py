"""Pins of the oracle's V-cycle and Krylov solvers (paper Section 4, eq. (4.3)).

Independent facts: the V-cycle's error propagation equals the textbook product
S^nu2 (I - P A_c^-1 P^T A) S^nu1 with S = I - omega D^-1 A (recursively for the
coarse solve); for the Galerkin coarse operator, the coarse-grid correction is
an A-orthogonal projection; the V-cycle with symmetric pre/post smoothing is a
symmetric operator; every solver converges to the sparse direct solution.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import agca, fem, mesh, mg
from workloads import AlignedCube, Sinkers


def _sinker_levels(L, ncomp, seed=2):
    levels = mesh.hierarchy(L)
    field = Sinkers(3, seed, radius=0.2, width=2.0 / 2 ** (L + 1), contrast=1e4)
    nu_levels = [field.nu(mesh.centroids_canonical(lv)) for lv in levels]
    return levels, nu_levels, field


@pytest.fixture(scope="module")
def scalar_h():
    levels, nu_levels, field = _sinker_levels(3, 1)
    return mg.build(3, nu_levels, 1, levels=levels), levels, field


def _vcycle_matrix(H, l):
    n = H.A[l].shape[0]
    return np.stack([mg.vcycle(H, e, l) for e in np.eye(n)], axis=1)


def test_vcycle_error_propagation_formula(scalar_h):
    H, _, _ = scalar_h
    # two coarsest levels are small enough for dense matrices
    for l in (1, 2):
        A = H.A[l].toarray()
        n = A.shape[0]
        S = np.eye(n) - H.omega * A / H.D[l][:, None]
        P = H.P[l - 1].toarray()
        Bc = np.linalg.inv(H.A[0].toarray()) if l == 1 else _vcycle_matrix(H, l - 1)
        E_ref = (np.linalg.matrix_power(S, H.nu2) @ (np.eye(n) - P @ Bc @ P.T @ A)
                 @ np.linalg.matrix_power(S, H.nu1))
        B = _vcycle_matrix(H, l)
        E = np.eye(n) - B @ A
        assert np.abs(E - E_ref).max() < 1e-10
        assert np.abs(B - B.T).max() < 1e-10 * np.abs(B).max()   # symmetric preconditioner


def test_galerkin_coarse_correction_is_projection():
    levels, nu_levels, _ = _sinker_levels(2, 1)
    H = mg.build(2, nu_levels, 1, mode=agca.FLAG_ALL, levels=levels)
    A = H.A[2].toarray()
    P = H.P[1].toarray()
    Ac = H.A[1].toarray()
    assert np.abs(Ac - P.T @ A @ P).max() < 1e-12 * np.abs(Ac).max()
    T = np.eye(A.shape[0]) - P @ np.linalg.solve(Ac, P.T @ A)
    assert np.abs(T @ T - T).max() < 1e-9
    assert np.abs(A @ T - (A @ T).T).max() < 1e-9 * np.abs(A).max()


def _exact(H, b):
    return spla.splu(H.A[H.L].tocsc()).solve(b)


def test_stationary_cube17_converges_to_direct_solution():
    levels = mesh.hierarchy(3)
    field = AlignedCube()
    nu_levels = [field.nu(mesh.centroids_canonical(lv)) for lv in levels]
    H = mg.build(3, nu_levels, 1, levels=levels)
    b = fem.load_vector(levels[3], np.ones(levels[3].tets.shape[0]), 1)[H.free[3]]
    # stationary V(2,2) converges, slowly: Galerkin coarse operators with linear
    # interpolation are A-orthogonal projections, but the jump is not aligned with
    # levels 0 and 1 (mesh widths 1/2 and 1/4), so a few error modes are poorly
    # represented there; CG acceleration removes them.
    res = mg.stationary(H, b, 1e-10, maxit=3000)
    assert res.converged, res.history[-1]
    xs = _exact(H, b)
    assert np.abs(res.x - xs).max() <= 1e-8 * np.abs(xs).max()
    res = mg.pcg(H.A[3], b, lambda r: mg.vcycle(H, r), 1e-10)
    assert res.converged and res.iterations < 25
    assert np.abs(res.x - xs).max() <= 1e-8 * np.abs(xs).max()
    # on level 2 (mesh width 1/8) the jump is grid-aligned: nothing is flagged and
    # AGCA equals DCA there (Section 4.2, eta_1); levels 0 and 1 differ
    Hd = mg.build(3, nu_levels, 1, mode=agca.FLAG_NONE, levels=levels)
    assert not H.flags[2].any()
    assert abs(Hd.A[2] - H.A[2]).max() <= 1e-12 * abs(H.A[2]).max()


@pytest.mark.parametrize("solver", ["pcg", "fcg", "ir", "fgmres", "minres"])
def test_krylov_solvers_reach_direct_solution(scalar_h, solver):
    H, levels, field = scalar_h
    b = fem.load_vector(levels[3], field.force(mesh.centroids_canonical(levels[3]), 1), 1)[H.free[3]]
    A = H.A[3]
    M = lambda r: mg.vcycle(H, r)
    fn = {"pcg": mg.pcg, "fcg": mg.fcg, "ir": mg.iterative_refinement,
          "fgmres": mg.fgmres, "minres": mg.minres}[solver]
    res = fn(A, b, M, 1e-11)
    assert res.converged
    xs = _exact(H, b)
    assert np.linalg.norm(res.x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert np.linalg.norm(b - A @ res.x) <= 1e-11 * np.linalg.norm(b) * 1.0001


def test_pcg_matches_scipy_cg_iteration_count(scalar_h):
    H, levels, field = scalar_h
    b = fem.load_vector(levels[3], field.force(mesh.centroids_canonical(levels[3]), 1), 1)[H.free[3]]
    M = lambda r: mg.vcycle(H, r)
    res = mg.pcg(H.A[3], b, M, 1e-10)
    it = [0]

    def cb(xk):
        it[0] += 1

    Mop = spla.LinearOperator(H.A[3].shape, matvec=M)
    spla.cg(H.A[3], b, rtol=1e-10, atol=0.0, M=Mop, callback=cb, maxiter=500)
    assert abs(it[0] - res.iterations) <= 1


def test_agca_beats_dca_on_unaligned_jump():
    """Section 4.2: with an unaligned jump, AGCA needs no more iterations than DCA."""
    levels = mesh.hierarchy(3)
    from workloads import AlignedCube as Box
    cube = Box(lo=11 / 24 - 1 / 8, hi=11 / 24 + 1 / 8, nu_in=1e3, nu_out=1e-3)
    nu_levels = [cube.nu(mesh.centroids_canonical(lv)) for lv in levels]
    iters = {}
    for mode in (agca.FLAG_RATIO, agca.FLAG_NONE):
        H = mg.build(3, nu_levels, 1, mode=mode, levels=levels)
        b = fem.load_vector(levels[3], np.ones(levels[3].tets.shape[0]), 1)[H.free[3]]
        iters[mode] = mg.pcg(H.A[3], b, lambda r: mg.vcycle(H, r), 1e-8).iterations
    assert iters[agca.FLAG_RATIO] <= iters[agca.FLAG_NONE]


def test_vector_pcg_converges():
    levels, nu_levels, field = _sinker_levels(2, 3)
    H = mg.build(2, nu_levels, 3, levels=levels)
    b = fem.load_vector(levels[2], field.force(mesh.centroids_canonical(levels[2]), 3), 3)[H.free[2]]
    res = mg.pcg(H.A[2], b, lambda r: mg.vcycle(H, r), 1e-10)
    assert res.converged
    xs = _exact(H, b)
    assert np.linalg.norm(res.x - xs) <= 1e-7 * np.linalg.norm(xs)


def test_minres_iterates_minimise_the_preconditioned_residual():
    """Each MINRES iterate is the minimiser of the M-norm of b - A x over the
    preconditioned Krylov space span{M b, (M A) M b, ...} (Paige and Saunders 1975),
    here found by brute force: an orthonormal (Arnoldi) basis of the space and a
    dense least-squares solve, on a small symmetric indefinite system."""
    rng = np.random.default_rng(3)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.concatenate([rng.uniform(1, 10, 25), -rng.uniform(0.5, 4, 15)])
    A = (Q * ev) @ Q.T
    C = np.tril(rng.standard_normal((n, n)) * 0.2) + np.eye(n)
    Mmat = C @ C.T
    b = rng.standard_normal(n)
    for k in (1, 2, 5, 9, 14):
        res = mg.minres(A, b, lambda r: Mmat @ r, tol=0.0, maxit=k)
        assert res.iterations == k
        # orthonormal basis by Arnoldi (each new vector M A v orthogonalised twice)
        basis = np.empty((n, k))
        v = Mmat @ b
        for j in range(k):
            for _ in range(2):
                v = v - basis[:, :j] @ (basis[:, :j].T @ v)
            basis[:, j] = v / np.linalg.norm(v)
            v = Mmat @ (A @ basis[:, j])
        # ||b - A x||_M with ||r||_M^2 = r . M r = ||C^T r||^2
        y = np.linalg.lstsq(C.T @ A @ basis, C.T @ b, rcond=None)[0]
        x_ref = basis @ y
        assert np.linalg.norm(res.x - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
