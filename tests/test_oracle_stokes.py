"""Pins of the oracle's Stokes pieces (paper Section 3.1): divergence B, lumped 1/nu
pressure mass, and the block-preconditioned FGMRES / MINRES solves.

B and m are checked against quantities fixed by calculus and by an independent
quadrature: B^T 1 = 0 on free velocities (divergence theorem), B u = -c int psi_k
for a linear field with constant divergence c, brute-force Gauss quadrature of
psi_k div Phi_j with psi_k located point by point in the coarse mesh, and
m_k = int psi_k for nu = 1.  The Krylov solutions must equal the bordered direct
solve.
"""

import numpy as np
import pytest

from oracle import fem, mesh, mg, stokes

# 4-point Gauss rule on the reference tetrahedron, exact for degree 2
_A, _B = 0.5854101966249685, 0.1381966011250105
_GP = np.array([[_A, _B, _B, _B], [_B, _A, _B, _B], [_B, _B, _A, _B], [_B, _B, _B, _A]])


def _hat_integrals(lv):
    """int psi_k over the domain: sum over elements containing k of |e| / 4."""
    _, vol = fem.element_geometry(lv.coords[lv.tets])
    out = np.zeros((lv.n + 1) ** 3)
    np.add.at(out, lv.node_id[lv.tets].ravel(), np.repeat(vol / 4.0, 4))
    return out


def test_divergence_theorem_and_linear_fields():
    levels = mesh.hierarchy(3)
    c, f = levels[2], levels[3]
    B = stokes.div_matrix(c, f)
    nn = (f.n + 1) ** 3
    free = fem.free_dofs(f, 3)
    ones = np.ones(B.shape[0])
    bt1 = (B.T @ ones)[free]
    assert np.abs(bt1).max() <= 1e-15 * np.abs(B).max() * 10
    X = np.zeros((nn, 3))
    X[f.node_id] = f.coords
    hat = _hat_integrals(c)
    for coef, div in (((1, 0, 0), 1.0), ((1, 2, 3), 6.0), ((0, -1, 0), -1.0)):
        u = np.concatenate([coef[k] * X[:, k] for k in range(3)])
        assert np.allclose(B @ u, -div * hat, rtol=0, atol=1e-14)


def test_divergence_brute_force_quadrature():
    levels = mesh.hierarchy(1)
    c, f = levels[0], levels[1]
    B = stokes.div_matrix(c, f).toarray()
    nn_c, nn_f = (c.n + 1) ** 3, (f.n + 1) ** 3
    ref = np.zeros((nn_c, 3 * nn_f))
    C4 = c.coords[c.tets]
    Minv = np.linalg.inv(np.concatenate([np.ones((C4.shape[0], 1, 4)), C4.transpose(0, 2, 1)], axis=1))
    g, vol = fem.element_geometry(f.coords[f.tets])
    for t in range(f.tets.shape[0]):
        x4 = f.coords[f.tets[t]]
        for q in range(4):
            xq = _GP[q] @ x4
            lam = Minv @ np.concatenate([[1.0], xq])            # coarse barycentrics, all tets
            tc = np.nonzero(np.all(lam > -1e-12, axis=1))[0][0]
            psi = np.zeros(nn_c)
            psi[c.node_id[c.tets[tc]]] = lam[tc]
            for b in range(4):
                for k in range(3):
                    ref[:, k * nn_f + f.node_id[f.tets[t, b]]] -= vol[t] / 4.0 * psi * g[t, b, k]
    assert np.abs(B - ref).max() <= 1e-14 * np.abs(ref).max()


def test_lumped_mass():
    levels = mesh.hierarchy(3)
    c, f = levels[2], levels[3]
    m1 = stokes.lumped_mass(c, f, np.ones(f.tets.shape[0]))
    assert np.allclose(m1, _hat_integrals(c), rtol=1e-13, atol=0)
    rng = np.random.default_rng(0)
    nu = np.exp(rng.uniform(-5, 5, f.tets.shape[0]))
    m = stokes.lumped_mass(c, f, nu)
    _, vol = fem.element_geometry(f.coords[f.tets])
    assert abs(m.sum() - (vol / nu[f.elem_id]).sum()) <= 1e-13 * m.sum()
    assert np.all(m > 0)


@pytest.mark.parametrize("solver", ["fgmres", "minres"])
def test_krylov_solutions_equal_direct(solver):
    from workloads import Sinkers
    L = 2
    levels = mesh.hierarchy(L)
    field = Sinkers(2, 3, radius=0.2, width=2.0 / 2 ** (L + 1), contrast=1e4)
    nu = [field.nu(mesh.centroids_canonical(lv)) for lv in levels]
    H = mg.build(L, nu, 3, levels=levels)
    S = stokes.StokesSystem(H)
    f = np.asarray(field.force(mesh.centroids_canonical(levels[L]), 3))
    bu = fem.load_vector(levels[L], f, 3)[H.free[L]]
    b = np.concatenate([bu, np.zeros(S.np_)])
    x_ref = S.direct(b)
    assert np.linalg.norm(S.K @ x_ref - b) <= 1e-10 * np.linalg.norm(b)
    assert np.abs(x_ref[S.nu_:].mean()) <= 1e-14 * np.abs(x_ref[S.nu_:]).max()
    res = S.solve(b, solver, tol=1e-10, restart=30, maxit=2000)
    assert res.converged, (solver, res.iterations)
    assert np.linalg.norm(res.x - x_ref) <= 1e-6 * np.linalg.norm(x_ref)


def test_triangular_preconditioner_with_exact_blocks_takes_two_steps():
    # With A~ = A and S~ = B A^-1 B^T (pseudo-inverse: constants are its kernel) the
    # upper block-triangular preconditioner makes K Q^-1 = [[I, 0], [B A^-1, I]], whose
    # minimal polynomial is (z - 1)^2: GMRES ends after two steps.  The other sign of
    # the pressure block does not (three distinct eigenvalues).
    from workloads import Sinkers
    L = 2
    levels = mesh.hierarchy(L)
    field = Sinkers(2, 3, radius=0.2, width=2.0 / 2 ** (L + 1), contrast=1e2)
    nu = [field.nu(mesh.centroids_canonical(lv)) for lv in levels]
    H = mg.build(L, nu, 3, levels=levels)
    S = stokes.StokesSystem(H)
    A_inv = np.linalg.inv(S.A.toarray())
    B = S.B.toarray()
    S_pinv = np.linalg.pinv(B @ A_inv @ B.T)
    f = np.asarray(field.force(mesh.centroids_canonical(levels[L]), 3))
    rng = np.random.default_rng(0)
    g = rng.standard_normal(S.np_)
    g -= g.mean()
    for gp in (np.zeros(S.np_), g):
        b = np.concatenate([fem.load_vector(levels[L], f, 3)[H.free[L]], gp])
        M = S.precond("triangular", a_inv=lambda r: A_inv @ r, s_inv=lambda r: S_pinv @ r)
        res = mg.fgmres(S.K, b, M, 1e-10, restart=30, maxit=50)
        assert res.converged and res.iterations <= 2, res.iterations

    def wrong_sign(r):
        ru, rp = S.split(r)
        q = S_pinv @ rp
        return np.concatenate([A_inv @ (ru + B.T @ q), q])
    res = mg.fgmres(S.K, b, wrong_sign, 1e-10, restart=30, maxit=50)
    assert res.iterations > 2
    # with the V-cycle and the lumped mass the triangular form still beats the diagonal one
    b0 = np.concatenate([fem.load_vector(levels[L], f, 3)[H.free[L]], np.zeros(S.np_)])
    it_d = S.solve(b0, "fgmres", tol=1e-8, restart=30, maxit=2000, precond="diagonal").iterations
    it_t = S.solve(b0, "fgmres", tol=1e-8, restart=30, maxit=2000, precond="triangular").iterations
    assert it_t < it_d, (it_t, it_d)


def _sinker_system(L, contrast=1e4):
    from workloads import Sinkers
    levels = mesh.hierarchy(L)
    field = Sinkers(3, 3, radius=0.2, width=2.0 / 2 ** (L + 1), contrast=contrast)
    nu = [field.nu(mesh.centroids_canonical(lv)) for lv in levels]
    H = mg.build(L, nu, 3, levels=levels)
    S = stokes.StokesSystem(H)
    f = np.asarray(field.force(mesh.centroids_canonical(levels[L]), 3))
    b = np.concatenate([fem.load_vector(levels[L], f, 3)[H.free[L]], np.zeros(S.np_)])
    return S, b


def test_bfbt_is_the_exact_schur_inverse_when_a_is_diagonal():
    # with A = W = diag(A), eq. (4.2) gives Z^+ (B W^-1 W W^-1 B^T) Z^+ = Z^+ and the
    # Schur complement B A^-1 B^T is Z itself: BFBT is exact, and the block-triangular
    # preconditioner with exact blocks makes K Q^-1 unipotent (two GMRES steps)
    import scipy.sparse as sp
    S, b = _sinker_system(2)
    S.A = sp.diags(S.A.diagonal()).tocsr()
    S.K = sp.bmat([[S.A, S.B.T], [S.B, None]]).tocsr()
    Z = S.z_operator().toarray()
    Zp = np.linalg.pinv(Z)
    s_inv = S.bfbt(z_solve=lambda r: Zp @ r)
    rng = np.random.default_rng(1)
    r = rng.standard_normal(S.np_)
    assert np.allclose(s_inv(r), Zp @ r, rtol=0, atol=1e-10 * np.abs(Zp @ r).max())
    w = S.A.diagonal()
    M = S.precond("triangular", a_inv=lambda ru: ru / w, s_inv=s_inv)
    res = mg.fgmres(S.K, b, M, 1e-10, restart=10, maxit=10)
    assert res.converged and res.iterations <= 2, res.iterations


def test_z_solve_fixed_steps():
    S, _ = _sinker_system(2)
    Z = S.z_operator()
    rng = np.random.default_rng(2)
    r = rng.standard_normal(S.np_)
    r -= r.mean()                      # the range of Z: B^T 1 = 0, so Z 1 = 0
    # Jacobi-preconditioned CG on the 125 pressure nodes (condition number about 900 on
    # the range): 50 steps solve it to rounding (steps beyond convergence only add noise)
    y = S.z_solve(50, Z)(r)
    assert np.linalg.norm(Z @ y - r) <= 1e-8 * np.linalg.norm(r)
    # fewer steps reduce the residual, monotonically in the Z-energy of the error
    yp = np.linalg.pinv(Z.toarray()) @ r
    errs = []
    for k in (1, 4, 16):
        e = S.z_solve(k, Z)(r) - yp
        errs.append(float(e @ (Z @ e)))
    assert errs[0] > errs[1] > errs[2]
    # a zero right-hand side (the pressure part of FGMRES's first vector) gives zero
    assert np.array_equal(S.z_solve(5, Z)(np.zeros(S.np_)), np.zeros(S.np_))


def test_bfbt_beats_the_lumped_mass_at_high_contrast():
    # the reason eq. (4.2) is used: with sharp viscosity jumps the 1/nu lumped mass is a
    # poor Schur approximation; BFBT (with 20-step Z solves) needs far fewer iterations
    S, b = _sinker_system(3, contrast=1e6)
    its = {}
    for schur in ("mass", "bfbt"):
        res = S.solve(b, "fgmres", tol=1e-8, restart=50, maxit=2000, precond="triangular",
                      schur=schur, schur_iters=20)
        assert res.converged
        its[schur] = res.iterations
    print(its)
    assert its["bfbt"] < 0.5 * its["mass"], its


def test_velocity_cycles_stationary_iteration():
    # k V-cycles from zero: k = 1 is the V-cycle itself; many cycles converge to A^-1 r;
    # the k-cycle operator is symmetric (V symmetric), so MINRES may use it
    import scipy.sparse.linalg as spla
    S, b = _sinker_system(2)
    rng = np.random.default_rng(12)
    r = rng.standard_normal(S.nu_)
    assert np.array_equal(S.velocity_cycles(1)(r), mg.vcycle(S.H, r))
    x = spla.spsolve(S.A.tocsc(), r)
    e = [np.linalg.norm(S.velocity_cycles(k)(r) - x) for k in (1, 2, 4, 40)]
    assert e[0] > e[1] > e[2] and e[3] <= 1e-10 * np.linalg.norm(x)
    s = rng.standard_normal(S.nu_)
    V2 = S.velocity_cycles(2)
    assert abs(s @ V2(r) - r @ V2(s)) <= 1e-12 * abs(s @ V2(r))
    for solver, pc in (("fgmres", "triangular"), ("minres", "diagonal")):
        res = S.solve(b, solver, tol=1e-10, restart=30, maxit=500, precond=pc, velocity_cycles=2)
        one = S.solve(b, solver, tol=1e-10, restart=30, maxit=500, precond=pc)
        assert res.converged and res.iterations < one.iterations, (solver, res.iterations, one.iterations)
        xd = S.direct(b)
        assert np.linalg.norm(res.x - xd) <= 1e-6 * np.linalg.norm(xd)
