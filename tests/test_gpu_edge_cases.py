"""Degenerate and boundary cases of the GPU path through the C ABI: the smallest
hierarchy (L = 1: 5^3 nodes, one free node on level 0), a zero right-hand side, a
start at the exact solution, a zero iteration budget, a constant coefficient (no
flags; DCA equals Galerkin coarsening), a zero Stokes right-hand side (every
preconditioner, BFBT included), and BFBT on the smallest Stokes hierarchy.
"""

import numpy as np
import pytest
import torch

from oracle import agca, fem, mesh, mg

from gpu_helpers import interior_full, oracle_apply_full, rand_full, rel_err, vcycle_errors

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pair(L, ncomp, nu_fn, smoother="jacobi"):
    from paper_2511_13109_amd import Hierarchy
    levels = mesh.hierarchy(L)
    nu = [nu_fn(mesh.centroids_canonical(lv)) for lv in levels]
    H = mg.build(L, nu, ncomp, levels=levels, smoother=smoother)
    G = Hierarchy(L, ncomp, _dev(nu[L]), [_dev(v) for v in nu[:L]], smoother=smoother)
    return levels, H, G


def _sinker_nu(pts):
    from workloads import Sinkers
    return Sinkers(2, 7, radius=0.2, width=0.05, contrast=1e4).nu(pts)


@pytest.mark.parametrize("smoother", ["jacobi", "chebyshev"])
@pytest.mark.parametrize("ncomp", [1, 3])
def test_smallest_hierarchy(ncomp, smoother):
    print(f"\n[L=1 ncomp={ncomp} {smoother}]", flush=True)
    levels, H, G = _pair(1, ncomp, _sinker_nu, smoother)
    try:
        rng = np.random.default_rng(1)
        for l in (0, 1):
            u = rand_full(H, l, rng)
            assert rel_err(G.apply(l, _dev(u)).cpu().numpy(), oracle_apply_full(H, l, u)) <= 1e-12
        b = rand_full(H, 1, rng)
        z = G.vcycle(_dev(b)).cpu().numpy()
        e_gpu, e_orc, vtol = vcycle_errors(H, b, z)
        print(f"[vcycle] library {e_gpu:.2e}, oracle FP64 {e_orc:.2e} (tolerance {vtol:.1e})", flush=True)
        assert e_gpu < vtol
        x, st = G.solve(_dev(b), solver="pcg", tol=1e-10, max_iter=200)
        ref = mg.pcg(H.A[1], b[H.free[1]], lambda r: mg.vcycle(H, r), 1e-10, maxit=200)
        assert st["converged"] and abs(st["iterations"] - ref.iterations) <= 1
    finally:
        G.close()


def test_zero_rhs_exact_start_and_zero_budget():
    levels, H, G = _pair(3, 3, _sinker_nu)
    try:
        nn = (levels[3].n + 1) ** 3
        zero = torch.zeros(3 * nn, dtype=torch.float64, device="cuda")
        x, st = G.solve(zero, solver="pcg", tol=1e-8)
        assert st["converged"] and st["iterations"] == 0 and float(x.abs().max()) == 0.0
        # start at (an FP64 rounding of) the exact solution: already converged
        rng = np.random.default_rng(2)
        b = rand_full(H, 3, rng)
        xs = np.zeros_like(b)
        import scipy.sparse.linalg as spla
        xs[H.free[3]] = spla.spsolve(H.A[3].tocsc(), b[H.free[3]])
        x0 = _dev(xs)
        x, st = G.solve(_dev(b), x=x0, solver="pcg", tol=1e-8)
        assert st["converged"] and st["iterations"] == 0
        # no iterations allowed: not converged, reported without raising
        x, st = G.solve(_dev(b), solver="pcg", tol=1e-8, max_iter=0, raise_on_noconv=False)
        assert not st["converged"] and st["iterations"] == 0
        assert abs(st["rel_residual"] - 1.0) <= 1e-12
    finally:
        G.close()


def test_constant_coefficient_has_no_flags_and_dca_equals_gca():
    from paper_2511_13109_amd import Hierarchy
    L = 3
    levels = mesh.hierarchy(L)
    nu = [np.full(lv.tets.shape[0], 2.5) for lv in levels]
    G = Hierarchy(L, 3, _dev(nu[L]), [_dev(v) for v in nu[:L]])
    Gg = Hierarchy(L, 3, _dev(nu[L]), [_dev(v) for v in nu[:L]], flag_mode="all")
    try:
        rng = np.random.default_rng(3)
        for l in range(L):
            assert G.query(l)["flagged"] == 0
            n = levels[l].n
            u = _dev(rng.standard_normal(3 * (n + 1) ** 3))
            a, g = G.apply(l, u).cpu().numpy(), Gg.apply(l, u).cpu().numpy()
            assert rel_err(a, g) <= 1e-12, l
    finally:
        G.close()
        Gg.close()


def test_stokes_zero_rhs():
    from paper_2511_13109_amd import Hierarchy, Stokes
    L = 2
    levels = mesh.hierarchy(L)
    nu = [_dev(_sinker_nu(mesh.centroids_canonical(lv))) for lv in levels]
    G = Hierarchy(L, 3, nu[L], nu[:L])
    try:
        S = Stokes(G)
        f = torch.zeros(3 * (levels[L].n + 1) ** 3, dtype=torch.float64, device="cuda")
        for solver, pc, schur in (("fgmres", "diagonal", "mass"), ("fgmres", "triangular", "mass"),
                                  ("minres", "diagonal", "mass"), ("fgmres", "triangular", "bfbt")):
            u, p, st = S.solve(f, solver=solver, precond=pc, tol=1e-8, schur=schur)
            assert st["converged"] and st["iterations"] == 0
            assert float(u.abs().max()) == 0.0 and float(p.abs().max()) == 0.0
    finally:
        G.close()


def test_stokes_smallest_hierarchy_bfbt():
    # L = 2 (the smallest Stokes hierarchy: 9^3 velocity, 5^3 pressure nodes), BFBT with
    # one and with 20 CG steps per Z solve, against the oracle's FGMRES
    from oracle import stokes
    from paper_2511_13109_amd import Hierarchy, Stokes
    L = 2
    levels = mesh.hierarchy(L)
    nu_h = [_sinker_nu(mesh.centroids_canonical(lv)) for lv in levels]
    H = mg.build(L, nu_h, 3, levels=levels)
    S = stokes.StokesSystem(H)
    from workloads import Sinkers
    f = np.asarray(Sinkers(2, 7, radius=0.2, width=0.05, contrast=1e4).force(
        mesh.centroids_canonical(levels[L]), 3))
    fu = fem.load_vector(levels[L], f, 3)
    b = np.concatenate([fu[H.free[L]], np.zeros(S.np_)])
    G = Hierarchy(L, 3, _dev(nu_h[L]), [_dev(v) for v in nu_h[:L]])
    try:
        for k in (1, 20):
            u, p, st = Stokes(G).solve(_dev(fu), solver="fgmres", restart=20, tol=1e-10,
                                       max_iter=500, precond="triangular", schur="bfbt",
                                       schur_iters=k)
            ref = S.solve(b, "fgmres", tol=1e-10, restart=20, maxit=500, precond="triangular",
                          schur="bfbt", schur_iters=k)
            assert st["converged"] and ref.converged
            n = min(len(st["history"]), len(ref.history), 15)
            assert np.allclose(st["history"][:n], ref.history[:n], rtol=1e-6, atol=1e-14), k
            assert abs(st["iterations"] - ref.iterations) <= 1, (k, st["iterations"], ref.iterations)
            xg = np.concatenate([u.cpu().numpy()[H.free[L]], p.cpu().numpy()])
            assert np.linalg.norm(b - S.K @ xg) <= 1.0001e-10 * np.linalg.norm(b)
    finally:
        G.close()
