"""GPU parity of the Stokes pieces (Section 3.1) against the oracle, through the C ABI:
divergence B, B^T, the lumped 1/nu pressure mass (1e-12 relative), and the
block-preconditioned FGMRES / MINRES solves (iteration counts within one of the
oracle's, residual histories, solutions against the bordered direct solve), both
solvers around the FP32 V-cycle (residual recomputed by the oracle), and FGMRES with its
Arnoldi basis stored in FP32.
"""

import numpy as np
import pytest
import torch

from oracle import fem, mesh, mg, stokes
from workloads import Sinkers

pytestmark = pytest.mark.gpu

CASES = [3, 4]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module", params=CASES, ids=lambda L: f"L{L}")
def case(request):
    from paper_2511_13109_amd import Hierarchy, Stokes
    L = request.param
    print(f"\n[stokes case L={L}]", flush=True)
    levels = mesh.hierarchy(L)
    field = Sinkers(2, 3, radius=0.2, width=2.0 / 2 ** (L + 1), contrast=1e2)
    nu = [field.nu(mesh.centroids_canonical(lv)) for lv in levels]
    H = mg.build(L, nu, 3, levels=levels)
    S = stokes.StokesSystem(H)
    f = np.asarray(field.force(mesh.centroids_canonical(levels[L]), 3))
    fu = fem.load_vector(levels[L], f, 3)
    G = Hierarchy(L, 3, _dev(nu[L]), [_dev(v) for v in nu[:L]])
    G32 = Hierarchy(L, 3, _dev(nu[L]), [_dev(v) for v in nu[:L]], mg_dtype="f32", mg_nu_dtype="f32")
    yield L, levels, H, S, fu, Stokes(G), Stokes(G32)
    G.close()
    G32.close()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_div_grad_mass(case):
    L, levels, H, S, fu, GS, _ = case
    rng = np.random.default_rng(0)
    nn = (levels[L].n + 1) ** 3
    u = rng.standard_normal(3 * nn)
    u_in = u.copy()
    u_in[np.setdiff1d(np.arange(3 * nn), H.free[L])] = 7.0     # boundary input is ignored
    q = GS.div(_dev(u_in)).cpu().numpy()
    Bfull = stokes.div_matrix(levels[L - 1], levels[L])
    uz = np.zeros(3 * nn)
    uz[H.free[L]] = u[H.free[L]]
    assert _rel(q, Bfull @ uz) <= 1e-12
    p = rng.standard_normal(S.np_)
    v = GS.grad(_dev(p)).cpu().numpy()
    ref = np.zeros(3 * nn)
    ref[H.free[L]] = S.B.T @ p
    assert _rel(v, ref) <= 1e-12
    m = GS.mass().cpu().numpy()
    assert _rel(m, S.m) <= 1e-12


@pytest.mark.parametrize("solver", ["fgmres", "minres"])
def test_solve_fp64_matches_oracle(case, solver):
    L, levels, H, S, fu, GS, _ = case
    nn = (levels[L].n + 1) ** 3
    b = np.concatenate([fu[H.free[L]], np.zeros(S.np_)])
    tol = 1e-9
    print(f"[{solver} L={L}] oracle solve", flush=True)
    ref = S.solve(b, solver, tol=tol, restart=30, maxit=3000)
    assert ref.converged
    u, p, st = GS.solve(_dev(fu), solver=solver, restart=30, tol=tol, max_iter=3000)
    print(f"[{solver} L={L}] gpu {st['iterations']} it, oracle {ref.iterations} it, "
          f"rel {st['rel_residual']:.2e}", flush=True)
    assert st["converged"] and st["rel_residual"] <= tol
    k = min(len(st["history"]), len(ref.history), 20)
    assert np.allclose(st["history"][:k], ref.history[:k], rtol=1e-6, atol=1e-14)
    # Hundreds of iterations of restarted FGMRES (whose progress stalls between
    # restarts) or of MINRES (whose 2-norm residual, used by the stopping test,
    # oscillates) amplify differences in the order of additions, so the crossing of
    # the tolerance may move by a few per cent; the history prefix above pins the
    # arithmetic of every step.
    assert abs(st["iterations"] - ref.iterations) <= max(1, int(0.05 * ref.iterations))
    # against the exact solution (sparse LU of the saddle-point matrix, affordable at
    # 17^3 velocity nodes) or else against the oracle's own Krylov solution
    x_ref = S.direct(b) if L <= 3 else ref.x
    xg = np.concatenate([u.cpu().numpy()[H.free[L]], p.cpu().numpy()])
    assert np.linalg.norm(xg - x_ref) <= 1e-5 * np.linalg.norm(x_ref)
    assert abs(p.cpu().numpy().mean()) <= 1e-12 * np.abs(p.cpu().numpy()).max()


@pytest.mark.parametrize("solver", ["fgmres", "minres"])
def test_solve_mixed_precision(case, solver):
    L, levels, H, S, fu, _, GS32 = case
    b = np.concatenate([fu[H.free[L]], np.zeros(S.np_)])
    u, p, st = GS32.solve(_dev(fu), solver=solver, restart=30, tol=1e-8, max_iter=3000)
    print(f"[{solver} FP32 V-cycle L={L}] {st['iterations']} it", flush=True)
    assert st["converged"] and st["rel_residual"] <= 1e-8
    xg = np.concatenate([u.cpu().numpy()[H.free[L]], p.cpu().numpy()])
    # residual recomputed by the oracle (FP64, assembled K)
    assert np.linalg.norm(b - S.K @ xg) <= 1.0001e-8 * np.linalg.norm(b)


@pytest.mark.parametrize("mg_dtype", ["f64", "f32"])
def test_triangular_preconditioner(case, mg_dtype):
    L, levels, H, S, fu, GS, GS32 = case
    G = GS if mg_dtype == "f64" else GS32
    b = np.concatenate([fu[H.free[L]], np.zeros(S.np_)])
    tol = 1e-9 if mg_dtype == "f64" else 1e-8
    u, p, st = G.solve(_dev(fu), solver="fgmres", restart=30, tol=tol, max_iter=3000,
                       precond="triangular")
    print(f"[fgmres triangular {mg_dtype} L={L}] {st['iterations']} it", flush=True)
    assert st["converged"] and st["rel_residual"] <= tol
    xg = np.concatenate([u.cpu().numpy()[H.free[L]], p.cpu().numpy()])
    assert np.linalg.norm(b - S.K @ xg) <= 1.0001 * tol * np.linalg.norm(b)
    if mg_dtype == "f64":
        ref = S.solve(b, "fgmres", tol=tol, restart=30, maxit=3000, precond="triangular")
        assert ref.converged
        k = min(len(st["history"]), len(ref.history), 20)
        assert np.allclose(st["history"][:k], ref.history[:k], rtol=1e-6, atol=1e-14)
        assert abs(st["iterations"] - ref.iterations) <= max(1, int(0.05 * ref.iterations))
        _, _, sd = G.solve(_dev(fu), solver="fgmres", restart=30, tol=tol, max_iter=3000)
        assert st["iterations"] < sd["iterations"]
    with pytest.raises(Exception):
        G.solve(_dev(fu), solver="minres", tol=tol, precond="triangular")


@pytest.mark.parametrize("mg_dtype", ["f64", "f32"])
def test_bfbt_schur_approximation(case, mg_dtype):
    # eq. (4.2) with 20-step Jacobi-CG Z solves, in both preconditioners: FP64 V-cycle
    # against the oracle's FGMRES (history prefix, iteration count), FP32 V-cycle by its
    # residual recomputed by the oracle
    L, levels, H, S, fu, GS, GS32 = case
    G = GS if mg_dtype == "f64" else GS32
    b = np.concatenate([fu[H.free[L]], np.zeros(S.np_)])
    tol = 1e-9 if mg_dtype == "f64" else 1e-8
    for precond in ("triangular", "diagonal"):
        u, p, st = G.solve(_dev(fu), solver="fgmres", restart=30, tol=tol, max_iter=3000,
                           precond=precond, schur="bfbt", schur_iters=20)
        print(f"[fgmres {precond} BFBT {mg_dtype} L={L}] {st['iterations']} it", flush=True)
        assert st["converged"] and st["rel_residual"] <= tol
        xg = np.concatenate([u.cpu().numpy()[H.free[L]], p.cpu().numpy()])
        assert np.linalg.norm(b - S.K @ xg) <= 1.0001 * tol * np.linalg.norm(b)
        if mg_dtype == "f64":
            ref = S.solve(b, "fgmres", tol=tol, restart=30, maxit=3000, precond=precond,
                          schur="bfbt", schur_iters=20)
            assert ref.converged
            k = min(len(st["history"]), len(ref.history), 20)
            assert np.allclose(st["history"][:k], ref.history[:k], rtol=1e-6, atol=1e-14)
            assert abs(st["iterations"] - ref.iterations) <= max(1, int(0.05 * ref.iterations))
    if mg_dtype == "f64":
        _, _, sm = G.solve(_dev(fu), solver="fgmres", restart=30, tol=tol, max_iter=3000,
                           precond="triangular")
        print(f"[fgmres triangular mass L={L}] {sm['iterations']} it", flush=True)
    with pytest.raises(Exception):
        G.solve(_dev(fu), solver="minres", tol=tol, schur="bfbt")
    with pytest.raises(Exception):
        G.solve(_dev(fu), solver="fgmres", tol=tol, schur="bfbt", schur_iters=0)


@pytest.mark.parametrize("solver,precond", [("fgmres", "triangular"), ("minres", "diagonal")])
def test_velocity_cycles_match_oracle(case, solver, precond):
    # two V-cycles per application of the velocity block's approximate inverse (a
    # stationary iteration from zero): FP64 V-cycle against the oracle (history prefix,
    # iteration counts), fewer iterations than with one cycle
    L, levels, H, S, fu, GS, _ = case
    b = np.concatenate([fu[H.free[L]], np.zeros(S.np_)])
    tol = 1e-9
    u, p, st = GS.solve(_dev(fu), solver=solver, restart=30, tol=tol, max_iter=3000, precond=precond,
                        velocity_cycles=2)
    ref = S.solve(b, solver, tol=tol, restart=30, maxit=3000, precond=precond, velocity_cycles=2)
    _, _, one = GS.solve(_dev(fu), solver=solver, restart=30, tol=tol, max_iter=3000, precond=precond)
    print(f"[{solver} {precond} 2 V-cycles L={L}] gpu {st['iterations']} it, oracle {ref.iterations} it, "
          f"one cycle {one['iterations']} it", flush=True)
    assert st["converged"] and ref.converged
    k = min(len(st["history"]), len(ref.history), 20)
    assert np.allclose(st["history"][:k], ref.history[:k], rtol=1e-6, atol=1e-14)
    assert abs(st["iterations"] - ref.iterations) <= max(1, int(0.05 * ref.iterations))
    assert st["iterations"] < one["iterations"]
    xg = np.concatenate([u.cpu().numpy()[H.free[L]], p.cpu().numpy()])
    assert np.linalg.norm(b - S.K @ xg) <= 1.0001 * tol * np.linalg.norm(b)
    with pytest.raises(Exception):
        GS.solve(_dev(fu), solver=solver, tol=tol, precond=precond, velocity_cycles=9)


@pytest.mark.parametrize("precond,schur", [("triangular", "mass"), ("diagonal", "mass"),
                                           ("triangular", "bfbt_mg")])
def test_fgmres_fp32_basis(case, precond, schur):
    # The Arnoldi basis stored in FP32 (FP64 dot products, preconditioned vectors and
    # iterate).  Within one restart cycle the basis's rounding (about 6e-8 relative) bounds
    # how far the cycle can take the residual, so down to 1e-6 the solve follows the FP64
    # basis's (iteration counts within a few percent, the first steps' history to the
    # basis's rounding); to 1e-9 it gets there over extra restarts, its residual recomputed
    # by the oracle
    L, levels, H, S, fu, GS, _ = case
    b = np.concatenate([fu[H.free[L]], np.zeros(S.np_)])
    kw = dict(solver="fgmres", restart=30, max_iter=3000, precond=precond, schur=schur, schur_iters=4)
    _, _, st = GS.solve(_dev(fu), basis="f32", tol=1e-6, **kw)
    _, _, ref = GS.solve(_dev(fu), basis="f64", tol=1e-6, **kw)
    print(f"[fgmres {precond} {schur} FP32 basis L={L}] to 1e-6: {st['iterations']} it, FP64 basis "
          f"{ref['iterations']} it", flush=True)
    assert st["converged"] and ref["converged"]
    assert abs(st["iterations"] - ref["iterations"]) <= max(2, int(0.05 * ref["iterations"]))
    k = min(len(st["history"]), len(ref["history"]), 10)
    assert np.allclose(st["history"][:k], ref["history"][:k], rtol=1e-5, atol=1e-14)
    tol = 1e-9
    u, p, st = GS.solve(_dev(fu), basis="f32", tol=tol, **kw)
    _, _, ref = GS.solve(_dev(fu), basis="f64", tol=tol, **kw)
    print(f"[fgmres {precond} {schur} FP32 basis L={L}] to 1e-9: {st['iterations']} it, FP64 basis "
          f"{ref['iterations']} it", flush=True)
    assert st["converged"] and st["iterations"] <= 1.5 * ref["iterations"] + 30
    xg = np.concatenate([u.cpu().numpy()[H.free[L]], p.cpu().numpy()])
    assert np.linalg.norm(b - S.K @ xg) <= 1.0001 * tol * np.linalg.norm(b)
    with pytest.raises(Exception):
        GS.solve(_dev(fu), solver="minres", tol=tol, basis="f32")


@pytest.mark.parametrize("case", [3], indirect=True, ids=["L3"])
def test_fgmres_below_the_rounding_floor_stays_finite(case):
    # asking for 1e-14 drives the Arnoldi process into near-dependent vectors (the
    # classical Gram-Schmidt second pass runs there); the solve must stay finite and
    # keep its residual at the rounding level (one size is enough)
    L, levels, H, S, fu, GS, _ = case
    b = np.concatenate([fu[H.free[L]], np.zeros(S.np_)])
    u, p, st = GS.solve(_dev(fu), solver="fgmres", restart=30, tol=1e-14, max_iter=700,
                        precond="triangular", raise_on_noconv=False)
    assert np.all(np.isfinite(st["history"]))
    xg = np.concatenate([u.cpu().numpy()[H.free[L]], p.cpu().numpy()])
    assert np.linalg.norm(b - S.K @ xg) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("case", [3], indirect=True, ids=["L3"])
def test_fgmres_stops_at_the_rounding_floor(case):
    # The true residual of an FP64 iterate cannot go below a floor set by rounding.
    # Measure that floor with an unreachable tolerance, then ask for a third of it: the
    # solve must stop by itself (floor_limited, AGCA_OK) long before max_iter, with a
    # residual within 10x of the tolerance and at most the velocity block's rounding floor.
    L, levels, H, S, fu, GS, _ = case
    b = np.concatenate([fu[H.free[L]], np.zeros(S.np_)])
    _, _, s0 = GS.solve(_dev(fu), solver="fgmres", restart=30, tol=1e-17, max_iter=1500,
                        precond="triangular", raise_on_noconv=False)
    assert not s0["converged"]
    floor = s0["rel_residual"]
    tol = floor / 3
    u, p, st = GS.solve(_dev(fu), solver="fgmres", restart=30, tol=tol, max_iter=3000,
                        precond="triangular")
    print(f"[fgmres floor L={L}] floor {floor:.2e} ({s0['iterations']} it, "
          f"floor_limited {s0['floor_limited']}); tol {tol:.2e}: {st['iterations']} it, "
          f"rel {st['rel_residual']:.2e}, floor_limited {st['floor_limited']}", flush=True)
    assert st["floor_limited"] and not st["converged"]
    assert tol < st["rel_residual"] < 10 * tol
    # the evidence the stop needs: at most the rounding floor of the velocity block
    assert 0 < st["floor_estimate"] and st["rel_residual"] <= max(tol, st["floor_estimate"])
    assert st["iterations"] < 3000
    xg = np.concatenate([u.cpu().numpy()[H.free[L]], p.cpu().numpy()])
    # recomputed by the oracle (assembled K, another order of additions): the same floor
    assert np.linalg.norm(b - S.K @ xg) <= 10 * floor * np.linalg.norm(b)
    # a reachable tolerance converges and is not reported as floor limited
    _, _, sr = GS.solve(_dev(fu), solver="fgmres", restart=30, tol=1e-9, max_iter=3000,
                        precond="triangular")
    assert sr["converged"] and not sr["floor_limited"]
