"""GPU parity: every hot-path kernel against the CPU oracle, through the C ABI.

Sizes: L = 2 (9^3 nodes), 3 (17^3) and 4 (33^3): the element loop's 15-node
tiles and its z chunks end in ragged tails at all three.  FP64 results must
match to 1e-12 relative; flags and flagged-id lists bit-exactly.
"""

import numpy as np
import pytest
import torch

from oracle import adjoint, agca, fem, floor, mesh, mg
from tests.gpu_helpers import (field_for, interior_full, oracle_apply_full, oracle_case, rand_full, rel_err,
                               vcycle_errors)

pytestmark = pytest.mark.gpu

TOL = 1e-12
CASES = [("cube", 3, 1), ("sinkers", 3, 1), ("sinkers", 3, 3), ("unaligned", 4, 1), ("sinkers", 2, 3),
         ("sinkers", 4, 3)]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _gpu(case, mode="ratio", mg_dtype="f64", mg_nu=None):
    from paper_2511_13109_amd import Hierarchy
    kind, L, ncomp = case
    H, nu_levels, _ = oracle_case(kind, L, ncomp, {"ratio": 0, "none": 2, "all": 3}[mode])
    nus = [_dev(v) for v in nu_levels]
    G = Hierarchy(L, ncomp, nus[L], nus[:L], flag_mode=mode, mg_dtype=mg_dtype, mg_nu_dtype=mg_nu)
    return H, G


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}-L{c[1]}-nc{c[2]}")
def pair(request):
    print(f"\n[case {request.param}]", flush=True)
    H, G = _gpu(request.param)
    yield request.param, H, G
    G.close()


def test_flags_bit_exact(pair):
    _, H, G = pair
    for l in range(H.L):
        ref = np.nonzero(H.flags[l])[0].astype(np.int32)
        got = G.flags(l)
        assert np.array_equal(got, ref), (l, got.size, ref.size)
        assert G.query(l)["flagged"] == ref.size


def test_blocks_match_local_galerkin(pair):
    _, H, G = pair
    Ps = H.P_full
    for l in range(H.L):
        ids = G.flags(l)
        if ids.size == 0:
            continue
        sel = ids if ids.size <= 64 else ids[np.linspace(0, ids.size - 1, 64).astype(int)]
        ref = agca.local_gca_blocks(H.levels, Ps, H.nu_levels[H.L], H.ncomp, l, sel)
        got = G.blocks(l)
        pos = np.searchsorted(ids, sel)
        assert rel_err(got[pos], ref) < TOL, l


def test_apply_every_level(pair):
    _, H, G = pair
    rng = np.random.default_rng(0)
    for l in range(H.L + 1):
        u = rand_full(H, l, rng)
        u_dev = _dev(u + 7.0 * (1 - interior_full(H, l)))   # boundary input must be ignored
        v = G.apply(l, u_dev).cpu().numpy()
        ref = oracle_apply_full(H, l, u)
        assert rel_err(v, ref) < TOL, l


def test_residual_and_jacobi_sweep(pair):
    _, H, G = pair
    rng = np.random.default_rng(1)
    for l in range(1, H.L + 1):
        x = rand_full(H, l, rng)
        b = rand_full(H, l, rng)
        r = G.residual(l, _dev(b), _dev(x)).cpu().numpy()
        assert rel_err(r, b - oracle_apply_full(H, l, x)) < TOL
        m = interior_full(H, l)
        xs = _dev(x)
        G.smooth(l, _dev(b), xs, 1)
        ref = np.zeros_like(x)
        ref[m] = mg.jacobi(H, l, b[m], x[m], 1)
        assert rel_err(xs.cpu().numpy(), ref) < TOL
        xs = _dev(x)
        G.smooth(l, _dev(b), xs, 3)
        ref[m] = mg.jacobi(H, l, b[m], x[m], 3)
        assert rel_err(xs.cpu().numpy(), ref) < TOL


def test_diagonal(pair):
    _, H, G = pair
    for l in range(H.L + 1):
        d = G.diagonal(l)
        ref = np.zeros_like(d)
        ref[interior_full(H, l)] = H.D[l]
        assert rel_err(d, ref) < TOL


def test_transfers(pair):
    _, H, G = pair
    rng = np.random.default_rng(2)
    for l in range(1, H.L + 1):
        rf = rand_full(H, l, rng)
        rc = G.restrict(l, _dev(rf)).cpu().numpy()
        mc, mf = interior_full(H, l - 1), interior_full(H, l)
        ref = np.zeros(mc.size)
        ref[mc] = H.P[l - 1].T @ rf[mf]
        assert rel_err(rc, ref) < TOL
        ec = rand_full(H, l - 1, rng)
        xf = rand_full(H, l, rng)
        out = G.prolong_add(l - 1, _dev(ec), _dev(xf)).cpu().numpy()
        ref = xf.copy()
        ref[mf] += H.P[l - 1] @ ec[mc]
        assert rel_err(out, ref) < TOL


def test_vcycle(pair):
    case, H, G = pair
    rng = np.random.default_rng(3)
    b = rand_full(H, H.L, rng)
    x = G.vcycle(_dev(b)).cpu().numpy()
    e_gpu, e_orc, tol = vcycle_errors(H, b, x)
    print(f"[vcycle {case}] library {e_gpu:.2e}, oracle FP64 {e_orc:.2e} from the extended-precision "
          f"cycle (tolerance {tol:.1e})", flush=True)
    assert e_gpu < tol


def test_dot_deterministic(pair):
    _, H, G = pair
    rng = np.random.default_rng(4)
    x = rand_full(H, H.L, rng)
    y = rand_full(H, H.L, rng)
    d1 = G.dot(H.L, _dev(x), _dev(y))
    d2 = G.dot(H.L, _dev(x), _dev(y))
    assert d1 == d2
    assert abs(d1 - x @ y) <= 1e-13 * np.abs(x).sum() * np.abs(y).max()


def test_pcg_solve(pair):
    case, H, G = pair
    lv = H.levels[H.L]
    field = field_for(case[0], H.L)
    f = field.force(mesh.centroids_canonical(lv), H.ncomp) if case[0] == "sinkers" else \
        np.ones(lv.tets.shape[0]) if H.ncomp == 1 else np.tile([0, 0, -1.0], (lv.tets.shape[0], 1))
    b = fem.load_vector(lv, f, H.ncomp)
    # load vector kernel parity
    fT = np.asarray(f).reshape(lv.tets.shape[0], -1).T.copy()
    bg = G.load_vector(_dev(fT.ravel())).cpu().numpy()
    assert rel_err(bg, b) < TOL
    m = interior_full(H, H.L)
    # 1e-10 for the 1e3-contrast cube; 1e-8 where the 1e6 contrast limits the attainable
    # true residual in FP64
    tol = 1e-10 if case[0] == "cube" else 1e-8
    ref = mg.pcg(H.A[H.L], b[m], lambda r: mg.vcycle(H, r), tol)
    x, st = G.solve(_dev(b), solver="pcg", tol=tol)
    assert st["converged"] and st["rel_residual"] <= tol
    assert abs(st["iterations"] - ref.iterations) <= 1
    _check_history(H, b, ref, st)
    xs = fem.restrict_free(H.ops_full[H.L], H.free[H.L])
    import scipy.sparse.linalg as spla
    exact = spla.splu(xs.tocsc()).solve(b[m])
    err = np.linalg.norm(x.cpu().numpy()[m] - exact) / np.linalg.norm(exact)
    assert err < 1e-4


def _check_history(H, b_full, ref, st):
    """PCG residual history against the oracle's, relative 1e-6, over the iterations whose
    residual is at least 1e7 times the rounding floor of the oracle's solution (below
    that the recurrences of the two FP64 runs, and the true residuals that replace the
    library's recurrence, differ by rounding in the leading digits)."""
    m = interior_full(H, H.L)
    xr = np.zeros_like(b_full)
    xr[m] = ref.x
    rho = floor.residual_floor(H.levels[H.L], H.nu_levels[H.L], H.ncomp, b_full, xr)
    hr = np.asarray(ref.history)
    k = min(len(st["history"]), int(np.sum(hr >= 1e7 * rho)))
    assert k >= 5, (k, rho)
    assert np.allclose(st["history"][:k], hr[:k], rtol=1e-6, atol=0), (st["history"][:k], hr[:k])


def test_adjoint_gradient_kernel(pair):
    _, H, G = pair
    rng = np.random.default_rng(5)
    u = rand_full(H, H.L, rng)
    w = rand_full(H, H.L, rng)
    g = G.grad_log_nu(_dev(u), _dev(w)).cpu().numpy()
    ref = adjoint.grad_log_nu(H.levels[H.L], H.nu_levels[H.L], H.ncomp, u, w)
    assert rel_err(g, ref) < TOL


@pytest.mark.parametrize("mode", ["none", "all"])
def test_flag_modes(mode):
    H, G = _gpu(("sinkers", 3, 3), mode=mode)
    try:
        rng = np.random.default_rng(6)
        for l in range(H.L):
            assert G.query(l)["flagged"] == (0 if mode == "none" else 6 * H.levels[l].n ** 3)
            u = rand_full(H, l, rng)
            assert rel_err(G.apply(l, _dev(u)).cpu().numpy(), oracle_apply_full(H, l, u)) < TOL
    finally:
        G.close()


def test_mixed_precision_fcg_reaches_fp64_residual():
    H, G = _gpu(("sinkers", 4, 3), mg_dtype="f32", mg_nu="f32")
    H2, G2 = _gpu(("sinkers", 4, 3), mg_dtype="f32", mg_nu="bf16")
    try:
        lv = H.levels[H.L]
        f = field_for("sinkers", H.L).force(mesh.centroids_canonical(lv), 3)
        b = _dev(fem.load_vector(lv, f, 3))
        m = interior_full(H, H.L)
        bn = b.cpu().numpy()[m]
        ref_fcg = mg.fcg(H.A[H.L], bn, lambda r: mg.vcycle(H, r), 1e-8).iterations
        for GG in (G, G2):
            # the stationary iteration (x += B r) needs ~430 FP64 V-cycles here
            for solver, cap in (("fcg", 300), ("ir", 1500)):
                x, st = GG.solve(b, solver=solver, tol=1e-8, max_iter=cap, raise_on_noconv=False)
                print(solver, GG.cfg.mg_nu_dtype, st["iterations"], st["rel_residual"], flush=True)
                assert st["converged"] and st["rel_residual"] <= 1e-8, (solver, st["iterations"],
                                                                        st["rel_residual"])
                if solver == "fcg":
                    # an FP32 V-cycle costs at most a few extra outer iterations
                    assert st["iterations"] <= ref_fcg + 5, (st["iterations"], ref_fcg)
        # FP32 level apply against the oracle at FP32 accuracy
        rng = np.random.default_rng(7)
        u = rand_full(H, H.L, rng)
        v = G.apply(H.L, _dev(u).float()).double().cpu().numpy()
        assert rel_err(v, oracle_apply_full(H, H.L, u)) < 1e-5
    finally:
        G.close()
        G2.close()


def test_invalid_coefficient_rejected():
    from paper_2511_13109_amd import AGCAError, Hierarchy
    H, nu_levels, _ = oracle_case("sinkers", 2, 1, 0)
    nus = [_dev(v) for v in nu_levels]
    bad = nus[2].clone()
    bad[17] = float("nan")
    with pytest.raises(AGCAError, match="AGCA_E_INVALID"):
        Hierarchy(2, 1, bad, nus[:2])
    bad[17] = -1.0
    with pytest.raises(AGCAError, match="AGCA_E_INVALID"):
        Hierarchy(2, 1, bad, nus[:2])


def test_memory_limit_gives_oom():
    from paper_2511_13109_amd import AGCAError, Hierarchy
    H, nu_levels, _ = oracle_case("sinkers", 2, 1, 0)
    nus = [_dev(v) for v in nu_levels]
    with pytest.raises(AGCAError, match="AGCA_E_OOM"):
        Hierarchy(2, 1, nus[2], nus[:2], mem_limit_bytes=4096)


def test_cast_round_to_nearest_even():
    from paper_2511_13109_amd import Hierarchy
    H, nu_levels, _ = oracle_case("sinkers", 2, 1, 0)
    nus = [_dev(v) for v in nu_levels]
    G = Hierarchy(2, 1, nus[2], nus[:2])
    try:
        rng = np.random.default_rng(8)
        x = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-20, 20, 1000),
                            [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -8 + 2 ** -40]])
        f32 = G.cast(_dev(x), "f32").cpu().numpy()
        assert np.array_equal(f32, x.astype(np.float32))
        bf = G.cast(_dev(x), "bf16").cpu().numpy().view(np.uint16).astype(np.uint32)
        back = (bf << 16).view(np.float32).astype(np.float64)
        # one rounding of the float64 value to 8 significant bits, ties to even
        m, e = np.frexp(x)
        ref = np.ldexp(np.round(m * 256.0), e - 8)
        assert np.array_equal(back, ref)
        # ties go to the even neighbour; anything above a tie rounds up
        assert back[-4] == 1.0 and back[-3] == 1.0 and back[-2] == 1.0 + 2 ** -6
        assert back[-1] == 1.0 + 2 ** -7
    finally:
        G.close()


# ---------------------------------------------------------------------------
# Chebyshev smoother (Section 4): eigenvalue estimates, V-cycle and PCG against
# the oracle, for degree 2 (first two passes fused on element-loop levels) and
# degree 3 (every pass separate)
# ---------------------------------------------------------------------------
CHEB_CASES = [("sinkers", 3, 3, 2), ("sinkers", 4, 3, 2), ("unaligned", 4, 1, 3), ("sinkers", 3, 3, 3)]


@pytest.mark.parametrize("case", CHEB_CASES, ids=lambda c: f"{c[0]}-L{c[1]}-nc{c[2]}-deg{c[3]}")
def test_chebyshev_smoother(case):
    from paper_2511_13109_amd import Hierarchy
    import copy
    kind, L, ncomp, deg = case
    print(f"\n[chebyshev {case}]", flush=True)
    H0, nu_levels, field = oracle_case(kind, L, ncomp, 0, "chebyshev")
    H = copy.copy(H0)
    H.nu1 = H.nu2 = deg
    nus = [_dev(v) for v in nu_levels]
    G = Hierarchy(L, ncomp, nus[L], nus[:L], smoother="chebyshev", pre=deg, post=deg)
    try:
        for l in range(1, L + 1):
            lam = G.query(l)["lambda_max"]
            assert abs(lam - H.lam[l]) <= 1e-10 * H.lam[l], (l, lam, H.lam[l])
        rng = np.random.default_rng(11)
        b = rand_full(H, L, rng)
        m = interior_full(H, L)
        x = G.vcycle(_dev(b)).cpu().numpy()
        e_gpu, e_orc, vtol = vcycle_errors(H, b, x)
        print(f"[chebyshev {case}] V-cycle: library {e_gpu:.2e}, oracle FP64 {e_orc:.2e} "
              f"(tolerance {vtol:.1e})", flush=True)
        assert e_gpu < vtol
        lv = H.levels[L]
        f = field.force(mesh.centroids_canonical(lv), ncomp) if kind == "sinkers" else \
            np.ones(lv.tets.shape[0])
        bb = fem.load_vector(lv, f, ncomp)
        tol = 1e-8
        r_ref = mg.pcg(H.A[L], bb[m], lambda r: mg.vcycle(H, r), tol)
        r_jac = mg.pcg(H.A[L], bb[m], lambda r: mg.vcycle(_jacobi_twin(H), r), tol)
        xg, st = G.solve(_dev(bb), solver="pcg", tol=tol)
        print(f"[chebyshev {case}] PCG gpu {st['iterations']} oracle {r_ref.iterations} "
              f"(Jacobi V-cycle {r_jac.iterations})", flush=True)
        assert st["converged"] and abs(st["iterations"] - r_ref.iterations) <= 1
        _check_history(H, bb, r_ref, st)
    finally:
        G.close()
    # the FP32 V-cycle with the Chebyshev smoother inside FCG reaches the FP64 residual
    G32 = Hierarchy(L, ncomp, nus[L], nus[:L], smoother="chebyshev", pre=deg, post=deg,
                    mg_dtype="f32", mg_nu_dtype="f32")
    try:
        _, st = G32.solve(_dev(bb), solver="fcg", tol=tol, max_iter=1500)
        assert st["converged"] and st["rel_residual"] <= tol
    finally:
        G32.close()


# Uneven and zero smoothing counts.  On these 17^3 hierarchies levels 1-2 (scalar) or
# level 1 (vector) run as one workgroup-resident kernel, the levels above as one launch
# per pass: both must follow the oracle's cycle pass for pass.
SWEEP_CASES = [("jacobi", 1, 3), ("jacobi", 3, 0), ("jacobi", 0, 2), ("chebyshev", 3, 1),
               ("chebyshev", 1, 4), ("chebyshev", 0, 3)]


@pytest.mark.parametrize("ncomp", [1, 3])
@pytest.mark.parametrize("sweeps", SWEEP_CASES, ids=lambda s: f"{s[0]}-{s[1]}-{s[2]}")
def test_vcycle_uneven_sweeps(sweeps, ncomp):
    from paper_2511_13109_amd import Hierarchy
    import copy
    smoother, pre, post = sweeps
    print(f"\n[uneven sweeps {sweeps} nc={ncomp}]", flush=True)
    H0, nu_levels, _ = oracle_case("sinkers", 3, ncomp, 0, smoother)
    H = copy.copy(H0)
    H.nu1, H.nu2 = pre, post
    nus = [_dev(v) for v in nu_levels]
    G = Hierarchy(3, ncomp, nus[3], nus[:3], smoother=smoother, pre=pre, post=post)
    try:
        rng = np.random.default_rng(12)
        for _ in range(2):  # the second call starts from the first one's buffers
            b = rand_full(H, 3, rng)
            x = G.vcycle(_dev(b)).cpu().numpy()
            e_gpu, e_orc, tol = vcycle_errors(H, b, x)
            print(f"[uneven sweeps {sweeps} nc={ncomp}] library {e_gpu:.2e}, oracle FP64 {e_orc:.2e} "
                  f"(tolerance {tol:.1e})", flush=True)
            assert e_gpu < tol
    finally:
        G.close()


def _jacobi_twin(H):
    import copy
    J = copy.copy(H)
    J.smoother = "jacobi"
    J.nu1 = J.nu2 = 2
    return J


def test_stationary_mg_cube17():
    # the scalar aligned-cube workload's solver: stationary V(2,2) iterations to 1e-10
    H, G = _gpu(("cube", 3, 1))
    try:
        lv = H.levels[H.L]
        b = fem.load_vector(lv, np.ones(lv.tets.shape[0]), 1)
        m = interior_full(H, H.L)
        ref = mg.stationary(H, b[m], 1e-10, maxit=3000)
        assert ref.converged
        x, st = G.solve(_dev(b), solver="stationary", tol=1e-10, max_iter=3000)
        print(f"\n[stationary cube17] gpu {st['iterations']} it, oracle {ref.iterations} it", flush=True)
        assert st["converged"] and st["rel_residual"] <= 1e-10
        assert abs(st["iterations"] - ref.iterations) <= 1
        k = min(len(st["history"]), len(ref.history), 50)
        assert np.allclose(st["history"][:k], ref.history[:k], rtol=1e-6, atol=0)
        assert rel_err(x.cpu().numpy()[m], ref.x) <= 1e-8
    finally:
        G.close()
