"""The rounding floor of the residual and the solver's stopping rule on the GPU, through
the C ABI: the floor kernel against the oracle (1e-12), the solve driven to stagnation
(floor_limited only at most max(tol, rho), solution against an exact solve within
the condition-number bound), and boundary slots of the inputs that must be ignored."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from oracle import fem, floor, mesh, mg
from tests.gpu_helpers import field_for, interior_full, oracle_case, rand_full, rel_err

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _gpu(case, **kw):
    from paper_2511_13109_amd import Hierarchy
    kind, L, ncomp = case
    H, nu_levels, field = oracle_case(kind, L, ncomp, 0)
    nus = [_dev(v) for v in nu_levels]
    return H, nu_levels, field, Hierarchy(L, ncomp, nus[L], nus[:L], **kw)


def _rhs(case, H, field):
    lv = H.levels[H.L]
    if case[0] == "sinkers":
        f = field.force(mesh.centroids_canonical(lv), H.ncomp)
    else:
        f = np.ones(lv.tets.shape[0]) if H.ncomp == 1 else np.tile([0, 0, -1.0], (lv.tets.shape[0], 1))
    return fem.load_vector(lv, f, H.ncomp)


@pytest.mark.parametrize("case", [("cube", 3, 1), ("sinkers", 3, 3), ("sinkers", 4, 3), ("unaligned", 4, 1)],
                         ids=lambda c: f"{c[0]}-L{c[1]}-nc{c[2]}")
def test_floor_kernel(case):
    print(f"\n[floor kernel {case}]", flush=True)
    H, nu, _, G = _gpu(case)
    try:
        rng = np.random.default_rng(0)
        lv = H.levels[H.L]
        for scale in (1.0, 1e-6):
            x = rand_full(H, H.L, rng)
            b = scale * rand_full(H, H.L, rng)
            m = interior_full(H, H.L)
            junk = 3.0 * (~m)                      # boundary slots must be ignored
            rho = G.residual_floor(_dev(b + junk), _dev(x + junk))
            ref = floor.residual_floor(lv, nu[H.L], H.ncomp, b, x)
            assert abs(rho - ref) <= 1e-12 * ref, (rho, ref)
    finally:
        G.close()


@pytest.mark.parametrize("case", [("cube", 3, 1), ("sinkers", 3, 3)], ids=lambda c: f"{c[0]}-L{c[1]}-nc{c[2]}")
def test_solve_to_stagnation(case):
    """PCG asked for an unreachable tolerance stops at the rounding floor: floor_limited,
    its true residual at most rho; rho equals the oracle's floor of the returned x;
    the solution matches an exact solve (sparse LU plus one refinement step with an
    extended-precision residual) within kappa_est (r_gpu + r_exact) / ||b||."""
    print(f"\n[stagnation {case}]", flush=True)
    H, nu, field, G = _gpu(case)
    try:
        b = _rhs(case, H, field)
        m = interior_full(H, H.L)
        x, st = G.solve(_dev(b), solver="pcg", tol=1e-17, max_iter=2000, raise_on_noconv=False)
        xg = x.cpu().numpy()
        rho = st["floor_estimate"]
        print(f"[stagnation {case}] {st['iterations']} it, {st['replacements']} replacements, "
              f"rel {st['rel_residual']:.3e}, rho {rho:.3e}, floor_limited {st['floor_limited']}", flush=True)
        assert st["floor_limited"] and st["status"] == 0
        assert st["rel_residual"] <= rho
        ref_rho = floor.residual_floor(H.levels[H.L], nu[H.L], H.ncomp, b, xg)
        assert abs(rho - ref_rho) <= 1e-12 * ref_rho
        A = H.A[H.L]
        lu = spla.splu(A.tocsc())
        xs = lu.solve(b[m])
        r = (b[m].astype(np.longdouble) - A.astype(np.longdouble) @ xs.astype(np.longdouble)).astype(np.float64)
        xs = xs + lu.solve(r)
        bn = np.linalg.norm(b[m])
        r_ex = np.linalg.norm(b[m] - A @ xs) / bn
        r_gpu = np.linalg.norm(b[m] - A @ xg[m]) / bn
        lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0]
        lmin = spla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
        bound = (lmax / lmin) * (r_gpu + r_ex)
        err = np.linalg.norm(xg[m] - xs) / np.linalg.norm(xs)
        print(f"[stagnation {case}] |x - x*| / |x*| = {err:.2e}, bound {bound:.2e} "
              f"(kappa {lmax / lmin:.2e}, residuals {r_gpu:.2e} / {r_ex:.2e})", flush=True)
        assert err <= bound
    finally:
        G.close()


def test_boundary_slots_of_b_are_ignored():
    """agca_solve norms b over the free dofs only: garbage in the boundary slots of b
    gives bit-identical results."""
    case = ("sinkers", 3, 3)
    H, nu, field, G = _gpu(case)
    try:
        b = _rhs(case, H, field)
        m = interior_full(H, H.L)
        rng = np.random.default_rng(1)
        junk = np.where(m, 0.0, 1e3 * rng.standard_normal(b.size))
        x1, s1 = G.solve(_dev(b), solver="pcg", tol=1e-8)
        x2, s2 = G.solve(_dev(b + junk), solver="pcg", tol=1e-8)
        assert s1["iterations"] == s2["iterations"] and s1["rel_residual"] == s2["rel_residual"]
        assert torch.equal(x1, x2)
    finally:
        G.close()


@pytest.mark.parametrize("mg_dtype", ["f64", "f32"])
def test_prolongation_ignores_coarse_boundary_slots(mg_dtype):
    case = ("sinkers", 3, 3)
    H, nu, field, G = _gpu(case, mg_dtype=mg_dtype, mg_nu_dtype=mg_dtype)
    try:
        rng = np.random.default_rng(2)
        dt = torch.float64 if mg_dtype == "f64" else torch.float32
        for l in range(1, H.L + 1):
            mc, mf = interior_full(H, l - 1), interior_full(H, l)
            ec = rand_full(H, l - 1, rng)
            xf = rand_full(H, l, rng)
            ec_junk = ec + np.where(mc, 0.0, 50.0 * rng.standard_normal(ec.size))
            out = G.prolong_add(l - 1, _dev(ec_junk).to(dt), _dev(xf).to(dt)).double().cpu().numpy()
            ref = xf.copy()
            ref[mf] += H.P[l - 1] @ ec[mc]
            assert rel_err(out, ref) < (1e-12 if mg_dtype == "f64" else 1e-6), l
    finally:
        G.close()
