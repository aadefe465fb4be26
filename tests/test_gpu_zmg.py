"""GPU parity of the BFBT pressure multigrid (eq. (4.2) with a geometric multigrid for
Z = B W^-1 B^T) through the C ABI, against the oracle's ZHierarchy: the 65-offset
stencils of every level assembled by probing (1e-12 of the level's largest entry),
one V-cycle (1e-10), the Schur approximations S^-1 r of all three kinds, and
triangular FGMRES with BFBT_MG (residual-history prefix, iteration counts).  At
129^3 pressure nodes (the 257^3 Stokes workload) the stencil and the cycle are checked
by properties that hold at any size: symmetry, zero row sums, the stencil's product
against the matrix-free Z = B W^-1 B^T on a random vector, and the V-cycle's symmetry
and energy-norm contraction.
"""

import numpy as np
import pytest
import torch

from oracle import fem, mesh, mg, stokes
from workloads import Sinkers

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _outside(n):
    """(65, (n+1)^3) mask: node k + o_i lies outside the lattice."""
    n1 = n + 1
    k = np.arange(n1 ** 3)
    kx, ky, kz = k % n1, (k // n1) % n1, k // n1 ** 2
    out = np.zeros((65, k.size), dtype=bool)
    for i, (dx, dy, dz) in enumerate(stokes.Z_OFFSETS):
        out[i] = (kx + dx < 0) | (kx + dx > n) | (ky + dy < 0) | (ky + dy > n) | (kz + dz < 0) | (kz + dz > n)
    return out


@pytest.fixture(scope="module", params=[2, 4, 5], ids=lambda L: f"L{L}")
def zcase(request):
    from paper_2511_13109_amd import Hierarchy, Stokes
    L = request.param
    print(f"\n[pressure multigrid case L={L}]", flush=True)
    levels = mesh.hierarchy(L)
    field = Sinkers(3, 5, radius=0.2, width=2.0 / 2 ** (L + 1), contrast=1e4)
    nu = [field.nu(mesh.centroids_canonical(lv)) for lv in levels]
    H = mg.build(L, nu, 3, levels=levels)
    S = stokes.StokesSystem(H)
    ZH = stokes.ZHierarchy(S)
    f = np.asarray(field.force(mesh.centroids_canonical(levels[L]), 3))
    fu = fem.load_vector(levels[L], f, 3)
    G = Hierarchy(L, 3, _dev(nu[L]), [_dev(v) for v in nu[:L]])
    yield L, H, S, ZH, fu, Stokes(G)
    G.close()


def test_stencils_match_oracle(zcase):
    L, H, S, ZH, fu, GS = zcase
    for l in range(L):
        got = GS.z_stencil(l).cpu().numpy()
        ref = ZH.stencil(l)
        err = _rel(got, ref)
        print(f"[stencil level {l}] {ref.shape[1]} nodes, rel err {err:.1e}", flush=True)
        assert err <= 1e-12, l
        # entries whose neighbour leaves the lattice are exactly zero (the stencil kernels
        # rely on it)
        assert np.all(got[_outside(2 ** (l + 1))] == 0.0)


def test_vcycle_matches_oracle(zcase):
    L, H, S, ZH, fu, GS = zcase
    rng = np.random.default_rng(L)
    r = rng.standard_normal(S.np_)
    r -= r.mean()
    y = GS.z_vcycle(_dev(r)).cpu().numpy()
    ref = ZH.vcycle(r)
    err = _rel(y, ref)
    print(f"[vcycle] rel err {err:.1e}", flush=True)
    assert err <= 1e-10
    # a second call gives the same bits (no state kept between cycles)
    assert np.array_equal(GS.z_vcycle(_dev(r)).cpu().numpy(), y)


@pytest.mark.parametrize("schur,k", [("mass", 1), ("bfbt", 5), ("bfbt_mg", 1), ("bfbt_mg", 4)])
def test_schur_apply_matches_oracle(zcase, schur, k):
    # few enough CG steps that no Z solve runs past convergence at 5^3 pressure nodes
    # (steps beyond it only amplify the order of additions)
    L, H, S, ZH, fu, GS = zcase
    rng = np.random.default_rng(10 + k)
    r = rng.standard_normal(S.np_)
    q = GS.schur_apply(_dev(r), schur, k).cpu().numpy()
    if schur == "mass":
        ref = r / S.m
    elif schur == "bfbt":
        ref = S.bfbt(k)(r)
    else:
        ref = S.bfbt(k, z_solve=ZH.z_solve(k))(r)
    err = _rel(q, ref)
    print(f"[S^-1 {schur} k={k}] rel err {err:.1e}", flush=True)
    assert err <= (1e-12 if schur == "mass" else 1e-8)


def test_fgmres_bfbt_mg_matches_oracle(zcase):
    L, H, S, ZH, fu, GS = zcase
    b = np.concatenate([fu[H.free[L]], np.zeros(S.np_)])
    tol = 1e-9
    u, p, st = GS.solve(_dev(fu), solver="fgmres", restart=30, tol=tol, max_iter=2000,
                        precond="triangular", schur="bfbt_mg", schur_iters=4)
    ref = S.solve(b, "fgmres", tol=tol, restart=30, maxit=2000, precond="triangular",
                  schur="bfbt_mg", schur_iters=4)
    print(f"[fgmres triangular BFBT_MG L={L}] gpu {st['iterations']} it, oracle {ref.iterations} it",
          flush=True)
    assert st["converged"] and ref.converged
    n = min(len(st["history"]), len(ref.history), 15)
    assert np.allclose(st["history"][:n], ref.history[:n], rtol=1e-6, atol=1e-14)
    assert abs(st["iterations"] - ref.iterations) <= max(1, int(0.05 * ref.iterations))
    xg = np.concatenate([u.cpu().numpy()[H.free[L]], p.cpu().numpy()])
    assert np.linalg.norm(b - S.K @ xg) <= 1.0001 * tol * np.linalg.norm(b)


@pytest.mark.parametrize("zcase", [4], indirect=True, ids=["L4"])
def test_bfbt_mg_with_the_fp32_velocity_cycle(zcase):
    # BFBT with multigrid Z solves around the FP32/FP32-coefficient V-cycle: converged,
    # residual recomputed by the oracle; velocity_cycles 0 and 1 are the same solve
    from paper_2511_13109_amd import Hierarchy, Stokes
    L, H, S, ZH, fu, GS = zcase
    nu_l = [np.asarray(v) for v in H.nu_levels]
    G32 = Hierarchy(L, 3, _dev(nu_l[L]), [_dev(v) for v in nu_l[:L]], mg_dtype="f32", mg_nu_dtype="f32")
    try:
        S32 = Stokes(G32)
        b = np.concatenate([fu[H.free[L]], np.zeros(S.np_)])
        tol = 1e-8
        u, p, st = S32.solve(_dev(fu), solver="fgmres", restart=30, tol=tol, max_iter=2000,
                             precond="triangular", schur="bfbt_mg", schur_iters=4)
        assert st["converged"]
        xg = np.concatenate([u.cpu().numpy()[H.free[L]], p.cpu().numpy()])
        assert np.linalg.norm(b - S.K @ xg) <= 1.0001 * tol * np.linalg.norm(b)
        _, _, st0 = S32.solve(_dev(fu), solver="fgmres", restart=30, tol=tol, max_iter=2000,
                              precond="triangular", schur="bfbt_mg", schur_iters=4, velocity_cycles=0)
        assert st0["history"] == st["history"]
        print(f"[fgmres triangular BFBT_MG FP32 V-cycle L={L}] {st['iterations']} it", flush=True)
    finally:
        G32.close()


def test_bad_arguments(zcase):
    L, H, S, ZH, fu, GS = zcase
    r = GS.pvec()
    with pytest.raises(Exception):
        GS.schur_apply(r, "bfbt_mg", 0)
    with pytest.raises(Exception):
        GS.z_stencil(L)
    with pytest.raises(Exception):
        GS.z_stencil(-1)
    with pytest.raises(Exception):
        GS.solve(_dev(fu), solver="minres", tol=1e-8, schur="bfbt_mg")


def test_stencils_follow_a_coefficient_rebuild():
    # the multigrid is assembled for the coefficient in place at its first use and again
    # after every rebuild: stencils and S^-1 against the oracle for the second field
    from paper_2511_13109_amd import Hierarchy, Stokes
    L = 3
    levels = mesh.hierarchy(L)
    fields = [Sinkers(3, 5, radius=0.2, width=2.0 / 2 ** (L + 1), contrast=1e4),
              Sinkers(2, 9, radius=0.25, width=2.0 / 2 ** (L + 1), contrast=1e3)]
    nus = [[f.nu(mesh.centroids_canonical(lv)) for lv in levels] for f in fields]
    G = Hierarchy(L, 3, _dev(nus[0][L]), [_dev(v) for v in nus[0][:L]])
    try:
        GS = Stokes(G)
        first = GS.z_stencil(L - 1).cpu().numpy()
        G.set_nu(_dev(nus[1][L]), [_dev(v) for v in nus[1][:L]])
        S = stokes.StokesSystem(mg.build(L, nus[1], 3, levels=levels))
        ZH = stokes.ZHierarchy(S)
        for l in range(L):
            assert _rel(GS.z_stencil(l).cpu().numpy(), ZH.stencil(l)) <= 1e-12, l
        assert _rel(GS.z_stencil(L - 1).cpu().numpy(), first) > 1e-3
        r = np.random.default_rng(8).standard_normal(S.np_)
        q = GS.schur_apply(_dev(r), "bfbt_mg", 2).cpu().numpy()
        assert _rel(q, S.bfbt(2, z_solve=ZH.z_solve(2))(r)) <= 1e-8
    finally:
        G.close()


def _stencil_apply_host(st, n, x):
    return stokes.stencil_apply(st, n, x)


def test_stokes257_stencil_properties():
    # 257^3 velocity, 129^3 pressure nodes (the Stokes workload's size): the assembled
    # top-level stencil is symmetric, annihilates constants, and its product equals the
    # matrix-free B W^-1 B^T (through the library's B, B^T and diag(A)) on a random vector
    from paper_2511_13109_amd import Hierarchy, Stokes
    from workloads import workload
    from workloads.lattice import element_centroids
    L = 7
    print(f"\n[stokes257 pressure stencil]", flush=True)
    w = workload("stokes257")
    field = w.make_field()
    nu = [_dev(field.nu(element_centroids(l))) for l in range(L + 1)]
    G = Hierarchy(L, 3, nu[L], nu[:L])
    try:
        GS = Stokes(G)
        n = 2 ** L
        n1 = n + 1
        st = GS.z_stencil(L - 1).cpu().numpy()
        scale = np.abs(st[32]).max()
        # symmetry: S[o](k) = S[-o](k + o), on a sample of nodes and every offset
        rng = np.random.default_rng(7)
        ks = rng.integers(0, n1 ** 3, 4000)
        kx, ky, kz = ks % n1, (ks // n1) % n1, ks // n1 ** 2
        for i, (dx, dy, dz) in enumerate(stokes.Z_OFFSETS):
            j = 64 - i                                   # the offset -o
            assert stokes.Z_OFFSETS[j] == (-dx, -dy, -dz)
            inside = (kx + dx >= 0) & (kx + dx <= n) & (ky + dy >= 0) & (ky + dy <= n) & \
                     (kz + dz >= 0) & (kz + dz <= n)
            a = st[i, ks[inside]]
            b = st[j, (ks + dx + n1 * (dy + n1 * dz))[inside]]
            assert np.abs(a - b).max() <= 1e-13 * scale, (dx, dy, dz)
            assert np.all(st[i, ks[~inside]] == 0.0)
        assert np.abs(st.sum(axis=0)).max() <= 1e-12 * scale
        # the V-cycle at this size: symmetric (u . V v = v . V u, to rounding) and an
        # energy-norm contraction on zero-sum vectors (checked through Z's stencil form)
        uu = rng.standard_normal(n1 ** 3)
        vv = rng.standard_normal(n1 ** 3)
        uu -= uu.mean()
        vv -= vv.mean()
        Vu = GS.z_vcycle(_dev(uu)).cpu().numpy()
        Vv = GS.z_vcycle(_dev(vv)).cpu().numpy()
        assert abs(uu @ Vv - vv @ Vu) <= 1e-10 * abs(uu @ Vv)
        e = uu
        Ze = _stencil_apply_host(st, n, e)
        e1 = e - GS.z_vcycle(_dev(Ze)).cpu().numpy()
        e1 -= e1.mean()
        ratio = np.sqrt((e1 @ _stencil_apply_host(st, n, e1)) / (e @ Ze))
        print(f"[stokes257] pressure V-cycle energy contraction on a random error {ratio:.3f}", flush=True)
        assert ratio < 0.9
        x = rng.standard_normal(n1 ** 3)
        diag = np.asarray(G.diagonal(L), dtype=np.float64)
        winv = np.where(diag != 0, 1.0 / np.where(diag != 0, diag, 1.0), 0.0)
        v = GS.grad(_dev(x))
        zx = GS.div(v * _dev(winv)).cpu().numpy()
        sx = _stencil_apply_host(st, n, x)
        err = _rel(sx, zx)
        print(f"[stokes257] stencil vs matrix-free Z: {err:.1e}", flush=True)
        assert err <= 1e-12
    finally:
        G.close()
