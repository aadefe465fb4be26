"""GPU parity of the macro-granularity coarsening (eqs. (2.8)-(2.9)) through the C ABI:
the per-macro gradient maxima against the oracle (1e-12 relative), the 24-of-48 count
of a sharp unaligned cube, per-level flag sets (bit-exact), and V-cycles and PCG
iteration counts of the macro-flag hierarchy against the oracle built with the same
flags.  At 129^3 (element-loop coarse level with stored blocks, the path the small
cases never reach) coarse-level rows are sampled and recomputed element by element.
"""

import numpy as np
import pytest
import torch

from oracle import agca, mesh, mg, sample
from workloads import Sinkers, workload
from workloads.lattice import element_centroids

from gpu_helpers import interior_full, rel_err, vcycle_errors

pytestmark = pytest.mark.gpu


def _node_xyz(L):
    n = 2 ** (L + 1)
    p = np.arange((n + 1) ** 3)
    return np.stack([p % (n + 1), (p // (n + 1)) % (n + 1), p // (n + 1) ** 2], axis=1) / n


def _sinker_field(L):
    return Sinkers(4, 2, radius=0.15, width=2.0 / 2 ** (L + 1), contrast=1e6)


@pytest.mark.parametrize("L", [2, 4])
def test_macro_gradient_matches_oracle(L):
    from paper_2511_13109_amd import macro_gradient
    print(f"\n[macro gradient L={L}]", flush=True)
    levels = mesh.hierarchy(L)
    eta = _sinker_field(L).nu(_node_xyz(L))
    g_dev = macro_gradient(L, torch.from_numpy(eta).cuda())
    g_ref = agca.macro_gradient_max(levels, eta)
    assert np.abs(g_dev - g_ref).max() <= 1e-12 * g_ref.max()
    # sharp unaligned cube [1/3, 7/12]^3: exactly the 24 macros it meets (Fig. 9)
    X = _node_xyz(L)
    box = np.where(np.all((X > 1 / 3) & (X < 7 / 12), axis=1), 1e3, 1.0)
    gb = macro_gradient(L, torch.from_numpy(box).cuda())
    assert int((gb > 0).sum()) == 24
    assert np.array_equal(gb > 0, agca.macro_gradient_max(levels, box) > 0)


@pytest.mark.parametrize("ncomp", [1, 3])
def test_macro_flag_hierarchy_matches_oracle(ncomp):
    from paper_2511_13109_amd import Hierarchy, macro_gradient
    L = 3
    print(f"\n[macro flags L={L} ncomp={ncomp}]", flush=True)
    levels = mesh.hierarchy(L)
    field = _sinker_field(L)
    nu = [field.nu(mesh.centroids_canonical(lv)) for lv in levels]
    g = macro_gradient(L, torch.from_numpy(field.nu(_node_xyz(L))).cuda())
    tol = float(np.median(g[g > 0]))              # a tolerance that splits the macros
    mf = g > tol
    assert 0 < mf.sum() < 48
    H = mg.build(L, nu, ncomp, mode=agca.FLAG_MACRO, levels=levels, macro_flags=mf)
    G = Hierarchy(L, ncomp, torch.from_numpy(nu[L]).cuda(), [torch.from_numpy(v).cuda() for v in nu[:L]],
                  flag_mode="macro", macro_flags=mf)
    try:
        for l in range(L):
            ref = np.nonzero(H.flags[l])[0]
            assert np.array_equal(G.flags(l), ref), l
            assert ref.size == int(mf.sum()) * 8 ** l
        rng = np.random.default_rng(ncomp)
        nn = (levels[L].n + 1) ** 3
        b = rng.standard_normal(ncomp * nn) * interior_full(H, L)
        z = G.vcycle(torch.from_numpy(b).cuda()).cpu().numpy()
        e_gpu, e_orc, vtol = vcycle_errors(H, b, z)
        print(f"[vcycle] library {e_gpu:.2e}, oracle FP64 {e_orc:.2e} (tolerance {vtol:.1e})", flush=True)
        assert e_gpu < vtol
        x, st = G.solve(torch.from_numpy(b).cuda(), solver="pcg", tol=1e-10, max_iter=500)
        ref = mg.pcg(H.A[L], b[H.free[L]], lambda r: mg.vcycle(H, r), 1e-10, maxit=500)
        assert abs(st["iterations"] - ref.iterations) <= 1, (st["iterations"], ref.iterations)
    finally:
        G.close()


@pytest.mark.parametrize("storage", ["blocks", "mean"])
def test_macro_flags_element_loop_level_sampled(storage):
    # 129^3: level 5 (65^3 nodes) runs the element loop on the flagged macros' elements,
    # with stored blocks (k_block_products + k_cube with blocks) or with the descendant
    # mean as their coefficient
    from paper_2511_13109_amd import Hierarchy, macro_gradient
    L, NC = 6, 3
    print(f"\n[macro flags 129^3, element-loop coarse level, {storage}]", flush=True)
    w = workload("sinker129")
    field = w.make_field()
    nu = [field.nu(element_centroids(l)) for l in range(L + 1)]
    g = macro_gradient(L, torch.from_numpy(field.nu(_node_xyz(L))).cuda())
    mf = np.zeros(48, dtype=bool)
    mf[np.argsort(-g)[:12]] = True                 # the 12 macros with the steepest gradient
    G = Hierarchy(L, NC, torch.from_numpy(nu[L]).cuda(), [torch.from_numpy(v).cuda() for v in nu[:L]],
                  flag_mode="macro", macro_flags=mf, coarse_storage=storage)
    try:
        level = 5
        assert G.query(level)["flagged"] == 12 * 8 ** level
        n = 2 ** (level + 1)
        nn = (n + 1) ** 3
        rng = np.random.default_rng(5)
        u = rng.standard_normal(NC * nn)
        v = G.apply(level, torch.from_numpy(u).cuda()).cpu().numpy()
        # nodes on both sides of flagged / unflagged macro boundaries and inside
        pts = [(n // 2, n // 2, n // 2), (n // 4, n // 2, 3 * n // 4), (1, 1, 1), (n - 1, n // 3, 5)]
        pts += [tuple(rng.integers(1, n, 3)) for _ in range(4)]
        for node in pts:
            ref = sample.coarse_apply_at_node(level, L, np.array(node) / n, nu[level], nu[L], NC, u,
                                              macro_flags=mf)
            pid = node[0] + (n + 1) * (node[1] + (n + 1) * node[2])
            got = np.array([v[c * nn + pid] for c in range(NC)])
            assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), node
    finally:
        G.close()
