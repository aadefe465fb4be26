"""Pins of the oracle's geometric multigrid for the BFBT operator Z = B W^-1 B^T
(eq. (4.2)) on the pressure lattice.

Z and its Galerkin coarsenings must keep the constant pressure in their kernel (B^T 1
= 0 by the divergence theorem, and P 1 = 1), couple only the 65 offsets that two Kuhn
edges reach, and match the 27-node brute-force product of the composite
interpolation; the stencil form must reproduce the sparse products; the coarse solve
must be the minimal-norm solution (pseudo-inverse); the V-cycle must be symmetric and
contract the Z-energy error; and CG with it must reach the zero-mean solution (a
grounded sparse LU solve) that the exact BFBT needs.
"""

import numpy as np
import pytest

from oracle import fem, mesh, mg, stokes, transfer


def _system(L, contrast=1e4):
    from workloads import Sinkers
    levels = mesh.hierarchy(L)
    field = Sinkers(3, 3, radius=0.2, width=2.0 / 2 ** (L + 1), contrast=contrast)
    nu = [field.nu(mesh.centroids_canonical(lv)) for lv in levels]
    H = mg.build(L, nu, 3, levels=levels)
    return stokes.StokesSystem(H)


@pytest.fixture(scope="module")
def sys4():
    return _system(4)


@pytest.fixture(scope="module")
def zh4(sys4):
    return stokes.ZHierarchy(sys4)


def _grounded_solve(Z, r):
    """The zero-mean solution of Z y = r (r of zero sum, Z's kernel the constants): fix
    y_0 = 0, solve the rest by sparse LU, remove the mean."""
    import scipy.sparse.linalg as spla
    Zr = Z[1:, 1:].tocsc()
    y = np.zeros(Z.shape[0])
    y[1:] = spla.splu(Zr).solve(r[1:])
    return y - y.mean()


def test_offsets_are_sums_of_two_kuhn_edges():
    # the Kuhn lattice edges: offsets in {0,1}^3 or {0,-1}^3 (15 with zero)
    K = {(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)}
    K |= {(-a, -b, -c) for (a, b, c) in K}
    sums = {(a[0] + b[0], a[1] + b[1], a[2] + b[2]) for a in K for b in K}
    assert len(K) == 15 and len(sums) == 65
    assert sums == set(stokes.Z_OFFSETS)
    assert stokes.Z_OFFSETS[32] == (0, 0, 0)       # the centre is the middle offset
    assert all((-a, -b, -c) in sums for (a, b, c) in sums)


def test_levels_keep_constants_and_the_stencil(zh4):
    for l, Z in enumerate(zh4.Z):
        n = zh4.levels[l].n
        assert Z.shape[0] == (n + 1) ** 3
        d = zh4.D[l]
        assert d.min() > 0
        assert np.abs(Z @ np.ones(Z.shape[0])).max() <= 1e-12 * d.max()
        assert abs(Z - Z.T).max() <= 1e-14 * d.max()
        st = zh4.stencil(l)                            # raises on an offset outside the 65
        x = np.random.default_rng(l).standard_normal(Z.shape[0])
        assert np.allclose(stokes.stencil_apply(st, n, x), Z @ x, rtol=0, atol=1e-13 * d.max())


def test_galerkin_levels_equal_the_composite_product(zh4):
    # Z_0 computed level by level equals P0^T Z_top P0 with P0 the composite
    # interpolation, built here column by column from the nodal values of the coarse
    # hats on the fine lattice (a hat is affine on each coarse tet)
    lv0, top = zh4.levels[0], zh4.levels[-1]
    nf = top.n + 1
    P0 = np.zeros((nf ** 3, 27))
    C = lv0.coords[lv0.tets]
    M = np.ones((C.shape[0], 4, 4))
    M[:, 1:, :] = C.transpose(0, 2, 1)
    Minv = np.linalg.inv(M)
    p = np.arange(nf ** 3)
    X = np.stack([p % nf, (p // nf) % nf, p // nf ** 2], 1) / top.n
    for k in range(X.shape[0]):
        lam = Minv @ np.concatenate([[1.0], X[k]])      # barycentrics in every coarse tet
        t = int(np.argmax(lam.min(axis=1)))             # a tet containing the point
        P0[k, lv0.node_id[lv0.tets[t]]] = lam[t]
    ref = P0.T @ (zh4.Z[-1] @ P0)
    assert np.allclose(zh4.Z[0].toarray(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_coarse_solve_is_the_pseudo_inverse(zh4):
    Z0 = zh4.Z[0].toarray()
    assert np.linalg.matrix_rank(Z0, tol=1e-10 * np.abs(Z0).max()) == 26
    assert np.allclose(zh4.coarse_inv, np.linalg.pinv(Z0), rtol=0, atol=1e-10 * np.abs(zh4.coarse_inv).max())


def test_vcycle_symmetric_and_contracting(zh4):
    n = zh4.Z[-1].shape[0]
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal((2, n))
    assert abs(u @ zh4.vcycle(v) - v @ zh4.vcycle(u)) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(zh4.vcycle(v))
    # error propagation E = I - V Z on the mean-zero space: its Z-energy norm, by power
    # iteration, is well below 1
    Z = zh4.Z[-1]
    e = rng.standard_normal(n)
    e -= e.mean()
    rho = 0.0
    for _ in range(30):
        e2 = e - zh4.vcycle(Z @ e)
        e2 -= e2.mean()
        rho = np.sqrt((e2 @ (Z @ e2)) / (e @ (Z @ e)))
        e = e2 / np.sqrt(e2 @ (Z @ e2))
    print(f"V-cycle energy contraction {rho:.3f}")
    assert rho < 0.7


def test_mg_cg_reaches_the_zero_mean_solution(sys4, zh4):
    Z = zh4.Z[-1]
    rng = np.random.default_rng(4)
    r = rng.standard_normal(Z.shape[0])
    r -= r.mean()
    y = zh4.z_solve(12)(r)
    assert np.linalg.norm(Z @ y - r) <= 1e-9 * np.linalg.norm(r)
    yp = _grounded_solve(Z, r)
    assert np.allclose(y - y.mean(), yp, rtol=0, atol=1e-8 * np.abs(yp).max())
    # fewer steps: a monotone Z-energy error, and far below Jacobi-CG's with as many

    def energy(k):
        e = zh4.z_solve(k)(r) - yp
        return float(e @ (Z @ e))
    e1 = [energy(k) for k in (1, 3, 6)]
    assert e1[0] > e1[1] > e1[2]
    ej = sys4.z_solve(6, Z)(r) - yp
    assert e1[2] < 1e-3 * float(ej @ (Z @ ej))
    assert np.array_equal(zh4.z_solve(4)(np.zeros(Z.shape[0])), np.zeros(Z.shape[0]))


def test_bfbt_mg_solves_like_the_jacobi_cg_form():
    S = _system(3, contrast=1e6)
    from workloads import Sinkers
    lv = S.H.levels[3]
    field = Sinkers(3, 3, radius=0.2, width=2.0 / 2 ** 4, contrast=1e6)
    f = np.asarray(field.force(mesh.centroids_canonical(lv), 3))
    b = np.concatenate([fem.load_vector(lv, f, 3)[S.free_u], np.zeros(S.np_)])
    its = {}
    for schur, k in (("bfbt", 20), ("bfbt_mg", 4)):
        res = S.solve(b, "fgmres", tol=1e-8, restart=50, maxit=500, precond="triangular",
                      schur=schur, schur_iters=k)
        assert res.converged
        its[schur] = res.iterations
        assert np.linalg.norm(S.K @ res.x - b) <= 1.01e-8 * np.linalg.norm(b)
    print(its)
    assert its["bfbt_mg"] <= its["bfbt"] + 2
