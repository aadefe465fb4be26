"""Pins of the oracle's operator assembly (paper eqs. (2.3), (3.5)).

Independent facts used: symmetry, zero row sums of the Neumann matrix, rigid
body modes in the kernel of the symmetric-gradient form, the textbook 7-point
Laplacian for nu = 1, brute-force energies computed with a different gradient
formula, and O(h^2) nodal convergence on a manufactured solution.
"""

import numpy as np
import pytest
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem, mesh


@pytest.fixture(scope="module")
def lv2():
    return mesh.hierarchy(2)


def _lognu(rng, T):
    return np.exp(rng.uniform(np.log(1e-3), np.log(1e3), T))


@pytest.mark.parametrize("ncomp", [1, 3])
def test_symmetric_zero_rowsum(lv2, ncomp):
    lv = lv2[2]
    rng = np.random.default_rng(1)
    nu = _lognu(rng, lv.tets.shape[0])
    A = fem.assemble(lv, nu, ncomp)
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
    nn = (lv.n + 1) ** 3
    for c in range(ncomp):
        one = np.zeros(ncomp * nn)
        one[c * nn:(c + 1) * nn] = 1.0
        assert np.abs(A @ one).max() <= 1e-12 * abs(A).max()


def test_rigid_body_rotations_in_kernel(lv2):
    lv = lv2[2]
    rng = np.random.default_rng(2)
    nu = _lognu(rng, lv.tets.shape[0])
    A = fem.assemble(lv, nu, 3)
    nn = (lv.n + 1) ** 3
    X = np.empty((nn, 3))
    X[lv.node_id] = lv.coords
    for w in np.eye(3):
        u = np.cross(w, X)                                  # infinitesimal rotation
        uu = np.concatenate([u[:, 0], u[:, 1], u[:, 2]])
        assert np.abs(A @ uu).max() <= 1e-11 * abs(A).max()


def test_scalar_unit_coefficient_is_7_point_laplacian(lv2):
    """nu = 1: A on free nodes equals h * (6 on the diagonal, -1 for the 6 axis neighbours)."""
    for lv in lv2[1:]:
        n = lv.n
        h = 1.0 / n
        A = fem.restrict_free(fem.assemble(lv, np.ones(lv.tets.shape[0]), 1), fem.free_dofs(lv, 1))
        m = n - 1
        T1 = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
        I = sp.identity(m)
        lap = sp.kron(sp.kron(I, I), T1) + sp.kron(sp.kron(I, T1), I) + sp.kron(sp.kron(T1, I), I)
        assert abs(A - h * lap).max() < 1e-14


def test_unit_coefficient_dst_solution(lv2):
    """Exact solve of h * Lap7 u = b by the type-I sine transform (textbook fast Poisson)."""
    lv = mesh.hierarchy(3)[3]
    n = lv.n
    h = 1.0 / n
    free = fem.free_dofs(lv, 1)
    A = fem.restrict_free(fem.assemble(lv, np.ones(lv.tets.shape[0]), 1), free)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(free.size)
    u = spla.spsolve(A.tocsc(), b)
    m = n - 1
    k = np.arange(1, m + 1)
    lam1 = 4 * np.sin(k * np.pi / (2 * n)) ** 2
    lam = lam1[None, None, :] + lam1[None, :, None] + lam1[:, None, None]
    B = b.reshape(m, m, m)
    U = scipy.fft.idstn(scipy.fft.dstn(B, type=1) / (h * lam), type=1)
    assert np.abs(U.ravel() - u).max() <= 1e-12 * np.abs(u).max()


def _edge_gradients(V):
    """Gradients of the barycentric coordinates from the 3x3 edge matrix (not the 4x4 inverse)."""
    E = V[:, 1:, :] - V[:, :1, :]                           # rows: v_k - v_0
    Einv = np.linalg.inv(E)                                 # columns give grad l_1..l_3
    g = np.empty((V.shape[0], 4, 3))
    g[:, 1:, :] = Einv.transpose(0, 2, 1)
    g[:, 0, :] = -g[:, 1:, :].sum(axis=1)
    return g, np.abs(np.linalg.det(E)) / 6.0


@pytest.mark.parametrize("L", [1, 2])
@pytest.mark.parametrize("ncomp", [1, 3])
def test_brute_force_bilinear_form(L, ncomp):
    """u^T A v equals sum_e nu_e |e| form(grad u_h, grad v_h) evaluated element by element,
    with gradients from the edge matrix, for random u, v and random log-uniform nu."""
    lv = mesh.hierarchy(L)[L]
    rng = np.random.default_rng(10 + L)
    nu = _lognu(rng, lv.tets.shape[0])
    A = fem.assemble(lv, nu, ncomp).toarray()
    nn = (lv.n + 1) ** 3
    g, vol = _edge_gradients(lv.coords[lv.tets])
    w = nu[lv.elem_id] * vol
    for _ in range(3):
        u = rng.standard_normal(ncomp * nn)
        v = rng.standard_normal(ncomp * nn)
        total = 0.0
        for e in range(lv.tets.shape[0]):
            nid = lv.node_id[lv.tets[e]]
            Gu = np.array([[sum(u[c * nn + nid[a]] * g[e, a, d] for a in range(4))
                            for d in range(3)] for c in range(ncomp)])
            Gv = np.array([[sum(v[c * nn + nid[a]] * g[e, a, d] for a in range(4))
                            for d in range(3)] for c in range(ncomp)])
            if ncomp == 1:
                total += w[e] * float(Gu[0] @ Gv[0])
            else:
                eu = 0.5 * (Gu + Gu.T)
                ev = 0.5 * (Gv + Gv.T)
                total += w[e] * 2.0 * float((eu * ev).sum())
        assert abs(u @ A @ v - total) <= 1e-11 * (abs(total) + np.abs(A).max())


def test_kuhn_element_matrix_is_path_laplacian():
    """Scalar unit element matrix of a Kuhn simplex = (h/6) * path Laplacian of its vertices."""
    lv = mesh.hierarchy(1)[1]
    h = 1.0 / lv.n
    K = fem.element_matrices(lv, np.ones(lv.tets.shape[0]), 1)
    X = np.rint(lv.coords * lv.n)
    order = np.argsort(X[lv.tets].sum(axis=2), axis=1)
    path = (h / 6.0) * np.array([[1, -1, 0, 0], [-1, 2, -1, 0], [0, -1, 2, -1], [0, 0, -1, 1.0]])
    for e in range(K.shape[0]):
        o = order[e]
        assert np.allclose(K[e][np.ix_(o, o)], path, atol=1e-15)


def _mms(L, ncomp):
    import sympy as s
    x, y, z = s.symbols("x y z")
    X = (x, y, z)
    us = s.sin(s.pi * x) * s.sin(s.pi * y) * s.sin(s.pi * z)
    nus = 1 + s.Rational(1, 2) * s.sin(2 * s.pi * x)
    if ncomp == 1:
        fs = [-sum(s.diff(nus * s.diff(us, X[d]), X[d]) for d in range(3))]
    else:
        U = [us, us, us]
        eps = [[(s.diff(U[i], X[j]) + s.diff(U[j], X[i])) / 2 for j in range(3)] for i in range(3)]
        fs = [-sum(s.diff(2 * nus * eps[i][j], X[j]) for j in range(3)) for i in range(3)]
    f_num = [s.lambdify(X, fi, "numpy") for fi in fs]
    u_num = s.lambdify(X, us, "numpy")
    nu_num = s.lambdify(X, nus, "numpy")
    lv = mesh.hierarchy(L)[L]
    cen = mesh.centroids_canonical(lv)
    nu = nu_num(cen[:, 0], cen[:, 1], cen[:, 2])
    fe = np.stack([fi(cen[:, 0], cen[:, 1], cen[:, 2]) for fi in f_num], axis=1)
    A = fem.assemble(lv, nu, ncomp)
    free = fem.free_dofs(lv, ncomp)
    b = fem.load_vector(lv, fe if ncomp > 1 else fe[:, 0], ncomp)
    uh = spla.spsolve(fem.restrict_free(A, free).tocsc(), b[free])
    nn = (lv.n + 1) ** 3
    Xn = np.empty((nn, 3))
    Xn[lv.node_id] = lv.coords
    ue = np.concatenate([u_num(Xn[:, 0], Xn[:, 1], Xn[:, 2])] * ncomp)[free]
    return np.abs(uh - ue).max()


@pytest.mark.parametrize("ncomp,Ls", [(1, (2, 3, 4)), (3, (1, 2, 3))])
def test_manufactured_solution_second_order(ncomp, Ls):
    errs = [_mms(L, ncomp) for L in Ls]
    rates = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert rates[-1] > 3.5, (errs, rates)
    assert all(r > 2.5 for r in rates), (errs, rates)


def test_load_vector_unit_source():
    """f = 1: every free node gets sum over its 24 Kuhn cells of |e|/4 = h^3."""
    lv = mesh.hierarchy(2)[2]
    b = fem.load_vector(lv, np.ones(lv.tets.shape[0]), 1)
    free = fem.free_dofs(lv, 1)
    assert np.allclose(b[free], 1.0 / lv.n ** 3, rtol=1e-13)
