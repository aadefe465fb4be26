"""Pins of transfers, flags and DCA/GCA/AGCA operators (paper Sections 2.1-2.3, eqs. (2.4)-(2.9)).

Independent facts used: interpolation reproduces constants and linear functions
exactly; its entries are the hat-function values 0, 1/2, 1; DCA equals GCA when
the coefficient is constant on every coarse element (Section 2.1 and Section
4.2, eta_1); the closed form of a local Galerkin block for linear interpolation
of P1 functions (mean finest coefficient times the unit element matrix, derived
from grad of a linear function being constant); flag counts derived from the
geometry of the aligned and unaligned cubes (and the 24/48 count printed in the
Figure 9 caption); brute-force descendant sets by point containment.
"""

import os

import numpy as np
import pytest

from oracle import agca, fem, mesh, transfer
from workloads import AlignedCube

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def h3():
    levels = mesh.hierarchy(3)
    return levels, transfer.prolongations(levels, 1)


def _node_coords(lv):
    X = np.empty(((lv.n + 1) ** 3, 3))
    X[lv.node_id] = lv.coords
    return X


def test_prolongation_exact_on_linear_functions(h3):
    levels, Ps = h3
    for l in range(3):
        P = Ps[l]
        Xc, Xf = _node_coords(levels[l]), _node_coords(levels[l + 1])
        assert np.allclose(P @ np.ones(P.shape[1]), 1.0, atol=1e-15)
        for d in range(3):
            assert np.allclose(P @ Xc[:, d], Xf[:, d], atol=1e-15)
        vals = np.unique(np.round(P.data, 15))
        assert set(vals.tolist()) <= {0.5, 1.0}
        # interior fine nodes: 1 parent (even) or 2 parents (odd)
        nnz = np.diff(P.indptr)
        assert set(nnz.tolist()) <= {1, 2}


def _coarse_const_nu(levels, l, rng):
    """Random coefficient constant on each level-l element: fine values and level-l values."""
    L = len(levels) - 1
    Tl = levels[l].tets.shape[0]
    nu_l = np.exp(rng.uniform(-5, 5, Tl))
    anc = mesh.ancestor(levels, l, L)
    nu_f = np.empty(levels[L].tets.shape[0])
    nu_f[levels[L].elem_id] = nu_l[levels[l].elem_id[anc]]
    return nu_f, nu_l


@pytest.mark.parametrize("ncomp", [1, 3])
def test_dca_equals_gca_for_coarse_constant_coefficient(h3, ncomp):
    levels, _ = h3
    Ps = transfer.prolongations(levels, ncomp)
    rng = np.random.default_rng(5)
    for l in range(0, 3):
        nu_f, nu_l = _coarse_const_nu(levels, l, rng)
        G = agca.gca_operator(levels, Ps, nu_f, ncomp, l)
        D = fem.assemble(levels[l], nu_l, ncomp)
        assert abs(G - D).max() <= 1e-12 * abs(D).max()


def _edge_grad_unit_matrix(V, ncomp):
    """Unit-coefficient element matrix from edge-matrix gradients (independent formula)."""
    E = V[1:] - V[:1]
    Einv = np.linalg.inv(E)
    g = np.empty((4, 3))
    g[1:] = Einv.T
    g[0] = -g[1:].sum(axis=0)
    vol = abs(np.linalg.det(E)) / 6.0
    if ncomp == 1:
        return vol * g @ g.T
    K = np.zeros((3, 4, 3, 4))
    for c in range(3):
        for d in range(3):
            K[c, :, d, :] = vol * ((g @ g.T) * (c == d) + np.outer(g[:, d], g[:, c]))
    return K.reshape(12, 12)


@pytest.mark.parametrize("ncomp", [1, 3])
def test_local_gca_block_closed_form(h3, ncomp):
    """block(m) = (mean of finest nu over m's descendants) * unit element matrix of m."""
    levels, _ = h3
    Ps = transfer.prolongations(levels, ncomp)
    L = 3
    rng = np.random.default_rng(7)
    nu = np.exp(rng.uniform(np.log(1e-3), np.log(1e3), levels[L].tets.shape[0]))
    for l in range(L):
        T = levels[l].tets.shape[0]
        elems = rng.choice(T, size=min(T, 12), replace=False)
        B = agca.local_gca_blocks(levels, Ps, nu, ncomp, l, elems)
        anc = mesh.ancestor(levels, l, L)
        pv = agca.path_order(levels[l])
        inv = np.empty(T, dtype=np.int64)
        inv[levels[l].elem_id] = np.arange(T)
        for k, e in enumerate(elems):
            d = levels[L].elem_id[anc == inv[e]]
            assert d.size == 8 ** (L - l)
            K1 = _edge_grad_unit_matrix(levels[l].coords[pv[inv[e]]], ncomp)
            ref = nu[d].mean() * K1
            assert np.abs(B[k] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("ncomp", [1, 3])
def test_local_blocks_sum_to_global_masked_galerkin(h3, ncomp):
    """Assembling the local blocks of a set of coarse elements reproduces Pi^T A_L(mask) Pi."""
    levels, _ = h3
    Ps = transfer.prolongations(levels, ncomp)
    L = 3
    rng = np.random.default_rng(8)
    nu = np.exp(rng.uniform(-4, 4, levels[L].tets.shape[0]))
    l = 1
    T = levels[l].tets.shape[0]
    sel = np.zeros(T, dtype=bool)
    sel[rng.choice(T, 40, replace=False)] = True
    elems = np.nonzero(sel)[0]
    B = agca.local_gca_blocks(levels, Ps, nu, ncomp, l, elems)
    nnc = (levels[l].n + 1) ** 3
    inv = np.empty(T, dtype=np.int64)
    inv[levels[l].elem_id] = np.arange(T)
    pv = agca.path_order(levels[l])
    G = np.zeros((ncomp * nnc, ncomp * nnc))
    for k, e in enumerate(elems):
        nid = levels[l].node_id[pv[inv[e]]]
        dofs = np.concatenate([c * nnc + nid for c in range(ncomp)])
        G[np.ix_(dofs, dofs)] += B[k]
    from oracle.transfer import composite
    Pi = composite(Ps, l, L)
    Af = fem.assemble(levels[L], nu, ncomp, elem_mask=agca.fine_mask_under(levels, sel, l))
    ref = (Pi.T @ Af @ Pi).toarray()
    assert np.abs(G - ref).max() <= 1e-12 * np.abs(ref).max()


def _brute_flags(levels, nu_fine, l, tau=10.0):
    """Descendants by centroid containment (barycentric test), then max > tau * min."""
    L = len(levels) - 1
    cen = mesh.centroids_canonical(levels[L])
    lv = levels[l]
    out = np.zeros(lv.tets.shape[0], dtype=bool)
    for k in range(lv.tets.shape[0]):
        V = lv.coords[lv.tets[k]]
        M = np.ones((4, 4))
        M[1:, :] = V.T
        lam = np.linalg.solve(M, np.vstack([np.ones(cen.shape[0]), cen.T]))
        inside = np.all(lam > 1e-12, axis=0)
        assert inside.sum() == 8 ** (L - l)
        v = nu_fine[inside]
        out[lv.elem_id[k]] = v.max() > tau * v.min()
    return out


def test_flags_brute_force_and_monotone(h3):
    levels, _ = h3
    rng = np.random.default_rng(9)
    L = 3
    nu = np.exp(rng.normal(0, 1.0, levels[L].tets.shape[0]))
    for l in range(L):
        f = agca.flags(levels, nu, l)
        assert np.array_equal(f, _brute_flags(levels, nu, l))
    # monotone: a flagged child has a flagged parent
    for l in range(1, L):
        fc, fp = agca.flags(levels, nu, l), agca.flags(levels, nu, l - 1)
        lv = levels[l]
        par = levels[l - 1].elem_id[lv.parent]
        assert np.all(fp[par[fc[lv.elem_id]]])


def test_flag_counts_aligned_cube(h3):
    """Aligned cube [0.375, 0.625]^3 on 17^3 nodes: 24/48, 24/384, 0/3072 flagged."""
    levels, _ = h3
    nu = AlignedCube().nu(mesh.centroids_canonical(levels[3]))
    counts = [int(agca.flags(levels, nu, l).sum()) for l in range(3)]
    assert counts == [24, 24, 0]


def test_flag_count_unaligned_cube_macro_level():
    """Figure 9 caption: the unaligned cube cuts 24 of the 48 macro elements."""
    vals = {}
    with open(os.path.join(GOLD, "fig9_gca_macros.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    c, r = vals["centre"], vals["half_width"]
    levels = mesh.hierarchy(3)
    cube = AlignedCube(lo=c - r, hi=c + r, nu_in=1e3, nu_out=1e-3)
    nu = cube.nu(mesh.centroids_canonical(levels[3]))
    f0 = agca.flags(levels, nu, 0)
    assert f0.size == int(vals["macro_elements"])
    assert int(f0.sum()) == int(vals["gca_macro_elements"])


def test_agca_modes_reduce_to_dca_and_gca(h3):
    levels, _ = h3
    ncomp = 1
    Ps = transfer.prolongations(levels, ncomp)
    rng = np.random.default_rng(11)
    L = 3
    nu_levels = [np.exp(rng.uniform(-3, 3, lv.tets.shape[0])) for lv in levels]
    none = agca.agca_operators(levels, Ps, nu_levels, ncomp, mode=agca.FLAG_NONE)["ops"]
    allg = agca.agca_operators(levels, Ps, nu_levels, ncomp, mode=agca.FLAG_ALL)["ops"]
    for l in range(L):
        D = fem.assemble(levels[l], nu_levels[l], ncomp)
        G = agca.gca_operator(levels, Ps, nu_levels[L], ncomp, l)
        assert abs(none[l] - D).max() <= 1e-13 * abs(D).max()
        assert abs(allg[l] - G).max() <= 1e-12 * abs(G).max()
