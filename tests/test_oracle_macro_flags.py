"""Pins of the oracle's macro-granularity gradient flag (paper eq. (2.8), Section 4.3
and Fig. 9) and of AGCA with macro flags (eq. (2.9)).

* The P1 interpolant of a linear function is the function itself: every finest
  element has gradient a, so every macro maximum is |a| (closed form).
* A sharp cube [1/3, 7/12]^3 (faces off the dyadic lattice) gives a non-zero
  gradient exactly on the 24 macro elements it meets: a Kuhn simplex of a macro
  cube meets an axis-aligned box iff its step order puts the box's "high" axes
  first, which gives 6 + 6 + 3*2 + 3*2 = 24 of 48 (Fig. 9's count).
* Macro flags reach every descendant: #flagged(level l) = #flagged macros * 8^l.
* All macros flagged reproduces pure Galerkin coarsening, none reproduces DCA.
"""

import os

import numpy as np
import pytest

from oracle import agca, mesh, transfer


def _nodes(level):
    X = np.empty((level.coords.shape[0], 3))
    X[level.node_id] = level.coords
    return X


@pytest.mark.parametrize("L", [1, 3])
def test_linear_field_has_constant_gradient(L):
    levels = mesh.hierarchy(L)
    a = np.array([0.3, -1.7, 2.2])
    eta = _nodes(levels[L]) @ a + 5.0
    g = agca.macro_gradient_max(levels, eta)
    assert g.shape == (48,)
    assert np.allclose(g, np.linalg.norm(a), rtol=1e-12, atol=0)


def _fig9():
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "fig9_gca_macros.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


@pytest.mark.parametrize("L", [2, 3, 4])
def test_sharp_unaligned_cube_meets_24_of_48_macros(L):
    fig9 = _fig9()
    lo, hi = fig9["centre"] - fig9["half_width"], fig9["centre"] + fig9["half_width"]
    levels = mesh.hierarchy(L)
    X = _nodes(levels[L])
    inside = np.all((X > lo) & (X < hi), axis=1)
    g = agca.macro_gradient_max(levels, np.where(inside, 1e3, 1.0))
    assert g.size == int(fig9["macro_elements"])
    assert int((g > 0).sum()) == int(fig9["gca_macro_elements"])
    # the flagged macros are the ones whose centroid-side of the box is right:
    # a macro meets the box iff it holds a node inside it
    lv0 = levels[0]
    anc = mesh.ancestor(levels, 0, L)
    has_inside = np.zeros(48, dtype=bool)
    fine = levels[L]
    np.logical_or.at(has_inside, lv0.elem_id[anc], inside[fine.node_id[fine.tets]].any(axis=1))
    assert np.array_equal(g > 0, has_inside)


def test_macro_flags_reach_every_descendant():
    L = 3
    levels = mesh.hierarchy(L)
    rng = np.random.default_rng(1)
    mf = rng.random(48) < 0.4
    for l in range(L + 1):
        f = agca.flags(levels, None, l, mode=agca.FLAG_MACRO, macro_flags=mf)
        assert int(f.sum()) == int(mf.sum()) * 8 ** l
    # consistency with the parent relation one level up
    for l in range(1, L + 1):
        f = agca.flags(levels, None, l, mode=agca.FLAG_MACRO, macro_flags=mf)
        fp = agca.flags(levels, None, l - 1, mode=agca.FLAG_MACRO, macro_flags=mf)
        par = levels[l - 1].elem_id[levels[l].parent]          # canonical parent per Bey child
        assert np.array_equal(f[levels[l].elem_id], fp[par])


def test_macro_of_an_element_contains_its_centroid():
    # brute force: barycentric coordinates of every level-2 centroid in all 48 macros
    L = 2
    levels = mesh.hierarchy(L)
    lv0 = levels[0]
    cen = mesh.centroids_canonical(levels[L])
    owner = -np.ones(cen.shape[0], dtype=np.int64)
    for t in range(48):
        V = lv0.coords[lv0.tets[t]]
        T = np.vstack([V[1:] - V[0]]).T
        lam = np.linalg.solve(T, (cen - V[0]).T).T
        inside = np.all(lam > 1e-12, axis=1) & (lam.sum(axis=1) < 1 - 1e-12)
        assert (owner[inside] == -1).all()
        owner[inside] = lv0.elem_id[t]
    assert (owner >= 0).all()
    for k in range(48):
        mf = np.zeros(48, dtype=bool)
        mf[k] = True
        f = agca.flags(levels, None, L, mode=agca.FLAG_MACRO, macro_flags=mf)
        assert np.array_equal(f, owner == k)


@pytest.mark.parametrize("ncomp", [1, 3])
def test_all_or_no_macros_reproduce_gca_and_dca(ncomp):
    L = 2
    levels = mesh.hierarchy(L)
    rng = np.random.default_rng(2)
    nu = [np.exp(rng.uniform(-2, 2, lv.tets.shape[0])) for lv in levels]
    Pf = transfer.prolongations(levels, ncomp)
    for mf, mode in ((np.ones(48, bool), agca.FLAG_ALL), (np.zeros(48, bool), agca.FLAG_NONE)):
        a = agca.agca_operators(levels, Pf, nu, ncomp, mode=agca.FLAG_MACRO, macro_flags=mf)
        b = agca.agca_operators(levels, Pf, nu, ncomp, mode=mode)
        for l in range(L + 1):
            assert abs(a["ops"][l] - b["ops"][l]).max() == 0.0
