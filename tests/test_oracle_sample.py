"""The element-by-element oracle (used for checks at full size) against the global oracle.

Both are oracle code, but the global one assembles sparse matrices of the whole
hierarchy and is pinned by closed forms, brute force and the paper's counts;
here the point-located single elements, node stars and local Galerkin products
must reproduce its apply, load vector, flags, blocks and adjoint gradient.
"""

import numpy as np
import pytest

from oracle import adjoint, agca, fem, mesh, sample, transfer
from workloads import workload

L = 3


@pytest.fixture(scope="module")
def case():
    levels = mesh.hierarchy(L)
    w = workload("sinker129", L=L)
    field = w.make_field()
    nu = [field.nu(mesh.centroids_canonical(levels[l])) for l in range(L + 1)]
    return levels, field, nu


def test_node_star_and_apply(case):
    levels, field, nu = case
    nc = 3
    n = levels[L].n
    nn = (n + 1) ** 3
    rng = np.random.default_rng(1)
    u = rng.standard_normal(nc * nn)
    fm = np.zeros(nc * nn, bool)
    fm[fem.free_dofs(levels[L], nc)] = True
    v = fem.assemble(levels[L], nu[L], nc) @ np.where(fm, u, 0.0)
    for node in [(1, 1, 1), (3, 5, 7), (8, 8, 8), (15, 2, 9)]:
        star = sample.elements_around(L, np.array(node) / n)
        assert len(star) == 24          # the Freudenthal star (checked via solid angles inside)
        y = sample.apply_at_node(L, np.array(node) / n, nu[L], nc, u)
        pid = node[0] + (n + 1) * (node[1] + (n + 1) * node[2])
        ref = np.array([v[c * nn + pid] for c in range(nc)])
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


def test_load_vector(case):
    levels, field, nu = case
    nc = 3
    n = levels[L].n
    nn = (n + 1) ** 3
    cen = mesh.centroids_canonical(levels[L])
    f = np.asarray(field.force(cen, nc))
    b = fem.load_vector(levels[L], f, nc)
    fT = f.T                               # (ncomp, elements)
    for node in [(2, 3, 4), (9, 9, 9)]:
        y = sample.load_at_node(L, np.array(node) / n, fT, nc)
        pid = node[0] + (n + 1) * (node[1] + (n + 1) * node[2])
        ref = np.array([b[c * nn + pid] for c in range(nc)])
        assert np.abs(y - ref).max() <= 1e-14 + 1e-13 * np.abs(ref).max()


def test_flags_and_blocks(case):
    levels, field, nu = case
    nc = 3
    Ps = transfer.prolongations(levels, nc)
    rng = np.random.default_rng(2)
    for l in range(L):
        flags = agca.flags(levels, nu[L], l)
        for p in rng.random((4, 3)):
            eid, fl = sample.flag_at_point(l, L, p, nu[L])
            assert fl == bool(flags[eid])
            eid, B = sample.block_at_point(l, L, p, nu[L], nc)
            ref = agca.local_gca_blocks(levels, Ps, nu[L], nc, l, np.array([eid]))[0]
            assert np.abs(B - ref).max() <= 1e-13 * np.abs(ref).max()


def test_gradient(case):
    levels, field, nu = case
    nc = 3
    n = levels[L].n
    nn = (n + 1) ** 3
    rng = np.random.default_rng(3)
    u = rng.standard_normal(nc * nn)
    w = rng.standard_normal(nc * nn)
    g = adjoint.grad_log_nu(levels[L], nu[L], nc, u, w)
    for p in rng.random((6, 3)):
        eid, ge = sample.grad_at_point(L, p, nu[L], nc, u, w)
        assert abs(ge - g[eid]) <= 1e-13 * np.abs(g).max()


def test_coarse_apply(case):
    levels, field, nu = case
    nc = 3
    Ps = transfer.prolongations(levels, nc)
    ops = agca.agca_operators(levels, Ps, nu, nc)["ops"]
    for l in (1, 2):
        n = levels[l].n
        nn = (n + 1) ** 3
        rng = np.random.default_rng(4)
        u = rng.standard_normal(nc * nn)
        free = fem.free_dofs(levels[l], nc)
        fm = np.zeros(nc * nn, bool)
        fm[free] = True
        v = np.zeros(nc * nn)
        v[free] = fem.restrict_free(ops[l], free) @ u[free]
        for node in [(1, 1, 1), (n // 2, n // 2 - 1, n // 2), (n - 1, 1, n // 2)]:
            y = sample.coarse_apply_at_node(l, L, np.array(node) / n, nu[l], nu[L], nc, u)
            pid = node[0] + (n + 1) * (node[1] + (n + 1) * node[2])
            ref = np.array([v[c * nn + pid] for c in range(nc)])
            assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def test_input_centroids_are_geometric():
    from workloads.lattice import element_centroids
    for l in range(3):
        assert np.array_equal(element_centroids(l), mesh.centroids_canonical(mesh.hierarchy(l)[l]))


def test_stokes_rows(case):
    # the element-by-element divergence, its transpose and the 1/nu pressure mass (support
    # of one pressure hat, interpolation on the pressure level) against the global oracle
    # (B = -P^T B_L assembled over all elements, m = P^T m_L)
    from oracle import stokes
    levels, field, nu = case
    coarse, fine = levels[L - 1], levels[L]
    n, nc_n = fine.n, coarse.n
    nn, npn = (n + 1) ** 3, (nc_n + 1) ** 3
    rng = np.random.default_rng(4)
    u = rng.standard_normal(3 * nn)
    fm = np.zeros(3 * nn, bool)
    fm[fem.free_dofs(fine, 3)] = True
    B = stokes.div_matrix(coarse, fine)
    q = B @ np.where(fm, u, 0.0)
    p = rng.standard_normal(npn)
    v = B.T @ p
    m = stokes.lumped_mass(coarse, fine, nu[L])
    for node in [(1, 1, 1), (2, 5, 3), (4, 4, 4), (7, 1, 6)]:         # pressure nodes
        k = node[0] + (nc_n + 1) * (node[1] + (nc_n + 1) * node[2])
        x = np.array(node) / nc_n
        assert abs(sample.div_at_pressure_node(L, x, u) - q[k]) <= 1e-13 * np.abs(q).max()
        assert abs(sample.mass_at_pressure_node(L, x, nu[L]) - m[k]) <= 1e-13 * m[k]
    for node in [(1, 1, 1), (3, 5, 7), (8, 8, 8), (15, 2, 9)]:        # velocity nodes
        j = node[0] + (n + 1) * (node[1] + (n + 1) * node[2])
        got = sample.grad_at_velocity_node(L, np.array(node) / n, p)
        ref = np.array([v[c * nn + j] for c in range(3)])
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(v).max(), node
