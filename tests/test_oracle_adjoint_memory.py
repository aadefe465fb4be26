"""Pins of the oracle's adjoint gradient and of the memory model (paper Section 5).

Adjoint: central finite differences of J(log nu) with exact sparse solves, and
the homogeneity identity sum_e dJ/dlog nu_e = -(u - u_obs) . u, which follows
from A(alpha nu) = alpha A(nu).
Memory: the constants printed in Section 5 (golden file).
"""

import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import adjoint, fem, memory, mesh
from workloads import GaussianLogField

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _problem(L, ncomp):
    lv = mesh.hierarchy(L)[L]
    g = GaussianLogField(seed=4)
    cen = mesh.centroids_canonical(lv)
    g.calibrate(cen)
    log_nu = g.log_nu(cen)
    f = g.force(cen, ncomp)
    b = fem.load_vector(lv, f, ncomp)
    free = fem.free_dofs(lv, ncomp)
    log_nu_obs = log_nu + g.noise(log_nu.size)

    def solve(lnu):
        A = fem.restrict_free(fem.assemble(lv, np.exp(lnu), ncomp), free)
        u = np.zeros(b.size)
        u[free] = spla.splu(A.tocsc()).solve(b[free])
        return u, A

    u_obs, _ = solve(log_nu_obs)
    return lv, log_nu, u_obs, solve, free


def _J(u, u_obs):
    return 0.5 * float(((u - u_obs) ** 2).sum())


@pytest.mark.parametrize("ncomp", [1, 3])
def test_adjoint_gradient_matches_finite_differences(ncomp):
    lv, log_nu, u_obs, solve, free = _problem(2, ncomp)
    u, A = solve(log_nu)
    w = np.zeros_like(u)
    w[free] = spla.splu(A.tocsc()).solve((u - u_obs)[free])
    g = adjoint.grad_log_nu(lv, np.exp(log_nu), ncomp, u, w)
    # homogeneity
    assert abs(g.sum() + (u - u_obs) @ u) <= 1e-10 * abs((u - u_obs) @ u)
    rng = np.random.default_rng(0)
    eps = 1e-5
    for e in rng.choice(log_nu.size, 6, replace=False):
        d = np.zeros_like(log_nu)
        d[e] = eps
        fd = (_J(solve(log_nu + d)[0], u_obs) - _J(solve(log_nu - d)[0], u_obs)) / (2 * eps)
        assert abs(fd - g[e]) <= 1e-6 * np.abs(g).max()
    for _ in range(2):
        d = rng.standard_normal(log_nu.size) * eps
        fd = (_J(solve(log_nu + d)[0], u_obs) - _J(solve(log_nu - d)[0], u_obs)) / 2.0
        assert abs(fd - g @ d) <= 1e-6 * abs(g @ d) + 1e-14


def _golden():
    vals = {}
    with open(os.path.join(GOLD, "memory_constants.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, v = line.split()[:2]
                vals[name] = float(v)
    return vals


def test_memory_constants_reproduce_section5():
    g = _golden()
    # the paper evaluates with c_u rounded to 0.95; exact limit 23/24 within 1.5 %
    c = g["c_u"]
    assert abs(memory.mem_A_L(c) - g["mem_A_L"]) < 0.05
    assert abs(memory.mem_K_L(c) - g["mem_K_L"]) < 0.06
    assert abs(memory.mem_gca_sparse(c_u=c) - g["mem_gca_sparse"]) < 0.01
    assert abs(memory.mem_gca_all_elements(c) - g["mem_gca_all_elements"]) < 0.25
    assert abs(memory.mem_agca_stencil() - g["mem_agca_stencil"]) < 0.05
    assert abs(float(memory.c_u_limit()) - c) < 0.01
    assert abs(memory.cells_per_vertex(4096) - g["cells_per_vertex"]) < 0.01
    # (5.1) at finite size approaches its limit
    assert abs(memory.c_u_at(512) - float(memory.c_u_limit())) < 1e-3
