"""The library's per-cell arithmetic (csrc/kuhn.h, cube_math.h, gca_math.h) and its
solver stopping rule (csrc/stop_rule.h), compiled for the host with g++ and compared
with the CPU oracle: element matrices of eq. (2.3) / (3.5), the element energy form of
the adjoint gradient, the Galerkin blocks of the element-wise recursion (2.7), and the
decisions of the rounding-floor stop."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import agca, mesh, transfer
from workloads import Sinkers

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2511_13109_amd", "csrc")
# axis step order of the Kuhn simplex s (canonical element id, Section 2.1 refinement)
ORDERS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("host") / "host_math")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Wno-unknown-pragmas", "-Werror", "-I", CSRC,
                    os.path.join(HERE, "host_math.cpp"), "-o", out], check=True)
    return out


def _run(exe, text):
    r = subprocess.run([exe], input=text, capture_output=True, text=True, check=True)
    return np.array([float(v) for v in r.stdout.split()])


@pytest.mark.parametrize("ncomp", [1, 3])
def test_element_matrices(exe, ncomp):
    M = 4 * ncomp
    got = _run(exe, f"elem {ncomp}\n").reshape(6, M, M)
    h = 0.125
    for s, order in enumerate(ORDERS):
        ref = agca.unit_element_matrix_path(h, ncomp, order)
        assert np.abs(got[s] * h / 6.0 - ref).max() <= 1e-14 * np.abs(ref).max(), s


@pytest.mark.parametrize("ncomp", [1, 3])
def test_element_energy(exe, ncomp):
    rng = np.random.default_rng(ncomp)
    U = rng.standard_normal((8, ncomp))
    W = rng.standard_normal((8, ncomp))
    txt = f"energy {ncomp} " + " ".join(f"{v:.17g}" for v in np.concatenate([U.ravel(), W.ravel()]))
    got = _run(exe, txt)
    h = 1.0
    for s, order in enumerate(ORDERS):
        K = agca.unit_element_matrix_path(h, ncomp, order) * 6.0 / h
        corners = [0]
        for ax in order:
            corners.append(corners[-1] | (1 << ax))
        u = np.concatenate([U[corners, c] for c in range(ncomp)])
        w = np.concatenate([W[corners, c] for c in range(ncomp)])
        assert got[s] == pytest.approx(u @ K @ w, rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("ncomp,l", [(1, 0), (1, 1), (3, 0), (3, 1)])
def test_galerkin_blocks(exe, ncomp, l):
    L = 2
    levels = mesh.hierarchy(L)
    field = Sinkers(3, 2, radius=0.2, width=0.05, contrast=1e6)
    nu = field.nu(mesh.centroids_canonical(levels[L]))
    Ps = transfer.prolongations(levels, ncomp)
    rng = np.random.default_rng(l)
    ids = np.sort(rng.choice(6 * levels[l].n ** 3, 12, replace=False))
    ref = agca.local_gca_blocks(levels, Ps, nu, ncomp, l, ids)
    txt = f"gca {ncomp} {l} {L} {ids.size} " + " ".join(str(int(e)) for e in ids) + " " + \
        " ".join(f"{v:.17g}" for v in nu)
    M = 4 * ncomp
    got = _run(exe, txt).reshape(ids.size, M, M)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def _stop(exe, tol, rho, checks):
    """checks: (true residual, iteration, full period) of each replacement above tol."""
    txt = f"stop {tol:.17g} {rho:.17g} {len(checks)} " + " ".join(
        f"{r:.17g} {it} {int(f)}" for r, it, f in checks)
    return [int(v) for v in _run(exe, txt)]


def test_stop_rule(exe):
    CONT, FLOOR, STALL = 0, 1, 2
    # a healthy phase halving every 10 iterations (full periods, to 6.25e-8 at it 50), then
    # stagnation at 3.4e-8 from it 52 with checks every 2 iterations: two windows of 10
    # iterations without a 10 % gain (its 62 and 72) stop it when rho is above the level
    healthy = [(1e-6 * 0.5 ** k, 10 * (k + 1), True) for k in range(5)]
    flat = [(3.4e-8 * (1 + 0.01 * (k % 3)), 50 + 2 * (k + 1), False) for k in range(40)]
    out = _stop(exe, 1e-8, 4e-8, healthy + flat)
    assert out[:15] == [CONT] * 15
    assert out[-1] == FLOOR and len(out) == 16        # the check at it 72
    # the same level above rho: six windows without progress (its 62 ... 112) give up
    out = _stop(exe, 1e-8, 2e-8, healthy + flat)
    assert out[-1] == STALL and len(out) == 5 + 31    # the check at it 112
    # a stop 75x above tol with a floor far below it is not success
    stuck = [(7.5e-7 * (1 + 0.01 * (k % 3)), 10 * (k + 1), True) for k in range(12)]
    assert _stop(exe, 1e-8, 1e-9, stuck) == [CONT] * 6 + [STALL]     # windows at its 20 ... 70
    assert _stop(exe, 1e-8, 1.6e-7, stuck)[-1] == STALL
    # a tolerance below the floor: stagnation at 1.5 x tol with rho of 2 x tol is a floor stop
    low = [(1.6e-8, 10, True), (1.5e-8, 20, True), (1.55e-8, 30, True), (1.52e-8, 40, True)]
    assert _stop(exe, 1e-8, 2e-8, low)[-1] == FLOOR
    # replacements that halve the true residual never stop, however many
    seq = [(0.5 ** k, 10 * (k + 1), True) for k in range(30)]
    assert _stop(exe, 1e-12, 2e-9, seq) == [CONT] * 30
    # a solve creeping to tol (checks every iteration, 1 % gain each, after a healthy phase
    # of 20 iterations per halving) keeps going: 10 % comes within its window
    creep = [(1e-5, 20, True), (2e-6, 40, True)] + [(1.05e-6 * 0.99 ** k, 41 + k, False) for k in range(40)]
    assert _stop(exe, 1e-6, 1e-9, creep) == [CONT] * len(creep)
    # with checks from the start (no full period yet) the window is the iteration count
    early = [(5e-7, 3, False), (4.9e-7, 4, False)] + [(4.9e-7, 6 * k, False) for k in range(1, 12)]
    out = _stop(exe, 1e-8, 1e-9, early)
    assert out[-1] == STALL and out[:-1] == [CONT] * (len(out) - 1)
    # the replacements of a measured FP32-multigrid FCG solve (513^3 sinkers, rho 7.28e-7):
    # near the floor the true residual of a replacement swings between 0.2 and 1.9 rho; the
    # solve goes two windows without progress at 1.2-1.8 rho (its 1789-1927) and keeps
    # going, reaches 0.6 rho at it 1928 and 0.2 rho at 2149, and stops there at the floor
    # two one-iteration windows later (every iteration halves the recurrence by then)
    fcg = [(4.0680e-01, 626, True), (1.8754e-01, 697, True), (8.4027e-02, 746, True),
           (4.1448e-02, 815, True), (1.4310e-02, 837, True), (7.0824e-03, 942, True),
           (3.5292e-03, 1011, True), (1.5526e-03, 1081, True), (7.4715e-04, 1138, True),
           (3.6875e-04, 1177, True), (1.7313e-04, 1263, True), (7.8038e-05, 1274, True),
           (2.6219e-05, 1378, True), (1.2500e-05, 1463, True), (9.0285e-06, 1472, False),
           (4.4383e-06, 1543, True), (2.9042e-06, 1574, False), (1.7946e-06, 1647, True),
           (1.4953e-06, 1711, False), (1.0326e-06, 1717, False), (9.1002e-07, 1718, False),
           (1.2881e-06, 1789, True), (1.1738e-06, 1840, True), (8.5659e-07, 1860, True),
           (1.2715e-06, 1927, False), (4.2877e-07, 1928, True), (9.9484e-07, 1972, False),
           (2.7801e-07, 1973, True), (2.3904e-07, 1974, False), (1.4000e-06, 2068, False),
           (2.3286e-07, 2069, True), (1.7666e-07, 2070, True), (1.2578e-06, 2147, False),
           (1.9937e-07, 2148, True), (1.4686e-07, 2149, True), (1.4866e-07, 2150, True),
           (1.4884e-07, 2151, True), (1.4825e-07, 2152, True)]
    assert _stop(exe, 1e-8, 7.28e-7, fcg) == [CONT] * 36 + [FLOOR]     # at it 2151
    # the same sequence under the earlier rule (a stall above the floor stops at once)
    # would have ended at it 1860, 1.2 rho, not converged


def test_pressure_stencil_offsets_and_probing_colours(exe):
    # csrc/zstencil.h: the 65 offsets in the oracle's order, and a probing colouring under
    # which the 65 neighbours k + o of every node k have 65 distinct colours (checked here
    # by brute force over a 9^3 lattice, every node whose whole stencil is inside)
    from oracle import stokes
    v = _run(exe, "zstencil\n").astype(int)
    offs = [tuple(t) for t in v[:65 * 3].reshape(65, 3)]
    assert offs == stokes.Z_OFFSETS
    col = v[65 * 3:].reshape(9, 9, 9)                     # [z, y, x]
    assert col.min() >= 0 and col.max() <= 64
    for z in range(2, 7):
        for y in range(2, 7):
            for x in range(2, 7):
                cs = {col[z + dz, y + dy, x + dx] for (dx, dy, dz) in offs}
                assert len(cs) == 65, (x, y, z)
