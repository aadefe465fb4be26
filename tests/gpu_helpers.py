"""Shared set-up of the GPU parity tests: the same seeded inputs for the oracle and the library."""

from __future__ import annotations

import numpy as np

from oracle import fem, mesh, mg
from workloads import AlignedCube, Sinkers

_CACHE = {}


def field_for(kind: str, L: int, seed: int = 2):
    if kind == "cube":
        return AlignedCube()
    if kind == "sinkers":
        return Sinkers(4, seed, radius=0.15, width=2.0 / 2 ** (L + 1), contrast=1e6)
    if kind == "unaligned":
        return AlignedCube(lo=11 / 24 - 1 / 8, hi=11 / 24 + 1 / 8, nu_in=1e3, nu_out=1e-3)
    raise ValueError(kind)


def oracle_case(kind: str, L: int, ncomp: int, mode: int = 0, smoother: str = "jacobi"):
    """Oracle hierarchy plus the per-level coefficients (canonical ids) for a field."""
    key = (kind, L, ncomp, mode, smoother)
    if key in _CACHE:
        return _CACHE[key]
    levels = mesh.hierarchy(L)
    field = field_for(kind, L)
    nu_levels = [field.nu(mesh.centroids_canonical(lv)) for lv in levels]
    H = mg.build(L, nu_levels, ncomp, mode=mode, levels=levels, smoother=smoother)
    _CACHE[key] = (H, nu_levels, field)
    return _CACHE[key]


def interior_full(H, l: int) -> np.ndarray:
    """Mask over all dofs (ncomp blocks of (n+1)^3) that are free."""
    m = np.zeros(H.ncomp * (H.levels[l].n + 1) ** 3, dtype=bool)
    m[H.free[l]] = True
    return m


def oracle_apply_full(H, l: int, u_full: np.ndarray) -> np.ndarray:
    """Free-DoF operator applied to a full vector (boundary input ignored, output zero)."""
    m = interior_full(H, l)
    out = np.zeros_like(u_full)
    out[m] = H.A[l] @ u_full[m]
    return out


def rand_full(H, l: int, rng) -> np.ndarray:
    v = rng.standard_normal(H.ncomp * (H.levels[l].n + 1) ** 3)
    return v * interior_full(H, l)


def rel_err(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / den)


def vcycle_extended(H, b_free: np.ndarray) -> np.ndarray:
    """The oracle's V-cycle (mg.vcycle, the same steps) evaluated in 80-bit extended
    precision: every level matrix, interpolation and diagonal converted to np.longdouble
    (the 1x1 / 3x3 level-0 solve stays FP64).  Used to measure how far one FP64
    V-cycle, the oracle's or the library's, lands from the exact one."""
    import copy
    E = copy.copy(H)
    E.A = [a.astype(np.longdouble) for a in H.A]
    E.P = [p.astype(np.longdouble) for p in H.P]
    E.D = [d.astype(np.longdouble) for d in H.D]
    return mg.vcycle(E, np.asarray(b_free, dtype=np.longdouble))


def vcycle_errors(H, b_full: np.ndarray, x_gpu_full: np.ndarray):
    """(library error, oracle FP64 error, tolerance) of one V-cycle, each relative to the
    extended-precision V-cycle (max-norm).  The tolerance is 1e-12, or 4x the oracle's own
    FP64 error where the cycle's cancellations make that larger: both are FP64
    evaluations of the same steps, in different summation orders."""
    m = interior_full(H, H.L)
    ext = vcycle_extended(H, b_full[m])
    x64 = mg.vcycle(H, b_full[m])
    den = float(np.abs(ext).max())
    e_gpu = float(np.abs(x_gpu_full[m] - ext).max()) / den
    e_orc = float(np.abs(x64 - ext).max()) / den
    return e_gpu, e_orc, max(1e-12, 4.0 * e_orc)
