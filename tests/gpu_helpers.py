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
