"""Viscosity and forcing fields of the sinker benchmarks, sampled at given points.

Paper, Section 3.2, eqs. (3.6)-(3.12): viscosities are built from characteristic
functions xi of cubes and balls, rescaled between eta_low = DR^-1/2 and
eta_high = DR^1/2 (3.9), and the forcing is f = (0, 0, -xi) (3.11).

Readings taken here (the paper is silent or garbled on these points):

* Several sinkers are combined as a union, xi = 1 - prod_j (1 - s_j).  Eq. (3.6)
  writes a plain product of ball indicators, which read literally would be
  their intersection (empty for separated sinkers).
* "Smoothed by a tanh of width 2h" means s_j = (1 - tanh((|x - p_j| - r_j) / w)) / 2
  with w = 2 h_L, h_L the finest mesh width.
* The random draws use numpy's PCG64 ``default_rng(seed)`` in a fixed order:
  centres first, then radii (when they are random), then anything else.

Every function takes an ``(N, 3)`` float64 array of points and returns float64
values; callers choose the points (element centroids of whatever grid they use).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

_CHUNK = 1 << 20


def _chunked(fn, pts: np.ndarray, out_cols: int = 0) -> np.ndarray:
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    n = pts.shape[0]
    out = np.empty((n,) if out_cols == 0 else (n, out_cols), dtype=np.float64)
    for s in range(0, n, _CHUNK):
        out[s:s + _CHUNK] = fn(pts[s:s + _CHUNK])
    return out


class AlignedCube:
    """Grid-aligned central cube: nu = nu_in on the closed box [lo, hi]^3, else nu_out.

    This is eta_1 of eq. (3.6)/(3.9) with the box [0.375, 0.625]^3 (half-width 1/8
    around the centre) and the levels 1 and 1e3; the forcing is the constant 1 of
    the scalar diffusion problem -div(nu grad u) = 1.
    """

    def __init__(self, lo: float = 0.375, hi: float = 0.625,
                 nu_in: float = 1e3, nu_out: float = 1.0):
        self.lo, self.hi, self.nu_in, self.nu_out = lo, hi, nu_in, nu_out

    def nu(self, pts: np.ndarray) -> np.ndarray:
        pts = np.asarray(pts, dtype=np.float64)
        inside = np.all((pts >= self.lo) & (pts <= self.hi), axis=1)
        return np.where(inside, self.nu_in, self.nu_out)

    def force(self, pts: np.ndarray, ncomp: int = 1) -> np.ndarray:
        pts = np.asarray(pts, dtype=np.float64)
        if ncomp == 1:
            return np.ones(pts.shape[0])
        f = np.zeros((pts.shape[0], ncomp))
        f[:, -1] = -1.0
        return f


class Sinkers:
    """Spherical sinkers with tanh-smoothed boundaries (eta_6 of eq. (3.6), smoothed like eta_3).

    nu = nu_lo + (nu_hi - nu_lo) * xi, f = (0, 0, -xi), xi the smoothed union of
    balls of radius r_j around centres p_j.
    """

    def __init__(self, n_sinkers: int, seed: int, radius=0.1, width: float = 2.0 / 128,
                 contrast: float = 1e6, centre_box: Tuple[float, float] = (0.2, 0.8)):
        rng = np.random.default_rng(seed)
        self.centres = rng.uniform(centre_box[0], centre_box[1], size=(n_sinkers, 3))
        if isinstance(radius, (tuple, list)):
            self.radii = rng.uniform(radius[0], radius[1], size=n_sinkers)
        else:
            self.radii = np.full(n_sinkers, float(radius))
        self.width = float(width)
        self.nu_hi = math.sqrt(contrast)        # eta_high = DR^(1/2), eq. (3.9)
        self.nu_lo = 1.0 / math.sqrt(contrast)  # eta_low  = DR^(-1/2)
        self.seed = seed

    def _xi(self, pts: np.ndarray) -> np.ndarray:
        keep = np.ones(pts.shape[0])
        for p, r in zip(self.centres, self.radii):
            d = np.sqrt(((pts - p) ** 2).sum(axis=1))
            s = 0.5 * (1.0 - np.tanh((d - r) / self.width))
            keep *= (1.0 - s)
        return 1.0 - keep

    def xi(self, pts: np.ndarray) -> np.ndarray:
        return _chunked(self._xi, pts)

    def nu(self, pts: np.ndarray) -> np.ndarray:
        return self.nu_lo + (self.nu_hi - self.nu_lo) * self.xi(pts)

    def force(self, pts: np.ndarray, ncomp: int = 3) -> np.ndarray:
        xi = self.xi(pts)
        if ncomp == 1:
            return xi
        f = np.zeros((pts.shape[0], ncomp))
        f[:, -1] = -xi
        return f

    def xi_torch(self, pts):
        """xi of the same field for a (N, 3) float64 torch tensor (any device): the same
        formula with torch operations, for inputs too large to evaluate on the host."""
        import torch
        keep = torch.ones(pts.shape[0], dtype=torch.float64, device=pts.device)
        for p, r in zip(self.centres, self.radii):
            c = torch.as_tensor(p, dtype=torch.float64, device=pts.device)
            d = torch.sqrt(((pts - c) ** 2).sum(dim=1))
            s = 0.5 * (1.0 - torch.tanh((d - float(r)) / self.width))
            keep *= (1.0 - s)
        return 1.0 - keep

    def nu_torch(self, pts):
        return self.nu_lo + (self.nu_hi - self.nu_lo) * self.xi_torch(pts)


class ShapeField:
    """eta_1 to eta_4 of eqs. (3.6)-(3.9): nu = eta_low + (eta_high - eta_low) xi with
    eta_high = DR^1/2, eta_low = DR^-1/2, and f = (0, 0, -xi) (3.11).

    kind 'cube'   : xi_1, the box of half-width 1/8 around (1/2, 1/2, 1/2) (grid-aligned)
         'ucube'  : xi_2, the same box around (11/24, 11/24, 11/24) (unaligned)
         'tcube'  : xi_3, the unaligned box smoothed by tanh with steepness omega:
                    prod_i (tanh(omega (x_i - c + 1/8)) - tanh(omega (x_i - c - 1/8))) / 2,
                    reading the auxiliary function of (3.7) as the one (3.6) names
         'sphere' : xi_4, the ball of radius 0.1 around (1/2, 1/2, 1/2)
    """

    C_UA = 11.0 / 24.0

    def __init__(self, kind: str, contrast: float, omega: float = 10.0):
        if kind not in ("cube", "ucube", "tcube", "sphere"):
            raise ValueError(kind)
        self.kind, self.omega = kind, float(omega)
        self.nu_hi = math.sqrt(contrast)
        self.nu_lo = 1.0 / math.sqrt(contrast)

    def _xi(self, pts: np.ndarray) -> np.ndarray:
        if self.kind == "cube":
            return np.all(np.abs(pts - 0.5) <= 0.125, axis=1).astype(np.float64)
        if self.kind == "ucube":
            return np.all(np.abs(pts - self.C_UA) <= 0.125, axis=1).astype(np.float64)
        if self.kind == "sphere":
            return (((pts - 0.5) ** 2).sum(axis=1) <= 0.01).astype(np.float64)
        w = self.omega
        c = self.C_UA
        t = 0.5 * (np.tanh(w * (pts - (c - 0.125))) - np.tanh(w * (pts - (c + 0.125))))
        return t.prod(axis=1)

    def xi(self, pts: np.ndarray) -> np.ndarray:
        return _chunked(self._xi, pts)

    def nu(self, pts: np.ndarray) -> np.ndarray:
        return self.nu_lo + (self.nu_hi - self.nu_lo) * self.xi(pts)

    def force(self, pts: np.ndarray, ncomp: int = 3) -> np.ndarray:
        xi = self.xi(pts)
        if ncomp == 1:
            return xi
        f = np.zeros((pts.shape[0], ncomp))
        f[:, -1] = -xi
        return f


class GaussianLogField:
    """log nu = affine rescale of a sum of Gaussians, with contrast exp(2*half_range).

    Raw field g(x) = sum_k a_k exp(-|x - c_k|^2 / (2 s_k^2)), a_k ~ U(-1, 1),
    c_k ~ U[0.1, 0.9]^3, s_k ~ U[0.05, 0.2].  ``calibrate`` fixes the affine map
    that sends [min g, max g] over the calibration points to
    [-half_range, +half_range]; half_range = ln 100 gives contrast 1e4.
    ``noise`` draws the per-element perturbation of log nu used to make the
    observations (10 % log-amplitude).
    """

    def __init__(self, n_gauss: int = 16, seed: int = 4, half_range: float = math.log(100.0)):
        rng = np.random.default_rng(seed)
        self.centres = rng.uniform(0.1, 0.9, size=(n_gauss, 3))
        self.widths = rng.uniform(0.05, 0.2, size=n_gauss)
        self.amps = rng.uniform(-1.0, 1.0, size=n_gauss)
        self.half_range = half_range
        self.seed = seed
        self.gmin: Optional[float] = None
        self.gmax: Optional[float] = None

    def _raw(self, pts: np.ndarray) -> np.ndarray:
        g = np.zeros(pts.shape[0])
        for c, s, a in zip(self.centres, self.widths, self.amps):
            g += a * np.exp(-((pts - c) ** 2).sum(axis=1) / (2.0 * s * s))
        return g

    def calibrate(self, pts: np.ndarray) -> None:
        g = _chunked(self._raw, pts)
        self.gmin, self.gmax = float(g.min()), float(g.max())

    def log_nu(self, pts: np.ndarray) -> np.ndarray:
        if self.gmin is None:
            raise RuntimeError("GaussianLogField.calibrate() must be called first")
        g = _chunked(self._raw, pts)
        t = (g - self.gmin) / (self.gmax - self.gmin)
        return -self.half_range + 2.0 * self.half_range * t

    def nu(self, pts: np.ndarray) -> np.ndarray:
        return np.exp(self.log_nu(pts))

    def noise(self, n: int, amplitude: float = 0.1, seed_offset: int = 1000) -> np.ndarray:
        rng = np.random.default_rng(self.seed + seed_offset)
        return amplitude * rng.standard_normal(n)

    def force(self, pts: np.ndarray, ncomp: int = 3) -> np.ndarray:
        f = np.zeros((np.asarray(pts).shape[0], ncomp))
        f[:, -1] = -1.0
        return f if ncomp > 1 else f[:, 0]


@dataclass
class Workload:
    """One benchmark problem: mesh depth, unknowns per node, fields and tolerances."""
    name: str
    L: int                 # finest refinement level of the 2x2x2-cube, 48-tet macro grid
    ncomp: int             # 1 = scalar diffusion, 3 = vector viscous block
    kind: str              # 'cube', 'sinkers', 'gauss', 'stokes'
    tol: float             # relative residual target
    seed: int = 0
    n_sinkers: int = 0
    radius: object = 0.1
    contrast: float = 1e6
    description: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return 2 ** (self.L + 1)

    def make_field(self):
        h = 1.0 / self.n
        if self.kind == "cube":
            return AlignedCube()
        if self.kind in ("sinkers", "stokes"):
            return Sinkers(self.n_sinkers, self.seed, radius=self.radius, width=2.0 * h,
                           contrast=self.contrast)
        if self.kind == "gauss":
            return GaussianLogField(n_gauss=16, seed=self.seed)
        raise ValueError(self.kind)


WORKLOADS = {
    # scalar diffusion, 17^3 nodes, 4 levels, aligned cube nu = 1e3, stationary V(2,2) to 1e-10
    "cube17": Workload("cube17", L=3, ncomp=1, kind="cube", tol=1e-10,
                       description="scalar -div(nu grad u)=1, 17^3 nodes, aligned cube nu=1e3"),
    # vector viscous block, 129^3 nodes, 8 tanh sinkers, contrast 1e6, PCG to 1e-8
    "sinker129": Workload("sinker129", L=6, ncomp=3, kind="sinkers", tol=1e-8, seed=2,
                          n_sinkers=8, radius=0.1,
                          description="vector -div(2 nu eps(u))=f, 129^3 nodes, 8 sinkers r=0.1, 1e6"),
    # generalized Stokes, P1-iso-P2 velocity 257^3 / pressure 129^3, 16 sinkers
    "stokes257": Workload("stokes257", L=7, ncomp=3, kind="stokes", tol=1e-8, seed=3,
                          n_sinkers=16, radius=0.1,
                          description="Stokes, velocity 257^3, pressure 129^3, 16 sinkers, 1e6"),
    # adjoint gradient on the 129^3 vector block, log-Gaussian viscosity, contrast 1e4
    "adjoint129": Workload("adjoint129", L=6, ncomp=3, kind="gauss", tol=1e-10, seed=4,
                           contrast=1e4,
                           description="dJ/dlog nu, 129^3 vector block, 16 Gaussians, 1e4"),
    # large vector run, 513^3 nodes, 64 sinkers r in [0.02, 0.06], mixed precision
    "sinker513": Workload("sinker513", L=8, ncomp=3, kind="sinkers", tol=1e-8, seed=5,
                          n_sinkers=64, radius=(0.02, 0.06),
                          description="vector block, 513^3 nodes, 64 sinkers, mixed precision"),
}


def workload(name: str, L: Optional[int] = None) -> Workload:
    """Return a workload, optionally at another refinement level (same fields and seed)."""
    w = WORKLOADS[name]
    if L is None:
        return w
    return Workload(w.name, L, w.ncomp, w.kind, w.tol, w.seed, w.n_sinkers, w.radius,
                    w.contrast, w.description, dict(w.extra))
