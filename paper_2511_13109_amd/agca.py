"""Python binding of the AGCA multigrid library (thin wrapper over include/agca.h).

Device memory and streams come from PyTorch: vectors are contiguous CUDA
(HIP) tensors and their data pointers are handed to the C ABI unchanged.  All
arithmetic runs in the library's HIP kernels; if libagca.so is missing, the
import of this module raises.
"""

from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import AGCAError, check  # noqa: F401

_DT = {"f64": _lib.F64, "f32": _lib.F32, "bf16": _lib.BF16}
_TORCH = {_lib.F64: torch.float64, _lib.F32: torch.float32}
_FLAG = {"ratio": _lib.FLAG_RATIO, "macro": _lib.FLAG_MACRO, "none": _lib.FLAG_NONE,
         "dca": _lib.FLAG_NONE, "all": _lib.FLAG_ALL, "gca": _lib.FLAG_ALL}
_SOLVER = {"pcg": _lib.SOLVER_PCG, "fcg": _lib.SOLVER_FCG, "ir": _lib.SOLVER_IR,
           "stationary": _lib.SOLVER_STATIONARY}


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return C.c_void_p(t.data_ptr())


def _dtype_of(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return _lib.F64
    if t.dtype == torch.float32:
        return _lib.F32
    raise ValueError(f"unsupported dtype {t.dtype}")


def default_config() -> _lib.Config:
    cfg = _lib.Config()
    _lib.load().agca_default_config(C.byref(cfg))
    return cfg


def validate_config(cfg: _lib.Config) -> int:
    return _lib.load().agca_validate_config(C.byref(cfg))


def macro_gradient(L: int, eta_nodes: torch.Tensor, stream=None, noalloc: bool = False) -> np.ndarray:
    """Largest |grad eta_h| over the finest elements of each of the 48 macro elements
    (eq. (2.8)); eta_nodes: (2^(L+1)+1)^3 float64 device tensor of nodal values.
    noalloc: the variant without device allocations (agca_macro_gradient_noalloc)."""
    if eta_nodes.dtype != torch.float64 or eta_nodes.numel() != (2 ** (L + 1) + 1) ** 3:
        raise ValueError("eta_nodes must hold (2^(L+1)+1)^3 float64 nodal values")
    st = stream if stream is not None else torch.cuda.current_stream(eta_nodes.device)
    out = np.zeros(48)
    name = "agca_macro_gradient_noalloc" if noalloc else "agca_macro_gradient"
    check(getattr(_lib.load(), name)(L, _ptr(eta_nodes), out.ctypes.data_as(C.c_void_p),
                                     C.c_void_p(st.cuda_stream)), name)
    return out


class Hierarchy:
    """AGCA multigrid hierarchy on levels 0..L (paper Section 2).

    nu_fine: (6 n_L^3,) float64 device tensor; nu_coarse: L tensors, level l holding
    6 n_l^3 float64 values (the DCA coefficient of that level).
    """

    def __init__(self, L: int, ncomp: int, nu_fine: torch.Tensor, nu_coarse: Sequence[torch.Tensor],
                 flag_mode: str = "ratio", tau: float = 10.0, mg_dtype: str = "f64",
                 mg_nu_dtype: Optional[str] = None, pre: int = 2, post: int = 2,
                 omega: float = 2.0 / 3.0, mem_limit_bytes: int = 0, stream=None,
                 smoother: str = "jacobi", macro_flags: Optional[Sequence[bool]] = None,
                 coarse_storage: str = "blocks"):
        self._lib = _lib.load()
        cfg = default_config()
        cfg.L, cfg.ncomp = L, ncomp
        cfg.flag_mode = _FLAG[flag_mode]
        cfg.flag_ratio = tau
        cfg.mg_dtype = _DT[mg_dtype]
        cfg.mg_nu_dtype = _DT[mg_nu_dtype or mg_dtype]
        cfg.pre_sweeps, cfg.post_sweeps, cfg.omega = pre, post, omega
        cfg.smoother = {"jacobi": _lib.SMOOTH_JACOBI, "chebyshev": _lib.SMOOTH_CHEBYSHEV}[smoother]
        cfg.mem_limit_bytes = mem_limit_bytes
        cfg.coarse_storage = {"blocks": _lib.STORE_BLOCKS, "mean": _lib.STORE_MEAN}[coarse_storage]
        if flag_mode == "macro":
            if macro_flags is None or len(macro_flags) != 48:
                raise ValueError("flag_mode 'macro' needs 48 macro flags")
            for k, f in enumerate(macro_flags):
                cfg.macro_flags[k] = 1 if f else 0
        self.cfg = cfg
        self.L, self.ncomp = L, ncomp
        self.mg_dtype = cfg.mg_dtype
        self.device = nu_fine.device
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._keep = [nu_fine] + list(nu_coarse)
        arr = (C.c_void_p * max(1, L))(*[t.data_ptr() for t in nu_coarse])
        self._check_nu(nu_fine, nu_coarse)
        h = C.c_void_p()
        check(self._lib.agca_create(C.byref(cfg), _ptr(nu_fine), arr,
                                    C.c_void_p(self._stream.cuda_stream), C.byref(h)), "agca_create")
        self._h = h
        self.version = 0   # bumped by every coefficient change

    def _check_nu(self, nu_fine, nu_coarse):
        if len(nu_coarse) != self.L:
            raise ValueError("need one coarse coefficient per level 0..L-1")
        for l, t in enumerate(list(nu_coarse) + [nu_fine]):
            lev = l if l < self.L else self.L
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("coefficients must be contiguous float64 device tensors")
            if t.numel() != 6 * (2 ** (lev + 1)) ** 3:
                raise ValueError(f"coefficient of level {lev} has the wrong size")

    # -- lifecycle --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.agca_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_nu(self, nu_fine: torch.Tensor, nu_coarse: Sequence[torch.Tensor]):
        self._check_nu(nu_fine, nu_coarse)
        arr = (C.c_void_p * max(1, self.L))(*[t.data_ptr() for t in nu_coarse])
        check(self._lib.agca_set_nu(self._h, _ptr(nu_fine), arr), "agca_set_nu")
        self._keep = [nu_fine] + list(nu_coarse)
        self.version += 1

    def set_log_nu(self, log_nu_fine: torch.Tensor, nu_coarse: Sequence[torch.Tensor]):
        """Rebuild from log nu on the finest level (exponentiated by the library)."""
        self._check_nu(log_nu_fine, nu_coarse)
        arr = (C.c_void_p * max(1, self.L))(*[t.data_ptr() for t in nu_coarse])
        check(self._lib.agca_set_log_nu(self._h, _ptr(log_nu_fine), arr), "agca_set_log_nu")
        self._keep = [log_nu_fine] + list(nu_coarse)
        self.version += 1

    # -- sizes ------------------------------------------------------------
    def n(self, level: int) -> int:
        return 2 ** (level + 1)

    def nodes(self, level: int) -> int:
        return (self.n(level) + 1) ** 3

    def vec(self, level: int, dtype=torch.float64) -> torch.Tensor:
        return torch.zeros(self.ncomp * self.nodes(level), dtype=dtype, device=self.device)

    def query(self, level: int) -> dict:
        info = _lib.LevelInfo()
        check(self._lib.agca_query(self._h, level, C.byref(info)), "agca_query")
        return {k: getattr(info, k) for k, _ in info._fields_}

    def device_bytes(self) -> int:
        return int(self._lib.agca_device_bytes(self._h))

    def flags(self, level: int) -> np.ndarray:
        n = C.c_int64()
        info = self.query(level)
        ids = np.zeros(max(1, info["flagged"]), dtype=np.int32)
        check(self._lib.agca_get_flags(self._h, level, ids.ctypes.data_as(C.c_void_p), ids.size,
                                       C.byref(n)), "agca_get_flags")
        return ids[:n.value].copy()

    def blocks(self, level: int) -> np.ndarray:
        info = self.query(level)
        M = 4 * self.ncomp
        out = np.zeros((max(1, info["flagged"]), M, M))
        check(self._lib.agca_get_blocks(self._h, level, out.ctypes.data_as(C.c_void_p), out.size),
              "agca_get_blocks")
        return out[:info["flagged"]].copy()

    def diagonal(self, level: int) -> np.ndarray:
        out = np.zeros(self.ncomp * self.nodes(level))
        check(self._lib.agca_get_diagonal(self._h, level, out.ctypes.data_as(C.c_void_p), out.size),
              "agca_get_diagonal")
        return out

    # -- level operations -------------------------------------------------
    def apply(self, level: int, u: torch.Tensor, v: Optional[torch.Tensor] = None) -> torch.Tensor:
        v = torch.empty_like(u) if v is None else v
        check(self._lib.agca_apply(self._h, level, _dtype_of(u), _ptr(u), _ptr(v)), "agca_apply")
        return v

    def residual(self, level: int, b: torch.Tensor, x: torch.Tensor,
                 r: Optional[torch.Tensor] = None) -> torch.Tensor:
        r = torch.empty_like(b) if r is None else r
        check(self._lib.agca_residual(self._h, level, _dtype_of(b), _ptr(b), _ptr(x), _ptr(r)),
              "agca_residual")
        return r

    def smooth(self, level: int, b: torch.Tensor, x: torch.Tensor, sweeps: int,
               omega: Optional[float] = None) -> torch.Tensor:
        om = self.cfg.omega if omega is None else omega
        check(self._lib.agca_smooth(self._h, level, _dtype_of(b), sweeps, om, _ptr(b), _ptr(x)),
              "agca_smooth")
        return x

    def restrict(self, fine_level: int, r_f: torch.Tensor, r_c: Optional[torch.Tensor] = None):
        r_c = self.vec(fine_level - 1, r_f.dtype) if r_c is None else r_c
        check(self._lib.agca_restrict(self._h, fine_level, _dtype_of(r_f), _ptr(r_f), _ptr(r_c)),
              "agca_restrict")
        return r_c

    def prolong_add(self, coarse_level: int, e_c: torch.Tensor, x_f: torch.Tensor):
        check(self._lib.agca_prolong_add(self._h, coarse_level, _dtype_of(e_c), _ptr(e_c), _ptr(x_f)),
              "agca_prolong_add")
        return x_f

    def vcycle(self, b: torch.Tensor, x: Optional[torch.Tensor] = None) -> torch.Tensor:
        x = torch.empty_like(b) if x is None else x
        check(self._lib.agca_vcycle(self._h, _dtype_of(b), _ptr(b), _ptr(x)), "agca_vcycle")
        return x

    def dot(self, level: int, x: torch.Tensor, y: torch.Tensor) -> float:
        out = C.c_double()
        check(self._lib.agca_dot(self._h, level, _dtype_of(x), _ptr(x), _ptr(y), C.byref(out)),
              "agca_dot")
        return out.value

    def cast(self, src: torch.Tensor, to: str) -> torch.Tensor:
        frm = _dtype_of(src)
        code = _DT[to]
        if code == _lib.BF16:
            dst = torch.empty(src.numel(), dtype=torch.int16, device=src.device)
        else:
            dst = torch.empty(src.numel(), dtype=_TORCH[code], device=src.device)
        check(self._lib.agca_cast(self._h, frm, code, _ptr(src), _ptr(dst), src.numel()), "agca_cast")
        return dst

    def solve(self, b: torch.Tensor, x: Optional[torch.Tensor] = None, solver: str = "pcg",
              tol: float = 1e-8, max_iter: int = 500, record_history: bool = True,
              raise_on_noconv: bool = True, milestones: Sequence[float] = ()):
        """milestones: tolerances above tol at which the solve records when its verified true
        residual first fell below each (stats["milestones"]: tol -> (iteration, seconds,
        residual), or None if never)."""
        opts = _lib.SolveOpts()
        opts.solver = _SOLVER[solver]
        opts.max_iter = max_iter
        opts.tol = tol
        opts.use_x0 = 0 if x is None else 1
        opts.record_history = 1 if record_history else 0
        if len(milestones) > _lib.MAX_MILESTONES:
            raise ValueError(f"at most {_lib.MAX_MILESTONES} milestones")
        opts.n_milestones = len(milestones)
        for i, m in enumerate(milestones):
            opts.milestones[i] = m
        x = torch.zeros_like(b) if x is None else x
        st = _lib.SolveStats()
        rc = self._lib.agca_solve(self._h, C.byref(opts), _ptr(b), _ptr(x), C.byref(st))
        stats = {"iterations": st.iterations, "converged": bool(st.converged),
                 "floor_limited": bool(st.floor_limited), "replacements": st.replacements,
                 "rel_residual": st.rel_residual,
                 "recursive_rel_residual": st.recursive_rel_residual,
                 "floor_estimate": st.floor_estimate, "seconds": st.seconds,
                 "history": list(st.history[:min(st.iterations + 1, _lib.MAX_HISTORY)])
                 if record_history else [], "status": rc,
                 "milestones": {m: ((st.milestone_iterations[i], st.milestone_seconds[i],
                                     st.milestone_residuals[i]) if st.milestone_iterations[i] >= 0 else None)
                                for i, m in enumerate(milestones)}}
        if rc != _lib.AGCA_OK and (rc != _lib.AGCA_E_NOCONV or raise_on_noconv):
            check(rc, "agca_solve")
        return x, stats

    def residual_floor(self, b: torch.Tensor, x: torch.Tensor) -> float:
        """Rounding floor rho of the relative residual of x (agca_residual_floor)."""
        out = C.c_double()
        check(self._lib.agca_residual_floor(self._h, _ptr(b), _ptr(x), C.byref(out)),
              "agca_residual_floor")
        return out.value

    def grad_log_nu(self, u: torch.Tensor, w: torch.Tensor, g: Optional[torch.Tensor] = None):
        g = torch.empty(6 * self.n(self.L) ** 3, dtype=torch.float64, device=u.device) if g is None else g
        check(self._lib.agca_grad_log_nu(self._h, _ptr(u), _ptr(w), _ptr(g)), "agca_grad_log_nu")
        return g

    def load_vector(self, f: torch.Tensor, b: Optional[torch.Tensor] = None) -> torch.Tensor:
        """b_i = sum_e f_e |e| / 4; f: component-major (ncomp, 6 n_L^3) per-element values
        by element id, flattened."""
        b = self.vec(self.L) if b is None else b
        check(self._lib.agca_load_vector(self._h, _ptr(f.contiguous()), _ptr(b)), "agca_load_vector")
        return b


class Stokes:
    """Generalized Stokes on a vector Hierarchy (Section 3.1): velocity on level L,
    pressure P1 on every node of level L-1."""

    def __init__(self, H: Hierarchy):
        if H.ncomp != 3:
            raise ValueError("Stokes needs the vector hierarchy")
        self.H = H
        self.np = H.nodes(H.L - 1)

    def pvec(self) -> torch.Tensor:
        return torch.zeros(self.np, dtype=torch.float64, device=self.H.device)

    def div(self, u: torch.Tensor, q: Optional[torch.Tensor] = None) -> torch.Tensor:
        q = self.pvec() if q is None else q
        check(self.H._lib.agca_stokes_div(self.H._h, _ptr(u), _ptr(q)), "agca_stokes_div")
        return q

    def grad(self, p: torch.Tensor, v: Optional[torch.Tensor] = None) -> torch.Tensor:
        v = self.H.vec(self.H.L) if v is None else v
        check(self.H._lib.agca_stokes_grad(self.H._h, _ptr(p), _ptr(v)), "agca_stokes_grad")
        return v

    def mass(self) -> torch.Tensor:
        m = self.pvec()
        check(self.H._lib.agca_stokes_mass(self.H._h, _ptr(m)), "agca_stokes_mass")
        return m

    SCHUR = {"mass": _lib.SCHUR_MASS, "bfbt": _lib.SCHUR_BFBT, "bfbt_mg": _lib.SCHUR_BFBT_MG}

    def schur_apply(self, rp: torch.Tensor, schur: str = "bfbt_mg", schur_iters: int = 4,
                    q: Optional[torch.Tensor] = None) -> torch.Tensor:
        """q = S^-1 rp, the pressure block of the block-diagonal preconditioner."""
        q = self.pvec() if q is None else q
        check(self.H._lib.agca_stokes_schur_apply(self.H._h, self.SCHUR[schur], schur_iters, _ptr(rp), _ptr(q)),
              "agca_stokes_schur_apply")
        return q

    def z_stencil(self, level: int) -> torch.Tensor:
        """(65, (n_level+1)^3) stencil of the pressure multigrid's operator on `level`."""
        out = torch.empty(65 * self.H.nodes(level), dtype=torch.float64, device=self.H.device)
        check(self.H._lib.agca_stokes_z_stencil(self.H._h, level, _ptr(out)), "agca_stokes_z_stencil")
        return out.view(65, -1)

    def z_vcycle(self, r: torch.Tensor) -> torch.Tensor:
        y = self.pvec()
        check(self.H._lib.agca_stokes_z_vcycle(self.H._h, _ptr(r), _ptr(y)), "agca_stokes_z_vcycle")
        return y

    def solve(self, f: torch.Tensor, g: Optional[torch.Tensor] = None, solver: str = "fgmres",
              restart: int = 30, tol: float = 1e-8, max_iter: int = 1000, record_history: bool = True,
              raise_on_noconv: bool = True, precond: str = "diagonal", schur: str = "mass",
              schur_iters: int = 20, velocity_cycles: int = 1, basis: str = "f64"):
        """schur: 'mass' (1/nu lumped mass), 'bfbt' (eq. (4.2), FGMRES only, each Z solve
        schur_iters Jacobi-CG steps) or 'bfbt_mg' (the same with each Z solve schur_iters
        CG steps preconditioned by a pressure multigrid V-cycle); velocity_cycles: V-cycles
        per application of the velocity block's approximate inverse (1: the paper's);
        basis: storage of the FGMRES Arnoldi basis, 'f64' or 'f32'."""
        opts = _lib.StokesOpts()
        opts.solver = {"fgmres": _lib.STOKES_FGMRES, "minres": _lib.STOKES_MINRES}[solver]
        opts.precond = {"diagonal": _lib.STOKES_DIAGONAL, "triangular": _lib.STOKES_TRIANGULAR}[precond]
        opts.schur = self.SCHUR[schur]
        opts.schur_iters = schur_iters
        opts.velocity_cycles = velocity_cycles
        opts.basis_dtype = {"f64": _lib.F64, "f32": _lib.F32}[basis]
        opts.restart, opts.max_iter, opts.tol = restart, max_iter, tol
        opts.record_history = 1 if record_history else 0
        g = self.pvec() if g is None else g
        u = self.H.vec(self.H.L)
        p = self.pvec()
        st = _lib.SolveStats()
        rc = self.H._lib.agca_stokes_solve(self.H._h, C.byref(opts), _ptr(f), _ptr(g), _ptr(u), _ptr(p),
                                           C.byref(st))
        stats = {"iterations": st.iterations, "converged": bool(st.converged),
                 "floor_limited": bool(st.floor_limited), "floor_estimate": st.floor_estimate,
                 "rel_residual": st.rel_residual, "seconds": st.seconds, "status": rc,
                 "history": list(st.history[:min(st.iterations + 1, _lib.MAX_HISTORY)])
                 if record_history else []}
        if rc != _lib.AGCA_OK and (rc != _lib.AGCA_E_NOCONV or raise_on_noconv):
            check(rc, "agca_stokes_solve")
        return u, p, stats


def coefficients_from_field(field, L: int, device="cuda") -> List[torch.Tensor]:
    """Sample a coefficient field at the element centroids of every level 0..L (host evaluation)."""
    from workloads.lattice import element_centroids
    out = []
    for l in range(L + 1):
        out.append(torch.from_numpy(np.ascontiguousarray(field.nu(element_centroids(l)))).to(device))
    return out
