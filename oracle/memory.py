"""Memory model of the paper (Section 5, eqs. (5.1)-(5.8), Table 1), in units of N_L.

Part of the CPU oracle: test infrastructure only (tests, smoke check, CPU baseline).

N_L is a fine-grid vector holding all velocity and pressure DoFs of the Stokes
problem.  The paper's printed constants are approximations of the limits
computed here; the tests compare these exact values against them.

Readings: in (5.2) and (5.3) the garbled "15 . 2+1" is read as (couplings x 2 + 1)
words per row: a value and a column index per nonzero plus one row pointer.
c_u is the limit 1 - 1/24 of (5.1) as printed (the paper quotes it as 0.95); the
printed constants are reproduced to within the paper's rounding.
"""

from __future__ import annotations

from fractions import Fraction


def vertices(n: int) -> int:
    """Vertices of the cube lattice with n cells per axis."""
    return (n + 1) ** 3


def c_u_limit() -> Fraction:
    """(5.1): velocity share, 1 - lim N_v(l) / (3 N_v(l+1)); N_v grows 8x per level."""
    return 1 - Fraction(1, 3 * 8)


def c_u_at(n: int) -> float:
    """(5.1) at a finite level: 1 - N_v(l) / (3 N_v(l+1)) with n cells per axis on level l."""
    return 1.0 - vertices(n) / (3.0 * vertices(2 * n))


def mem_A_L(c_u=None) -> float:
    """(5.2): (3 x 15 nonzeros x 2 words + 1 row pointer) per velocity row, times c_u."""
    c_u = c_u_limit() if c_u is None else c_u
    return float((3 * 15 * 2 + 1) * c_u)


def mem_K_L(c_u=None) -> float:
    """(5.3): Mem_A_L + 2 x (15 x 2 + 1) words per pressure row, times c_p = 1 - c_u."""
    c_u = c_u_limit() if c_u is None else c_u
    return mem_A_L(c_u) + float(2 * (15 * 2 + 1) * (1 - c_u))


def mem_gca_sparse(n_fill_in: float = 1.0, c_u=None) -> float:
    """(5.4): fill-in times Mem_A_L / 8."""
    return n_fill_in * mem_A_L(c_u) / 8.0


def mem_gca_all_elements(c_u=None) -> float:
    """(5.6): 3 components x 16 entries x 6 cells per vertex x 1/8 x c_u."""
    c_u = c_u_limit() if c_u is None else c_u
    return float(3 * 16 * 6 * Fraction(1, 8) * c_u)


def mem_agca_stencil(c_u=None) -> float:
    """(5.8): 3 components x 15 stencil entries x 1/8 x c_u."""
    c_u = c_u_limit() if c_u is None else c_u
    return float(3 * 15 * Fraction(1, 8) * c_u)


def cells_per_vertex(n: int) -> float:
    """(5.5) at finite size: Kuhn cells per lattice vertex, 6 n^3 / (n+1)^3 -> 6."""
    return 6.0 * n ** 3 / vertices(n)


def table1(c_agca: float, n_restart: int = 30) -> dict:
    """Table 1 columns in units of N_L."""
    return {
        "matrix_based": {"fine": mem_K_L(), "coarse": mem_gca_sparse()},
        "sparse_gca": {"fine": 0.0, "coarse": mem_gca_sparse()},
        "agca": {"fine": 0.0, "coarse": c_agca * mem_gca_all_elements()},
        "agca_stencil": {"fine": 0.0, "coarse": c_agca * mem_agca_stencil()},
        "dca": {"fine": 0.0, "coarse": 0.0},
        "fgmres": 2 + 2 * n_restart,
        "pde": 2,
        "preconditioner": 4,
    }
