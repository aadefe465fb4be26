"""AGCA multigrid for MI355X: adaptive Galerkin coarse-grid approximation with
hand-written HIP kernels behind a C ABI (include/agca.h).

Paper: "Large-scale multigrid with adaptive Galerkin coarsening" (Boehm, Kohl,
Koestler, Ruede).  ``Hierarchy`` is the entry point.
"""


def __getattr__(name):
    # the binding loads libagca.so on first use and fails loudly if it is missing
    if name in ("Hierarchy", "Stokes", "coefficients_from_field", "AGCAError", "default_config",
                "validate_config", "macro_gradient"):
        from . import agca
        return getattr(agca, name)
    if name == "autograd":
        from . import autograd
        return autograd
    if name == "AGCASolve":
        from .autograd import AGCASolve
        return AGCASolve
    raise AttributeError(name)
