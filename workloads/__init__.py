"""Seeded synthetic inputs: coefficient fields and right-hand sides.

This package holds only the problem data of the sinker benchmarks (viscosity
functions and forcing terms evaluated at given points, plus the random draws
that place the sinkers).  It knows nothing about meshes, elements, operators or
solvers: callers pass the points (element centroids) at which a field is
sampled.  Both the CPU oracle and the GPU path draw their inputs from here.
"""

from .fields import (  # noqa: F401
    AlignedCube,
    GaussianLogField,
    Sinkers,
    Workload,
    workload,
    WORKLOADS,
)
