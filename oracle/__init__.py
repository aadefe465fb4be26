"""Plain FP64 CPU oracle for AGCA multigrid.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it, and it
imports nothing from the GPU library: it builds the mesh by generic Bey
refinement on coordinates, assembles global sparse matrices from element
matrices obtained by inverting barycentric matrices, forms global Galerkin
products P^T A P with SciPy, and runs its multigrid and Krylov loops as plain
Python loops over those matrices.

Paper: "Large-scale multigrid with adaptive Galerkin coarsening" (Boehm, Kohl,
Koestler, Ruede).  Each function cites the section or equation it follows.

Parity status: every function is pinned by a test in ``tests/test_oracle_*.py``
against a fact fixed independently of this code (closed forms, a textbook
special case, brute force, invariants or a count printed in the paper), except
where a function's docstring says "parity unpinned".
"""
