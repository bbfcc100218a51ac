"""Plain FP64 CPU oracle for the implicit-Coriolis Newton-Krylov Jacobian-vector product.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package:
only the tests, the smoke check and the CPU-baseline leg of the benchmark use it.
It shares no code, tables or constants with the GPU library; both sides read the
same seeded inputs (seeded_inputs.py) and nothing else.

Paper: Gonzalez Sembla, Rambert, Feudel, Tuckerman, "Convection in a rapidly
rotating spherical shell: Newton's method using implicit Coriolis integration",
Mathematics 13, 2113 (2025), arXiv 2508.16635.

Modules:
  grids      radial Chebyshev/Gauss-Lobatto grid, dealiasing maps, Gauss-Legendre
             nodes, normalized associated Legendre tables, azimuthal sector grid
  sht        scalar / vector spherical-harmonic synthesis and analysis (direct sums)
  physics    potentials -> physical fields, (linearized) nonlinear terms, curl projections
  operators  M and K blocks with the implicit Coriolis coupling, boundary rows,
             equilibrated banded LU solve with iterative refinement
  solver     step, Newton residual, jvp with the traveling-wave phase slot,
             restarted GMRES and Newton

Parity status of each function is stated in its docstring; every function is
pinned by a test in tests/test_oracle_*.py unless it says "parity unpinned".
"""
