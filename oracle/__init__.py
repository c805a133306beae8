"""Plain FP64 CPU oracle of the two-grid GMsFEM-preconditioned mixed Darcy solver.

TEST INFRASTRUCTURE ONLY.  This package exists to check the HIP path: only
the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The product path never calls it and shares no code with it.

Every function follows one passage of the paper (Yang, Fu, Chung, "A two-grid
preconditioner with an adaptive coarse space for flow simulations in highly
heterogeneous media"), cited by section and equation label in its docstring.
The local, coarse and smoother problems are written exactly as the paper
defines them -- restrictions R L R^T of the global saddle-point matrix --
and solved by a sparse direct factorisation of the bordered saddle system
(one mean-zero pressure multiplier), which is deliberately a different
method from the stream-function and Cholesky forms the HIP path uses.

Parity status of each part is recorded in the module docstrings; every part
is pinned by a test under ``tests/test_oracle_*.py`` against closed forms,
invariants or brute force.
"""
from .discretization import Grid2D, mass_matrix, div_matrix, source_vector  # noqa: F401
from .solver import OracleSolver  # noqa: F401
