"""Plain, slow FP64 CPU oracle of the monolithic multilevel GDSW method.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may import,
call or link anything here; only the tests, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path:
it reads the same harness-built problem arrays and recomputes everything from
the definitions of section 2.1 (overlapping Schwarz, GDSW coarse space,
Galerkin operator), section 2.2 (the recursion and eq. (2.2)) and section 3
(restarted flexible GMRES), using NumPy/SciPy (SuperLU for sparse local and
interior solves, LAPACK for the coarsest dense solve).

Every function here is pinned by a test under tests/ against closed forms,
invariants, special cases or brute force; see the docstrings.
"""
from .levels import Mesh, LevelMaps, level1_mesh, build_level, next_mesh  # noqa: F401
from .gdsw import Hierarchy, setup, apply, solve_direct  # noqa: F401
from .fgmres import fgmres  # noqa: F401
from .mg import two_grid_setup, two_grid_cycle, two_grid_solve  # noqa: F401
