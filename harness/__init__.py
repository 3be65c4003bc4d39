"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package builds the *problem* that the GDSW method is applied to: voxel
meshes, the Q2 velocity / P1-discontinuous pressure saddle-point matrix of
eq. (2.1) (stationary Stokes, section 2) with a constant or Carreau viscosity
(section 3), Dirichlet elimination, right-hand sides and part hierarchies.
It contains none of the preconditioner's arithmetic (no overlap, interface,
coarse basis, Galerkin product, local factorization or Krylov step): both the
oracle and the HIP library receive its output as plain arrays.
"""
from .problems import Problem, unit_cube_problem, die_problem, random_vector  # noqa: F401
