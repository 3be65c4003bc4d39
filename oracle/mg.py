"""Two-grid geometric multigrid with the GDSW-preconditioned FGMRES as coarse solver (section 3).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 3 uses the method in a second role: the coarsest problem of a
geometric multigrid for the same Stokes system is solved by FGMRES
preconditioned by the multilevel GDSW method, only to a relative residual
reduction of 1e-1.  The fine problem there is one uniform refinement of the
coarse one (13.2M over 2.1M and 94.1M over 13.2M dofs), so the cycle here has
two grids: the refined die (fine) and the die (coarse), with the nested
Q2 / P1disc prolongation P and restriction P^T.  The smoother, which the
paper does not name, is a damped one-level restricted overlapping Schwarz
step on the fine grid's 2^3-voxel parts.  One cycle on r, z0 = 0:

  nu_pre times:  z <- z + omega S (r - K_f z)
  coarse:        z <- z + P FGMRES(K_c, B_GDSW, P^T (r - K_f z), tol)
  nu_post times: z <- z + omega S (r - K_f z)

The whole solve is FGMRES on K_f with this (inexact, hence flexible) cycle as
preconditioner.
"""
import numpy as np

from .gdsw import setup, apply
from .fgmres import fgmres


class TwoGrid:
    pass


def two_grid_setup(fine, coarse, P, nu_pre=2, nu_post=2, omega=1.0, coarse_tol=1e-1):
    """fine: the refined problem with its smoother parts (one level, two-level hierarchy arrays); coarse:
    the problem the GDSW hierarchy is built on; P: prolongation (fine free dofs x coarse free dofs)."""
    M = TwoGrid()
    M.Kf = fine.K().tocsr()
    M.Kc = coarse.K().tocsr()
    M.P = P.tocsr()
    M.PT = P.T.tocsr()
    M.S = setup(fine, no_coarse=True, levels=2)
    M.Hc = setup(coarse)
    M.nu_pre, M.nu_post, M.omega, M.coarse_tol = nu_pre, nu_post, omega, coarse_tol
    M.coarse_its = []
    return M


def two_grid_cycle(M, r):
    r = np.asarray(r, dtype=np.float64)
    z = np.zeros_like(r)
    for _ in range(M.nu_pre):
        z = z + M.omega * apply(M.S, r - M.Kf @ z)
    dc = M.PT @ (r - M.Kf @ z)
    ec, info = fgmres(lambda v: M.Kc @ v, lambda v: apply(M.Hc, v), dc, tol=M.coarse_tol)
    M.coarse_its.append(info["iterations"])
    z = z + M.P @ ec
    for _ in range(M.nu_post):
        z = z + M.omega * apply(M.S, r - M.Kf @ z)
    return z


def two_grid_solve(M, b, tol=1e-8, restart=30, max_it=1000):
    return fgmres(lambda v: M.Kf @ v, lambda v: two_grid_cycle(M, v), b, tol=tol, restart=restart, max_it=max_it)
