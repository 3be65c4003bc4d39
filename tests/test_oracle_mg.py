"""Pins of the oracle's two-grid multigrid with the GDSW-preconditioned coarse solver (section 3).

  * without smoothing and with a coarse solve to 1e-13, one cycle is the
    coarse-grid correction P K_c^{-1} P^T r (a sparse direct solve here);
  * with smoothing, FGMRES preconditioned by the cycle reaches 1e-8 in a few
    iterations, its solution agrees with the direct solve of the fine
    system, and each coarse FGMRES stops at its 1e-1 reduction.
"""
import numpy as np
import scipy.sparse.linalg as spl

import oracle
from harness import die_problem, random_vector
from harness.problems import prolongation
from tests.conftest import cached


def _pair():
    def make():
        Pc = die_problem(8, 4, 4, seed=0, levels=2)
        Pf = die_problem(8, 4, 4, seed=0, levels=2, refine=2)
        return Pc, Pf, prolongation(Pc, Pf)
    return cached(("mg_pair", 8), make)


def test_cycle_without_smoothing_is_the_coarse_grid_correction():
    Pc, Pf, P = _pair()
    M = oracle.two_grid_setup(Pf, Pc, P, nu_pre=0, nu_post=0, coarse_tol=1e-13)
    r = random_vector(Pf.n, 3)
    z = oracle.two_grid_cycle(M, r)
    ref = P @ spl.spsolve(Pc.K().tocsc(), P.T @ r)
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)


def test_two_grid_fgmres_solves_the_fine_system():
    Pc, Pf, P = _pair()
    M = oracle.two_grid_setup(Pf, Pc, P, nu_pre=2, nu_post=2)
    x, info = oracle.two_grid_solve(M, Pf.b, tol=1e-8)
    assert info["converged"] and info["iterations"] <= 15
    xd = spl.spsolve(Pf.K().tocsc(), Pf.b)
    assert np.linalg.norm(x - xd) <= 1e-5 * np.linalg.norm(xd)
    Kc = Pc.K()
    assert all(1 <= k <= 30 for k in M.coarse_its)
