"""Two-grid geometric multigrid with the GDSW solver as coarse solver (section 3, second role) on the GPU.

A seeded die (the coarse problem, three-level GDSW, FGMRES to a 1e-1
reduction) and its uniform refinement (the fine problem, smoothed by a damped
one-level restricted Schwarz step on its 2^3-voxel parts), with the nested
Q2 / P1disc prolongation (pinned by polynomial reproduction).  Checked against
the oracle's two-grid method: one cycle element by element, and the FGMRES
solve on the fine system preconditioned by the cycle.
"""
import sys

import numpy as np
import pytest

import oracle
from harness import die_problem, random_vector
from harness.problems import prolongation
from tests.conftest import cached

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def _pair():
    def make():
        Pc = die_problem(16, 8, 8, seed=0, levels=3)
        Pf = die_problem(16, 8, 8, seed=0, levels=2, refine=2)
        return Pc, Pf, prolongation(Pc, Pf)
    return cached(("mg16", 0), make)


def test_two_grid_cycle_and_solve_match_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_01433_amd import gdsw
    gdsw.load_library()
    Pc, Pf, P = _pair()
    _say("two-grid: fine n =", Pf.n, "coarse n =", Pc.n)
    M = cached(("mg16_orc", 0), lambda: oracle.two_grid_setup(Pf, Pc, P, nu_pre=2, nu_post=2, omega=1.0))
    r = random_vector(Pf.n, 51)
    M.coarse_its.clear()
    zo = oracle.two_grid_cycle(M, r)
    its_cycle = list(M.coarse_its)
    M.coarse_its.clear()
    xo, info_o = oracle.two_grid_solve(M, Pf.b, tol=1e-8)
    with gdsw.Context(Pf, no_coarse=True, tol=1e-8) as fine, gdsw.Context(Pc, tol=1e-1) as coarse:
        with gdsw.MultiGrid(fine, coarse, P, nu_pre=2, nu_post=2, omega=1.0) as mg:
            z = mg.apply(torch.as_tensor(r, device="cuda")).cpu().numpy()
            c1 = mg.counts()
            x, info = mg.solve(torch.as_tensor(Pf.b, device="cuda"))
            c2 = mg.counts()
    x = x.cpu().numpy()
    err = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    emax = np.abs(z - zo).max() / np.abs(zo).max()
    res = np.linalg.norm(Pf.b - Pf.K() @ x) / np.linalg.norm(Pf.b)
    xerr = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    _say("cycle vs oracle", err, emax, "| coarse its", c1["coarse_iterations"], "oracle", its_cycle,
         "| outer its", info["iterations"], "oracle", info_o["iterations"], "| residual", res, "| x vs oracle", xerr,
         "| coarse its per cycle", (c2["coarse_iterations"] - c1["coarse_iterations"]) / max(1, c2["cycles"] - c1["cycles"]))
    assert c1["cycles"] == 1 and c1["coarse_iterations"] == its_cycle[0]
    assert err <= 1e-8 and emax <= 1e-8
    assert info["converged"] and res <= 1e-8 * 1.0001
    assert abs(info["iterations"] - info_o["iterations"]) <= 1
    assert xerr <= 1e-5
