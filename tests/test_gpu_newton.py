"""The Newton step of section 3's alternating Picard-Newton iteration on the GPU.

The Newton matrix of the Carreau operator (the velocity block gains the
derivative of the viscosity, pinned by a finite-difference test of the input
generator) goes through the same library: its local blocks are factored with
partial pivoting, the coarse basis and Galerkin operators are built from it,
and FGMRES solves it.  Checked against the oracle: the three-level apply
element by element, and the FGMRES solve (iterations within 2, true residual,
solution).
"""
import sys

import numpy as np
import pytest

import oracle
from harness import die_problem, random_vector
from tests.conftest import cached

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_newton_step_apply_and_solve_match_oracle(precision):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_01433_amd import gdsw
    gdsw.load_library()
    P = cached(("newton", 16), lambda: die_problem(16, 8, 8, seed=0, levels=3, n_exp=0.3, lam=10.0,
                                                   linearization="newton"))
    Pp = cached(("picard", 16), lambda: die_problem(16, 8, 8, seed=0, levels=3, n_exp=0.3, lam=10.0))
    assert np.abs(P.val - Pp.val).max() > 1e-3 * np.abs(Pp.val).max()     # a different operator
    H = cached(("newton_h", 16), lambda: oracle.setup(P))
    K = P.K()
    r = random_vector(P.n, 21)
    zo = oracle.apply(H, r)
    xo, info_o = cached(("newton_x", 16),
                        lambda: oracle.fgmres(lambda v: K @ v, lambda v: oracle.apply(H, v), P.b, tol=1e-8))
    _say("newton step", precision, "n =", P.n, "oracle iterations", info_o["iterations"])
    with gdsw.Context(P, tol=1e-8, precision=precision) as ctx:
        z = ctx.apply(torch.as_tensor(r, device="cuda")).cpu().numpy()
        x, info = ctx.solve(torch.as_tensor(P.b, device="cuda"))
    x = x.cpu().numpy()
    err = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    emax = np.abs(z - zo).max() / np.abs(zo).max()
    res = np.linalg.norm(P.b - K @ x) / np.linalg.norm(P.b)
    xerr = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    _say("  apply", err, emax, "| iterations", info["iterations"], "| residual", res, "| x vs oracle", xerr)
    tol = 1e-10 if precision == "fp64" else 1e-3
    assert err <= tol and emax <= tol
    assert info["converged"] and res <= 1e-8 * 1.0001
    assert abs(info["iterations"] - info_o["iterations"]) <= 2
    assert xerr <= 1e-5
