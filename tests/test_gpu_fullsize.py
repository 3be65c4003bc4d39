"""GPU parity at the size of the three-level FP64 workload (32x16x16 die, 914 parts).

  * the level-1 local solves (batched pivoted LU + substitution, the register
    panels for tall blocks and the compact update grids) on sampled dofs: a
    one-level restricted apply must equal, at each sampled dof g, the entry of
    A_i^{-1} R_i r of g's owning part, computed on the CPU with a dense LU of the
    local block taken from the oracle's maps (section 2.1);
  * the whole three-level apply of eq. (2.2) against the oracle's, element by
    element (coarsest of order 1655: the tall-panel factorization and the
    register-resident inverse);
  * the FGMRES solve against the oracle's FGMRES with the oracle's
    preconditioner: convergence, the true residual recomputed on the CPU,
    iteration counts within 2, and the two solutions.
"""
import sys

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import levels as olevels
from harness import die_problem, random_vector
from tests.conftest import cached

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_01433_amd import gdsw
    gdsw.load_library()
    return gdsw


def _die(levels):
    return cached(("die32", levels), lambda: die_problem(32, 16, 16, seed=0, nu0=1.0, lam=1.0, n_exp=0.5,
                                                         levels=levels))


def _dev(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), device="cuda")


def test_fullsize_local_solves_on_sampled_dofs(gd):
    P = _die(2)
    mesh = olevels.level1_mesh(P)
    maps = olevels.build_level(mesh, 1)
    owner = oracle.gdsw.ras_owner(mesh, maps)
    r = random_vector(P.n, 11)
    _say("fullsize one-level RAS apply, n =", P.n)
    with gd.Context(P, no_coarse=True) as ctx:
        z = ctx.apply(_dev(r)).cpu().numpy()
    K = P.K().tocsr()
    rng = np.random.Generator(np.random.PCG64(5))
    sample = rng.choice(P.n, size=24, replace=False)
    worst = 0.0
    for g in sample:
        i = int(owner[g])
        D = np.asarray(maps.dom[i])
        Ai = K[D][:, D].toarray()
        y = sla.lu_solve(sla.lu_factor(Ai), r[D])
        a = int(np.searchsorted(D, g))
        assert D[a] == g
        err = abs(z[g] - y[a]) / max(np.abs(y).max(), 1e-300)
        worst = max(worst, err)
    _say("worst sampled relative error", worst)
    assert worst <= 1e-10


def _errs(z, zo):
    return (float(np.linalg.norm(z - zo) / np.linalg.norm(zo)),
            float(np.abs(z - zo).max() / np.abs(zo).max()))


def test_fullsize_three_level_apply_and_solve_match_oracle(gd):
    P = _die(3)
    _say("fullsize three-level oracle setup, n =", P.n)
    H = cached(("die32_h", 3), lambda: oracle.setup(P))
    K = P.K()
    r = random_vector(P.n, 12)
    zo = oracle.apply(H, r)
    _say("oracle FGMRES")
    xo, info_o = oracle.fgmres(lambda v: K @ v, lambda v: oracle.apply(H, v), P.b, tol=1e-8)
    with gd.Context(P, tol=1e-8) as ctx:
        z = ctx.apply(_dev(r)).cpu().numpy()
        x, info = ctx.solve(_dev(P.b))
        st = ctx.stats()
    x = x.cpu().numpy()
    err, emax = _errs(z, zo)
    res = np.linalg.norm(P.b - K @ x) / np.linalg.norm(P.b)
    xerr, xmax = _errs(x, xo)
    _say("apply rel err", err, "max err", emax, "| iterations gpu", info["iterations"], "oracle",
         info_o["iterations"], "| true residual", res, "| solution vs oracle", xerr, xmax,
         "| coarsest order", st["n"][2])
    assert st["n"][2] == H.K_coarsest.shape[0] > 1536      # the coarsest takes the tall-panel path
    assert err <= 1e-10 and emax <= 1e-10
    assert info["converged"] and info_o["converged"]
    assert res <= 1e-8 * 1.0001
    assert abs(info["iterations"] - info_o["iterations"]) <= 2
    assert xerr <= 1e-5 and xmax <= 1e-5
