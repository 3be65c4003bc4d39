"""Several right-hand sides at once (gdsw_apply_multi, gdsw_solve_multi), through the C ABI.

The local solves stream each factor once per chunk of right-hand sides and
update on the matrix cores; every other step runs per vector with the
single-vector kernels.  So each column must agree with the single apply of that
column to rounding (FP64 and FP32 factors, ragged chunks, blocks of order 2295),
the FP64 apply must match the oracle's eq. (2.2) element by element, and the
lockstep solves must follow the single solves (same iteration counts up to one,
true residuals below the tolerance, solutions agreeing far below it).
The low-accuracy regime of section 3 (FGMRES to a 1e-1 reduction, the solver
used as the coarse solver of an outer method) is covered by the lockstep solve.
"""
import sys

import numpy as np
import pytest

import oracle
from harness import unit_cube_problem, die_problem, random_vector
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


def _block(n, k, seed):
    return torch.as_tensor(np.stack([random_vector(n, seed + q) for q in range(k)]), device="cuda")


_CASES = {
    "die16_L4_uneven": lambda: die_problem(16, 8, 8, seed=3, levels=4, frac3=0.3),
    "cube9_b3_L2": lambda: unit_cube_problem(n=9, block=3, levels=2),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,k", [("die16_L4_uneven", 5), ("die16_L4_uneven", 11), ("cube9_b3_L2", 3)])
def test_apply_multi_columns_equal_single_applies(gd, name, k, precision):
    P = cached(("gpu", name), _CASES[name])
    R = _block(P.n, k, 40)
    _say("apply_multi", name, "k =", k, precision)
    with gd.Context(P, precision=precision) as ctx:
        Z = ctx.apply_multi(R).cpu().numpy()
        bound = 1e-12 if precision == "fp64" else 1e-4
        worst = 0.0
        for q in range(k):
            zq = ctx.apply(R[q].contiguous()).cpu().numpy()
            d = np.abs(Z[q] - zq).max() / np.abs(zq).max()
            worst = max(worst, d)
            assert d <= bound, (q, d)
        _say("  largest column difference from the single apply", worst)
    if precision == "fp64":
        H = cached(("orc", name, "RAS", False), lambda: oracle.setup(P))
        for q in (0, k - 1):
            zo = oracle.apply(H, R[q].cpu().numpy())
            err = np.linalg.norm(Z[q] - zo) / np.linalg.norm(zo)
            emax = np.abs(Z[q] - zo).max() / np.abs(zo).max()
            _say("  column", q, "vs oracle", err, emax)
            assert err <= 1e-10 and emax <= 1e-10


@pytest.mark.parametrize("tol", [1e-1, 1e-8])
def test_solve_multi_equals_single_solves(gd, tol):
    P = cached(("gpu", "die16_L3"), lambda: die_problem(16, 8, 8, seed=0, levels=3))
    k = 6
    B = _block(P.n, k, 60)
    B[0] = torch.as_tensor(P.b, device="cuda")
    _say("solve_multi k =", k, "tol", tol)
    with gd.Context(P, tol=tol) as ctx:
        X, infos = ctx.solve_multi(B)
        X = X.cpu().numpy()
        K = P.K()
        for q in range(k):
            x1, i1 = ctx.solve(B[q].contiguous())
            x1 = x1.cpu().numpy()
            assert infos[q]["converged"] and i1["converged"]
            assert abs(infos[q]["iterations"] - i1["iterations"]) <= 1, q
            bq = B[q].cpu().numpy()
            res = np.linalg.norm(bq - K @ X[q]) / np.linalg.norm(bq)
            assert res <= tol * 1.0001
            if infos[q]["iterations"] == i1["iterations"]:
                assert np.linalg.norm(X[q] - x1) <= 1e-8 * np.linalg.norm(x1), q
    _say("  iterations", [i["iterations"] for i in infos])


def test_solve_multi_long_restart_equals_single_solves(gd):
    """Lockstep solves past 32 Krylov columns (FGMRES(60) to 1e-10): the unfused Gram-Schmidt passes and
    the per-system second-pass decisions follow each system's single solve."""
    P = cached(("gpu", "die16_L3"), lambda: die_problem(16, 8, 8, seed=0, levels=3))
    k = 3
    B = _block(P.n, k, 80)
    _say("solve_multi restart 60, k =", k)
    with gd.Context(P, tol=1e-10, restart=60) as ctx:
        X, infos = ctx.solve_multi(B)
        X = X.cpu().numpy()
        K = P.K()
        for q in range(k):
            x1, i1 = ctx.solve(B[q].contiguous())
            x1 = x1.cpu().numpy()
            assert infos[q]["converged"] and i1["converged"]
            assert i1["iterations"] > 32 and abs(infos[q]["iterations"] - i1["iterations"]) <= 1, q
            assert abs(infos[q]["reorthogonalizations"] - i1["reorthogonalizations"]) <= 2, q
            bq = B[q].cpu().numpy()
            assert np.linalg.norm(bq - K @ X[q]) <= 1e-10 * np.linalg.norm(bq) * 1.0001
            assert np.linalg.norm(X[q] - x1) <= 1e-6 * np.linalg.norm(x1), q
    _say("  iterations", [i["iterations"] for i in infos], "second passes",
         [i["reorthogonalizations"] for i in infos])


def test_solve_multi_reports_notconv_per_system(gd):
    P = cached(("gpu", "die16_L3"), lambda: die_problem(16, 8, 8, seed=0, levels=3))
    B = _block(P.n, 3, 70)
    _say("solve_multi notconv")
    with gd.Context(P, tol=1e-12, max_it=5) as ctx:
        X, infos = ctx.solve_multi(B)
        x1, i1 = ctx.solve(B[1].contiguous())
    assert infos[0]["code"] == gd.NOTCONV
    assert all(not i["converged"] and i["iterations"] == 5 for i in infos)
    x1 = x1.cpu().numpy()
    assert np.linalg.norm(X[1].cpu().numpy() - x1) <= 1e-10 * np.linalg.norm(x1)
    assert abs(infos[1]["rel_residual"] - i1["rel_residual"]) <= 1e-8 * i1["rel_residual"]
