"""Pins of the oracle's FGMRES(m)."""
import numpy as np

import oracle


def test_distinct_eigenvalues_bound_iterations():
    """Unpreconditioned GMRES on a diagonal matrix with k distinct eigenvalues ends in k steps."""
    k = 7
    d = np.repeat(np.arange(1.0, k + 1), 11)
    b = np.random.Generator(np.random.PCG64(0)).standard_normal(d.size)
    x, info = oracle.fgmres(lambda v: d * v, lambda v: v, b, tol=1e-12, restart=30)
    assert info["iterations"] == k and info["converged"]
    np.testing.assert_allclose(x, b / d, rtol=1e-10)


def test_exact_preconditioner_one_iteration():
    rng = np.random.Generator(np.random.PCG64(1))
    A = rng.standard_normal((40, 40)) + 40 * np.eye(40)
    Ainv = np.linalg.inv(A)
    b = rng.standard_normal(40)
    x, info = oracle.fgmres(lambda v: A @ v, lambda v: Ainv @ v, b, tol=1e-12)
    assert info["iterations"] == 1


def test_restart_and_true_residual():
    rng = np.random.Generator(np.random.PCG64(2))
    d = rng.uniform(1.0, 100.0, 300)
    b = rng.standard_normal(300)
    x, info = oracle.fgmres(lambda v: d * v, lambda v: v, b, tol=1e-9, restart=5, max_it=2000)
    assert info["converged"] and info["restarts"] > 1
    assert np.linalg.norm(d * x - b) <= 1e-9 * np.linalg.norm(b)


def test_flexible_preconditioner_varies():
    """A preconditioner that changes every call is allowed (flexible variant) and still converges."""
    rng = np.random.Generator(np.random.PCG64(3))
    d = rng.uniform(1.0, 10.0, 100)
    b = rng.standard_normal(100)
    calls = [0]

    def prec(v):
        calls[0] += 1
        return v / (d * (1.0 + 0.1 * (calls[0] % 3)))
    x, info = oracle.fgmres(lambda v: d * v, prec, b, tol=1e-10)
    assert info["converged"]
    assert np.linalg.norm(d * x - b) <= 1e-10 * np.linalg.norm(b)
