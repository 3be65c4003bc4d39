"""Restarted right-preconditioned flexible GMRES (section 3, FGMRES(m)).

Arnoldi with modified Gram-Schmidt, Givens rotations on the Hessenberg
matrix, x0 = 0.  A cycle stops when the estimated relative residual
|g_{j+1}| / ||b|| reaches tol; the true residual ||b - K x|| / ||b|| is then
checked and the method restarts from x if it is still above tol.  The
iteration count is the total number of inner iterations.
"""
import numpy as np


def fgmres(matvec, precond, b, tol=1e-8, restart=30, max_it=1000):
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    info = dict(iterations=0, restarts=0, converged=False, rel_residual=0.0)
    if bnorm == 0.0:
        info["converged"] = True
        return x, info
    its = 0
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        info["rel_residual"] = beta / bnorm
        if beta / bnorm <= tol:
            info["converged"] = True
            break
        if its >= max_it:
            break
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        Hh = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                Hh[i, j] = np.dot(w, V[i])
                w = w - Hh[i, j] * V[i]
            Hh[j + 1, j] = np.linalg.norm(w)
            if Hh[j + 1, j] != 0.0:
                V[j + 1] = w / Hh[j + 1, j]
            for i in range(j):
                t = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                Hh[i + 1, j] = -sn[i] * Hh[i, j] + cs[i] * Hh[i + 1, j]
                Hh[i, j] = t
            den = np.hypot(Hh[j, j], Hh[j + 1, j])
            cs[j] = Hh[j, j] / den
            sn[j] = Hh[j + 1, j] / den
            Hh[j, j] = den
            Hh[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            if abs(g[j + 1]) / bnorm <= tol or its >= max_it or Hh[j + 1, j] == 0.0 and den == 0.0:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(Hh[i, i + 1:k], y[i + 1:k])) / Hh[i, i]
        x = x + y @ Z[:k]
        info["restarts"] += 1
    info["iterations"] = its
    return x, info
