"""GDSW coarse basis, Galerkin operator, recursion and the preconditioner of eq. (2.2).

Section 2.1:
  * local blocks A_i = R_i A R_i^T, applied exactly (SuperLU);
  * Phi_Gamma: per (entity, velocity direction) the indicator of that entity's
    dofs in that direction (translations only), per part the indicator of its
    constant pressure modes;
  * Phi_I = -A_II^{-1} A_{I Gamma} Phi_Gamma, part by part (A_II is block
    diagonal over parts);
  * A_0 = Phi^T A Phi;  B = Phi A_0^{-1} Phi^T + sum_i R_i^T A_i^{-1} R_i.
Section 2.2: A_0^(l) = Phi^(l)^T A_0^(l-1) Phi^(l), each coarse problem but the
last approximated by the two-level method on the next decomposition; the last
one is solved directly (dense LU here).

Summation order of the apply: z starts at 0.0, local solutions are added in
ascending part order (each z[g] accumulates left to right), then the coarse
correction Phi y is added.

Combination of overlapping values: eq. (2.2) prints the additive form
R_i^T A_i^{-1} R_i.  With three or more levels that form does not converge on
saddle-point problems of this kind (a reading of this project, measured on the
seeded dies and on constant-viscosity cubes), while the restricted form, in
which each dof keeps only the local solution of its owner (the lowest part
containing its node for velocity, the part of its element for pressure),
converges with iteration counts that grow mildly with the number of levels,
as Table 1 reports.  The restricted form is therefore the default; the
additive one stays available.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from .levels import level1_mesh, build_level, next_mesh


def gamma_basis(n, maps):
    """Phi_Gamma as an n x n_coarse 0/1 matrix."""
    rows, cols = [], []
    for c, dofs in enumerate(maps.col_dofs):
        rows.extend(dofs)
        cols.extend([c] * len(dofs))
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, maps.n_coarse))


def coarse_basis(K, maps):
    """Phi = [Phi_I; Phi_Gamma] with the discrete saddle-point extension into each part's interior."""
    n = K.shape[0]
    PhiG = gamma_basis(n, maps)
    rows, cols, vals = [], [], []
    G = PhiG.tocoo()
    rows.extend(G.row.tolist())
    cols.extend(G.col.tolist())
    vals.extend(G.data.tolist())
    for I in maps.inter:
        if len(I) == 0:
            continue
        KII = K[I][:, I].tocsc()
        rhs = -(K[I, :] @ PhiG).tocsr()          # -A_{I Gamma} Phi_Gamma (Phi_Gamma vanishes on I)
        used = np.unique(rhs.indices)            # columns with a nonzero right-hand side
        if len(used) == 0:
            continue
        X = spl.splu(KII).solve(rhs[:, used].toarray())
        for a, g in enumerate(I):
            rows.extend([int(g)] * len(used))
            cols.extend(used.tolist())
            vals.extend(X[a].tolist())
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, maps.n_coarse))


class Level:
    pass


class Hierarchy:
    """levels[0..L-2]: Schwarz levels (K, maps, local factors, Phi); coarsest: dense LU."""

    def __init__(self):
        self.levels = []
        self.K_coarsest = None
        self.lu_coarsest = None
        self.no_coarse = False


def setup(problem, delta=1, levels=None, no_coarse=False, combine="RAS", pressure_gamma="constants"):
    """Build the L-level hierarchy of eq. (2.2) for a harness Problem.

    combine="AS" sums every local solution over its whole overlapping set
    (R_i^T as printed in eq. (2.2)); combine="RAS" (default) keeps, for every
    dof, only the solution of the part that owns it.  no_coarse drops the
    coarsest correction (one-level Schwarz when L = 2).  pressure_gamma: see
    levels.build_level ("all": the extension of the coarse basis is velocity-only).
    """
    L = problem.levels if levels is None else levels
    H = Hierarchy()
    H.no_coarse = no_coarse
    H.combine = combine
    K = problem.K().tocsr()
    mesh = level1_mesh(problem)
    for ell in range(1, L):
        lev = Level()
        lev.K = K
        lev.mesh = mesh
        lev.maps = build_level(mesh, delta, pressure_gamma)
        lev.lu = [spl.splu(K[D][:, D].tocsc()) for D in lev.maps.dom]
        lev.owner = ras_owner(mesh, lev.maps) if combine == "RAS" else None
        H.levels.append(lev)
        last = (ell == L - 1)
        if no_coarse and last:
            return H
        lev.Phi = coarse_basis(K, lev.maps)
        K = (lev.Phi.T @ K @ lev.Phi).tocsr()
        if not last:
            parent = problem.part_parent[ell - 1]
            n_next = problem.n_parts[ell]
            mesh = next_mesh(mesh, lev.maps, parent, n_next)
            if n_next == 1:
                break                       # a single part: this level becomes the coarsest
    H.K_coarsest = K
    H.lu_coarsest = sla.lu_factor(K.toarray())
    return H


def ras_owner(mesh, maps):
    """Restricted variant: each dof is kept by one part (lowest part of S(v); pressure by its element)."""
    owner = -np.ones(mesh.n_dof, dtype=np.int64)
    for v in range(mesh.n_nodes):
        if maps.S[v]:
            for x in mesh.node_dof[v]:
                if x >= 0:
                    owner[x] = min(maps.S[v])
    for e in range(len(mesh.elem_nodes)):
        for x in mesh.elem_pdof[e]:
            if x >= 0:
                owner[x] = mesh.elem_part[e]
    return owner


def _apply_level(H, k, r):
    lev = H.levels[k]
    z = np.zeros_like(r)
    for i, (D, lu) in enumerate(zip(lev.maps.dom, lev.lu)):
        w = lu.solve(r[D])
        if lev.owner is not None:
            w = np.where(lev.owner[D] == i, w, 0.0)
        z[D] += w
    if H.no_coarse and k == len(H.levels) - 1:
        return z
    rc = lev.Phi.T @ r
    if k + 1 < len(H.levels):
        yc = _apply_level(H, k + 1, rc)
    else:
        yc = sla.lu_solve(H.lu_coarsest, rc)
    return z + lev.Phi @ yc


def apply(H, r):
    """z = B r, eq. (2.2) (two-level formula of section 2.1 when L = 2)."""
    r = np.asarray(r, dtype=np.float64)
    if not H.levels:
        return sla.lu_solve(H.lu_coarsest, r)
    return _apply_level(H, 0, r)


def solve_direct(problem, b=None):
    """The plain definition of solve: x = K^{-1} b."""
    b = problem.b if b is None else b
    return spl.spsolve(problem.K().tocsc(), b)
