"""Q2-P1disc assembly of the Stokes saddle-point matrix (eq. (2.1)).

Velocity forms: 'laplace' is mu * grad u : grad v (section 2); 'sym' is
2 nu(x) D(u) : D(v) with the symmetric gradient D (section 3), nu given per
Gauss point.  The divergence block is B[q, v] = -int q div v, so that
K = [[A, B^T], [B, 0]] is symmetric.  The sparsity pattern is the element
connectivity (all couplings an element creates are stored, including those
that integrate to zero); the Laplace form omits the cross-component velocity
couplings, which it never creates.
"""
import numpy as np
import scipy.sparse as sp

from .q2 import quadrature_points, q2_tables, p1_tables

_PTS, _WTS = quadrature_points()
_PHI, _DPHI = q2_tables(_PTS)          # (q, a), (q, a, dir)
_PSI = p1_tables(_PTS)                 # (q, m)


def velocity_tables(form):
    """M[q] with A_e = (h/2) * sum_q nu_q M[q]; local velocity dof = 3a + i."""
    G = _DPHI                                               # (q, a, k)
    lap = np.einsum("qak,qbk->qab", G, G)                   # (q, a, b)
    eye = np.eye(3)
    M = np.einsum("qab,ij->qaibj", lap, eye)
    if form == "sym":
        M = M + np.einsum("qaj,qbi->qaibj", G, G)
    elif form != "laplace":
        raise ValueError(form)
    M = M * _WTS[:, None, None, None, None]
    return M.reshape(27, 81, 81)


def divergence_table():
    """B_e = -(h/2)^2 * T with T[m, 3b+j] = sum_q w_q psi_m dphi_{b,j}."""
    T = np.einsum("q,qm,qbj->mbj", _WTS, _PSI, _DPHI)
    return T.reshape(4, 81)


def load_table():
    """int phi_a over the reference cube: F_e[3a+i] = (h/2)^3 * f_i * L[a]."""
    return np.einsum("q,qa->a", _WTS, _PHI)


def gauss_gradients(mesh, nodal_u):
    """grad u at the 27 Gauss points of each element from the Q2 interpolant: (E, q, i, k)."""
    ue = nodal_u[mesh.elem_node]                            # (E, a, i)
    return np.einsum("eai,qak->eqik", ue, _DPHI) * (2.0 / mesh.h)


ASSEMBLY_CHUNK = 65536


def newton_vectors(mesh, D_q):
    """t[e, q, 3a + i] = (D_q G_a)_i: the derivative of D(u_k):D(v) at Gauss point q of element e with
    respect to the velocity dof (a, i) of v, up to the factor 2/h (D_q: (E, 27, 3, 3) symmetric
    gradients of the linearization point in physical units, G_a: reference gradients of node a)."""
    return np.einsum("eqik,qak->eqai", D_q, _DPHI).reshape(D_q.shape[0], 27, 81)


def assemble(mesh, nu_q, form, f=(0.0, 0.0, 0.0), newton=None):
    """Full (unconstrained) K in COO-summed CSR over all dofs and the load vector.

    Full dof numbering: velocity 3*node + i, then pressure 3*n_nodes + 4*e + m.
    nu_q: (E, 27) viscosity at Gauss points.
    newton: None (Picard: the viscosity frozen at the linearization point), or
    (c_q, D_q) adding the derivative of the viscosity to the velocity block,
    (h/2) sum_q w_q c_q t_q t_q^T per element with t from newton_vectors (the
    Newton term of section 3's alternating Picard-Newton iteration; c_q =
    4 nu'(gamma_dot) / gamma_dot at the Gauss points).
    """
    h = mesh.h
    E = mesh.n_elem
    nv = 3 * mesh.n_nodes
    ntot = nv + 4 * E
    M = velocity_tables(form)
    Be = -(0.5 * h) ** 2 * divergence_table()              # same for every element
    if form == "laplace":
        comp = np.tile(np.arange(3), 27)
        mask = comp[:, None] == comp[None, :]
    else:
        mask = np.ones((81, 81), dtype=bool)
    ii, jj = np.nonzero(mask)

    def block(e0, e1):
        En = e1 - e0
        Ae = (0.5 * h) * (nu_q[e0:e1] @ M.reshape(27, 81 * 81)).reshape(En, 81, 81)
        if newton is not None:
            c_q, D_q = newton
            t = newton_vectors(mesh, D_q[e0:e1])
            Ae = Ae + (0.5 * h) * np.einsum("eq,eqx,eqy->exy", c_q[e0:e1] * _WTS[None, :], t, t)
        vd = (3 * mesh.elem_node[e0:e1, :, None] + np.arange(3)[None, None, :]).reshape(En, 81)
        pd = nv + 4 * np.arange(e0, e1)[:, None] + np.arange(4)[None, :]
        rows = [vd[:, ii].ravel(), pd[:, :, None].repeat(81, 2).ravel(), vd[:, None, :].repeat(4, 1).ravel()]
        cols = [vd[:, jj].ravel(), vd[:, None, :].repeat(4, 1).ravel(), pd[:, :, None].repeat(81, 2).ravel()]
        vals = [Ae[:, ii, jj].ravel(), np.broadcast_to(Be, (En, 4, 81)).ravel(),
                np.broadcast_to(Be, (En, 4, 81)).ravel()]
        r = np.concatenate(rows)
        c = np.concatenate(cols)
        v = np.concatenate(vals)
        return sp.coo_matrix((v, (r, c)), shape=(ntot, ntot)).tocsr()

    # one COO pass for meshes up to ASSEMBLY_CHUNK elements; larger meshes are
    # summed per chunk first (bounding the host memory of the triplets), then the
    # chunk sums are summed in one more COO pass; explicit zeros stay in the pattern
    if E <= ASSEMBLY_CHUNK:
        K = block(0, E)
    else:
        parts = [block(e0, min(E, e0 + ASSEMBLY_CHUNK)).tocoo() for e0 in range(0, E, ASSEMBLY_CHUNK)]
        r = np.concatenate([q.row for q in parts])
        c = np.concatenate([q.col for q in parts])
        v = np.concatenate([q.data for q in parts])
        del parts
        K = sp.coo_matrix((v, (r, c)), shape=(ntot, ntot)).tocsr()
    K.sort_indices()
    vd = (3 * mesh.elem_node[:, :, None] + np.arange(3)[None, None, :]).reshape(E, 81)
    L = load_table()
    F = np.zeros(ntot)
    fe = (0.5 * h) ** 3 * L[:, None] * np.asarray(f, dtype=np.float64)[None, :]   # (a, i)
    np.add.at(F, vd.ravel(), np.broadcast_to(fe.ravel(), (E, 81)).ravel())
    return K, F


def eliminate(K, F, free_mask, fixed_values):
    """Restrict to free dofs; move the fixed values to the right-hand side (lifting)."""
    free = np.nonzero(free_mask)[0]
    fixed = np.nonzero(~free_mask)[0]
    Kff = K[free][:, free].tocsr()
    Kff.sort_indices()
    b = F[free] - K[free][:, fixed] @ fixed_values[fixed]
    return Kff, b, free
