"""Problem builders: the manufactured unit-cube case and seeded voxel dies.

A Problem holds exactly what the library's setup call receives: the CSR
matrix K over free dofs (velocity 3*node+d first, then pressure 4*elem+m,
each compacted in that order), node_dof / elem_node / elem_pdof / elem_part
maps, the part hierarchy, and a right-hand side.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .mesh import VoxelMesh, axis_segments, part_hierarchy, die_voxels, FACES
from .assemble import assemble, eliminate, gauss_gradients


@dataclass
class Problem:
    name: str
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    b: np.ndarray
    n_nodes: int
    node_dof: np.ndarray          # (n_nodes*3,) int32, -1 = Dirichlet
    n_elem: int
    elem_node: np.ndarray         # (n_elem*27,) int32
    elem_pdof: np.ndarray         # (n_elem*4,) int32, -1 = pinned
    elem_part: np.ndarray         # (n_elem,) int32
    levels: int
    n_parts: List[int]
    part_parent: List[np.ndarray]
    node_xyz: np.ndarray
    x_exact: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    def K(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def with_hierarchy(self, elem_part, n_parts, part_parent, levels):
        import copy
        q = copy.copy(self)
        q.elem_part = np.asarray(elem_part, dtype=np.int32)
        q.n_parts = list(n_parts)
        q.part_parent = [np.asarray(p, dtype=np.int32) for p in part_parent]
        q.levels = levels
        return q


def uniform_segments(n, block):
    return (np.arange(n) // block).astype(np.int64)


def _number_dofs(mesh, dir_node, pinned_p):
    nv = 3 * mesh.n_nodes
    free = np.ones(nv + 4 * mesh.n_elem, dtype=bool)
    free[(3 * np.nonzero(dir_node)[0][:, None] + np.arange(3)).ravel()] = False
    for e, m in pinned_p:
        free[nv + 4 * e + m] = False
    idx = -np.ones(free.shape[0], dtype=np.int64)
    idx[free] = np.arange(int(free.sum()))
    node_dof = idx[:nv].astype(np.int32)
    elem_pdof = idx[nv:].astype(np.int32)
    return free, node_dof, elem_pdof


def _build(name, mesh, nu_q, form, f, dir_node, dir_values, pinned_p, pin_values,
           elem_part, n_parts, part_parent, levels, x_full=None, meta=None, newton=None, rhs_extra=None):
    K, F = assemble(mesh, nu_q, form, f, newton=newton)
    if rhs_extra is not None:
        F = F + rhs_extra
    free, node_dof, elem_pdof = _number_dofs(mesh, dir_node, pinned_p)
    fixed_vals = np.zeros(free.shape[0])
    nv = 3 * mesh.n_nodes
    fixed_vals[:nv] = dir_values.ravel()
    for (e, m), v in zip(pinned_p, pin_values):
        fixed_vals[nv + 4 * e + m] = v
    Kff, b, free_idx = eliminate(K, F, free, fixed_vals)
    x_exact = None if x_full is None else x_full[free_idx]
    return Problem(name=name, n=Kff.shape[0], rowptr=Kff.indptr.astype(np.int64),
                   col=Kff.indices.astype(np.int32), val=Kff.data.astype(np.float64), b=b,
                   n_nodes=mesh.n_nodes, node_dof=node_dof, n_elem=mesh.n_elem,
                   elem_node=mesh.elem_node.ravel().astype(np.int32), elem_pdof=elem_pdof,
                   elem_part=np.asarray(elem_part, dtype=np.int32), levels=levels,
                   n_parts=list(n_parts), part_parent=[np.asarray(p, np.int32) for p in part_parent],
                   node_xyz=mesh.node_xyz, x_exact=x_exact, meta=meta or {})


def manufactured_u(xyz):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return np.stack([x * x + y * z, -2 * x * y + x * z, y * y], axis=1)


def manufactured_p(xyz):
    return xyz[:, 0] + 2 * xyz[:, 1] - 3 * xyz[:, 2]


MANUFACTURED_F = (-1.0, 2.0, -5.0)        # -lap u + grad p for the pair above


def unit_cube_problem(n=4, block=2, levels=2, pin=True, form="laplace", mu=1.0):
    """Unit cube, n^3 voxels, all-Dirichlet with the manufactured quadratic velocity.

    Parts are block^3 voxel blocks; coarser levels group part blocks 2x2x2.
    With pin=True the constant pressure mode of element 0 is fixed to its
    exact value so that the pressure is unique.
    """
    mesh = VoxelMesh(np.ones((n, n, n), dtype=bool), 1.0 / n)
    dir_node = np.zeros(mesh.n_nodes, dtype=bool)
    for e, fc in mesh.boundary_faces():
        dir_node[mesh.face_nodes(e, fc)] = True
    uex = manufactured_u(mesh.node_xyz)
    dir_values = np.where(dir_node[:, None], uex, 0.0)
    # exact P1disc modes: p(c) + (h/2)(p_x xi + p_y eta + p_z zeta)
    cen = (mesh.elem_ijk + 0.5) * mesh.h
    pmodes = np.stack([manufactured_p(cen), np.full(mesh.n_elem, 0.5 * mesh.h * 1.0),
                       np.full(mesh.n_elem, 0.5 * mesh.h * 2.0), np.full(mesh.n_elem, 0.5 * mesh.h * -3.0)], axis=1)
    x_full = np.concatenate([uex.ravel(), pmodes.ravel()])
    pinned = [(0, 0)] if pin else []
    pin_vals = [pmodes[0, 0]] if pin else []
    seg = uniform_segments(n, block)
    elem_part, n_parts, part_parent = part_hierarchy(mesh, seg, seg, seg, levels)
    nu_q = np.full((mesh.n_elem, 27), float(mu))
    return _build(f"cube{n}_b{block}_L{levels}", mesh, nu_q, form, MANUFACTURED_F, dir_node, dir_values,
                  pinned, pin_vals, elem_part, n_parts, part_parent, levels, x_full=x_full,
                  meta=dict(kind="cube", nx=n, ny=n, nz=n, h=mesh.h, form=form, mu=mu, pin=pin))


def carreau(gamma_dot, nu0, lam, n_exp):
    """Carreau law (section 3): nu = nu0 (1 + (lam * gamma_dot)^2)^((n-1)/2)."""
    return nu0 * (1.0 + (lam * gamma_dot) ** 2) ** ((n_exp - 1.0) / 2.0)


def shear_rate(grad):
    """gamma_dot = sqrt(2 D:D) with D the symmetric part of grad (last two axes i, k)."""
    D = 0.5 * (grad + np.swapaxes(grad, -1, -2))
    return np.sqrt(2.0 * np.sum(D * D, axis=(-1, -2)))


def _field_terms(rng):
    terms = []
    for _ in range(4):
        a = rng.standard_normal(3)
        k = rng.integers(1, 4, size=3)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        terms.append((a, k, ph))
    return terms


def _field_at(terms, x):
    u = np.zeros((x.shape[0], 3))
    for a, k, ph in terms:
        u += a[None, :] * np.sin(np.pi * (x @ k) + ph)[:, None]
    return u


def linearization_field(mesh, rng, lam, target=10.0, scale_mesh=None):
    """Seeded smooth velocity u_k = sum_q a_q sin(pi k_q . x + phi_q), scaled so max lam*gamma_dot = target
    (the maximum taken over the Gauss points of scale_mesh, default mesh: a refined mesh given its
    coarse mesh here carries the same function)."""
    terms = _field_terms(rng)
    ref = mesh if scale_mesh is None else scale_mesh
    gd = shear_rate(gauss_gradients(ref, _field_at(terms, ref.node_xyz)))
    return _field_at(terms, mesh.node_xyz) * (target / (lam * gd.max()))


def carreau_slope(gamma_dot, nu0, lam, n_exp):
    """nu'(gamma_dot) / gamma_dot = nu0 (n - 1) lam^2 (1 + (lam gamma_dot)^2)^((n-3)/2), finite at 0."""
    return nu0 * (n_exp - 1.0) * lam * lam * (1.0 + (lam * gamma_dot) ** 2) ** ((n_exp - 3.0) / 2.0)


def symmetric_gradients(grad):
    return 0.5 * (grad + np.swapaxes(grad, -1, -2))


def die_problem(nx=32, ny=16, nz=16, seed=0, nu0=1.0, lam=1.0, n_exp=0.5, levels=3,
                frac3=0.0, masked=0.20, inflow_speed=1.0, linearization="picard", refine=1):
    """Seeded die-like voxel channel with Carreau viscosity linearized at a smooth field.

    Inflow: two rectangular windows on x = 0 with a parabolic x-velocity;
    outflow: the x = x_max face (do-nothing); all other boundary faces no-slip.
    linearization: "picard" freezes the viscosity at the linearization point
    u_k (K = the Stokes operator with nu(u_k)); "newton" is the Newton step of
    the same nonlinear operator at u_k: the velocity block gains the
    derivative of nu, and the right-hand side is the one of the Newton update
    J(u_k) u_{k+1} = (J(u_k) - A(u_k)) u_k + f, i.e. the Newton term applied to
    u_k (with the same Dirichlet data).
    refine = 2: the same die with every voxel split into 2x2x2 (h halved; same
    obstacles, inflow windows and linearization field u_k(x)); its parts are
    2-voxel segments of the refined grid.  The pair (refine 1, refine 2) is a
    nested hierarchy for geometric multigrid (prolongation()).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    active = die_voxels(nx, ny, nz, rng, target=masked)
    h = 1.0 / ny
    coarse_mesh = None
    if refine == 2:
        coarse_mesh = VoxelMesh(active, h)
        active = active.repeat(2, 0).repeat(2, 1).repeat(2, 2)
        h = 0.5 * h
        nx, ny, nz = 2 * nx, 2 * ny, 2 * nz
    elif refine != 1:
        raise ValueError(refine)
    mesh = VoxelMesh(active, h)
    # boundary classification
    dir_node = np.zeros(mesh.n_nodes, dtype=bool)
    for e, fc in mesh.boundary_faces():
        axis, side = FACES[fc]
        if axis == 0 and side == 1 and mesh.elem_ijk[e, 0] == nx - 1:
            continue                      # outflow: natural condition
        dir_node[mesh.face_nodes(e, fc)] = True
    # two inflow windows on x = 0 (voxel-aligned), one in each half of y
    wins = []
    cny, cnz = ny // refine, nz // refine
    for half in range(2):
        wy = int(rng.integers(max(1, cny // 5), max(2, cny // 3) + 1))
        wz = int(rng.integers(max(1, cnz // 5), max(2, cnz // 3) + 1))
        ylo, yhi = (1, cny // 2 - wy) if half == 0 else (cny // 2, cny - 1 - wy)
        y0 = int(rng.integers(ylo, max(ylo, yhi) + 1))
        z0 = int(rng.integers(1, max(1, cnz - 1 - wz) + 1))
        hc = h * refine
        wins.append((y0 * hc, (y0 + wy) * hc, z0 * hc, (z0 + wz) * hc))
    g = np.zeros((mesh.n_nodes, 3))
    xyz = mesh.node_xyz
    on_in = dir_node & (mesh.node_lat[:, 0] == 0)
    for (ya, yb, za, zb) in wins:
        s = (xyz[:, 1] - ya) / (yb - ya)
        t = (xyz[:, 2] - za) / (zb - za)
        inside = on_in & (s >= 0) & (s <= 1) & (t >= 0) & (t <= 1)
        g[inside, 0] = inflow_speed * 16.0 * s[inside] * (1 - s[inside]) * t[inside] * (1 - t[inside])
    seg_rng = np.random.Generator(np.random.PCG64(seed + 1000))
    sx = axis_segments(nx, seg_rng, frac3)
    sy = axis_segments(ny, seg_rng, frac3)
    sz = axis_segments(nz, seg_rng, frac3)
    elem_part, n_parts, part_parent = part_hierarchy(mesh, sx, sy, sz, levels)
    uk = linearization_field(mesh, rng, lam, scale_mesh=coarse_mesh)
    grad = gauss_gradients(mesh, uk)
    gd = shear_rate(grad)                                     # (E, 27)
    nu_q = carreau(gd, nu0, lam, n_exp)
    newton = rhs_extra = None
    if linearization == "newton":
        newton = (4.0 * carreau_slope(gd, nu0, lam, n_exp), symmetric_gradients(grad))
        N = assemble(mesh, np.zeros_like(nu_q), "sym", (0.0, 0.0, 0.0), newton=newton)[0]
        u_full = np.concatenate([uk.ravel(), np.zeros(4 * mesh.n_elem)])
        rhs_extra = N @ u_full
        rhs_extra[3 * mesh.n_nodes:] = 0.0         # N holds the divergence blocks too: velocity rows only
    elif linearization != "picard":
        raise ValueError(linearization)
    tag = ("" if linearization == "picard" else "_newton") + ("" if refine == 1 else "_refined")
    return _build(f"die{nx}x{ny}x{nz}_s{seed}_L{levels}{tag}", mesh, nu_q, "sym", (0.0, 0.0, 0.0), dir_node, g,
                  [], [], elem_part, n_parts, part_parent, levels, newton=newton, rhs_extra=rhs_extra,
                  meta=dict(kind="die", nx=nx, ny=ny, nz=nz, h=h, seed=seed, nu0=nu0, lam=lam, n_exp=n_exp,
                            linearization=linearization, refine=refine,
                            elem_ijk=mesh.elem_ijk.copy(),
                            masked=float(1.0 - active.mean()), windows=wins, frac3=frac3,
                            nu_min=float(nu_q.min()), nu_max=float(nu_q.max())))


def random_vector(n, seed):
    """Seeded N(0, 1) vector (PCG64)."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n)


def prolongation_full(coarse, fine):
    """Prolongation of the nested Q2 / P1disc spaces from a die to its refinement (die_problem with
    refine = 2 of the same arguments), over all dofs before Dirichlet elimination: velocity 3 node + d,
    then pressure 4 elem + m (fine rows, coarse columns).  P u_c is the coarse finite element function
    evaluated on the fine dofs.  Velocity: every fine node takes the Q2 interpolant of a coarse element
    that contains it (the values agree on shared faces); pressure: every fine element takes the linear
    function of its parent element (constant mode c0 + (o . c) / 2 with o = +-1 the child's offset
    per axis, linear modes halved)."""
    import scipy.sparse as sp
    from .q2 import lagrange_1d
    hc, hf = coarse.meta["h"], fine.meta["h"]
    assert abs(hf - 0.5 * hc) < 1e-15 * hc
    cijk = coarse.meta["elem_ijk"]
    fijk = fine.meta["elem_ijk"]
    grid = -np.ones((coarse.meta["nx"], coarse.meta["ny"], coarse.meta["nz"]), dtype=np.int64)
    grid[cijk[:, 0], cijk[:, 1], cijk[:, 2]] = np.arange(cijk.shape[0])
    cen = coarse.elem_node.reshape(-1, 27).astype(np.int64)
    nvf, nvc = 3 * fine.n_nodes, 3 * coarse.n_nodes
    # velocity: a coarse element holding each fine node
    xf = fine.node_xyz / hc                                  # in coarse voxel units
    base = np.floor(xf + 1e-12).astype(np.int64)
    shape = np.array(grid.shape)
    elem = -np.ones(xf.shape[0], dtype=np.int64)
    cell = np.zeros_like(base)
    for ox in (0, -1):
        for oy in (0, -1):
            for oz in (0, -1):
                c = base + np.array([ox, oy, oz])
                ok = (elem < 0) & np.all((c >= 0) & (c < shape), axis=1) & np.all(xf - c <= 1.0 + 1e-12, axis=1)
                e = np.full(xf.shape[0], -1, dtype=np.int64)
                e[ok] = grid[c[ok, 0], c[ok, 1], c[ok, 2]]
                take = ok & (e >= 0)
                elem[take] = e[take]
                cell[take] = c[take]
    assert np.all(elem >= 0), "a fine node lies in no active coarse element"
    xi = 2.0 * (xf - cell) - 1.0
    phi = [lagrange_1d(xi[:, d])[0] for d in range(3)]
    k = np.arange(27)
    w = phi[0][:, k % 3] * phi[1][:, (k // 3) % 3] * phi[2][:, k // 9]      # (fine nodes, 27)
    cn = cen[elem]                                                          # (fine nodes, 27)
    keep = np.abs(w) > 1e-14
    vi, ai = np.nonzero(keep)
    rows = [3 * vi + d for d in range(3)]
    cols = [3 * cn[vi, ai] + d for d in range(3)]
    vals = [w[vi, ai]] * 3
    # pressure
    par = grid[fijk[:, 0] // 2, fijk[:, 1] // 2, fijk[:, 2] // 2]
    assert np.all(par >= 0)
    o = 2 * (fijk % 2) - 1
    ef = np.arange(fijk.shape[0])
    rows.append(nvf + 4 * ef)
    cols.append(nvc + 4 * par)
    vals.append(np.ones(ef.shape[0]))
    for m in range(3):
        rows.append(nvf + 4 * ef)
        cols.append(nvc + 4 * par + m + 1)
        vals.append(0.5 * o[:, m].astype(np.float64))
        rows.append(nvf + 4 * ef + m + 1)
        cols.append(nvc + 4 * par + m + 1)
        vals.append(np.full(ef.shape[0], 0.5))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    return sp.csr_matrix((v, (r, c)), shape=(nvf + 4 * fine.n_elem, nvc + 4 * coarse.n_elem))


def free_dof_index(P):
    """Full dof id (velocity 3 node + d, then pressure 4 elem + m) of every free dof, in free-dof order."""
    full = np.concatenate([np.asarray(P.node_dof, np.int64), np.asarray(P.elem_pdof, np.int64)])
    idx = np.full(P.n, -1, dtype=np.int64)
    ids = np.nonzero(full >= 0)[0]
    idx[full[ids]] = ids
    return idx


def prolongation(coarse, fine):
    """The prolongation between the free dofs (fine free x coarse free): the rows and columns of
    prolongation_full at the free dofs.  Coarse Dirichlet dofs contribute nothing (a coarse correction
    vanishes there); fine Dirichlet dofs have no row."""
    Pf = prolongation_full(coarse, fine)
    return Pf[free_dof_index(fine)][:, free_dof_index(coarse)].tocsr()
