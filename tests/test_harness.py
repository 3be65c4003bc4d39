"""Pins of the seeded problem builder (it feeds both the oracle and the library)."""
import itertools

import numpy as np
import pytest

from harness import unit_cube_problem, die_problem
from harness.problems import carreau, shear_rate


@pytest.mark.parametrize("form", ["laplace", "sym"])
@pytest.mark.parametrize("n", [2, 4])
def test_manufactured_solution_is_exact(n, form):
    """Q2/P1disc contains the quadratic velocity / linear pressure pair, so K x_exact = b."""
    P = unit_cube_problem(n=n, block=max(1, n // 2), form=form)
    r = P.K() @ P.x_exact - P.b
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(P.b)


def test_matrix_symmetric(cube4):
    K = cube4.K()
    assert abs(K - K.T).max() <= 1e-15 * abs(K).max()


def _brute_force_nnz(P, cross_components):
    """Count free-dof pairs that share an element (the element-connectivity pattern)."""
    en = P.elem_node.reshape(-1, 27)
    pairs = set()
    for e in range(P.n_elem):
        vd = [(int(P.node_dof[3 * v + d]), d) for v in en[e] for d in range(3)]
        vd = [(g, d) for g, d in vd if g >= 0]
        pd = [int(x) for x in P.elem_pdof[4 * e:4 * e + 4] if x >= 0]
        for (g, d), (h, c) in itertools.product(vd, vd):
            if cross_components or d == c:
                pairs.add((g, h))
        for q in pd:
            for g, _ in vd:
                pairs.add((q, g))
                pairs.add((g, q))
    return len(pairs)


@pytest.mark.parametrize("form,cross", [("laplace", False), ("sym", True)])
def test_pattern_is_element_connectivity(form, cross):
    P = unit_cube_problem(n=4, form=form)
    assert len(P.col) == _brute_force_nnz(P, cross)
    # dof counts of the 4^3 cube: 7^3 free Q2 nodes, 64 elements x 4 modes minus the pin
    assert P.n == 3 * 7 ** 3 + 4 * 64 - 1 == 1284


def test_carreau_closed_forms():
    g = np.array([0.0, 0.5, 2.0, 10.0])
    assert np.all(carreau(g, 3.0, 7.0, 1.0) == 3.0)                       # n = 1: Newtonian
    assert carreau(np.array([0.0]), 2.5, 10.0, 0.4)[0] == 2.5              # nu(0) = nu0
    np.testing.assert_allclose(carreau(np.array([1.0]), 1.0, 1.0, 0.5), 2.0 ** (-0.25), rtol=1e-15)


def test_shear_rate_of_simple_shear():
    """u = (s y, 0, 0): D has entries s/2 at (x,y),(y,x), so gamma_dot = sqrt(2 * 2 (s/2)^2) = |s|."""
    s = 3.0
    grad = np.zeros((1, 3, 3))
    grad[0, 0, 1] = s
    np.testing.assert_allclose(shear_rate(grad), [s], rtol=1e-15)


def test_die_generator_recipe():
    P = die_problem(16, 8, 8, seed=0, levels=3)
    m = P.meta
    assert 0.17 <= m["masked"] <= 0.24
    assert P.n_parts[0] > P.n_parts[1] >= 1
    # outflow: free nodes exist on x = x_max, hence no pressure pin is needed
    assert np.all(P.elem_pdof >= 0)
    again = die_problem(16, 8, 8, seed=0, levels=3)
    assert np.array_equal(again.val, P.val) and np.array_equal(again.b, P.b)


def test_chunked_assembly_keeps_pattern_and_values(monkeypatch):
    """Large meshes are assembled in element chunks: same pattern (explicit zeros kept), same values to rounding."""
    import harness.assemble as A
    P0 = die_problem(8, 4, 4, seed=2, levels=2)
    monkeypatch.setattr(A, "ASSEMBLY_CHUNK", 37)
    P1 = die_problem(8, 4, 4, seed=2, levels=2)
    assert np.array_equal(P0.rowptr, P1.rowptr) and np.array_equal(P0.col, P1.col)
    assert np.abs(P0.val - P1.val).max() <= 8 * np.finfo(np.float64).eps * np.abs(P0.val).max()
    assert np.array_equal(P0.b, P1.b)


def test_newton_term_is_the_derivative_of_the_carreau_operator():
    """Finite-difference check of the Newton linearization (section 3's Picard-Newton iteration): with
    A(w) the velocity block assembled with nu(w) at the Gauss points, the Newton matrix J(u) = A(u) + N(u)
    satisfies J(u) d = (A(u + e d)(u + e d) - A(u - e d)(u - e d)) / (2 e) + O(e^2).  Also J = J^T (the
    operator is the gradient of a dissipation potential) and N differs from zero."""
    import numpy as np
    from harness.mesh import VoxelMesh
    from harness.assemble import assemble, gauss_gradients
    from harness.problems import carreau, carreau_slope, shear_rate, symmetric_gradients
    rng = np.random.Generator(np.random.PCG64(5))
    mesh = VoxelMesh(np.ones((2, 2, 1), dtype=bool), 0.5)
    nu0, lam, n_exp = 2.0, 3.0, 0.4
    u = rng.standard_normal((mesh.n_nodes, 3))
    d = rng.standard_normal((mesh.n_nodes, 3))
    nv = 3 * mesh.n_nodes

    def A_of(w):
        gdw = shear_rate(gauss_gradients(mesh, w))
        return assemble(mesh, carreau(gdw, nu0, lam, n_exp), "sym")[0].toarray()[:nv, :nv]

    grad = gauss_gradients(mesh, u)
    gd = shear_rate(grad)
    newton = (4.0 * carreau_slope(gd, nu0, lam, n_exp), symmetric_gradients(grad))
    J = assemble(mesh, carreau(gd, nu0, lam, n_exp), "sym", newton=newton)[0].toarray()[:nv, :nv]
    eps = 1e-5
    fd = (A_of(u + eps * d) @ (u + eps * d).ravel() - A_of(u - eps * d) @ (u - eps * d).ravel()) / (2 * eps)
    jd = J @ d.ravel()
    assert np.linalg.norm(jd - fd) <= 1e-7 * np.linalg.norm(jd)
    assert np.abs(J - J.T).max() <= 1e-12 * np.abs(J).max()
    assert np.linalg.norm(J - A_of(u)) >= 1e-3 * np.linalg.norm(J)


def test_carreau_slope_closed_form():
    import numpy as np
    from harness.problems import carreau, carreau_slope
    g = np.array([0.3, 1.7, 4.0])
    h = 1e-6
    fd = (carreau(g + h, 2.0, 3.0, 0.4) - carreau(g - h, 2.0, 3.0, 0.4)) / (2 * h) / g
    assert np.allclose(carreau_slope(g, 2.0, 3.0, 0.4), fd, rtol=1e-7)


def _quadratic_fields(xyz):
    import numpy as np
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return np.stack([x * x - 3 * y * z + 2 * x, x * y + z * z - 1.0, 4 * x * z - y * y + y], axis=1)


def test_prolongation_reproduces_quadratic_velocity_and_linear_pressure():
    """Nested Q2 / P1disc spaces: P u_c equals the fine interpolant of any coarse Q2 velocity and P1disc
    pressure exactly; here a global quadratic velocity and linear pressure (both in the coarse space),
    sampled on the coarse dofs, must come out as the same functions sampled on the fine dofs.  The free-dof
    prolongation is the sub-block of the full one at the free dofs."""
    import numpy as np
    from harness import die_problem
    from harness.problems import prolongation_full, prolongation, free_dof_index
    Pc = die_problem(8, 4, 4, seed=0, levels=2)
    Pf = die_problem(8, 4, 4, seed=0, levels=2, refine=2)
    assert abs(Pf.meta["h"] - Pc.meta["h"] / 2) < 1e-15
    F = prolongation_full(Pc, Pf)

    def sample(P):
        u = _quadratic_fields(P.node_xyz)
        h = P.meta["h"]
        cen = (P.meta["elem_ijk"] + 0.5) * h
        gp = np.array([1.5, -2.0, 0.75])
        modes = np.stack([cen @ gp + 0.25] + [np.full(cen.shape[0], 0.5 * h * gp[m]) for m in range(3)], axis=1)
        return np.concatenate([u.ravel(), modes.ravel()])

    xc, xf = sample(Pc), sample(Pf)
    assert np.abs(F @ xc - xf).max() <= 1e-12 * np.abs(xf).max()
    P = prolongation(Pc, Pf)
    assert P.shape == (Pf.n, Pc.n)
    sub = F[free_dof_index(Pf)][:, free_dof_index(Pc)]
    assert np.abs((P - sub)).max() == 0.0
