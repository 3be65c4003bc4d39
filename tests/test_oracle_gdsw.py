"""Pins of the oracle's coarse basis, Galerkin operator and preconditioner."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spl

import oracle
from harness import unit_cube_problem, random_vector
from oracle.gdsw import gamma_basis, coarse_basis
from tests.conftest import cached


def test_partition_of_unity(cube4_h, cube4):
    lev = cube4_h.levels[0]
    m = lev.maps
    PhiG = gamma_basis(cube4.n, m).toarray()
    nd = cube4.node_dof.reshape(-1, 3)
    for d in range(3):
        s = PhiG[:, m.col_dir == d].sum(axis=1)
        gdofs = [int(nd[v, d]) for v in m.gamma_nodes if nd[v, d] >= 0]
        assert np.all(s[gdofs] == 1.0)
        assert s.sum() == len(gdofs)
    sp_ = PhiG[:, m.col_dir == 3].sum(axis=1)
    p0 = [int(x) for x in cube4.elem_pdof.reshape(-1, 4)[:, 0] if x >= 0]
    assert np.all(sp_[p0] == 1.0) and sp_.sum() == len(p0)


def test_translations_reproduced_on_floating_parts():
    """Sum of all (entity, d) columns equals the translation e_d on parts whose closure is Dirichlet-free."""
    P = cached(("cube", 6, 2), lambda: unit_cube_problem(n=6, block=2, levels=2))
    H = cached(("cube6h",), lambda: oracle.setup(P))
    lev = H.levels[0]
    m = lev.maps
    Phi = lev.Phi.toarray()
    centre = 13
    I = m.inter[centre]
    nd = P.node_dof.reshape(-1, 3)
    for d in range(3):
        s = Phi[:, m.col_dir == d].sum(axis=1)
        vel_d = set(int(x) for x in nd[:, d] if x >= 0)
        want = np.array([1.0 if int(g) in vel_d else 0.0 for g in I])
        np.testing.assert_allclose(s[I], want, atol=1e-12)


def test_extension_annihilates_interior_rows(cube4_h):
    lev = cube4_h.levels[0]
    KPhi = (lev.K @ lev.Phi).toarray()
    allI = np.concatenate(lev.maps.inter)
    assert np.abs(KPhi[allI]).max() <= 1e-12 * np.abs(KPhi).max()


def test_pressure_columns_have_no_interior_part(cube4_h):
    """B^T chi_i vanishes at nodes inside part i (the divergence theorem), so the extension is zero.

    Part 0 holds the pinned constant of element 0, so its column is not a constant over the
    whole part and does get an interior part.
    """
    lev = cube4_h.levels[0]
    Phi = lev.Phi.toarray()
    m = lev.maps
    allI = np.concatenate(m.inter)
    pcols = np.nonzero(m.col_dir == 3)[0]
    assert np.abs(Phi[np.ix_(allI, pcols[1:])]).max() <= 1e-13
    assert np.abs(Phi[np.ix_(m.inter[0], pcols[:1])]).max() > 1e-3


def test_galerkin_equals_schur_complement(cube4_h):
    """Phi^T K Phi = Phi_G^T (K_GG - K_GI K_II^-1 K_IG) Phi_G, computed densely."""
    lev = cube4_h.levels[0]
    K = lev.K.toarray()
    m = lev.maps
    I = np.concatenate(m.inter)
    G = m.gamma_dofs
    S = K[np.ix_(G, G)] - K[np.ix_(G, I)] @ np.linalg.solve(K[np.ix_(I, I)], K[np.ix_(I, G)])
    PhiG = gamma_basis(K.shape[0], m).toarray()[G]
    A0 = cube4_h.K_coarsest.toarray()
    np.testing.assert_allclose(A0, PhiG.T @ S @ PhiG, atol=1e-12 * np.abs(A0).max())
    assert np.abs(A0 - A0.T).max() <= 1e-13 * np.abs(A0).max()
    pp = np.nonzero(m.col_dir == 3)[0][1:]
    assert np.abs(A0[np.ix_(pp, pp)]).max() <= 1e-13 * np.abs(A0).max()


def test_unpinned_coarse_operator_has_constant_pressure_null_vector():
    P = cached(("cube4_nopin",), lambda: unit_cube_problem(pin=False))
    H = oracle.setup(P)
    A0 = H.K_coarsest.toarray()
    m = H.levels[0].maps
    v = (m.col_dir == 3).astype(float)
    assert np.linalg.norm(A0 @ v) <= 1e-12 * np.abs(A0).max()
    sv = np.linalg.svd(A0, compute_uv=False)
    assert sv[-1] <= 1e-12 * sv[0] < sv[-2]


def _dense_B(P, combine, L=None):
    """B of eq. (2.2) from explicit dense restriction matrices (brute force, tiny meshes)."""
    H = oracle.setup(P, combine=combine, levels=L)
    K = P.K().toarray()

    def level(k, Kk):
        lev = H.levels[k]
        n = Kk.shape[0]
        B = np.zeros((n, n))
        for i, D in enumerate(lev.maps.dom):
            R = np.zeros((len(D), n))
            R[np.arange(len(D)), D] = 1.0
            Rt = R.T.copy()
            if combine == "RAS":
                Rt[:, lev.owner[D] != i] = 0.0
            B += Rt @ np.linalg.inv(R @ Kk @ R.T) @ R
        Phi = lev.Phi.toarray()
        K0 = Phi.T @ Kk @ Phi
        if k + 1 < len(H.levels):
            inner = level(k + 1, K0)
        else:
            inner = np.linalg.inv(K0)
        return B + Phi @ inner @ Phi.T
    return H, level(0, K)


@pytest.mark.parametrize("combine", ["AS", "RAS"])
def test_apply_equals_dense_operator_two_level(cube4, combine):
    H, B = _dense_B(cube4, combine)
    for s in range(3):
        r = random_vector(cube4.n, s)
        np.testing.assert_allclose(oracle.apply(H, r), B @ r, rtol=0, atol=1e-10 * np.abs(B @ r).max())


def test_apply_equals_dense_operator_three_level():
    P = cached(("cube4_b1_L3",), lambda: unit_cube_problem(n=4, block=1, levels=3))
    assert P.n_parts == [64, 8]
    H, B = _dense_B(P, "RAS")
    r = random_vector(P.n, 7)
    np.testing.assert_allclose(oracle.apply(H, r), B @ r, rtol=0, atol=1e-10 * np.abs(B @ r).max())


def test_additive_operator_is_symmetric(cube4):
    H = oracle.setup(cube4, combine="AS")
    r1, r2 = random_vector(cube4.n, 1), random_vector(cube4.n, 2)
    a, b = r1 @ oracle.apply(H, r2), r2 @ oracle.apply(H, r1)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_single_part_one_level_is_exact_inverse(cube4):
    P = cube4.with_hierarchy(np.zeros(cube4.n_elem), [1], [], 2)
    H = oracle.setup(P, no_coarse=True)
    r = random_vector(P.n, 3)
    x = spl.spsolve(P.K().tocsc(), r)
    np.testing.assert_allclose(oracle.apply(H, r), x, atol=1e-12 * np.abs(x).max())
    K = P.K()
    xs, info = oracle.fgmres(lambda v: K @ v, lambda v: oracle.apply(H, v), P.b, tol=1e-10)
    assert info["iterations"] == 1 and info["converged"]


def test_three_levels_with_one_subregion_is_two_level(cube4):
    P3 = cube4.with_hierarchy(cube4.elem_part, [8, 1], [np.zeros(8)], 3)
    H2 = oracle.setup(cube4)
    H3 = oracle.setup(P3)
    r = random_vector(cube4.n, 4)
    assert np.array_equal(oracle.apply(H2, r), oracle.apply(H3, r))


def test_solve_matches_manufactured_solution(cube4, cube4_h):
    K = cube4.K()
    x, info = oracle.fgmres(lambda v: K @ v, lambda v: oracle.apply(cube4_h, v), cube4.b, tol=1e-10)
    assert info["converged"]
    assert np.linalg.norm(K @ x - cube4.b) <= 1e-10 * np.linalg.norm(cube4.b)
    np.testing.assert_allclose(x, cube4.x_exact, atol=1e-7)
    np.testing.assert_allclose(oracle.solve_direct(cube4), cube4.x_exact, atol=1e-11)
