"""Pins of the oracle's index maps (overlap, interface, entities, interior sets).

Expected values are closed-form counts on cubes, derived in the comments.
"""
import numpy as np
import pytest

import oracle
from harness import unit_cube_problem
from tests.conftest import cached


def _maps(P, delta=1):
    return oracle.build_level(oracle.level1_mesh(P), delta)


def test_config1_interface_and_entities(cube4):
    m = _maps(cube4)
    # Gamma: interior nodes of the planes x = y = z = 1/2 of the 9^3 lattice:
    # three planes of 7x7 free nodes, pairwise sharing 7-node lines, all three the centre
    assert len(m.gamma_nodes) == 3 * 49 - 3 * 7 + 1 == 127
    sizes = sorted(len(e) for e in m.entities)
    # each plane minus its two centre lines: 4 quadrants of 3x3 (faces); each centre
    # line minus the centre: 2 segments of 3 (edges); the centre point (vertex)
    assert sizes == [1] + [3] * 6 + [9] * 12
    kinds = np.bincount(m.entity_kind, minlength=3)
    assert list(kinds) == [1, 6, 12]
    for E, parts in zip(m.entities, m.entity_parts):
        assert len(parts) == {1: 8, 3: 4, 9: 2}[len(E)]
    # 19 entities x 3 translations + 8 part constants
    assert m.n_coarse == 57 + 8 == 65


def test_config1_local_sizes(cube4):
    m = _maps(cube4)
    # closure of a corner part: lattice 0..4 per axis; one node layer -> 0..5; the wall
    # layer 0 is Dirichlet -> 5^3 free nodes, 375 velocity dofs + 8 elements x 4 modes
    assert [len(d) for d in m.dom] == [406] + [407] * 7       # part 0 holds the pinned mode
    # interior: nodes strictly inside the part (lattice 1..3), 27 x 3, plus 8 x 3 linear modes
    assert [len(i) for i in m.inter] == [105] * 8


@pytest.mark.parametrize("n,block", [(6, 2), (9, 3)])
def test_interior_block_formula(n, block):
    """Central part of an n^3 cube, b^3 blocks: 3(2b+3)^3 + 4b^3 overlapping dofs, 3(2b-1)^3 + 3b^3 interior."""
    P = cached(("cube", n, block), lambda: unit_cube_problem(n=n, block=block, levels=2))
    m = _maps(P)
    c = n // block // 2
    nb = n // block
    centre = c + nb * (c + nb * c)
    b = block
    assert len(m.dom[centre]) == 3 * (2 * b + 3) ** 3 + 4 * b ** 3
    assert len(m.inter[centre]) == 3 * (2 * b - 1) ** 3 + 3 * b ** 3


def test_overlap_matches_geometric_box():
    """On a cube with box-shaped parts, one node layer = the closure box grown by one lattice step."""
    P = cached(("cube", 6, 2), lambda: unit_cube_problem(n=6, block=2, levels=2))
    m = _maps(P)
    lat = np.rint(P.node_xyz / (0.5 * (1.0 / 6))).astype(int)
    nd = P.node_dof.reshape(-1, 3)
    ep = P.elem_pdof.reshape(-1, 4)
    for i in range(P.n_parts[0]):
        bx, by, bz = i % 3, (i // 3) % 3, i // 9
        lo = np.array([4 * bx, 4 * by, 4 * bz]) - 1
        hi = np.array([4 * bx + 4, 4 * by + 4, 4 * bz + 4]) + 1
        inbox = np.all((lat >= lo) & (lat <= hi), axis=1)
        want = set(int(x) for x in nd[inbox].ravel() if x >= 0)
        want |= set(int(x) for e in np.nonzero(P.elem_part == i)[0] for x in ep[e] if x >= 0)
        assert list(m.dom[i]) == sorted(want)


def test_every_free_dof_is_interior_or_interface(cube4):
    m = _maps(cube4)
    seen = np.zeros(cube4.n, dtype=int)
    for I in m.inter:
        seen[I] += 1
    seen[m.gamma_dofs] += 1
    assert np.all(seen == 1)
    for D, I in zip(m.dom, m.inter):
        assert set(I) <= set(D)
        assert np.all(np.diff(D) > 0)


def test_next_level_mesh(cube4):
    mesh = oracle.level1_mesh(cube4)
    m = oracle.build_level(mesh)
    nxt = oracle.next_mesh(mesh, m, np.zeros(8, dtype=int), 1)
    assert nxt.n_nodes == 19 and nxt.n_dof == 65
    # each part touches 3 faces, 3 edges and the vertex
    assert all(len(e) == 7 for e in nxt.elem_nodes)
    assert list(nxt.elem_pdof[:, 0]) == list(range(57, 65))
    # the vertex is adjacent to the 6 edges and the 12 faces (they all touch the centre's 3^3 lattice cell)
    v = int(np.nonzero(m.entity_kind == 0)[0][0])
    assert len(nxt.adj[v]) == 18
