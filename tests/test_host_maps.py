"""Host (CPU) checks of the library: exported symbols and bit-exact index maps.

The library's map builder runs on the host; gdsw_plan_* exposes it without a
GPU, so its integer output is compared element by element with the oracle's.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from oracle.gdsw import ras_owner
from harness import unit_cube_problem, die_problem
from tests.conftest import cached

gdsw = pytest.importorskip("paper_2606_01433_amd.gdsw")
HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "gdsw.h")


def _lib():
    try:
        return gdsw.load_library()
    except RuntimeError as e:
        pytest.skip(str(e))


def test_library_exports_every_declared_function():
    lib = _lib()
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(gdsw_[a-z_]+)\s*\(", text))
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(gdsw.SIGNATURES), declared ^ set(gdsw.SIGNATURES)


def _oracle_levels(P, delta=1):
    """Oracle maps of every level, following the recursion without any numerics."""
    mesh = oracle.level1_mesh(P)
    out = []
    for ell in range(1, P.levels):
        m = oracle.build_level(mesh, delta)
        out.append((mesh, m))
        if ell == P.levels - 1:
            break
        n_next = P.n_parts[ell]
        mesh = oracle.next_mesh(mesh, m, P.part_parent[ell - 1], n_next)
        if n_next == 1:
            break
    return out


def _compare(P, delta=1):
    lib_maps, has_coarsest = gdsw.plan_maps(P, overlap=delta)
    orc = _oracle_levels(P, delta)
    assert len(lib_maps) == len(orc)
    for lm, (mesh, om) in zip(lib_maps, orc):
        assert lm["n_dof"] == mesh.n_dof and lm["n_parts"] == mesh.n_parts
        assert np.array_equal(lm["dom_ptr"][1:] - lm["dom_ptr"][:-1], [len(d) for d in om.dom])
        assert np.array_equal(lm["dom"], np.concatenate(om.dom))
        assert np.array_equal(lm["int_ptr"][1:] - lm["int_ptr"][:-1], [len(d) for d in om.inter])
        assert np.array_equal(lm["inter"], np.concatenate(om.inter))
        assert np.array_equal(lm["gamma_nodes"], om.gamma_nodes)
        assert np.array_equal(lm["ent_ptr"][1:] - lm["ent_ptr"][:-1], [len(e) for e in om.entities])
        assert np.array_equal(lm["ent_nodes"], np.concatenate(om.entities))
        assert np.array_equal(lm["ent_kind"], om.entity_kind)
        assert lm["n_coarse"] == om.n_coarse
        assert np.array_equal(lm["col_entity"], om.col_entity)
        assert np.array_equal(lm["col_dir"], om.col_dir)
        assert np.array_equal(lm["owner"], ras_owner(mesh, om))
    return lib_maps


def test_maps_cube_two_level(cube4):
    _lib()
    _compare(cube4)


@pytest.mark.parametrize("delta", [0, 2])
def test_maps_other_overlaps(cube4, delta):
    _lib()
    _compare(cube4, delta)


def test_maps_cube_three_level():
    _lib()
    P = cached(("cube", 8, 2, 3), lambda: unit_cube_problem(n=8, block=2, levels=3))
    _compare(P)


def test_maps_die_four_level_uneven():
    _lib()
    P = cached(("die16", 4, 0.3), lambda: die_problem(16, 8, 8, seed=3, levels=4, frac3=0.3))
    maps = _compare(P)
    assert len(maps) == 3


def test_maps_with_permuted_dof_numbering():
    """Dof ids in no particular order (velocity ids no longer grow with the node, so the builder sorts
    each overlapping set's dofs instead of merging them in node order): the maps still equal the
    oracle's on the same numbering."""
    _lib()
    import copy
    P0 = cached(("die16", 4, 0.3), lambda: die_problem(16, 8, 8, seed=3, levels=4, frac3=0.3))
    P = copy.copy(P0)
    perm = np.random.default_rng(5).permutation(P0.n).astype(np.int32)
    nd = np.asarray(P0.node_dof).copy()
    nd[nd >= 0] = perm[nd[nd >= 0]]
    pd = np.asarray(P0.elem_pdof).copy()
    pd[pd >= 0] = perm[pd[pd >= 0]]
    P.node_dof, P.elem_pdof = nd, pd
    _compare(P)


def test_invalid_inputs_are_rejected(cube4):
    _lib()
    bad = cube4.with_hierarchy(cube4.elem_part.copy(), [8], [], 2)
    bad.elem_part[3] = 99
    with pytest.raises(gdsw.GdswError, match="EINVAL"):
        gdsw.plan_maps(bad)
    import copy
    dup = copy.copy(cube4)
    dup.node_dof = cube4.node_dof.copy()
    free = np.nonzero(dup.node_dof >= 0)[0]
    dup.node_dof[free[1]] = dup.node_dof[free[0]]          # one dof id used twice
    with pytest.raises(gdsw.GdswError, match="EINVAL"):
        gdsw.plan_maps(dup)
    assert gdsw.footprint_bytes(bad) == 0


def test_maps_all_pressure_modes_on_the_interface():
    """pressure_gamma = all: the library's host maps equal the oracle's for that reading."""
    from harness import die_problem
    P = die_problem(16, 8, 8, seed=0, levels=3)
    H = oracle.setup(P, pressure_gamma="all")
    maps, _ = gdsw.plan_maps(P, pressure_gamma="all")
    for k, lev in enumerate(H.levels):
        assert np.array_equal(maps[k]["inter"], np.concatenate([np.asarray(i, np.int64) for i in lev.maps.inter]))
        assert np.array_equal(maps[k]["dom"], np.concatenate(lev.maps.dom))
        assert np.array_equal(maps[k]["col_entity"], lev.maps.col_entity)
