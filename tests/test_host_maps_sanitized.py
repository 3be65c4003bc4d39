"""The host map builder (csrc/maps.cpp) under AddressSanitizer and UndefinedBehaviorSanitizer.

A host-only driver (tests/host/maps_driver.cpp) is compiled with g++
-fsanitize=address,undefined together with maps.cpp, run on problems of
several shapes (two to four levels, uneven parts, overlap 1 and 2), and its
maps must equal the oracle's bit for bit (section 2.1 per level, the recursion
of section 2.2) with no sanitizer report.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle.gdsw import ras_owner
from harness import unit_cube_problem, die_problem
from tests.conftest import cached

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("asan")
    exe = str(d / "maps_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", os.path.join(ROOT, "tests", "host", "maps_driver.cpp"),
           os.path.join(ROOT, "paper_2606_01433_amd", "csrc", "maps.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _write(P, d, overlap):
    meta = np.array([P.n, P.n_nodes, P.n_elem, P.levels, overlap] + list(P.n_parts), dtype=np.int64)
    meta.tofile(os.path.join(d, "meta.bin"))
    np.asarray(P.node_dof, np.int32).tofile(os.path.join(d, "node_dof.bin"))
    np.asarray(P.elem_node, np.int32).tofile(os.path.join(d, "elem_node.bin"))
    np.asarray(P.elem_pdof, np.int32).tofile(os.path.join(d, "elem_pdof.bin"))
    np.asarray(P.elem_part, np.int32).tofile(os.path.join(d, "elem_part.bin"))
    for l, par in enumerate(P.part_parent):
        np.asarray(par, np.int32).tofile(os.path.join(d, f"parent{l + 1}.bin"))


@pytest.mark.parametrize("name,overlap", [("cube4_L2", 1), ("cube8_L3", 1), ("die16_L4_uneven", 1),
                                          ("die16_L3", 2)])
def test_maps_under_sanitizers_match_oracle(driver, tmp_path, name, overlap):
    make = {"cube4_L2": lambda: unit_cube_problem(),
            "cube8_L3": lambda: unit_cube_problem(n=8, block=2, levels=3),
            "die16_L4_uneven": lambda: die_problem(16, 8, 8, seed=3, levels=4, frac3=0.3),
            "die16_L3": lambda: die_problem(16, 8, 8, seed=0, levels=3)}[name]
    P = cached(("asan", name), make)
    ind, outd = tmp_path / "in", tmp_path / "out"
    ind.mkdir()
    outd.mkdir()
    _write(P, str(ind), overlap)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, str(ind), str(outd)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    H = oracle.setup(P, delta=overlap)
    for k, lev in enumerate(H.levels):
        p = str(outd / f"L{k + 1}_")
        rd = lambda f, dt: np.fromfile(p + f, dtype=dt)
        assert np.array_equal(rd("dom.bin", np.int32), np.concatenate(lev.maps.dom))
        assert np.array_equal(rd("inter.bin", np.int32), np.concatenate([np.asarray(i, np.int64) for i in lev.maps.inter]))
        assert np.array_equal(rd("ent_nodes.bin", np.int32), np.concatenate(lev.maps.entities))
        assert np.array_equal(rd("col_entity.bin", np.int32), lev.maps.col_entity)
        assert np.array_equal(rd("owner.bin", np.int32), ras_owner(lev.mesh, lev.maps))
