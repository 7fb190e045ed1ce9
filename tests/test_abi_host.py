"""Host-side tests of the C ABI (no GPU needed): the library loads, exports every symbol the header
declares, validates descriptors, and builds the same neighbour tables as the oracle."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2501_06717_amd import binding as bd
from paper_2501_06717_amd import workloads as wk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bmhd.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bmhd_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = declared_functions()
    assert set(bd.EXPORTS) == set(names), names


def test_library_exports_every_declared_symbol():
    L = bd.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", bd.LIB_PATH], capture_output=True, text=True).stdout
    for name in declared_functions():
        assert re.search(rf"\bT {name}\b", out), name
    assert bd.lib().bmhd_version() >= 100


@pytest.mark.parametrize("make", [
    lambda: wk.uniform_state((1, 1, 1)),
    lambda: wk.uniform_state((2, 1, 1), bc=(1, 2, 0, 0, 1, 1)),
    lambda: wk.odd_box(),
    lambda: wk.two_level_box(),
    lambda: wk.two_level_box(bc=(1, 2, 0, 0, 2, 1)),
    lambda: wk.two_level_magnetosphere(48),
    lambda: wk.fast_wave((4, 2, 2), refine_octant=True),
])
def test_neighbors_match_oracle(oracle_mod, make):
    wl = make()
    g = bd.Grid.from_workload(wl)
    o = oracle_mod.Grid.from_workload(wl)
    assert np.array_equal(g.neighbors(), o.neighbors())


def test_two_level_magnetosphere_counts():
    wl = wk.two_level_magnetosphere(144)
    assert wl.n_blocks == 7456 and wl.n_cells == 3817472
    assert int((wl.level == 1).sum()) == 1856
    g = bd.Grid.from_workload(wl)
    assert g.info.n_flux_faces == 264


def _expect_einval(level, ijk, sim, sims):
    with pytest.raises(bd.BmhdError, match="error -1"):
        bd.Grid(level, ijk, sim, sims)


def test_descriptor_validation():
    s = wk.Sim((2, 1, 1), (0, 0, 0), 1.0)
    _expect_einval([0, 0], [[0, 0, 0], [0, 0, 0]], [0, 0], [s])          # overlap
    _expect_einval([0], [[0, 0, 0]], [0], [s])                            # uncovered root
    _expect_einval(np.zeros(0), np.zeros((0, 3)), np.zeros(0), [s])       # no blocks at all
    _expect_einval([0, 1], [[0, 0, 0], [2, 0, 0]], [0, 0], [s])           # partial refinement
    _expect_einval([0, 0], [[0, 0, 0], [1, 0, 0]], [0, 1], [s])           # bad simulation id
    _expect_einval([0, 2], [[0, 0, 0], [1, 0, 0]], [0, 0], [s])           # bad level
    _expect_einval([0, 0], [[0, 0, 0], [2, 0, 0]], [0, 0], [s])           # outside the root box
    s2 = wk.Sim((2, 1, 1), (0, 0, 0), 1.0, bc=(0, 1, 0, 0, 0, 0))
    _expect_einval([0, 0], [[0, 0, 0], [1, 0, 0]], [0, 0], [s2])          # unpaired periodic
    s3 = wk.Sim((2, 1, 1), (0, 0, 0), 0.0)
    _expect_einval([0, 0], [[0, 0, 0], [1, 0, 0]], [0, 0], [s3])          # zero cell size


def test_calls_before_upload_fail():
    wl = wk.uniform_state((1, 1, 1))
    g = bd.Grid.from_workload(wl)
    L = bd.lib()
    rc = L.bmhd_set_state(g.h, ctypes.c_void_p(8), ctypes.c_void_p(8), None)
    assert rc == -1 and b"upload" in L.bmhd_last_error()
    o = bd.make_opts()
    rc = L.bmhd_advance(g.h, ctypes.c_void_p(8), ctypes.c_void_p(16), ctypes.c_void_p(24), 2, ctypes.byref(o), None, None)
    assert rc == -1
    rc = L.bmhd_grid_upload(g.h, ctypes.c_void_p(8), ctypes.c_size_t(1 << 20), None)
    assert rc == -1 and b"aligned" in L.bmhd_last_error()
    rc = L.bmhd_grid_upload(g.h, ctypes.c_void_p(256), ctypes.c_size_t(16), None)
    assert rc == -3 and b"too small" in L.bmhd_last_error()
