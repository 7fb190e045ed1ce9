"""Error returns of the C ABI on an uploaded grid (GPU): every one is detected on the host before any
kernel is launched, returns its code and leaves a message in bmhd_last_error."""
import ctypes

import numpy as np
import pytest

from paper_2501_06717_amd import workloads as wk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EINVAL, EUNSUPPORTED = -1, -4


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2501_06717_amd import binding as bd
    wl = wk.two_level_box()
    g = bd.Grid.from_workload(wl).upload()
    U0 = g.set_state(torch.from_numpy(wl.W).cuda())
    U1 = torch.zeros_like(U0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    return bd, g, U0, U1, dt


def call_advance(bd, g, U0p, U1p, dtp, n, o):
    return bd.lib().bmhd_advance(g.h, ctypes.c_void_p(U0p), ctypes.c_void_p(U1p), ctypes.c_void_p(dtp), n,
                                 ctypes.byref(o), None, None)


def test_bad_pointers_and_counts(env):
    bd, g, U0, U1, dt = env
    L = bd.lib()
    o = bd.make_opts(flux="hlle", powell=True)
    p0, p1, pd = U0.data_ptr(), U1.data_ptr(), dt.data_ptr()
    assert call_advance(bd, g, 0, p1, pd, 2, o) == EINVAL and b"state pointers" in L.bmhd_last_error()
    assert call_advance(bd, g, p0 + 4, p1, pd, 2, o) == EINVAL
    assert call_advance(bd, g, p0, p0, pd, 2, o) == EINVAL
    assert call_advance(bd, g, p0, p1, pd, -1, o) == EINVAL and b"n_stages" in L.bmhd_last_error()
    og = bd.make_opts(flux="hlle", use_graph=True)
    assert call_advance(bd, g, p0, p1, pd, 3, og) == EINVAL and b"even" in L.bmhd_last_error()
    assert L.bmhd_fill_ghosts(g.h, ctypes.c_void_p(p0 + 8 * 3 + 4), ctypes.c_void_p(p1), None) == EINVAL
    assert L.bmhd_reduce_dt(g.h, ctypes.c_void_p(p0), ctypes.c_double(0.0), ctypes.c_void_p(pd), None) == EINVAL


@pytest.mark.parametrize("field,value,msg", [
    ("flux", 7, b"flux"), ("precision", 5, b"precision"), ("slab", 6, b"slab"), ("scheme", 9, b"scheme"),
    ("persist_wgs", -1, b"persist"), ("local_dt", 2, b"local_dt"), ("cfl", -0.5, b"cfl"),
])
def test_bad_options(env, field, value, msg):
    bd, g, U0, U1, dt = env
    o = bd.make_opts(flux="hlle")
    setattr(o, field, value)
    assert call_advance(bd, g, U0.data_ptr(), U1.data_ptr(), dt.data_ptr(), 2, o) == EINVAL
    assert msg in bd.lib().bmhd_last_error()


def test_unsupported_combinations(env):
    bd, g, U0, U1, dt = env
    mlp = bd.Mlp(32)
    stats = torch.zeros(80)
    stats[32:64] = 1.0
    stats[72:80] = 1.0
    L = g.learned(mlp, stats)
    # the learned form needs a single-level grid: this one has a resolution change
    with pytest.raises(bd.BmhdError, match="single-level"):
        g.advance(U0, U1, dt, 2, flux="hlle", learned=L)
    L.mode = 3
    with pytest.raises(bd.BmhdError, match="mode"):
        g.advance(U0, U1, dt, 2, flux="hlle", learned=L)
    # the binding checks the size of a per-cell dt
    with pytest.raises(bd.BmhdError, match="local_dt"):
        g.advance(U0, U1, dt, 2, flux="hlle", local_dt=True)


def test_state_is_untouched_by_a_refused_call(env):
    bd, g, U0, U1, dt = env
    before = U0.clone()
    o = bd.make_opts(flux="hlle")
    o.slab = 3
    assert call_advance(bd, g, U0.data_ptr(), U1.data_ptr(), dt.data_ptr(), 2, o) == EINVAL
    torch.cuda.synchronize()
    assert torch.equal(U0, before)
