"""The stage's side stream. On a grid with blocks near a body, those blocks run on a side stream of the
grid beside the block form's launch, forked from the caller's stream by an event and joined back into it;
while the caller's stream is being captured into a graph everything stays on that stream. The state after
eager steps on the default stream, eager steps on another stream and graph-replayed steps on either must
be the same bit for bit, and synchronising the caller's stream alone must be enough to read it."""
import sys

import numpy as np
import pytest

from paper_2501_06717_amd import workloads as wk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2501_06717_amd import binding
    binding.lib()
    return binding


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def near_body_blocks(wl):
    """Blocks whose cells or 2-deep face halos can meet a body sphere (a superset test on the host: the
    block's box grown by two cells against the sphere)."""
    n = 0
    for lv, ijk, sid in zip(wl.level, wl.ijk, wl.sim):
        s = wl.sims[sid]
        if not s.body_r > 0:
            continue
        dx = s.dx0 / (1 << int(lv))
        lo = np.array(s.origin) + (np.array(ijk) * 8 - 2) * dx
        hi = lo + 12 * dx
        c = np.array(s.body_c)
        d = np.maximum(np.maximum(lo - c, 0.0), c - hi)
        n += int((d * d).sum() <= s.body_r ** 2)
    return n


def steps(bd, wl, n_stages, stream, **kw):
    g = bd.Grid.from_workload(wl).upload()
    U0 = g.set_state(torch.from_numpy(wl.W).cuda())
    U1 = torch.zeros_like(U0)
    dt = torch.zeros(len(wl.sims), dtype=torch.float64, device="cuda")
    faults = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()  # the state is set on the current stream; the steps may run on another
    g.advance(U0, U1, dt, n_stages, faults=faults, stream=stream, **kw)
    (stream if stream is not None else torch.cuda.current_stream()).synchronize()
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
        out = (U0.cpu().numpy(), dt.cpu().numpy(), int(faults.item()))
    del U0, U1, g
    return out


@pytest.mark.parametrize("name", ["magnetosphere_64", "two_level_magnetosphere_48"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_flux"])
def test_side_stream_eager_and_graph_agree(bd, name, precision):
    wl = wk.magnetosphere(64) if name == "magnetosphere_64" else wk.two_level_magnetosphere(48)
    nn = near_body_blocks(wl)
    say(name, precision, wl.n_blocks, "blocks,", nn, "near the body")
    assert 0 < nn < wl.n_blocks
    kw = dict(flux="hlle", powell=True, cfl=0.8, precision=precision)
    side = torch.cuda.Stream()
    ref, rdt, rf = steps(bd, wl, 6, None, **kw)
    for stream, graph in ((side, False), (None, True), (side, True)):
        got, dt, f = steps(bd, wl, 6, stream, use_graph=graph, **kw)
        say("  stream", "side" if stream is not None else "default", "graph", graph)
        assert f == rf
        assert np.array_equal(dt, rdt)
        assert np.array_equal(got, ref)
    assert np.all(np.isfinite(ref))
