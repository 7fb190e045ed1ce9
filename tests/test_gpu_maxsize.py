"""GPU at the largest uniform grid one MI355X holds in FP64 with both stage buffers: 1024^3 cells
(2,097,152 blocks of 8^3). Each state array then holds 2^33 values (68.7 GB), so every device offset is
past 32 bits and the stage grid has 4.2 M workgroups.

The state depends on x only and repeats every 64 cells (8 blocks), with random values per x cell so the
limiter and the Powell source act everywhere. One step of the 1024^3 grid must then equal, block for
block and bit for bit, the same step on a periodic 8 x 2 x 2-block grid that holds one period (the
global dt is a maximum over the same set of cell values, so it is equal too); the small grid's step is
checked against the oracle within 1e-12, and sampled blocks of the large grid, the highest indices
among them, are checked against the oracle directly."""
import gc
import sys

import numpy as np
import pytest

from paper_2501_06717_amd import workloads as wk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_AXIS = 128                  # blocks per axis of the large grid
SMALL = (8, 2, 2)             # one period along x, two blocks along y and z
GROUPS = {"rho": [0], "mom": [1, 2, 3], "B": [4, 5, 6], "e": [7]}
TOL = 1e-12
KW = dict(flux="hlle", powell=True, cfl=0.8)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2501_06717_amd import binding
    binding.lib()
    return binding


def x_profile(seed):
    """Primitive values for the 64 x cells of one period: rho, p in [0.8, 1.2], u in [-0.1, 0.1],
    B in [0.3, 0.7]."""
    rng = np.random.default_rng(seed)
    prof = np.empty((8, 64))
    prof[0] = 1.0 + 0.2 * rng.uniform(-1, 1, 64)
    prof[1:4] = 0.1 * rng.uniform(-1, 1, (3, 64))
    prof[4:7] = 0.5 + 0.2 * rng.uniform(-1, 1, (3, 64))
    prof[7] = 1.0 + 0.2 * rng.uniform(-1, 1, 64)
    return prof


def small_workload(prof):
    lv, ijk, sid = wk.uniform_blocks(SMALL)
    sim = wk.Sim(SMALL, (0.0, 0.0, 0.0), 1.0)
    W = np.empty((8, len(lv), 8, 8, 8))
    for b in range(len(lv)):
        x0 = 8 * int(ijk[b, 0])
        W[:, b] = prof[:, None, None, x0:x0 + 8]
    return wk.Workload("x_period", lv, ijk, sid, [sim], W, **KW)


def group_err(got, ref):
    return {g: float(np.abs(got[vs] - ref[vs]).max() / max(np.abs(ref[vs]).max(), 1e-300)) for g, vs in GROUPS.items()}


def test_1024_cubed_one_step(bd, oracle_mod):
    gc.collect()
    torch.cuda.empty_cache()
    nb = N_AXIS ** 3
    state_bytes = 8 * nb * 512 * 8
    free, _ = torch.cuda.mem_get_info()
    if free < 2 * state_bytes + (8 << 30):
        pytest.skip(f"needs {2 * state_bytes / 1e9:.0f} GB of free device memory, {free / 1e9:.0f} GB free")

    wl = small_workload(x_profile(11))
    o = oracle_mod.Grid.from_workload(wl)
    R = o.set_state(wl.W)
    R1 = np.zeros_like(R)
    rdt, rf = o.advance(R, R1, np.zeros(1), 2, **KW)
    assert rf == 0

    gs = bd.Grid.from_workload(wl).upload()
    S0 = gs.set_state(torch.from_numpy(wl.W).cuda())
    S1 = torch.empty_like(S0)
    sdt = torch.zeros(1, dtype=torch.float64, device="cuda")
    sf = torch.zeros(1, dtype=torch.int32, device="cuda")
    S_in = S0.clone()
    gs.advance(S0, S1, sdt, 2, faults=sf, **KW)
    torch.cuda.synchronize()
    err = group_err(S0.cpu().numpy(), R)
    say("small grid vs oracle", err, "dt", float(sdt.item()), float(rdt[0]))
    assert int(sf.item()) == 0 and max(err.values()) <= TOL, err
    assert abs(float(sdt.item()) - float(rdt[0])) <= 1e-14 * float(rdt[0])

    lv, ijk, sid = wk.uniform_blocks((N_AXIS,) * 3)
    big = wk.Sim((N_AXIS,) * 3, (0.0, 0.0, 0.0), 1.0)
    g = bd.Grid(lv, ijk, sid, [big]).upload()
    # the small-grid block holding the same cell values as each large-grid block (i-fastest listing)
    src = (ijk[:, 0] % SMALL[0]) + SMALL[0] * ((ijk[:, 1] % SMALL[1]) + SMALL[1] * (ijk[:, 2] % SMALL[2]))
    idx = torch.from_numpy(src.astype(np.int64)).cuda()
    del lv, ijk, sid
    say("large grid:", nb, "blocks,", nb * 512, "cells,", 2 * state_bytes / 1e9, "GB of state")
    U0 = torch.empty((8, nb, 8, 8, 8), dtype=torch.float64, device="cuda")
    torch.index_select(S_in, 1, idx, out=U0)
    U1 = torch.empty_like(U0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    faults = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    g.advance(U0, U1, dt, 2, faults=faults, **KW)
    torch.cuda.synchronize()
    del U1
    say("  one step done; dt", float(dt.item()), "faults", int(faults.item()))
    assert int(faults.item()) == 0
    assert float(dt.item()) == float(sdt.item())

    # every block, bit for bit, against the small grid's step
    bad = 0
    chunk = 1 << 16
    for s in range(0, nb, chunk):
        e = min(nb, s + chunk)
        ref = torch.index_select(S0, 1, idx[s:e])
        bad += int((U0[:, s:e] != ref).flatten(2).any(dim=2).any(dim=0).sum().item())
        del ref
    say("  blocks differing from the one-period grid:", bad)
    assert bad == 0

    # sampled blocks against the oracle directly: the first, the last and random ones
    rng = np.random.default_rng(3)
    sample = np.unique(np.concatenate([np.arange(8), np.arange(nb - 8, nb), rng.integers(0, nb, 48)]))
    got = U0[:, torch.from_numpy(sample).cuda()].cpu().numpy()
    ref = R[:, src[sample]]
    err = group_err(got, ref)
    say("  sampled blocks vs oracle", err)
    assert max(err.values()) <= TOL, err
    del U0, S0, S1, S_in, g, gs
    gc.collect()
    torch.cuda.empty_cache()
