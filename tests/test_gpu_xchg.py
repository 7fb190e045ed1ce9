"""GPU ghost exchange between virtual processes (Sec. 4.2-4.4, Algorithm 4) through the C ABI: every
process packs its messages (copies, restrictions by finer senders, prolongations by coarser senders from
their pass-1 ghost cells) into one buffer per receiver, the buffers move by device copies standing in for
the transfers between GPUs, every process unpacks them by their headers and fills its boundary ghost
cells; the gathered views must equal bmhd_fill_ghosts' padded view bit for bit, for uniform and two-level
grids, every boundary type, and assignments from one process to one block per process. The full-size
case splits the 256^3 magnetosphere into eight 128^3 processes (4,096 blocks each)."""
import numpy as np
import pytest

from paper_2501_06717_amd import workloads as wk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GRIDS = {
    "periodic_2x2x2": lambda: wk.uniform_state((2, 2, 2)),
    "one_block_periodic": lambda: wk.uniform_state((1, 1, 1)),
    "odd_box_mixed_bc": lambda: wk.odd_box(),
    "two_level_periodic": lambda: wk.two_level_box(),
    "two_level_mixed_bc": lambda: wk.two_level_box(bc=(1, 2, 0, 0, 2, 1)),
    "two_roots_one_refined": lambda: wk.two_level_box(nroot=(2, 1, 1), refine=((1, 0, 0),)),
    "fast_wave_octant": lambda: wk.fast_wave((2, 2, 2), refine_octant=True),
    "magnetosphere_cut": lambda: wk.magnetosphere_cut(32),
    "two_level_magnetosphere_48": lambda: wk.two_level_magnetosphere(48),
}


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2501_06717_amd import binding
    binding.lib()
    return binding


def ranks(wl, kind, seed=0):
    nb = wl.n_blocks
    if kind == "one":
        return np.zeros(nb, np.int32), 1
    if kind == "each":
        return np.arange(nb, dtype=np.int32), nb
    if kind == "halves":
        return (np.arange(nb) * 2 // nb).astype(np.int32), 2
    rng = np.random.default_rng(seed)
    return rng.integers(0, 3, nb).astype(np.int32), 3


def gather(views, rank, n, nb):
    out = torch.empty((8, nb, 12, 12, 12), dtype=torch.float64, device=views[0].device)
    for r in range(n):
        ids = torch.from_numpy(np.nonzero(rank == r)[0]).to(views[0].device)
        if len(ids):
            out[:, ids] = views[r]
    return out


@pytest.mark.parametrize("kind", ["one", "halves", "random3", "each"])
@pytest.mark.parametrize("grid", list(GRIDS))
def test_exchange_equals_ghost_fill(bd, grid, kind):
    wl = GRIDS[grid]()
    if kind == "each" and wl.n_blocks > 64:
        pytest.skip("one process per block: small grids only")
    rank, n = ranks(wl, kind, seed=len(grid))
    print("xchg", grid, kind, n, "processes", wl.n_blocks, "blocks", flush=True)
    g = bd.Grid.from_workload(wl).upload()
    x = bd.Xchg(g, rank, n).upload()
    for field in ("unique", "random"):
        W = wk.unique_id_field(wl) if field == "unique" else wk.random_positive_state(wl, seed=2)
        U = torch.from_numpy(W).cuda() if field == "unique" else g.set_state(torch.from_numpy(W).cuda())
        ref = g.fill_ghosts(U)
        bad = torch.zeros(1, dtype=torch.int32, device="cuda")
        got = gather(x.run(U, bad=bad), rank, n, wl.n_blocks)
        torch.cuda.synchronize()
        assert int(bad.item()) == 0
        assert torch.equal(got, ref), (grid, kind, field, int((got != ref).sum()))


def test_eight_processes_of_128_cubed(bd):
    """The 256^3 magnetosphere as 2 x 2 x 2 processes of 128^3 cells (4,096 blocks each): face, edge and
    corner messages between them, outflow and inflow boundaries, equal to the single-process fill."""
    wl = wk.magnetosphere(256)
    ijk = np.asarray(wl.ijk).reshape(-1, 3)
    rank = ((ijk[:, 0] // 16) + 2 * (ijk[:, 1] // 16) + 4 * (ijk[:, 2] // 16)).astype(np.int32)
    g = bd.Grid.from_workload(wl).upload()
    x = bd.Xchg(g, rank, 8).upload()
    assert np.all(x.nloc == 4096)
    U = g.set_state(torch.from_numpy(wl.W).cuda())
    views = x.run(U)
    del U
    ref = g.fill_ghosts(g.set_state(torch.from_numpy(wl.W).cuda()))
    for r in range(8):
        ids = torch.from_numpy(np.nonzero(rank == r)[0]).cuda()
        assert torch.equal(views[r], ref[:, ids]), r


def test_damaged_header_is_skipped_and_counted(bd):
    """A receive buffer whose first header names another block is not unpacked (the view keeps its
    cells) and the message is counted."""
    wl = wk.uniform_state((2, 2, 2))
    rank = (np.arange(wl.n_blocks) % 2).astype(np.int32)
    g = bd.Grid.from_workload(wl).upload()
    x = bd.Xchg(g, rank, 2).upload()
    U = g.set_state(torch.from_numpy(wk.random_positive_state(wl, seed=3)).cuda())
    views = [x.new_view(r) for r in range(2)]
    for r in range(2):
        x.interior(r, U, views[r])
    sends = [torch.empty(x.send_len(1, s), dtype=torch.float64, device="cuda") for s in range(2)]
    recvs = [torch.empty(x.recv_len(1, r), dtype=torch.float64, device="cuda") for r in range(2)]
    for s in range(2):
        x.pack(1, s, views[s], sends[s])
    x.transfer(1, sends, recvs)
    recvs[0][0] = recvs[0][0] + 1.0           # the first message to process 0 now names another block
    before = views[0].clone()
    bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    x.unpack(1, 0, recvs[0], views[0], bad=bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 1
    lb, lo, hi = int(recvs[0][0].item()) - 1, recvs[0][1:4].long().cpu().numpy() + 2, recvs[0][4:7].long().cpu().numpy() + 2
    box = (slice(None), lb, slice(lo[2], hi[2] + 1), slice(lo[1], hi[1] + 1), slice(lo[0], hi[0] + 1))
    assert torch.equal(views[0][box], before[box])


SHARDED = {
    "magnetosphere_cut_hlle_powell": (lambda: wk.magnetosphere_cut(32), dict(flux="hlle", powell=True)),
    "two_level_box_body_hlle_powell": (lambda: wk.two_level_box(body=True), dict(flux="hlle", powell=True)),
    "two_level_mixed_bc_rusanov_fp32": (lambda: wk.two_level_box(bc=(1, 2, 0, 0, 2, 1)),
                                        dict(flux="rusanov", precision="fp32_flux")),
    "fast_wave_octant_linde_powell": (lambda: wk.fast_wave((2, 2, 2), refine_octant=True),
                                      dict(flux="linde", powell=True)),
}


def single_process_steps(g, U, n_steps, faults, **kw):
    """The reference: bmhd_advance step by step with the same per-step dt (CFL 0.8 minimum)."""
    U1 = torch.empty_like(U)
    for _ in range(n_steps):
        dt = g.reduce_dt(U, 0.8)
        g.advance(U, U1, dt, 2, recompute_dt=False, faults=faults, **kw)


@pytest.mark.parametrize("for_stage", [False, True])
@pytest.mark.parametrize("kind", ["halves", "random3", "each"])
@pytest.mark.parametrize("case", list(SHARDED))
def test_sharded_steps_equal_single_process(bd, case, kind, for_stage):
    """Two steps with every process advancing only its own blocks (both exchange passes, then each
    process's stage reading the ghost cells of faces with a neighbour on another process or level from its
    view and the rest in place, then the flux corrections) equal bmhd_advance bit for bit: the same stage
    kernels read the same ghost values, whether they come from the neighbours' interiors and the
    level-change halos or from messages. With complete views and with the stage-mode maps, whose views
    hold only what the stage and the packs read."""
    make, kw = SHARDED[case]
    wl = make()
    if kind == "each" and wl.n_blocks > 64:
        pytest.skip("one process per block: small grids only")
    rank, n = ranks(wl, kind, seed=len(case))
    print("sharded", case, kind, for_stage, n, "processes", wl.n_blocks, "blocks", flush=True)
    g = bd.Grid.from_workload(wl).upload()
    x = bd.Xchg(g, rank, n, for_stage=for_stage).upload()
    W = torch.from_numpy(wk.random_positive_state(wl, seed=7) if case.startswith("two_level") else wl.W).cuda()
    R = g.set_state(W)
    fa = torch.zeros(1, dtype=torch.int32, device="cuda")
    single_process_steps(g, R, 2, fa, **kw)
    U = g.set_state(W)
    U1 = torch.empty_like(U)
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    x.advance(U, U1, 2, cfl=0.8, faults=fb, **kw)
    torch.cuda.synchronize()
    assert int(fa.item()) == int(fb.item()) == 0
    assert torch.equal(U, R), (case, kind, float((U - R).abs().max()))


def test_sharded_step_of_eight_128_cubed_processes(bd):
    """One step of the 256^3 magnetosphere as 2 x 2 x 2 processes of 128^3 cells (stage-mode maps) equals
    the single-process step bit for bit."""
    wl = wk.magnetosphere(256)
    ijk = np.asarray(wl.ijk).reshape(-1, 3)
    rank = ((ijk[:, 0] // 16) + 2 * (ijk[:, 1] // 16) + 4 * (ijk[:, 2] // 16)).astype(np.int32)
    g = bd.Grid.from_workload(wl).upload()
    x = bd.Xchg(g, rank, 8, for_stage=True).upload()
    W = torch.from_numpy(wl.W).cuda()
    R = g.set_state(W)
    fa = torch.zeros(1, dtype=torch.int32, device="cuda")
    single_process_steps(g, R, 1, fa, flux="hlle", powell=True)
    U = g.set_state(W)
    U1 = torch.empty_like(U)
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    x.advance(U, U1, 1, cfl=0.8, faults=fb, flux="hlle", powell=True)
    torch.cuda.synchronize()
    assert int(fa.item()) == int(fb.item()) == 0
    assert torch.equal(U, R)


def test_sharded_stage_refuses_what_it_does_not_take(bd):
    wl = wk.uniform_state((2, 2, 2))
    g = bd.Grid.from_workload(wl).upload()
    x = bd.Xchg(g, np.zeros(wl.n_blocks, np.int32), 1).upload()
    U = g.set_state(torch.from_numpy(wl.W).cuda())
    view = x.run(U)[0]
    dt = g.reduce_dt(U, 0.8)
    with pytest.raises(bd.BmhdError):
        x.stage(0, 2, view, U, U, torch.empty_like(U), dt)
    with pytest.raises(bd.BmhdError):
        x.stage(0, 0, view, U, U, torch.empty_like(U), dt, local_dt=True)
    with pytest.raises(bd.BmhdError):
        x.stage(0, 0, view, U, U, torch.empty_like(U), dt, persist_wgs=256)
