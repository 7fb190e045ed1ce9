"""Pins of the oracle's message passing between processes (Sec. 4.2-4.4, Algorithm 4), CPU only.

The exchange over simulated processes (copy, restriction by the finer sender, prolongation by the coarser
sender from its pass-1 ghost cells, boundary cells filled by the receiver) must leave every block's
padded array equal, bit for bit, to the single-process ghost fill, whatever the assignment of blocks to
processes; the message lists must follow the counting loop (start offsets with the n_C = 7 header)."""
import numpy as np
import pytest

from paper_2501_06717_amd import workloads as wk

GRIDS = {
    "periodic_2x2x2": lambda: wk.uniform_state((2, 2, 2)),
    "one_block_periodic": lambda: wk.uniform_state((1, 1, 1)),
    "odd_box_mixed_bc": lambda: wk.odd_box(),
    "two_level_periodic": lambda: wk.two_level_box(),
    "two_level_mixed_bc": lambda: wk.two_level_box(bc=(1, 2, 0, 0, 2, 1)),
    "two_roots_one_refined": lambda: wk.two_level_box(nroot=(2, 1, 1), refine=((1, 0, 0),)),
    "fast_wave_octant": lambda: wk.fast_wave((2, 2, 2), refine_octant=True),
}


def _ranks(wl, kind, seed=0):
    nb = wl.n_blocks
    if kind == "one":
        return np.zeros(nb, np.int32), 1
    if kind == "each":
        return np.arange(nb, dtype=np.int32), nb
    if kind == "halves":
        return (np.arange(nb) * 2 // nb).astype(np.int32), 2
    rng = np.random.default_rng(seed)
    return rng.integers(0, 3, nb).astype(np.int32), 3


@pytest.mark.parametrize("kind", ["one", "halves", "random3", "each"])
@pytest.mark.parametrize("grid", list(GRIDS))
def test_exchange_equals_single_process_ghost_fill(oracle_mod, grid, kind):
    wl = GRIDS[grid]()
    rank, n = _ranks(wl, kind, seed=len(grid))
    g = oracle_mod.Grid.from_workload(wl)
    for U in (wk.unique_id_field(wl), g.set_state(wk.random_positive_state(wl, seed=2))):
        ref = g.fill_ghosts(U)
        got = g.xchg_run(U, rank, n)
        assert np.array_equal(got, ref), np.argwhere(got != ref)[:5]


def test_message_list_follows_the_counting_loop(oracle_mod):
    wl = wk.two_level_box(bc=(1, 2, 0, 0, 2, 1))
    rank, n = _ranks(wl, "random3", seed=4)
    g = oracle_mod.Grid.from_workload(wl)
    M = g.xchg_messages(rank, n)
    assert len(M) > 0
    kinds = set(M[:, 9].tolist())
    assert kinds == {0, 1, 2}                          # copy, restriction, prolongation all occur
    assert np.all((M[:, 9] == 2) == (M[:, 2] == 2))    # prolongations, and only they, travel in pass 2
    for key in {tuple(r) for r in M[:, :3].tolist()}:
        rows = M[(M[:, 0] == key[0]) & (M[:, 1] == key[1]) & (M[:, 2] == key[2])]
        assert np.array_equal(rows[:, 3], np.arange(len(rows)))            # i_M = 0, 1, 2, ...
        cells = np.prod(rows[:, 13:16] - rows[:, 10:13] + 1, axis=1)
        start = np.concatenate([[0], np.cumsum(7 + 8 * cells)[:-1]])
        assert np.array_equal(rows[:, 4], start)                             # start(i_M) with the header
        assert np.all(np.diff(rows[:, 5]) >= 0)                              # the local block order
        assert np.all(rank[rows[:, 5]] == key[0]) and np.all(rank[rows[:, 7]] == key[1])
    # message sizes: a same-level face message carries 8 x 8 x 2 cells, a restriction 4 x 4 x 2, a
    # prolongation onto a fine face 8 x 8 x 2 (the ghost layers of the finer block)
    cells = np.prod(M[:, 13:16] - M[:, 10:13] + 1, axis=1)
    assert cells[M[:, 9] == 0].max() == 128 and cells[M[:, 9] == 1].max() == 32 and cells[M[:, 9] == 2].max() >= 128


@pytest.mark.parametrize("grid", list(GRIDS))
def test_every_ghost_cell_is_sent_exactly_once(oracle_mod, grid):
    """Each ghost cell inside the domain (or across a periodic face) is written by exactly one message;
    interior cells and ghost cells beyond an outflow or inflow face by none."""
    wl = GRIDS[grid]()
    rank, n = _ranks(wl, "random3", seed=1)
    M = oracle_mod.Grid.from_workload(wl).xchg_messages(rank, n)
    cnt = np.zeros((wl.n_blocks, 12, 12, 12), np.int64)
    for r in M:
        b, lo, hi = r[7], r[10:13] + 2, r[13:16] + 2
        cnt[b, lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += 1
    sim = wl.sims[0]
    idx = np.arange(12) - 2
    for b in range(wl.n_blocks):
        lv = wl.level[b]
        inside = np.ones((12, 12, 12), bool)
        ghost = np.zeros((12, 12, 12), bool)
        for a in range(3):
            N = sim.nroot[a] * 8 * 2 ** lv
            G = wl.ijk[b][a] * 8 + idx
            ok = (G >= 0) & (G < N)
            periodic = sim.bc[2 * a] == 0 and sim.bc[2 * a + 1] == 0
            shape = [1, 1, 1]
            shape[2 - a] = 12
            inside &= (ok | periodic).reshape(shape)
            ghost |= ((idx < 0) | (idx > 7)).reshape(shape)
        want = (inside & ghost).astype(np.int64)
        assert np.array_equal(cnt[b], want), (b, np.argwhere(cnt[b] != want)[:4])
