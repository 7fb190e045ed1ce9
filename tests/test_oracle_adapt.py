"""Pins of the oracle's refinement criterion and grid adaptation (the grid adapts between steps, Sec. 2-3;
the criterion is a reading: the largest normalised jump of the density and of |B|^2 between a cell's two
face neighbours), CPU only."""
import numpy as np
import pytest

from paper_2501_06717_amd import workloads as wk


def test_uniform_state_refines_nothing_and_coarsens_everything(oracle_mod):
    wl = wk.uniform_state((2, 2, 2))
    g = oracle_mod.Grid.from_workload(wl)
    ind = g.block_indicator(g.set_state(wl.W))
    assert np.array_equal(ind, np.zeros(wl.n_blocks))
    lv, ijk, sim = g.adapt(ind, 0.1, 0.05)
    assert np.array_equal(lv, wl.level) and np.array_equal(ijk, np.asarray(wl.ijk).reshape(-1, 3))
    tl = wk.with_state(wk.two_level_box(), None)
    g2 = oracle_mod.Grid.from_workload(tl)
    W = np.ones((8, tl.n_blocks, 8, 8, 8))
    ind2 = g2.block_indicator(g2.set_state(W))
    assert np.all(ind2 == 0.0)
    lv2, _, _ = g2.adapt(ind2, 0.1, 0.05)
    assert np.all(lv2 == 0) and len(lv2) == np.prod(tl.sims[0].nroot)


def test_indicator_of_a_linear_density_ramp(oracle_mod):
    """rho = 1 + a x in a periodic-free box (outflow): the jump across a cell is 2 a dx / (2 rho(x)), the
    largest where rho is smallest; at the first cell the outflow ghost repeats it, halving the jump."""
    wl = wk.uniform_state((2, 1, 1), bc=(1, 1, 1, 1, 1, 1), W0=(1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0))
    a = 0.25
    W = wl.W.copy()
    for b in range(wl.n_blocks):
        for i in range(8):
            x = (wl.ijk[b][0] * 8 + i + 0.5) * wl.sims[0].dx0
            W[0, b, :, :, i] = 1.0 + a * x
    g = oracle_mod.Grid.from_workload(wl)
    ind = g.block_indicator(g.set_state(W))
    dx = wl.sims[0].dx0
    rho = lambda i: 1.0 + a * (i + 0.5) * dx
    # block 0: the largest jump is at cell 1 (neighbours 0 and 2); cell 0 sees (0, 1) only
    want0 = max(abs(rho(2) - rho(0)) / (rho(2) + rho(0)), abs(rho(1) - rho(0)) / (rho(1) + rho(0)))
    want1 = abs(rho(9) - rho(7)) / (rho(9) + rho(7))     # block 1's first cell, its neighbour in block 0
    assert ind[0] == pytest.approx(want0, rel=1e-14) and ind[1] == pytest.approx(want1, rel=1e-14)


def test_a_density_jump_refines_the_roots_that_touch_it(oracle_mod):
    """A density ratio of 3 across the plane x = 16 in a 4 x 2 x 2 root box (outflow): the blocks whose
    cells see both sides (the two root columns next to the plane) get 0.5, all others 0; with thresholds
    0.3 / 0.1 exactly those roots are refined, and coarsening the result with a uniform state returns the
    root grid."""
    wl = wk.uniform_state((4, 2, 2), bc=(1,) * 6, W0=(1.0, 0.0, 0.0, 0.0, 0.2, 0.1, 0.0, 1.0))
    W = wl.W.copy()
    ijk = np.asarray(wl.ijk).reshape(-1, 3)
    W[0, ijk[:, 0] >= 2] = 3.0
    g = oracle_mod.Grid.from_workload(wl)
    ind = g.block_indicator(g.set_state(W))
    touch = (ijk[:, 0] == 1) | (ijk[:, 0] == 2)
    assert np.all(ind[touch] == 0.5) and np.all(ind[~touch] == 0.0)
    lv, nijk, sim = g.adapt(ind, 0.3, 0.1)
    assert len(lv) == 16 - 8 + 8 * 8
    refined_roots = {tuple(c // 2) for c, l in zip(nijk, lv) if l == 1}
    assert refined_roots == {tuple(c) for c in ijk[touch]}
    # the adapted grid is accepted and, with a uniform state, coarsens back to the roots
    new = wk.Workload("adapted", lv, nijk, sim, wl.sims, np.ones((8, len(lv), 8, 8, 8)))
    g2 = oracle_mod.Grid.from_workload(new)
    lv2, ijk2, _ = g2.adapt(g2.block_indicator(g2.set_state(new.W)), 0.3, 0.1)
    assert np.all(lv2 == 0) and np.array_equal(ijk2, ijk)


def test_hysteresis_keeps_a_refined_root_between_the_thresholds(oracle_mod):
    wl = wk.two_level_box(nroot=(2, 1, 1), refine=((1, 0, 0),))
    g = oracle_mod.Grid.from_workload(wl)
    ind = np.zeros(wl.n_blocks)
    ind[wl.level == 1] = 0.2                      # between r_coarsen = 0.1 and r_refine = 0.3
    lv, _, _ = g.adapt(ind, 0.3, 0.1)
    assert np.sum(lv == 1) == 8 and np.sum(lv == 0) == 1
    lv, _, _ = g.adapt(ind * 0.25, 0.3, 0.1)      # all children below r_coarsen
    assert np.all(lv == 0) and len(lv) == 2


def test_adaptive_run_conserves_totals(oracle_mod):
    """Criterion, remap and stages, three times: on a periodic box with a dense blob the totals of all
    eight conserved variables stay constant to round-off through refinement and coarsening."""
    base = wk.uniform_state((2, 2, 2), W0=(1.0, 0.3, 0.1, 0.0, 0.4, 0.2, 0.1, 1.0))
    W = base.W.copy()
    ijk = np.asarray(base.ijk).reshape(-1, 3)
    W[0, (ijk[:, 0] == 0) & (ijk[:, 1] == 0) & (ijk[:, 2] == 0), 2:6, 2:6, 2:6] = 2.0
    wl = base
    g = oracle_mod.Grid.from_workload(wl)
    U = g.set_state(W)

    def totals(wl, U):
        vol = (wl.sims[0].dx0 / 2.0 ** np.asarray(wl.level)) ** 3
        return np.array([np.sum(U[v].sum(axis=(1, 2, 3)) * vol) for v in range(8)])

    t0 = totals(wl, U)
    levels = []
    for _ in range(3):
        lv, nijk, sim = g.adapt(g.block_indicator(U), 0.05, 0.01)
        new = wk.Workload("adapted", lv, nijk, sim, wl.sims, np.zeros((8, len(lv), 8, 8, 8)))
        g2 = oracle_mod.Grid.from_workload(new)
        U = g.remap(U, g2)
        wl, g = new, g2
        levels.append(int(np.sum(lv == 1)))
        U1 = np.zeros_like(U)
        _, faults = g.advance(U, U1, [0.0], 2, flux="hlle", powell=False)
        assert faults == 0
    assert levels[0] > 0
    t1 = totals(wl, U)
    assert np.all(np.abs(t1 - t0) <= 1e-13 * np.abs(t0).max())
