"""GPU refinement criterion and grid adaptation against the oracle (the grid adapts between steps on the
host, Sec. 2-3): the per-block indicator bit for bit, the adapted block list equal, and an adaptive run
(criterion, new grid, remap, steps; three rounds) within 1e-12 of the oracle doing the same."""
import numpy as np
import pytest

from paper_2501_06717_amd import workloads as wk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2501_06717_amd import binding
    binding.lib()
    return binding


def blob_box():
    base = wk.uniform_state((3, 2, 2), bc=(1, 2, 0, 0, 1, 1), W0=(1.0, 0.3, 0.1, 0.0, 0.4, 0.2, 0.1, 1.0))
    W = base.W.copy()
    ijk = np.asarray(base.ijk).reshape(-1, 3)
    W[0, (ijk[:, 0] == 1) & (ijk[:, 1] == 0) & (ijk[:, 2] == 1), 3:7, 2:6, 1:5] = 2.5
    return wk.with_state(base, W)


CASES = {
    "blob_box": blob_box,
    "magnetosphere_cut": lambda: wk.magnetosphere_cut(32),
    "two_level_magnetosphere_48": lambda: wk.two_level_magnetosphere(48),
    "random_two_level": lambda: wk.with_state(wk.two_level_box(), wk.random_positive_state(wk.two_level_box(), seed=4)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_indicator_and_block_list_equal_the_oracle(bd, oracle_mod, case):
    wl = CASES[case]()
    o = oracle_mod.Grid.from_workload(wl)
    R = o.set_state(wl.W)
    ref = o.block_indicator(R)
    g = bd.Grid.from_workload(wl).upload()
    got = g.block_indicator(torch.from_numpy(R).cuda()).cpu().numpy()
    print("indicator", case, float(ref.max()), flush=True)
    assert np.array_equal(got, ref)
    for rr, rc in ((0.05, 0.01), (float(np.median(ref)), 0.5 * float(np.median(ref)))):
        lv, ijk, sim = g.adapt_blocks(got, rr, rc)
        olv, oijk, osim = o.adapt(ref, rr, rc)
        assert np.array_equal(lv, olv) and np.array_equal(ijk, oijk) and np.array_equal(sim, osim)


@pytest.mark.parametrize("case,flux", [("blob_box", "hlle"), ("random_two_level", "rusanov")])
def test_adaptive_run_matches_the_oracle(bd, oracle_mod, case, flux):
    """Both grids refine and coarsen over the rounds (thresholds at the indicators' quantiles for the
    random state)."""
    wl = CASES[case]()
    o = oracle_mod.Grid.from_workload(wl)
    R = o.set_state(wl.W)
    g = bd.Grid.from_workload(wl).upload()
    U = torch.from_numpy(R.copy()).cuda()
    sims = wl.sims
    if case == "blob_box":
        rr, rc = 0.05, 0.01
    else:
        ind0 = o.block_indicator(R)
        rr, rc = float(np.quantile(ind0, 0.6)), float(np.quantile(ind0, 0.3))
    levels = []
    for rnd in range(3):
        g, U = g.adapt(U, rr, rc)
        lv, ijk, sim = o.adapt(o.block_indicator(R), rr, rc)
        levels.append(lv.copy())
        o2 = oracle_mod.Grid.from_workload(wk.Workload("adapted", lv, ijk, sim, sims, None))
        R = o.remap(R, o2)
        o = o2
        assert g.nb == o.nb and np.array_equal(g.level, lv)
        U1 = torch.zeros_like(U)
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        faults = torch.zeros(1, dtype=torch.int32, device="cuda")
        g.advance(U, U1, dt, 2, flux=flux, powell=True, faults=faults)
        R1 = np.zeros_like(R)
        rdt, rf = o.advance(R, R1, [0.0], 2, flux=flux, powell=True)
        torch.cuda.synchronize()
        got = U.cpu().numpy()
        err = max(float(np.abs(got[vs] - R[vs]).max() / np.abs(R[vs]).max())
                  for vs in ([0], [1, 2, 3], [4, 5, 6], [7]))        # per variable group
        print("adaptive", case, rnd, g.nb, "blocks,", int(np.sum(lv == 1)), "refined; err", err, flush=True)
        assert int(faults.item()) == 0 and rf == 0
        assert err <= TOL
        assert abs(float(dt.item()) - rdt[0]) <= 1e-14 * rdt[0]
    assert any(np.any(lv == 1) for lv in levels)
