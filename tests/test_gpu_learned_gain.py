"""What the trained flux-correction network gains over the plain method (GPU): the network shipped with
the package (trained by `python -m paper_2501_06717_amd.learn` on 32 solar-wind states, written to
paper_2501_06717_amd/trained/) on held-out solar-wind states it never saw, against the fine 256^3 FP64
run restricted to 128^3: 200 coarse steps of the learned path against 200 of the plain path, one coarse
step likewise, and one step with the exact a-priori target (the bound for a correction of this form)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NET = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2501_06717_amd", "trained",
                   "flux_mlp_h128.npz")


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2501_06717_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("seed", [1005, 2005])
def test_trained_network_gains_over_the_plain_path(bd, seed):
    from paper_2501_06717_amd import learn
    mlp, stats, meta = learn.load(NET)
    cfg = learn.Config(hidden=meta["hidden"])
    states = learn.solar_wind_states(2, seed)
    ev = learn.evaluate(bd, cfg, mlp, stats, states, log=lambda *m: print(*m, flush=True))
    for e in ev:
        assert e["learned"]["faults"] == 0 and e["plain"]["faults"] == 0
        # the exact target improves one step several-fold: the comparison itself is sound
        assert e["one_step_exact_target"]["gain"] > 3.0
    # the network improves on the plain path locally and over 200 coarse steps
    assert min(e["one_step"]["gain"] for e in ev) > 1.0
    assert np.mean([e["gain"] for e in ev]) > 1.0
