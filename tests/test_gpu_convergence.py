"""Second-order convergence of the GPU path on the circularly polarised Alfven wave, an exact nonlinear
solution (FP64, Rusanov, MC, Heun; one wave period): the L1 error of the transverse field against the
exact solution from 32^3 to 256^3 cells. The GPU path matches the oracle to 1e-12 on this wave (the
parity tests); the larger grids are out of the oracle's reach in a test, not the GPU's."""
import math
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


def cp_error(bd, n):
    wl = wk.cp_alfven(n)
    g = bd.Grid.from_workload(wl).upload()
    U0 = g.set_state(torch.from_numpy(wl.W).cuda())
    U1 = torch.zeros_like(U0)
    T = 1.0 / math.sqrt(2.0)
    dt_cfl = float(g.reduce_dt(U0, 0.8).item())
    nsteps = int(math.ceil(T / dt_cfl))
    dt = torch.tensor([T / nsteps], dtype=torch.float64, device="cuda")
    g.advance(U0, U1, dt, 2 * nsteps, flux="rusanov", powell=False, recompute_dt=False)
    torch.cuda.synchronize()
    exact = wk.cp_alfven_field(wl.sims[0], wl.level, wl.ijk, 0.0)
    err = float(np.mean(np.abs(U0[4:7].cpu().numpy() - exact[4:7])))
    print(f"cp alfven {n}^3: {nsteps} steps, L1 error {err:.4e}", flush=True)
    sys.stdout.flush()
    return err


def test_cp_alfven_order_approaches_two(bd):
    errs = {n: cp_error(bd, n) for n in (32, 64, 128, 256)}
    orders = {f"{n}->{2 * n}": math.log2(errs[n] / errs[2 * n]) for n in (32, 64, 128)}
    print("orders", orders, flush=True)
    # the MC limiter clips the wave's extrema, which costs order at coarse resolution; the order rises
    # toward 2 as the grid resolves the wave
    assert orders["32->64"] < orders["64->128"] < orders["128->256"] + 0.02
    # measured: 1.73, 1.90, 2.00
    assert orders["128->256"] >= 1.95, orders
