"""GPU parity of local time stepping (every fluid cell advances with its own CFL step, d_dt one value per
cell): the HIP path through the C ABI against the CPU oracle on grids with a body, a resolution change
(flux correction) and mixed boundaries, both work splits of the stage kernel, FP64 within 1e-12 per
variable group and the per-cell steps within 1e-14; graph replay; the refusal with the learned form."""
import sys

import numpy as np
import pytest

from paper_2501_06717_amd import workloads as wk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GROUPS = {"rho": [0], "mom": [1, 2, 3], "B": [4, 5, 6], "e": [7]}
TOL = 1e-12
FP32_TOL = 1e-5


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


def group_err(got, ref):
    return {g: float(np.abs(got[vs] - ref[vs]).max() / max(np.abs(ref[vs]).max(), 1e-300)) for g, vs in GROUPS.items()}


CASES = {
    "body": lambda: wk.magnetosphere_cut(32),
    "two_level": lambda: wk.two_level_box(),
    "odd_box": lambda: wk.odd_box(),
    "batch": lambda: wk.batched_waves(n_sims=3, n_lo=8, n_hi=27),
}


def gpu_local(bd, wl, n_stages, dt0=None, **kw):
    g = bd.Grid.from_workload(wl).upload()
    U0 = g.set_state(torch.from_numpy(wl.W).cuda())
    U1 = torch.zeros_like(U0)
    dt = torch.zeros((wl.n_blocks, 8, 8, 8), dtype=torch.float64, device="cuda")
    if dt0 is not None:
        dt.copy_(torch.from_numpy(dt0))
    faults = torch.zeros(1, dtype=torch.int32, device="cuda")
    g.advance(U0, U1, dt, n_stages, faults=faults, local_dt=True, **kw)
    torch.cuda.synchronize()
    return U0.cpu().numpy(), dt.cpu().numpy(), int(faults.item())


@pytest.mark.parametrize("scheme", ["plane", "face"])
@pytest.mark.parametrize("case", list(CASES))
def test_local_dt_matches_oracle(bd, oracle_mod, case, scheme):
    wl = CASES[case]()
    kw = dict(flux="hlle", powell=True, cfl=0.8)
    say("local dt", case, scheme)
    o = oracle_mod.Grid.from_workload(wl)
    R = o.set_state(wl.W)
    rdt, rf = o.advance(R, np.zeros_like(R), 0.0, 6, local_dt=True, **kw)
    G, dt, f = gpu_local(bd, wl, 6, scheme=scheme, **kw)
    assert f == rf
    fluid = rdt > 0.0
    assert np.array_equal(dt > 0.0, fluid)
    assert np.all(np.abs(dt[fluid] - rdt[fluid]) <= 1e-14 * rdt[fluid])
    err = group_err(G, R)
    say("  fp64", err)
    assert max(err.values()) <= TOL, err
    G32, _, f32 = gpu_local(bd, wl, 6, scheme=scheme, precision="fp32_flux", **kw)
    err32 = group_err(G32, R)
    say("  fp32_flux", err32)
    assert f32 == rf and max(err32.values()) <= FP32_TOL, err32


def test_local_dt_given_steps(bd, oracle_mod):
    """Without recompute_dt the per-cell steps are read as given (here: a random field of steps)."""
    wl = wk.two_level_box()
    rng = np.random.default_rng(3)
    dt0 = rng.uniform(0.02, 0.08, (wl.n_blocks, 8, 8, 8))
    kw = dict(flux="rusanov", powell=False, recompute_dt=False)
    o = oracle_mod.Grid.from_workload(wl)
    R = o.set_state(wl.W)
    rdt, _ = o.advance(R, np.zeros_like(R), dt0, 4, local_dt=True, **kw)
    G, dt, _ = gpu_local(bd, wl, 4, dt0=dt0, **kw)
    assert np.array_equal(dt, dt0) and np.array_equal(rdt, dt0)
    err = group_err(G, R)
    assert max(err.values()) <= TOL, err


def test_local_dt_with_a_uniform_bound_is_the_global_step(bd):
    """Same CFL bound in every cell: one step of local time stepping is one step of the global scheme (up to
    multiply-add contraction in the two kernels that form the bound)."""
    wl = wk.odd_box()
    wl = wk.with_state(wl, wk.uniform_bound_state(wl, seed=1))
    G, dloc, _ = gpu_local(bd, wl, 2, flux="hlle", powell=True, cfl=0.8)
    g = bd.Grid.from_workload(wl).upload()
    U0 = g.set_state(torch.from_numpy(wl.W).cuda())
    U1 = torch.zeros_like(U0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    g.advance(U0, U1, dt, 2, flux="hlle", powell=True, cfl=0.8)
    torch.cuda.synchronize()
    dtg = float(dt.item())
    assert np.all(np.abs(dloc - dtg) <= 1e-15 * dtg)
    err = group_err(G, U0.cpu().numpy())
    assert max(err.values()) <= 1e-14, err


def test_local_dt_graph_replay_matches_eager(bd):
    wl = wk.two_level_box()
    kw = dict(flux="hlle", powell=True, cfl=0.8)
    a, adt, _ = gpu_local(bd, wl, 8, **kw)
    b, bdt, _ = gpu_local(bd, wl, 8, use_graph=True, **kw)
    assert np.array_equal(a, b) and np.array_equal(adt, bdt)


def test_local_dt_refused_with_the_learned_form(bd):
    wl = wk.magnetosphere_cut(32)
    g = bd.Grid.from_workload(wl).upload()
    U0 = g.set_state(torch.from_numpy(wl.W).cuda())
    U1 = torch.zeros_like(U0)
    dt = torch.zeros((wl.n_blocks, 8, 8, 8), dtype=torch.float64, device="cuda")
    mlp = bd.Mlp(32)
    stats = torch.zeros(80); stats[32:64] = 1.0; stats[72:80] = 1.0
    L = g.learned(mlp, stats)
    with pytest.raises(bd.BmhdError, match="local time stepping"):
        g.advance(U0, U1, dt, 2, flux="hlle", powell=True, learned=L, local_dt=True, scheme="plane", slab=4)
