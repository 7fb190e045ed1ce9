"""GPU parity of the state remap after a refinement change (bmhd_remap through the C ABI) against the
oracle: bit-exact for refinement, coarsening and both at once (copy, prolongation and restriction are
evaluated without contraction on both sides); a run that adapts its grid between steps within 1e-12 of
the oracle doing the same; the refusal of a grid of another domain."""
import numpy as np
import pytest

from paper_2501_06717_amd import workloads as wk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GROUPS = {"rho": [0], "mom": [1, 2, 3], "B": [4, 5, 6], "e": [7]}


@pytest.fixture(scope="module")
def bd():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2501_06717_amd import binding
    binding.lib()
    return binding


def box(refine, seed=5, bc=(1, 2, 0, 0, 1, 1)):
    return wk.two_level_box(nroot=(4, 4, 3), refine=refine, bc=bc, seed=seed)


GEOMS = {
    "single": (),
    "a": ((1, 1, 1), (2, 2, 1), (3, 0, 2)),
    "b": ((1, 1, 1), (0, 3, 0), (2, 1, 2)),
}
PAIRS = [("single", "a"), ("a", "single"), ("a", "b"), ("b", "a")]


@pytest.mark.parametrize("src,dst", PAIRS)
def test_remap_is_bit_exact(bd, oracle_mod, src, dst):
    wa, wb = box(GEOMS[src]), box(GEOMS[dst])
    oa, ob = oracle_mod.Grid.from_workload(wa), oracle_mod.Grid.from_workload(wb)
    U = oa.set_state(wa.W)
    ref = oa.remap(U, ob)
    ga, gb = bd.Grid.from_workload(wa).upload(), bd.Grid.from_workload(wb).upload()
    got = ga.remap(torch.from_numpy(U).cuda(), gb).cpu().numpy()
    assert np.array_equal(got, ref)


def test_adaptive_run_matches_oracle(bd, oracle_mod):
    """Two steps on grid a, remap to grid b (some blocks refined, others coarsened), two more steps."""
    wa, wb = box(GEOMS["a"]), box(GEOMS["b"])
    kw = dict(flux="hlle", powell=True, cfl=0.8)
    oa, ob = oracle_mod.Grid.from_workload(wa), oracle_mod.Grid.from_workload(wb)
    R = oa.set_state(wa.W)
    oa.advance(R, np.zeros_like(R), 0.0, 4, **kw)
    R = oa.remap(R, ob)
    rdt, _ = ob.advance(R, np.zeros_like(R), 0.0, 4, **kw)
    ga, gb = bd.Grid.from_workload(wa).upload(), bd.Grid.from_workload(wb).upload()
    U = ga.set_state(torch.from_numpy(wa.W).cuda())
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    ga.advance(U, torch.zeros_like(U), dt, 4, **kw)
    V = ga.remap(U, gb)
    gb.advance(V, torch.zeros_like(V), dt, 4, **kw)
    torch.cuda.synchronize()
    G = V.cpu().numpy()
    assert abs(float(dt.item()) - float(rdt[0])) <= 1e-14 * float(rdt[0])
    for g, vs in GROUPS.items():
        err = np.abs(G[vs] - R[vs]).max() / np.abs(R[vs]).max()
        assert err <= 1e-12, (g, err)


def test_remap_refuses_another_domain(bd):
    wa = box(())
    wb = wk.two_level_box(nroot=(4, 4, 2), refine=(), bc=(1, 2, 0, 0, 1, 1), seed=5)
    ga, gb = bd.Grid.from_workload(wa).upload(), bd.Grid.from_workload(wb).upload()
    U = ga.set_state(torch.from_numpy(wa.W).cuda())
    with pytest.raises(bd.BmhdError, match="remap"):
        ga.remap(U, gb)
