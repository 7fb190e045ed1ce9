"""GPU tests of the learned flux-correction form: per-face data, the zero-correction identity, and the
fallback to the plain flux."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def face_index(d, i, j, z):
    return ((z * 8 + j) * 9 + i) if d == 0 else (((z * 9 + j) * 8 + i) if d == 1 else ((z * 8 + j) * 8 + i))


def compact_rows(wl):
    """Row of every face of bmhd_face_data's layout in the network path's compact layout (each face once:
    per block and direction the 512 faces at positions 0..7 along it, (z 8 + j) 8 + i; then 64 faces per
    high face plane with no neighbour across it, numbered block by block and direction by direction,
    t2 8 + t1 over the other two axes), for single-level grids of one simulation."""
    sim = wl.sims[0]
    ijk = np.asarray(wl.ijk).reshape(-1, 3)
    index = {tuple(int(v) for v in q): b for b, q in enumerate(ijk)}
    nb = len(ijk)
    nbr = np.full((nb, 3), -1, np.int64)
    for b in range(nb):
        for d in range(3):
            q = [int(v) for v in ijk[b]]
            q[d] += 1
            if q[d] >= sim.nroot[d]:
                if sim.bc[2 * d + 1] != 0:
                    continue
                q[d] = 0
            nbr[b, d] = index[tuple(q)]
    hb = np.full((nb, 3), -1, np.int64)
    n = 0
    for b in range(nb):
        for d in range(3):
            if nbr[b, d] < 0:
                hb[b, d] = n
                n += 1
    rows = np.empty((nb, 3, 576), np.int64)
    for b in range(nb):
        for d in range(3):
            for f in range(576):
                if d == 0:
                    p = [f % 9, (f // 9) % 8, f // 72]
                elif d == 1:
                    p = [f % 8, (f // 8) % 9, f // 72]
                else:
                    p = [f % 8, (f // 8) % 8, f // 64]
                if p[d] < 8:
                    rows[b, d, f] = b * 1536 + d * 512 + (p[2] * 8 + p[1]) * 8 + p[0]
                elif nbr[b, d] >= 0:
                    p[d] = 0
                    rows[b, d, f] = nbr[b, d] * 1536 + d * 512 + (p[2] * 8 + p[1]) * 8 + p[0]
                else:
                    t = [p[a] for a in range(3) if a != d]
                    rows[b, d, f] = nb * 1536 + hb[b, d] * 64 + t[1] * 8 + t[0]
    return torch.from_numpy(rows.reshape(-1))


def test_face_fluxes_reproduce_the_stage(bd):
    """One forward-Euler stage equals U + dt * (-sum_d (F_d+ - F_d-) / dx) built from bmhd_face_data's
    fluxes (rotated back from the face-normal frame)."""
    wl = wk.with_state(wk.uniform_state((2, 2, 2)), wk.random_positive_state(wk.uniform_state((2, 2, 2)), 3))
    g = bd.Grid.from_workload(wl).upload()
    U0 = g.set_state(dev(wl.W))
    _, F = g.face_data(U0, flux="rusanov", want_x=False)
    U1 = torch.zeros_like(U0)
    dt = torch.tensor([0.01], dtype=torch.float64, device="cuda")
    Ua = U0.clone()
    g.advance(Ua, U1, dt, 1, flux="rusanov", powell=False, recompute_dt=False, alpha=(0.0, 0.5), beta=(1.0, 0.5))
    L = ((U1 - U0) / 0.01).cpu().numpy()
    F = F.cpu().numpy().reshape(wl.n_blocks, 3, 576, 8).astype(np.float64)
    # back to x, y, z components
    Fx = np.empty_like(F)
    for d in range(3):
        Fx[:, d, :, 0] = F[:, d, :, 0]
        Fx[:, d, :, 7] = F[:, d, :, 7]
        for a in range(3):
            Fx[:, d, :, 1 + (d + a) % 3] = F[:, d, :, 1 + a]
            Fx[:, d, :, 4 + (d + a) % 3] = F[:, d, :, 4 + a]
    ref = np.zeros((8, wl.n_blocks, 8, 8, 8))
    for z in range(8):
        for j in range(8):
            for i in range(8):
                for d in range(3):
                    lo = face_index(d, i, j, z)
                    hi = face_index(d, i + (d == 0), j + (d == 1), z + (d == 2))
                    ref[:, :, z, j, i] -= (Fx[:, d, hi, :] - Fx[:, d, lo, :]).T
    scale = np.abs(ref).max()
    assert np.abs(L - ref).max() <= 1e-5 * scale


def test_features_are_normal_frame_stencils(bd):
    wl = wk.with_state(wk.uniform_state((2, 1, 1)), wk.random_positive_state(wk.uniform_state((2, 1, 1)), 5))
    g = bd.Grid.from_workload(wl).upload()
    U0 = g.set_state(dev(wl.W))
    X, _ = g.face_data(U0, want_f=False)
    X = X.cpu().numpy().reshape(wl.n_blocks, 3, 576, 32)
    W = wl.W
    # interior face of block 0 along y at (i=3, j=4, z=5): stencil cells j = 2..5
    f = face_index(1, 3, 4, 5)
    for q in range(4):
        cell = W[:, 0, 5, 2 + q, 3]
        expect = np.array([cell[0], cell[2], cell[3], cell[1], cell[5], cell[6], cell[4], cell[7]])
        assert np.allclose(X[0, 1, f, q * 8:(q + 1) * 8], expect, rtol=1e-6, atol=1e-6)


def _learned_run(bd, wl, mlp, stats, n_stages, precision, flux, powell, fallback=None):
    g = bd.Grid.from_workload(wl).upload()
    U0 = g.set_state(dev(wl.W))
    U1 = torch.zeros_like(U0)
    dt = torch.zeros(len(wl.sims), dtype=torch.float64, device="cuda")
    faults = torch.zeros(1, dtype=torch.int32, device="cuda")
    L = g.learned(mlp, stats, fallback=fallback) if mlp is not None else None
    # the learned stage runs the wave-per-layer kernel on 8x8x4 slabs: compare with the same plain kernel
    g.advance(U0, U1, dt, n_stages, faults=faults, flux=flux, powell=powell, precision=precision, learned=L,
              scheme="plane", slab=4)
    torch.cuda.synchronize()
    return U0.cpu().numpy(), dt.cpu().numpy(), int(faults.item())


@pytest.mark.parametrize("precision", ["fp64", "fp32_flux"])
def test_zero_correction_equals_plain(bd, precision):
    wl = wk.magnetosphere_cut(32)
    mlp = bd.Mlp(32)                                 # all parameters zero: the network outputs 0
    stats = torch.zeros(80); stats[32:64] = 1.0; stats[72:80] = 1.0
    a, adt, af = _learned_run(bd, wl, mlp, stats, 4, precision, "hlle", True)
    b, bdt, bf = _learned_run(bd, wl, None, None, 4, precision, "hlle", True)
    assert af == 0 and bf == 0
    assert np.array_equal(adt, bdt)
    # the learned and plain stages are different kernel instantiations, whose multiply-add contraction
    # may differ: equal to a unit or two in the last place
    rel = max(np.abs(a[v] - b[v]).max() / np.abs(b[v]).max() for v in range(8))
    print("zero-correction max relative difference", rel, flush=True)
    assert rel <= 1e-15


def test_bad_correction_falls_back_to_plain(bd):
    wl = wk.magnetosphere_cut(32)
    rng = np.random.default_rng(0)
    mlp = bd.Mlp(32, torch.from_numpy(rng.normal(scale=0.3, size=bd.lib().bmhd_mlp_n_params(32)).astype(np.float32)))
    stats = torch.zeros(80); stats[32:64] = 1.0
    stats[64:72] = 0.0; stats[72:80] = 1e3                    # huge corrections
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    a, _, af = _learned_run(bd, wl, mlp, stats, 2, "fp64", "hlle", True, fallback=fb)
    b, _, _ = _learned_run(bd, wl, None, None, 2, "fp64", "hlle", True)
    print("flagged cells", int(fb.item()), "of", wl.n_cells * 2, flush=True)
    assert int(fb.item()) > wl.n_cells // 2
    err = max(np.abs(a[v] - b[v]).max() / np.abs(b[v]).max() for v in range(8))
    assert err <= 1e-8, err


def test_learned_stage_adds_the_network_increment(bd):
    """One learned stage: the features it builds equal bmhd_face_data's z-scored features, and its result
    differs from the plain stage by the flux differences of the network's de-normalised increments,
    rotated back to x, y, z (small increments: no cell is flagged)."""
    wl = wk.with_state(wk.uniform_state((2, 2, 2)), wk.random_positive_state(wk.uniform_state((2, 2, 2)), 7))
    g = bd.Grid.from_workload(wl).upload()
    U0 = g.set_state(dev(wl.W))
    rng = np.random.default_rng(2)
    mlp = bd.Mlp(32, torch.from_numpy(rng.normal(scale=0.3, size=bd.lib().bmhd_mlp_n_params(32)).astype(np.float32)))
    stats = torch.zeros(80)
    stats[0:32] = torch.from_numpy(rng.uniform(-0.5, 0.5, 32).astype(np.float32))
    stats[32:64] = torch.from_numpy(rng.uniform(0.5, 2.0, 32).astype(np.float32))
    stats[64:72] = 1e-4
    stats[72:80] = torch.from_numpy(rng.uniform(1e-4, 1e-3, 8).astype(np.float32))
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    L = g.learned(mlp, stats, fallback=fb)
    dt = torch.tensor([0.01], dtype=torch.float64, device="cuda")
    kw = dict(flux="hlle", powell=True, recompute_dt=False)
    Ua, U1a = U0.clone(), torch.zeros_like(U0)
    g.advance(Ua, U1a, dt, 1, learned=L, **kw)
    torch.cuda.synchronize()
    # the BF16 network's stage keeps its features in BF16, in the first half of the scratch buffer, each
    # face once (the compact layout); spread back to bmhd_face_data's layout
    rows = compact_rows(wl).cuda()
    nc = int(rows.max()) + 1
    X_in = g._lx.view(-1)[: nc * 16].view(torch.bfloat16).view(nc, 32).float()[rows]
    Xref, _ = g.face_data(U0, flux="hlle", stats=stats.cuda(), want_f=False)
    assert int(fb.item()) == 0
    # equal up to the rounding to BF16 (one BF16 unit where the FP32 values differ in the last places)
    bound = 2.0 ** -8 * Xref.abs() + 1e-5
    assert bool(((X_in - Xref).abs() <= bound).all()), float(((X_in - Xref).abs() - bound).max())
    assert float((X_in == Xref.to(torch.bfloat16).float()).float().mean()) > 0.99
    Ub, U1b = U0.clone(), torch.zeros_like(U0)
    g.advance(Ub, U1b, dt, 1, scheme="plane", slab=4, **kw)
    # the stage de-normalises in FP32 (a multiply-add per component)
    Y = mlp.forward(X_in).cpu().numpy()
    s = stats.numpy()
    dF = (Y * s[72:80] + s[64:72]).astype(np.float64).reshape(wl.n_blocks, 3, 576, 8)
    dFx = np.empty_like(dF)          # face-normal frame -> x, y, z components
    for d in range(3):
        dFx[:, d, :, 0] = dF[:, d, :, 0]
        dFx[:, d, :, 7] = dF[:, d, :, 7]
        for a in range(3):
            dFx[:, d, :, 1 + (d + a) % 3] = dF[:, d, :, 1 + a]
            dFx[:, d, :, 4 + (d + a) % 3] = dF[:, d, :, 4 + a]
    expect = np.zeros((8, wl.n_blocks, 8, 8, 8))
    for z in range(8):
        for j in range(8):
            for i in range(8):
                for d in range(3):
                    lo = face_index(d, i, j, z)
                    hi = face_index(d, i + (d == 0), j + (d == 1), z + (d == 2))
                    expect[:, :, z, j, i] -= 0.01 * (dFx[:, d, hi, :] - dFx[:, d, lo, :]).T
    got = (U1a - U1b).cpu().numpy()
    scale = np.abs(expect).max()
    print("increment scale", scale, "max deviation", np.abs(got - expect).max(), flush=True)
    assert scale > 1e-7
    # bound: FP32 rounding of the de-normalised increments, and FP64 rounding of the stage sums
    assert np.abs(got - expect).max() <= 1e-6 * scale + 1e-14 * np.abs(U1b.cpu().numpy()).max()


def test_given_corrections_equal_the_network_path(bd):
    """Mode 2 of the learned form takes the normalised corrections as given: handing it the network's own
    outputs for the step's input reproduces the network path bit for bit (one stage)."""
    wl = wk.magnetosphere_cut(32)
    g = bd.Grid.from_workload(wl).upload()
    U0 = g.set_state(dev(wl.W))
    rng = np.random.default_rng(4)
    mlp = bd.Mlp(32, torch.from_numpy(rng.normal(scale=0.3, size=bd.lib().bmhd_mlp_n_params(32)).astype(np.float32)))
    stats = torch.zeros(80)
    stats[32:64] = 1.0
    stats[64:72] = 1e-4
    stats[72:80] = 1e-3
    dt = torch.tensor([0.005], dtype=torch.float64, device="cuda")
    kw = dict(flux="hlle", powell=True, recompute_dt=False, scheme="plane", slab=4)
    Ua, U1a = U0.clone(), torch.zeros_like(U0)
    g.advance(Ua, U1a, dt, 1, learned=g.learned(mlp, stats), **kw)
    torch.cuda.synchronize()
    y = g._ly[compact_rows(wl).cuda()].contiguous()   # the network's outputs in bmhd_face_data's layout
    Ub, U1b = U0.clone(), torch.zeros_like(U0)
    g.advance(Ub, U1b, dt, 1, learned=g.given_corrections(y, stats), **kw)
    torch.cuda.synchronize()
    assert torch.equal(U1a, U1b)


def _group_err(a, b):
    return {k: float(np.abs(a[v] - b[v]).max() / np.abs(b[v]).max())
            for k, v in (("rho", [0]), ("mom", [1, 2, 3]), ("B", [4, 5, 6]), ("e", [7]))}


def test_features_match_the_oracle(bd, oracle_mod):
    """bmhd_face_data's z-scored stencil features against the oracle's (or_face_features, FP64) on the
    same conserved state, every face of every block of a box with a body, an inflow and outflow faces.
    The GPU rounds each primitive to FP32 and z-scores in FP32, (x - mean) / std: three roundings of at
    most half an FP32 unit each, so |X - ref| <= 2^-24 (|w| / std + 2 |ref|) with |w| <= |ref| std +
    |mean|; the test allows twice that."""
    base = wk.uniform_state((4, 4, 4), bc=(1, 2, 0, 0, 1, 1), body_r=5.0)
    wl = wk.with_state(base, wk.random_positive_state(base, seed=21))
    o = oracle_mod.Grid.from_workload(wl)
    R = o.set_state(wl.W)
    rng = np.random.default_rng(22)
    stats = np.zeros(80)
    stats[0:32] = rng.uniform(-0.5, 0.5, 32)
    stats[32:64] = rng.uniform(0.5, 2.0, 32)
    st32 = stats.astype(np.float32)
    g = bd.Grid.from_workload(wl).upload()
    X, _ = g.face_data(dev(R), stats=torch.from_numpy(st32).cuda(), want_f=False)
    X = X.cpu().numpy().astype(np.float64)
    mean, std = st32[0:32].astype(np.float64), st32[32:64].astype(np.float64)
    ref = o.face_features(R, stats=st32.astype(np.float64))
    assert X.shape == ref.shape
    bound = 2.0 ** -23 * ((np.abs(ref) * std + np.abs(mean)) / std + 2.0 * np.abs(ref))
    excess = (np.abs(X - ref) / bound).max()
    print("features: max error / FP32 bound", float(excess), flush=True)
    assert excess <= 1.0
    # the unnormalised features are the primitives rounded once to FP32 (the nearest FP32 value, or its
    # neighbour where the GPU's FP64 primitive and the oracle's straddle a rounding boundary)
    X0, _ = g.face_data(dev(R), want_f=False)
    X0 = X0.cpu().numpy().astype(np.float64)
    ref0 = o.face_features(R)
    assert np.all(np.abs(X0 - ref0) <= 2.0 ** -23 * np.abs(ref0))


@pytest.mark.parametrize("flux", ["hlle", "rusanov"])
def test_learned_stage_matches_the_oracle(bd, oracle_mod, flux):
    """One step of the learned form with corrections given per face (mode 2) against the oracle's learned
    stage (or_advance_learned): same provisional update, same flag rule on the old 7-point range, the
    fallback on both sides of every face of a flagged cell. Corrections are multiples of 1/64 scaled by a
    power of two, exact in FP32, so both sides add the same increments; they are sized so that about a
    tenth of the cells is flagged per stage. The grid has a body, an inflow face and outflow faces."""
    base = wk.uniform_state((4, 4, 4), bc=(1, 2, 0, 0, 1, 1), body_r=5.0)
    wl = wk.with_state(base, wk.random_positive_state(base, seed=31))
    o = oracle_mod.Grid.from_workload(wl)
    R0 = o.set_state(wl.W)
    R1 = np.zeros_like(R0)
    rng = np.random.default_rng(32)
    y = (np.round(rng.normal(size=(wl.n_blocks * 1728, 8)) * 64.0) / 64.0).astype(np.float32)
    ystats = np.zeros(16)
    ystats[8:16] = 2.0 ** -3
    rdt, rf, rflag = o.advance_learned(R0, R1, [0.0], 2, y.astype(np.float64), ystats, tau=0.1, flux=flux,
                                       powell=True)
    g = bd.Grid.from_workload(wl).upload()
    U0 = dev(o.set_state(wl.W))
    U1 = torch.zeros_like(U0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    faults = torch.zeros(1, dtype=torch.int32, device="cuda")
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    stats = torch.zeros(80)
    stats[64:72] = torch.from_numpy(ystats[:8].astype(np.float32))
    stats[72:80] = torch.from_numpy(ystats[8:].astype(np.float32))
    L = g.given_corrections(dev(y), stats, tau=0.1, fallback=fb)
    g.advance(U0, U1, dt, 2, faults=faults, flux=flux, powell=True, learned=L, scheme="plane", slab=4)
    torch.cuda.synchronize()
    err = _group_err(U0.cpu().numpy(), R0)
    nflag = int(fb.item())
    print("learned vs oracle", flux, err, "flagged", nflag, "oracle", rflag, "of", 2 * wl.n_cells, flush=True)
    assert int(faults.item()) == 0 and rf == 0
    assert abs(float(dt.item()) - rdt[0]) <= 1e-14 * rdt[0]
    assert 0.05 * 2 * wl.n_cells <= rflag <= 0.3 * 2 * wl.n_cells
    assert nflag == rflag
    assert max(err.values()) <= 1e-12, err


@pytest.mark.parametrize("floor_rel", [0.0, 0.02])
def test_range_floor_matches_the_oracle(bd, oracle_mod, floor_rel):
    """The acceptance test's range floor against the oracle: density and pressure uniform, velocity and
    field of random sign per cell (every old 7-point range is zero), corrections given per face. With no
    floor every cell whose density or pressure changes at all is flagged; with the floor h = floor_rel *
    max(|lo|, |hi|) only changes beyond tau * h are. Flag counts equal the oracle's and states agree to
    1e-12 per variable group."""
    base = wk.uniform_state((2, 2, 2))
    wl = wk.with_state(base, wk.uniform_bound_state(base, seed=41, rho=1.1, p=0.7, u0=0.002, b0=0.002))
    o = oracle_mod.Grid.from_workload(wl)
    R0 = o.set_state(wl.W)
    R1 = np.zeros_like(R0)
    rng = np.random.default_rng(42)
    y = (np.round(rng.normal(size=(wl.n_blocks * 1728, 8)) * 64.0) / 64.0).astype(np.float32)
    ystats = np.zeros(16)
    ystats[8:16] = 2.0 ** -8
    rdt, rf, rflag = o.advance_learned(R0, R1, [0.0], 2, y.astype(np.float64), ystats, tau=0.1,
                                       floor_rel=floor_rel, flux="hlle", powell=True)
    g = bd.Grid.from_workload(wl).upload()
    U0 = dev(o.set_state(wl.W))
    U1 = torch.zeros_like(U0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    stats = torch.zeros(80)
    stats[72:80] = torch.from_numpy(ystats[8:].astype(np.float32))
    L = g.given_corrections(dev(y), stats, tau=0.1, fallback=fb, floor_rel=floor_rel)
    g.advance(U0, U1, dt, 2, flux="hlle", powell=True, learned=L, scheme="plane", slab=4)
    torch.cuda.synchronize()
    err = _group_err(U0.cpu().numpy(), R0)
    nflag = int(fb.item())
    print("floor", floor_rel, "flagged", nflag, "oracle", rflag, "of", 2 * wl.n_cells, err, flush=True)
    assert nflag == rflag
    # (the oracle flags 7,369 and 2,765 of 8,192 cell-stages)
    if floor_rel == 0.0:
        assert rflag >= 0.8 * 2 * wl.n_cells
    else:
        assert 0.1 * 2 * wl.n_cells <= rflag <= 0.5 * 2 * wl.n_cells
    assert max(err.values()) <= 1e-12, err


@pytest.mark.parametrize("precision", ["fp64", "fp32_flux"])
def test_unchanged_uniform_state_is_never_flagged(bd, precision):
    """A uniform state whose density and pressure are not FP32 numbers (1.1, 0.7) stays exactly as it is
    under zero corrections, in both precisions: the acceptance test compares it with the FP64 range of
    its neighbourhood, so no cell is flagged even with no range floor."""
    wl = wk.uniform_state((2, 2, 2), W0=(1.1, 0.1, -0.2, 0.3, 0.5, -0.4, 0.3, 0.7))
    g = bd.Grid.from_workload(wl).upload()
    U0 = g.set_state(dev(wl.W))
    Uref = U0.clone()
    U1 = torch.zeros_like(U0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    y = torch.zeros((wl.n_blocks * 1728, 8), dtype=torch.float32, device="cuda")
    L = g.given_corrections(y, torch.zeros(80), tau=0.1, fallback=fb)
    g.advance(U0, U1, dt, 2, flux="hlle", powell=True, learned=L, precision=precision)
    torch.cuda.synchronize()
    assert int(fb.item()) == 0
    assert torch.equal(U0, Uref)


@pytest.mark.parametrize("nroot", [(2, 1, 1), (2, 2, 2)])
def test_face_targets_match_the_oracle(bd, oracle_mod, nroot):
    """bmhd_face_targets against the oracle bit for bit: on random face data (every fine face read from
    the right block and slot), and on the face fluxes of a state on the refined grid and of its
    restriction by bmhd_remap."""
    sim_wl = wk.magnetosphere_cut(8 * nroot[0]) if nroot == (2, 2, 2) else wk.uniform_state(nroot)
    sim = sim_wl.sims[0]
    lv, ijk, sid = wk.uniform_blocks(sim.nroot)
    coarse = wk.Workload("coarse", lv, ijk, sid, [sim], wk._empty_W(len(lv)))
    lvf, ijkf, sidf = wk.two_level_blocks(sim.nroot, np.ones(sim.nroot[::-1], bool))
    fine = wk.Workload("fine", lvf, ijkf, sidf, [sim], wk._empty_W(len(lvf)))
    fine = wk.with_state(fine, wk.random_positive_state(fine, seed=9))
    gf = bd.Grid.from_workload(fine).upload()
    gc = bd.Grid.from_workload(coarse).upload()
    rng = np.random.default_rng(10)
    Ff = rng.normal(size=(fine.n_blocks * 1728, 8)).astype(np.float32)
    Fc = rng.normal(size=(coarse.n_blocks * 1728, 8)).astype(np.float32)
    got = gf.face_targets(dev(Ff), gc, dev(Fc)).cpu().numpy()
    ref = oracle_mod.face_targets(Ff, ijkf, Fc, ijk)
    assert np.array_equal(got, ref)
    Uf = gf.set_state(dev(fine.W))
    Uc = gf.remap(Uf, gc)
    _, Ffd = gf.face_data(Uf, flux="hlle", want_x=False)
    _, Fcd = gc.face_data(Uc, flux="hlle", want_x=False)
    got = gf.face_targets(Ffd, gc, Fcd).cpu().numpy()
    ref = oracle_mod.face_targets(Ffd.cpu().numpy(), ijkf, Fcd.cpu().numpy(), ijk)
    assert np.array_equal(got, ref)


def test_face_targets_refuse_unrelated_grids(bd):
    base = wk.uniform_state((2, 1, 1))
    g2 = bd.Grid.from_workload(base).upload()
    two = wk.two_level_box(nroot=(2, 1, 1), refine=((1, 0, 0),))
    g3 = bd.Grid.from_workload(two).upload()
    F = torch.zeros((max(base.n_blocks, two.n_blocks) * 1728, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(bd.BmhdError):
        g3.face_targets(F, g2, F)        # not every root refined
    with pytest.raises(bd.BmhdError):
        g2.face_targets(F, g3, F)        # the coarse grid has level-1 blocks
