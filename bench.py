"""Benchmark: FP64 cell-updates/s of the explicit block-adaptive MHD update on one MI355X.

Workload (the metric's configuration): the magnetosphere-shaped uniform grid of 256^3 cells in 32^3
blocks of 8^3 (dipole along -z, solar-wind inflow, reflecting body of radius 2.5 cells, outflow
elsewhere), HLLE flux with the Powell source, MC limiter, Heun stages, CFL 0.8. A step is one full time
step of the whole hot path: dt reduction, two fused stage kernels (ghost gather, reconstruction, fluxes,
source, update, next-dt bound). Inputs are resident in HBM before the timed region starts.

Prints one JSON line (rank 0). Extra fields: "roofline" for the dominant kernel (the stage kernel, timed
live with HIP events that the library records on its stream; its "valu" object puts the same timing
against the VALU issue peak, the bound this FP64 kernel actually meets), "cpu_baseline" (the CPU oracle
on the host's cores over a bounded sample), "forms" (the FP32-flux form on the same workload with its
error against the FP64 path, local time stepping, the 64-simulation batch, the learned correction) and
"paper_context" (the paper's one-GPU fast-wave run on the same grid geometry, beside its published
one-A100 time).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/sec (FP64 plain vs FP32-flux vs learned) at stated L1 err; % HBM roofline"
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the FP64 stage kernel on this workload (stage 1, stage 2), from rocprofv3
# FETCH_SIZE and WRITE_SIZE runs scaled by a plain device copy (the summaries under profiles/); valid
# only for the kernel version they were taken on, keyed by (scheme, tile depth)
TRAFFIC = {
    ("face", 8): (1.722e9 + 1.074e9, 2.807e9 + 1.074e9),
    ("plane", 4): (2.019e9 + 1.074e9, 3.007e9 + 1.074e9),
    ("block", 8): (2.336e9 + 1.073e9, 3.381e9 + 1.073e9),
}


# VALU lane instructions per cell and stage of the FP64 stage kernel on this workload (mean of the two
# stages, SQ_INSTS_VALU x 64 / cells from a rocprofv3 counter run; the summary under profiles/), keyed
# like TRAFFIC; the VALU issue peak is one wave64 instruction per CU per clock (4 SIMDs x 16 lanes):
# 256 CUs x 2.4 GHz x 64 lanes
VALU_PER_CELL_STAGE = {("plane", 4): 1917.0, ("block", 8): 2138.0}
VALU_PEAK_LANE_OPS = 256 * 2.4e9 * 64


def resolve_shape(scheme, slab, precision, persist=0):
    """The launch shape the library picks for scheme / slab 0 ("default") requests."""
    sc = ("plane" if (slab == 4 or persist) else "block") if scheme == "default" else scheme
    ks = slab if slab else (8 if ((precision == "fp64" and sc == "face") or sc == "block") else 4)
    return sc, ks
# algorithmic HBM bytes per cell and stage: stage 1 reads U^n and writes U^1 (2 x 64 B); stage 2 reads
# U^1 and U^n and writes U^{n+1} (3 x 64 B): 320 B per cell-update
BYTES_STAGE = (128.0, 192.0)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--n", type=int, default=256, help="cells per axis of the magnetosphere grid")
    p.add_argument("--slab", type=int, default=0)
    p.add_argument("--scheme", default="default", choices=["default", "face", "plane", "block"],
                   help="work split of the stage kernel")
    p.add_argument("--persist", type=int, default=0, help="persistent grid size of the stage kernel (0: off)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-forms", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=1)
    p.add_argument("--form-steps", type=int, default=20, help="timed steps of the batched and learned forms")
    p.add_argument("--profile", action="store_true", help="short run for a profiler: no CPU leg, no forms")
    p.add_argument("--calib", action="store_true",
                   help="also run a plain 256 MiB device copy (scales the HBM byte counters of a profiler run)")
    p.add_argument("--precision", default="fp64", choices=["fp64", "fp32_flux"],
                   help="precision of the timed magnetosphere run (the metric is quoted for fp64)")
    p.add_argument("--form", default="plain", choices=["plain", "batched", "learned", "two_level", "exchange"],
                   help="with --profile: run only this form (batched: the 64-simulation batch, graph-replayed; "
                        "learned: the learned correction on the 128^3 grid; two_level: the two-level "
                        "magnetosphere, FP64 and FP32 flux)")
    p.add_argument("--two-level-steps", type=int, default=200, help="steps of the two-level form")
    return p.parse_args()


def time_form(g, W, steps, warmup, precision, slab, persist=0, scheme="default"):
    import torch
    from paper_2501_06717_amd import binding
    U0 = g.set_state(W)
    U1 = torch.empty_like(U0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    faults = torch.zeros(1, dtype=torch.int32, device="cuda")
    base = dict(flux="hlle", powell=True, precision=precision, cfl=0.8, slab=slab, persist_wgs=persist,
                scheme=scheme)
    if warmup:
        g.advance(U0, U1, dt, 2 * warmup, faults=faults, **base)
        U0 = g.set_state(W)  # restart from the initial state: the timed run is the first `steps` steps
    torch.cuda.synchronize()
    events = [torch.cuda.Event(enable_timing=True) for _ in range(4 * steps)]
    for e in events:  # torch creates the HIP event lazily, on its first record
        e.record()
    torch.cuda.synchronize()
    opts = binding.make_opts(events=events, **base)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.advance(U0, U1, dt, 2 * steps, opts=opts, faults=faults)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = [[], []]
    for s in range(2 * steps):
        st[s % 2].append(events[2 * s].elapsed_time(events[2 * s + 1]) * 1e-3)
    return U0, wall, st, int(faults.item()), float(dt.item())


def time_advance(g, U0, U1, dt, steps, after_warmup=None, **opts):
    """Wall time of `steps` steps on the current stream, inputs resident."""
    import torch
    g.advance(U0, U1, dt, 2, **opts)   # warm-up (and graph capture)
    if after_warmup is not None:
        after_warmup()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.advance(U0, U1, dt, 2 * steps, **opts)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def bench_batched(steps):
    """64 independent periodic simulations (block counts log-uniform in 64..4096, 8 linear waves each),
    Rusanov, FP32 flux with FP64 state, per-simulation dt: one persistent kernel per stage over all
    blocks and graph-replayed steps, launch shape from the autotuner."""
    import torch
    from paper_2501_06717_amd import binding, workloads as wk
    wl = wk.batched_waves()
    g = binding.Grid.from_workload(wl).upload()
    W = torch.from_numpy(wl.W).cuda()
    U0 = g.set_state(W)
    U1 = torch.empty_like(U0)
    dt = torch.zeros(len(wl.sims), dtype=torch.float64, device="cuda")
    base = dict(flux="rusanov", powell=False, precision="fp32_flux", cfl=0.8)
    best, ms = g.autotune(U0.clone(), U1, dt, n_steps=2, **base)
    shape = dict(scheme=int(best.scheme), slab=int(best.slab), persist_wgs=int(best.persist_wgs))
    U0 = g.set_state(W)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()  # the state is set on the current stream, the timed steps run on `stream`
    with torch.cuda.stream(stream):
        t = time_advance(g, U0, U1, dt, steps, use_graph=True, **shape, **base)
    cells = wl.n_cells
    log(f"batched: {len(wl.sims)} simulations, {cells} cells, {t * 1e3:.2f} ms for {steps} steps, shape {shape}")
    return {"value": cells * steps / t, "unit": "cell-updates/s", "workload": f"{len(wl.sims)} simulations, "
            f"{wl.n_blocks} blocks, {cells} cells, Rusanov, FP32 flux / FP64 state", "steps": steps,
            "ms_per_step": t * 1e3 / steps, "shape": shape, "autotune_ms": ms, "graph": True,
            # algorithmic bytes (320 B per cell-update) over the whole graph-replayed step, against 8 TB/s
            "hbm_frac_of_step": cells * steps * (BYTES_STAGE[0] + BYTES_STAGE[1]) / t / (HBM_PEAK_GBS * 1e9)}


def bench_learned(steps, floor_rel=None):
    """The learned flux correction on the 128^3 magnetosphere grid (dx = 2) with the network shipped in
    paper_2501_06717_amd/trained (MLP 32-128-128-128-8 on BF16 matrix cores), HLLE + Powell, FP64 update,
    beside the plain FP64 path on the same grid. Both are timed from the developed state the one-step
    gain uses (the 256^3 run after 100 steps, restricted), with the share of flagged cell-stages of the
    timed window; then what the learned form gains over the plain path on that held-out solar-wind state
    against the restricted 256^3 run (200 coarse steps from the start, and one step), and the equal-cost
    comparison with a plain 192^3 run against a 384^3 reference."""
    import torch
    from paper_2501_06717_amd import binding, learn
    net = os.path.join(ROOT, "paper_2501_06717_amd", "trained", "flux_mlp_h128.npz")
    mlp, stats, meta = learn.load(net)
    cfg = learn.Config(hidden=meta["hidden"])
    if floor_rel is not None:
        cfg.floor_rel = floor_rel
    state = learn.solar_wind_states(1, 1005)[0]
    gf, g, coarse, Uf, _, Uc0 = learn.developed_state(binding, state, 256)
    del gf, Uf
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    res = {}
    for name, L in (("plain", None), ("learned", g.learned(mlp, stats, fallback=fb, floor_rel=cfg.floor_rel))):
        U0 = Uc0.clone()
        U1 = torch.empty_like(U0)
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        t = time_advance(g, U0, U1, dt, steps, flux="hlle", powell=True, learned=L, after_warmup=fb.zero_)
        res[name] = coarse.n_cells * steps / t
    cells = coarse.n_cells
    flagged = int(fb.item()) / (2.0 * steps * cells)
    del g, Uc0
    ev = learn.evaluate(binding, cfg, mlp, stats, [state], log=log)[0]
    eq = learn.equal_cost(binding, cfg, mlp, stats, state)
    log(f"learned: {res['learned']:.3e} vs plain {res['plain']:.3e} cell-updates/s on {cells} cells, "
        f"{100 * flagged:.2f} % of cell-stages flagged")
    return {"value": res["learned"], "unit": "cell-updates/s", "plain_value": res["plain"],
            "workload": f"magnetosphere 128^3 ({cells} cells), developed state (256^3 run after 100 steps, "
                        f"restricted), MLP 32-128-128-128-8 BF16, HLLE + Powell",
            "steps": steps, "floor_rel": cfg.floor_rel, "flagged_share_per_stage": flagged,
            "weights": "trained (paper_2501_06717_amd/trained/flux_mlp_h128.npz, strength %.2f)" % meta["strength"],
            "accuracy": {"state": state, "reference": "256^3 FP64 run restricted to 128^3, same time",
                         "l1_rel_plain": ev["plain"]["l1_rel_mean"], "l1_rel_learned": ev["learned"]["l1_rel_mean"],
                         "gain_200_steps": ev["gain"], "flagged_share_200_steps": ev["learned"]["flagged_share"],
                         "gain_one_step": ev["one_step"]["gain"],
                         "flagged_share_one_step": ev["one_step"]["flagged_share"],
                         "gain_one_step_exact_target": ev["one_step_exact_target"]["gain"]},
            "equal_cost": eq}


def copy_bandwidth():
    """Achievable HBM bandwidth: a 2 GiB device-to-device copy (read + write), best of 5, HIP events."""
    import torch
    n = 256 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = 1e30
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del src, dst
    return 2 * n * 8 / best / 1e9


def bench_local_dt(g, W, cells, steps):
    """Local time stepping (the steady-state mode: every cell advances with its own CFL step) on the same
    workload, FP64, default launch shape: the per-cell step is formed in the first stage from its input."""
    import torch
    U0 = g.set_state(W)
    U1 = torch.empty_like(U0)
    dt = torch.zeros((g.nb, 8, 8, 8), dtype=torch.float64, device="cuda")
    faults = torch.zeros(1, dtype=torch.int32, device="cuda")
    t = time_advance(g, U0, U1, dt, steps, flux="hlle", powell=True, cfl=0.8, local_dt=True, faults=faults)
    d = dt.cpu().numpy()
    fluid = d > 0.0
    log(f"local_dt: {cells * steps / t:.3e} cell-updates/s")
    return {"value": cells * steps / t, "unit": "cell-updates/s", "steps": steps, "faults": int(faults.item()),
            "dt_ratio_max_min": float(d[fluid].max() / d[fluid].min()),
            "workload": "the same grid, FP64, HLLE + Powell, each fluid cell its own CFL 0.8 step"}


def bench_paper_fast_wave():
    """The paper's one-GPU fast-wave run (Sec. 5.1, Eq. 6, Table 2 at m = 6) in 8^3 blocks: the periodic
    domain [-32, 32]^3 as 10^3 root blocks (dx = 0.8) with the octant [-32, 0]^3 refined once, 1,875
    blocks = 960,000 cells as in the paper's 960 blocks of 10^3; FP64, the Linde-type flux (the paper's
    Linde flux as read here) + Powell, MC, Heun, CFL 0.8, 500 steps; HLLE beside it. Context beside Table
    3's one-A100 total, not a target."""
    import torch
    from paper_2501_06717_amd import binding, workloads as wk
    wl = wk.fast_wave((10, 10, 10), refine_octant=True)
    g = binding.Grid.from_workload(wl).upload()
    U0 = g.set_state(torch.from_numpy(wl.W).cuda())
    U1 = torch.empty_like(U0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    faults = torch.zeros(1, dtype=torch.int32, device="cuda")
    steps = 500
    t = time_advance(g, U0, U1, dt, steps, flux="linde", powell=True, cfl=0.8, faults=faults)
    U0 = g.set_state(torch.from_numpy(wl.W).cuda())
    th = time_advance(g, U0, U1, dt, steps, flux="hlle", powell=True, cfl=0.8)
    cells = wl.n_cells
    log(f"paper fast wave: {cells} cells, {steps} steps in {t:.3f} s (Linde-type flux), {th:.3f} s (HLLE)")
    return {"value": cells * steps / t, "unit": "cell-updates/s", "wall_s": t, "steps": steps,
            "workload": f"fast wave (Eq. 6), [-32,32]^3 periodic, 10^3 root blocks of 8^3 + refined octant: "
                        f"{wl.n_blocks} blocks, {cells} cells, FP64, Linde-type flux (HLLE + contact "
                        f"anti-diffusion) + Powell, MC, Heun, CFL 0.8",
            "hlle": {"value": cells * steps / th, "wall_s": th},
            "faults": int(faults.item()),
            "paper_one_a100": {"wall_s": 5.76, "value": 960000 * 500 / 5.76, "unit": "cell-updates/s",
                               "workload": "960 blocks of 10^3 cells, Linde flux, 500 steps (Table 3, m = 6)"},
            "ratio_to_paper": cells * steps / t / (960000 * 500 / 5.76)}


def bench_two_level(steps):
    """The two-level magnetosphere (level-1 shell 3-10 body radii around the dipole: 7,456 blocks,
    3,817,472 cells, 264 coarse-fine block faces), HLLE + Powell, FP64 and FP32 flux with FP64 update, each
    from the initial state over `steps` steps; the FP32-flux result against the FP64 one. The stage
    includes the level-change ghost fill (restriction, prolongation) and the flux correction."""
    import torch
    from paper_2501_06717_amd import binding, workloads as wk
    wl = wk.two_level_magnetosphere(144)
    g = binding.Grid.from_workload(wl).upload()
    W = torch.from_numpy(wl.W).cuda()
    out = {"workload": f"two-level magnetosphere: {wl.n_blocks} blocks, {wl.n_cells} cells, "
                       f"{int(g.info.n_level_faces)} level-change block faces, HLLE + Powell, CFL 0.8",
           "steps": steps}
    res = {}
    for precision in ("fp64", "fp32_flux"):
        U0 = g.set_state(W)
        U1 = torch.empty_like(U0)
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        faults = torch.zeros(1, dtype=torch.int32, device="cuda")
        g.advance(U0, U1, dt, 2, flux="hlle", powell=True, cfl=0.8, precision=precision)  # warm-up
        U0 = g.set_state(W)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.advance(U0, U1, dt, 2 * steps, faults=faults, flux="hlle", powell=True, cfl=0.8, precision=precision)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res[precision] = U0.cpu().numpy()
        out[precision] = {"value": wl.n_cells * steps / t, "unit": "cell-updates/s", "wall_s": t,
                          "faults": int(faults.item())}
        del U0, U1
        log(f"two-level {precision}: {wl.n_cells * steps / t:.3e} cell-updates/s over {steps} steps")
    ref, got = res["fp64"], res["fp32_flux"]
    out["fp32_flux"]["l1_rel_vs_fp64"] = float(np.abs(got - ref).sum() / np.abs(ref).sum())
    out["fp32_flux"]["linf_rel_vs_fp64"] = {k: float(np.abs(got[v] - ref[v]).max() / np.abs(ref[v]).max())
                                            for k, v in (("rho", [0]), ("mom", [1, 2, 3]), ("B", [4, 5, 6]),
                                                         ("e", [7]))}
    del g, W, res
    torch.cuda.synchronize()
    return out


def bench_exchange(reps=20):
    """The ghost exchange between processes (Algorithm 4) at one process's share of the 256^3
    magnetosphere split into 2 x 2 x 2 processes of 128^3 cells (4,096 blocks each): the pack kernel of
    process 0 (its messages to the 7 other processes: 3 faces, 3 edges, 1 corner of sub-cubes), the unpack
    of the messages it receives (plus its local messages and boundary ghosts), with the transfers as device
    copies between them. Per call: HIP events around each kernel launch, mean over `reps`."""
    import torch
    from paper_2501_06717_amd import binding, workloads as wk
    wl = wk.magnetosphere(256)
    ijk = np.asarray(wl.ijk).reshape(-1, 3)
    rank = ((ijk[:, 0] // 16) + 2 * (ijk[:, 1] // 16) + 4 * (ijk[:, 2] // 16)).astype(np.int32)
    g = binding.Grid.from_workload(wl).upload()
    x = binding.Xchg(g, rank, 8).upload()
    U = g.set_state(torch.from_numpy(wl.W).cuda())
    views = [x.new_view(r) for r in range(8)]
    for r in range(8):
        x.interior(r, U, views[r])
    sends = [torch.empty(x.send_len(1, s), dtype=torch.float64, device="cuda") for s in range(8)]
    recvs = [torch.empty(x.recv_len(1, r), dtype=torch.float64, device="cuda") for r in range(8)]
    for s in range(8):
        x.pack(1, s, views[s], sends[s])
    x.transfer(1, sends, recvs)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    tp = tu = 0.0
    for _ in range(reps):
        ev[0].record()
        x.pack(1, 0, views[0], sends[0])
        ev[1].record()
        ev[2].record()
        x.unpack(1, 0, recvs[0], views[0])
        ev[3].record()
        torch.cuda.synchronize()
        tp += ev[0].elapsed_time(ev[1]) * 1e-3 / reps
        tu += ev[2].elapsed_time(ev[3]) * 1e-3 / reps
    msgs = x.messages()
    m0 = msgs[(msgs[:, 0] == 0) & (msgs[:, 1] != 0)]
    r0 = msgs[(msgs[:, 1] == 0) & (msgs[:, 0] != 0)]
    sent, recv = 8 * x.send_len(1, 0), 8 * x.recv_len(1, 0)
    out = {"workload": "256^3 magnetosphere as 2 x 2 x 2 processes of 128^3 cells (4,096 blocks each); "
                       "process 0's pass 1 (copies)",
           "messages_sent": int(len(m0)), "messages_received": int(len(r0)),
           "bytes_sent": sent, "bytes_received": recv,
           "pack_us": tp * 1e6, "unpack_us": tu * 1e6,
           "pack_GBs": sent / tp / 1e9, "unpack_GBs": recv / tu / 1e9,
           "note": "unpack also copies process 0's local messages (every ghost face inside its sub-cube) and "
                   "fills its outflow/inflow ghost cells"}
    log(f"exchange: pack {tp * 1e6:.1f} us ({sent / 1e6:.1f} MB), unpack {tu * 1e6:.1f} us ({recv / 1e6:.1f} MB)")
    del views, sends, recvs
    # whole steps with the eight processes advanced separately from their exchanged views (every process's
    # exchange and stage run one after another on this one GPU), beside the single-process step on the
    # same grid with the same per-step dt; the first step of each warms up
    steps = 3
    walls = {}
    x = binding.Xchg(g, rank, 8, for_stage=True).upload()
    for name in ("sharded", "single"):
        U = g.set_state(torch.from_numpy(wl.W).cuda())
        U1 = torch.empty_like(U)
        for k in range(steps + 1):
            if k == 1:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            if name == "sharded":
                x.advance(U, U1, 1, cfl=0.8, flux="hlle", powell=True)
            else:
                dt = g.reduce_dt(U, 0.8)
                g.advance(U, U1, dt, 2, recompute_dt=False, flux="hlle", powell=True)
        torch.cuda.synchronize()
        walls[name] = (time.perf_counter() - t0) / steps
        del U, U1
    out["sharded_step_ms"] = walls["sharded"] * 1e3
    out["single_step_ms"] = walls["single"] * 1e3
    out["sharded_note"] = ("stage-mode maps: each process's stage reads the ghost cells of faces whose neighbour is "
                           "on another process from its view and the rest in place; the exchange copies only the "
                           "sending blocks' interiors; on one GPU the eight processes run one after another")
    log(f"exchange: sharded step {walls['sharded'] * 1e3:.2f} ms, single-process step {walls['single'] * 1e3:.2f} ms")
    del x, g
    torch.cuda.synchronize()
    return out


def accuracy_vs_oracle(binding, wl, R, steps):
    """L1 and per-group L-infinity error of the FP64 path and of the FP32-flux form against the oracle's
    result R after the same steps from the same state (the workload the benchmark times, full size)."""
    import torch
    g = binding.Grid.from_workload(wl).upload()
    W = torch.from_numpy(wl.W).cuda()
    out = {"steps": steps, "reference": "the CPU oracle (FP64) on the same steps of the same workload"}
    for precision in ("fp64", "fp32_flux"):
        U0 = g.set_state(W)
        U1 = torch.empty_like(U0)
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        faults = torch.zeros(1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        g.advance(U0, U1, dt, 2 * steps, faults=faults, flux="hlle", powell=True, cfl=0.8, precision=precision)
        torch.cuda.synchronize()
        got = U0.cpu().numpy()
        del U0, U1
        out[precision] = {"l1_rel": float(np.abs(got - R).sum() / np.abs(R).sum()),
                          "linf_rel": {k: float(np.abs(got[v] - R[v]).max() / np.abs(R[v]).max())
                                       for k, v in (("rho", [0]), ("mom", [1, 2, 3]), ("B", [4, 5, 6]), ("e", [7]))},
                          "faults": int(faults.item())}
        del got
    del g, W
    torch.cuda.synchronize()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2501_06717_amd import binding, workloads as wk

    torch.cuda.set_device(0)
    if a.profile and a.form != "plain":
        fn = {"batched": bench_batched, "learned": bench_learned, "two_level": bench_two_level,
              "exchange": bench_exchange}[a.form]
        log(json.dumps(fn(a.steps)))
        return
    wl = wk.magnetosphere(a.n, n_steps=a.steps)
    log(f"workload {wl.name}: {wl.n_blocks} blocks, {wl.n_cells} cells")
    g = binding.Grid.from_workload(wl).upload()
    W = torch.from_numpy(wl.W).cuda()
    steps, warm = a.steps, a.warmup

    U64, wall, st, faults, dt_last = time_form(g, W, steps, warm, a.precision, a.slab, a.persist, a.scheme)
    cells = wl.n_cells
    value = cells * steps / wall
    t1, t2 = float(np.mean(st[0])), float(np.mean(st[1]))
    achieved = cells * (BYTES_STAGE[0] + BYTES_STAGE[1]) / (t1 + t2) / 1e9
    scheme, ks = resolve_shape(a.scheme, a.slab, a.precision, a.persist)
    fp64 = a.precision == "fp64"
    prec = 'double' if fp64 else 'float'
    kname = {"plane": f"k_stage_wp<{ks}, {prec}, HLLE, Powell>", "face": f"k_stage<{ks}, {prec}, HLLE, Powell>",
             "block": f"k_stage_blk<{prec}, HLLE, Powell>"}[scheme]
    meas = TRAFFIC.get((scheme, ks)) if (a.n == 256 and not a.persist and fp64) else None
    traffic = 0.5 * (meas[0] + meas[1]) if meas else None
    vpc = VALU_PER_CELL_STAGE.get((scheme, ks)) if (a.n == 256 and not a.persist and fp64) else None
    valu = None
    if vpc:
        rate = vpc * cells * 2 / (t1 + t2)
        valu = {"bound": "alu", "achieved": rate / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12,
                "unit": "T VALU lane-instructions/s", "frac": rate / VALU_PEAK_LANE_OPS,
                "instructions_per_cell_stage": vpc,
                "hbm_frac_at_full_valu_issue": VALU_PEAK_LANE_OPS / (2 * vpc) * 320 / (HBM_PEAK_GBS * 1e9)}
    log(f"{a.precision}: {wall * 1e3:.2f} ms for {steps} steps, stage kernels {t1 * 1e6:.1f} / {t2 * 1e6:.1f} us, "
        f"faults {faults}, dt {dt_last:.4e}")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else "f32 flux / f64 state",
        "data": "synthetic",
        "config": {"workload": f"magnetosphere {a.n}^3 cells ({wl.n_blocks} blocks of 8^3), dipole + solar-wind "
                               "inflow, body r=2.5, HLLE + Powell, MC, Heun, CFL 0.8, "
                               + ("FP64" if fp64 else "FP32 reconstruction/flux, FP64 update"),
                   "cells": cells, "blocks": wl.n_blocks, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per stage-kernel launch, mean of the two stages",
                     "algorithmic_bytes_per_launch": 0.5 * cells * (BYTES_STAGE[0] + BYTES_STAGE[1]),
                     "kernel": kname + " (both stages; " + {"plane": "wave per cell layer",
                                                            "face": "face per thread",
                                                            "block": "wave per cell layer, one workgroup per block"}[scheme]
                               + f", tile 8x8x{ks})",
                     "stage_us": [t1 * 1e6, t2 * 1e6], "bytes_per_cell_update": 320,
                     "valu": valu},
        "faults": faults,
    }
    if not a.profile:
        bw = copy_bandwidth()
        out["roofline"]["measured_copy_GBs"] = bw
        out["roofline"]["frac_of_measured_copy"] = achieved / bw
        log(f"device copy: {bw:.0f} GB/s")
    if a.calib:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not (a.no_forms or a.profile) and fp64:
        U32, wall32, st32, f32, _ = time_form(g, W, steps, warm, "fp32_flux", a.slab, a.persist, a.scheme)
        ref = U64.cpu().numpy()
        got = U32.cpu().numpy()
        l1 = float(np.abs(got - ref).sum() / np.abs(ref).sum())
        linf = {k: float(np.abs(got[v] - ref[v]).max() / np.abs(ref[v]).max())
                for k, v in (("rho", [0]), ("mom", [1, 2, 3]), ("B", [4, 5, 6]), ("e", [7]))}
        t1_32, t2_32 = float(np.mean(st32[0])), float(np.mean(st32[1]))
        ach32 = cells * (BYTES_STAGE[0] + BYTES_STAGE[1]) / (t1_32 + t2_32) / 1e9
        out["forms"] = {"fp32_flux": {"value": cells * steps / wall32, "unit": "cell-updates/s",
                                      "stage_us": [t1_32 * 1e6, t2_32 * 1e6],
                                      "roofline": {"bound": "hbm", "achieved": ach32, "peak": HBM_PEAK_GBS,
                                                   "unit": "GB/s", "frac": ach32 / HBM_PEAK_GBS,
                                                   "kernel": "k_stage_blk<float, HLLE, Powell> (both stages)"
                                                   if resolve_shape(a.scheme, a.slab, "fp32_flux", a.persist)[0]
                                                   == "block" else "stage kernel (both stages)"},
                                      "l1_rel_vs_fp64": l1, "linf_rel_vs_fp64": linf, "faults": f32,
                                      "error_reference": "the FP64 GPU path on the same steps (itself within "
                                                         "1e-12 of the CPU oracle)"}}
        log(f"fp32_flux: {wall32 * 1e3:.2f} ms, L1 {l1:.3e}")
        del U32
        out["forms"]["local_dt"] = bench_local_dt(g, W, cells, a.form_steps)
    del U64
    torch.cuda.synchronize()
    if not (a.no_forms or a.profile) and fp64:
        del g, W
        out.setdefault("forms", {})
        out["forms"]["two_level"] = bench_two_level(a.two_level_steps)
        out["forms"]["exchange"] = bench_exchange()
        out["forms"]["batched"] = bench_batched(a.form_steps)
        out["forms"]["learned"] = bench_learned(a.form_steps)
        out["paper_context"] = {"fast_wave": bench_paper_fast_wave()}
    if not (a.no_cpu_baseline or a.profile):
        import oracle
        o = oracle.Grid.from_workload(wl)
        U0 = o.set_state(wl.W)
        U1 = np.zeros_like(U0)
        cores = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        o.advance(U0, U1, [0.0], 2 * a.cpu_steps, flux="hlle", powell=True, cfl=0.8)
        tc = time.perf_counter() - t0
        threads = int(os.environ.get("OMP_NUM_THREADS", cores))
        out["cpu_baseline"] = {"value": cells * a.cpu_steps / tc, "unit": "cell-updates/s",
                               "cores": min(cores, threads), "kind": "oracle",
                               "sample": f"{a.cpu_steps} full step(s) of the same {a.n}^3 workload "
                                         f"({tc:.1f} s, OpenMP over blocks)"}
        log(f"cpu oracle: {tc:.1f} s for {a.cpu_steps} step(s)")
        out["accuracy_vs_oracle"] = accuracy_vs_oracle(binding, wl, U0, a.cpu_steps)
        log(f"accuracy vs oracle: {json.dumps(out['accuracy_vs_oracle'])}")
        if "two_level" in out.get("forms", {}):
            # the two-level form after one step against the oracle doing the same step
            tl = wk.two_level_magnetosphere(144)
            ot = oracle.Grid.from_workload(tl)
            R0 = ot.set_state(tl.W)
            R1 = np.zeros_like(R0)
            ot.advance(R0, R1, [0.0], 2, flux="hlle", powell=True, cfl=0.8)
            out["forms"]["two_level"]["accuracy_vs_oracle"] = accuracy_vs_oracle(binding, tl, R0, 1)
            del R0, R1
            log("two-level accuracy vs oracle: " + json.dumps(out["forms"]["two_level"]["accuracy_vs_oracle"]))
        # one thread on a 64^3 cut of the same workload (the per-cell work is the same), for the GPU's
        # equivalent in host cores
        import ctypes
        gomp = ctypes.CDLL("libgomp.so.1")
        cut = wk.magnetosphere_cut(64)
        oc = oracle.Grid.from_workload(cut)
        V0 = oc.set_state(cut.W)
        V1 = np.zeros_like(V0)
        gomp.omp_set_num_threads(1)
        t0 = time.perf_counter()
        oc.advance(V0, V1, [0.0], 2, flux="hlle", powell=True, cfl=0.8)
        t1c = time.perf_counter() - t0
        gomp.omp_set_num_threads(min(cores, threads))
        one = cut.n_cells / t1c
        out["cpu_baseline"]["one_thread"] = {"value": one, "unit": "cell-updates/s",
                                             "sample": f"1 step of the {cut.n_cells}-cell cut of the same workload "
                                                       f"({t1c:.1f} s, one thread)"}
        out["cpu_baseline"]["gpu_equivalent_cores"] = value / one
        log(f"cpu oracle, one thread: {one:.3e} cell-updates/s; GPU = {value / one:.0f} cores")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
