"""Learned flux correction for coarse magnetosphere grids: data, training and evaluation.

The network corrects the plain HLLE flux of a coarse grid (128^3 cells, dx = 2) toward the flux a grid
twice as fine would put through the same face. Training data come from plain FP64 runs on the fine
grid (256^3, dx = 1: the coarse grid's simulation with every root refined once) of solar-wind states
drawn at random:

* every `snap_every` fine steps, the fine state is restricted to the coarse grid (mean of the 8 fine
  cells); the target of a coarse face is the mean of the 4 fine face fluxes covering it minus the plain
  HLLE flux of the restricted coarse state, both in the face-normal frame;
* the inputs are the 4-cell stencils of coarse primitives in the face-normal frame;
* per snapshot and direction, a share `top_frac` of the sampled faces comes from the top decile of the
  target magnitude and the rest is uniform; inputs and targets are z-scored with training-set statistics;
* optionally (`pair`) the samples are the two faces of a coarse cell along each direction and the loss
  weighs the error of their difference, which is what the cell update sees;
* the stage applies `strength` times the network's correction (folded into the output statistics).

Evaluation on held-out states: coarse plain and coarse learned runs against the fine run restricted, over
many steps and over one step; the one-step test also runs with the exact target of that state given as
the correction (no network), the bound for any correction of this form.

Training and inference run in the library's kernels (BF16 matrix cores, FP32 master weights, Adam), and
so do restriction (bmhd_remap) and the face targets (bmhd_face_targets); sampling and statistics use torch
tensor operations on the GPU.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import sys
import time

import numpy as np

from . import workloads as wk

GAMMA = 5.0 / 3.0


def solar_wind_states(n, seed):
    """Random solar-wind states: rho ~ U[1, 20], speed ~ U[300, 800] along -x, Bz ~ U[-10, 10]; pressure
    from sonic Mach 8."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        rho = rng.uniform(1.0, 20.0)
        speed = rng.uniform(300.0, 800.0)
        bz = rng.uniform(-10.0, 10.0)
        out.append(dict(rho=rho, ux=-speed, bz=bz))
    return out


def magnetosphere_pair(state, n_fine=256, M=7.9e4):
    """Fine and coarse workloads of one solar-wind state: the coarse grid (n_fine/2)^3, dx = 2, level-0
    blocks; the fine grid the same simulation with every root refined once (all blocks level 1, dx = 1),
    so that bmhd_remap restricts fine states onto the coarse grid and bmhd_face_targets pairs the faces."""
    sim = wk.magnetosphere_sim(n_fine // 2, **state)
    lv, ijk, sid = wk.uniform_blocks(sim.nroot)
    coarse = wk.Workload(f"coarse_{n_fine // 2}", lv, ijk, sid, [sim], wk.magnetosphere_state(sim, lv, ijk, M),
                         flux="hlle", powell=True, cfl=0.8)
    lvf, ijkf, sidf = wk.two_level_blocks(sim.nroot, np.ones(sim.nroot[::-1], bool))
    fine = wk.Workload(f"fine_{n_fine}", lvf, ijkf, sidf, [sim], wk.magnetosphere_state(sim, lvf, ijkf, M),
                       flux="hlle", powell=True, cfl=0.8)
    return fine, coarse


def low_faces(nb, d):
    """Rows of the per-block face layout (bmhd_face_data: [block][3][576]) of direction d whose position
    along d is 0..7: every face of the grid once (faces on the domain's high side excepted)."""
    import torch
    f = torch.arange(576)
    a = (f % 9) if d == 0 else (((f >> 3) % 9) if d == 1 else (f >> 6))
    sel = f[a < 8]
    return (torch.arange(nb).reshape(-1, 1) * 1728 + d * 576 + sel.reshape(1, -1)).reshape(-1)


def face_pairs(nb, d):
    """Row pairs (low face, high face) of every cell along direction d in the per-block face layout."""
    import torch
    k, j, i = torch.meshgrid(torch.arange(8), torch.arange(8), torch.arange(8), indexing="ij")
    i, j, k = i.reshape(-1), j.reshape(-1), k.reshape(-1)   # cell (i, j, k) = (x, y, z)
    if d == 0:
        lo, hi = (k * 8 + j) * 9 + i, (k * 8 + j) * 9 + i + 1
    elif d == 1:
        lo, hi = (k * 9 + j) * 8 + i, (k * 9 + j + 1) * 8 + i
    else:
        lo, hi = (k * 8 + j) * 8 + i, ((k + 1) * 8 + j) * 8 + i
    base = torch.arange(nb).reshape(-1, 1) * 1728 + d * 576
    return (base + lo.reshape(1, -1)).reshape(-1), (base + hi.reshape(1, -1)).reshape(-1)


# --------------------------------------------------------------------------------------------------
# global arrays from per-block data

def to_global(U, nb):
    """[8, nb^3 blocks (i fastest), 8, 8, 8] -> [8, N, N, N] (z, y, x)."""
    v = U.shape[0]
    t = U.reshape(v, nb, nb, nb, 8, 8, 8)           # (bz, by, bx, k, j, i)
    return t.permute(0, 1, 4, 2, 5, 3, 6).reshape(v, nb * 8, nb * 8, nb * 8)


def from_global(G, nb):
    v = G.shape[0]
    t = G.reshape(v, nb, 8, nb, 8, nb, 8)           # (bz, k, by, j, bx, i)
    return t.permute(0, 1, 3, 5, 2, 4, 6).reshape(v, nb ** 3, 8, 8, 8).contiguous()


def restrict_by(Uf, nbf, k):
    """Mean of the k^3 fine cells of each coarse cell (conserved variables); nbf^3 fine blocks of 8^3 in
    i-fastest order. Used where no remap applies: the equal-cost comparison restricts a 384^3 uniform run
    by 3 and by 2."""
    G = to_global(Uf, nbf)
    n = G.shape[1] // k
    Gc = G.reshape(8, n, k, n, k, n, k).mean(dim=(2, 4, 6))
    return from_global(Gc, nbf // k)


# --------------------------------------------------------------------------------------------------
# data generation

@dataclasses.dataclass
class Config:
    n_fine: int = 256
    train_states: int = 32
    heldout_states: int = 2
    fine_steps: int = 200          # fine steps per training state (a snapshot every snap_every)
    eval_fine_steps: int = 400     # evaluation horizon in fine steps (the coarse runs take half as many)
    snap_every: int = 20
    samples_per_dir: int = 16384
    top_frac: float = 0.0          # share of each snapshot's samples drawn from the top decile of |target|
    pair: float = 0.0              # > 0: samples are the two faces of a coarse cell along each direction, and
                                   # this weight goes to the error of their difference (what the cell update
                                   # sees); the rest to the error of each face
    hidden: int = 128
    epochs: int = 24
    strength: float = 0.25         # the correction applied is this fraction of the network's output
    floor_rel: float = 0.01        # least neighbourhood range of the acceptance test, relative to its magnitude
    batch: int = 4096
    lr: float = 1e-3
    seed_train: int = 5
    seed_heldout: int = 1005


def fine_dt(g, U, cfl=0.8):
    return g.reduce_dt(U, cfl)


def snapshot_targets(gf, gc, Uf):
    """Coarse stencil features Xc [nbc * 1728, 32] and flux-correction targets T [nbc * 1728, 8] of one
    fine snapshot (the fine state restricted by bmhd_remap; targets by bmhd_face_targets)."""
    Uc = gf.remap(Uf, gc)
    Xc, Fc = gc.face_data(Uc, flux="hlle")
    _, Ff = gf.face_data(Uf, flux="hlle", want_x=False)
    T = gf.face_targets(Ff, gc, Fc)
    del Ff, Fc, Uc
    return Xc, T


def sample(n, mag, gen):
    """Indices 0..n-1: `samples` of them, a share `top_frac` from the top decile of `mag`, the rest
    uniform."""
    import torch
    kt = int(round(gen["samples"] * gen["top_frac"]))
    ku = gen["samples"] - kt
    top = torch.topk(mag, max(n // 10, kt)).indices
    pick_top = top[torch.randint(0, top.numel(), (kt,), generator=gen["g"], device=top.device)]
    pick_uni = torch.randint(0, n, (ku,), generator=gen["g"], device=top.device)
    return torch.cat([pick_uni, pick_top])


def snapshot_data(bd, gf, gc, Uf, gen):
    """(X, T) samples of one fine snapshot: coarse stencil features and flux corrections."""
    import torch
    Xc, T = snapshot_targets(gf, gc, Uf)
    xs, ts = [], []
    for d in range(3):
        rows = low_faces(gc.nb, d).to(T.device)
        Td, Xd = T[rows], Xc[rows]
        idx = sample(Td.shape[0], (Td / (Td.std(dim=0) + 1e-30)).norm(dim=1), gen)
        xs.append(Xd[idx])
        ts.append(Td[idx])
    return torch.cat(xs), torch.cat(ts)


def snapshot_pairs(bd, gf, gc, Uf, gen):
    """Samples of one fine snapshot as face pairs: the low and high face of a coarse cell along each
    direction, X [n, 2, 32] (coarse stencil features) and T [n, 2, 8] (flux corrections). A share
    `top_frac` comes from the top decile of the difference of the two corrections, the rest is uniform."""
    import torch
    Xc, T = snapshot_targets(gf, gc, Uf)
    xs, ts = [], []
    for d in range(3):
        lo, hi = (r.to(T.device) for r in face_pairs(gc.nb, d))
        Ta, Tb, Xa, Xb = T[lo], T[hi], Xc[lo], Xc[hi]
        dT = Tb - Ta
        idx = sample(Ta.shape[0], (dT / (dT.std(dim=0) + 1e-30)).norm(dim=1), gen)
        xs.append(torch.stack([Xa[idx], Xb[idx]], dim=1))
        ts.append(torch.stack([Ta[idx], Tb[idx]], dim=1))
    return torch.cat(xs), torch.cat(ts)


def generate(bd, cfg: Config, states, log=print):
    """Training samples from fine plain FP64 runs of the given solar-wind states."""
    import torch
    gen = {"g": torch.Generator(device="cuda"), "samples": cfg.samples_per_dir, "top_frac": cfg.top_frac}
    gen["g"].manual_seed(cfg.seed_train)
    X, T = [], []
    for si, st in enumerate(states):
        fine, coarse = magnetosphere_pair(st, cfg.n_fine)
        gf = bd.Grid.from_workload(fine).upload()
        gc = bd.Grid.from_workload(coarse).upload()
        U0 = gf.set_state(torch.from_numpy(fine.W).cuda())
        U1 = torch.empty_like(U0)
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        t0 = time.time()
        for s0 in range(0, cfg.fine_steps, cfg.snap_every):
            gf.advance(U0, U1, dt, 2 * cfg.snap_every, flux="hlle", powell=True, cfl=0.8)
            x, t = (snapshot_pairs if cfg.pair > 0 else snapshot_data)(bd, gf, gc, U0, gen)
            X.append(x)
            T.append(t)
        torch.cuda.synchronize()
        log(f"state {si}: {st}, {cfg.fine_steps} fine steps + snapshots in {time.time() - t0:.1f} s")
        del gf, gc, U0, U1
    return torch.cat(X), torch.cat(T)


def train(bd, cfg: Config, X, T, log=print, init=None):
    """Adam on z-scored inputs and targets; returns (mlp, stats[80], loss history). `init`: parameters to
    start from (a network written by save(), trained on the same data statistics), else He-style random."""
    import torch
    pairs = X.dim() == 3
    Xf, Tf = (X.reshape(-1, 32), T.reshape(-1, 8)) if pairs else (X, T)
    xm, xs = Xf.mean(0), Xf.std(0) + 1e-12
    tm, ts = Tf.mean(0), Tf.std(0) + 1e-30
    Xn = ((X - xm) / xs).contiguous()
    Tn = ((T - tm) / ts).contiguous()
    wd = cfg.pair if pairs else 0.0
    stats = torch.cat([xm, xs, tm, ts]).float()
    rng = np.random.default_rng(cfg.seed_train)
    npar = int(bd.lib().bmhd_mlp_n_params(cfg.hidden))
    # He-style initialisation of the FP32 master weights
    p = np.zeros(npar, np.float32)
    o = 0
    for (nout, nin) in [(cfg.hidden, 32), (cfg.hidden, cfg.hidden), (cfg.hidden, cfg.hidden), (8, cfg.hidden)]:
        p[o:o + nout * nin] = rng.normal(scale=math.sqrt(2.0 / nin), size=nout * nin)
        o += nout * nin + nout
    if init is not None:
        p = np.load(init, allow_pickle=False)["params"].astype(np.float32)
    mlp = bd.Mlp(cfg.hidden, torch.from_numpy(p))
    n = Xn.shape[0]
    hist = []
    g = torch.Generator(device="cuda")
    g.manual_seed(cfg.seed_train)
    steps = cfg.epochs * (n // cfg.batch)
    it = 0
    for ep in range(cfg.epochs):
        perm = torch.randperm(n, generator=g, device="cuda")
        tot, nb = 0.0, 0
        for b0 in range(0, n - cfg.batch + 1, cfg.batch):
            idx = perm[b0:b0 + cfg.batch]
            if pairs:
                # difference loss through the face loss's gradient: the pseudo-target of each face is
                # (1 - wd) * its target + wd * (the other face's prediction + the target difference), so the
                # gradient is (1 - wd) * face error + wd * error of the difference
                xa, xb = Xn[idx, 0].contiguous(), Xn[idx, 1].contiguous()
                ta, tb = Tn[idx, 0], Tn[idx, 1]
                ya, yb = mlp.forward(xa), mlp.forward(xb)
                dT = ta - tb
                pa = (1.0 - wd) * ta + wd * (yb + dT)
                pb = (1.0 - wd) * tb + wd * (ya - dT)
                loss, grad = mlp.loss_grad(torch.cat([xa, xb]), torch.cat([pa, pb]).contiguous())
                loss = ((ya - yb) - dT).pow(2).mean()
            else:
                loss, grad = mlp.loss_grad(Xn[idx].contiguous(), Tn[idx].contiguous())
            # cosine decay of the learning rate to a tenth over the run
            lr = cfg.lr * (0.1 + 0.45 * (1.0 + math.cos(math.pi * it / max(steps, 1))))
            mlp.adam(grad, lr=lr)
            it += 1
            tot += float(loss)
            nb += 1
        hist.append(tot / max(nb, 1))
        log(f"epoch {ep}: mean batch loss {hist[-1]:.4f}")
    return mlp, stats, hist


def developed_state(bd, st, n_fine, warm_steps=100):
    """The fine run of solar-wind state `st` after `warm_steps` fine steps (HLLE + Powell, CFL 0.8) and its
    restriction to the coarse grid: (fine grid, coarse grid, coarse workload, fine state, the fine dt of
    that state, restricted coarse state). The flow has then left the uniform start."""
    import torch
    fine, coarse = magnetosphere_pair(st, n_fine)
    gf = bd.Grid.from_workload(fine).upload()
    gc = bd.Grid.from_workload(coarse).upload()
    Uf = gf.set_state(torch.from_numpy(fine.W).cuda())
    U1 = torch.empty_like(Uf)
    dtf = torch.zeros(1, dtype=torch.float64, device="cuda")
    gf.advance(Uf, U1, dtf, 2 * warm_steps, flux="hlle", powell=True, cfl=0.8)
    dtf = gf.reduce_dt(Uf, 0.8)
    return gf, gc, coarse, Uf, dtf, gf.remap(Uf, gc)


def one_step_gain(bd, cfg: Config, mlp, stats, st, warm_steps=100):
    """Local (one coarse step) error: from the restricted fine state after `warm_steps` fine steps, one
    coarse step (dt = 2 fine dt) plain and learned against the fine run advanced two steps and restricted.
    L1 of the change of state, per variable, relative to the fine change; and the flagged share of the
    learned step's cell-stages."""
    import torch
    gf, gc, coarse, Uf, dtf, Uc0 = developed_state(bd, st, cfg.n_fine, warm_steps)
    U1 = torch.empty_like(Uf)
    gf.advance(Uf, U1, dtf, 4, flux="hlle", powell=True, recompute_dt=False)
    dref = gf.remap(Uf, gc) - Uc0
    out = {}
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    for name, learned in (("plain", None), ("learned", gc.learned(mlp, stats, fallback=fb, floor_rel=cfg.floor_rel))):
        U = Uc0.clone()
        Ub = torch.empty_like(U)
        gc.advance(U, Ub, dtf * 2.0, 2, flux="hlle", powell=True, recompute_dt=False, learned=learned)
        d = U - Uc0
        out[name] = [float((d[v] - dref[v]).abs().sum() / dref[v].abs().sum()) for v in range(8)]
    out["gain"] = float(np.mean(out["plain"]) / max(np.mean(out["learned"]), 1e-300))
    out["flagged_share"] = int(fb.item()) / (2.0 * coarse.n_cells)
    return out


def exact_target_one_step(bd, cfg: Config, st, warm_steps=100):
    """The one_step_gain test with the exact a-priori target (from the fine state, not a network) given to
    the learned stage as its correction: the best a correction of this form can do from this state."""
    import torch
    gf, gc, coarse, Uf, dtf, Uc0 = developed_state(bd, st, cfg.n_fine, warm_steps)
    U1 = torch.empty_like(Uf)
    _, Fc = gc.face_data(Uc0, flux="hlle", want_x=False)
    _, Ff = gf.face_data(Uf, flux="hlle", want_x=False)
    y = gf.face_targets(Ff, gc, Fc)
    del Ff, Fc
    gf.advance(Uf, U1, dtf, 4, flux="hlle", powell=True, recompute_dt=False)
    dref = gf.remap(Uf, gc) - Uc0
    stats = torch.zeros(80)
    stats[32:64] = 1.0
    stats[72:80] = 1.0
    out = {}
    for name in ("plain", "exact"):
        L = gc.given_corrections(y, stats, tau=1e30) if name == "exact" else None
        U = Uc0.clone()
        Ub = torch.empty_like(U)
        gc.advance(U, Ub, dtf * 2.0, 2, flux="hlle", powell=True, recompute_dt=False, learned=L)
        d = U - Uc0
        out[name] = [float((d[v] - dref[v]).abs().sum() / dref[v].abs().sum()) for v in range(8)]
    out["gain"] = float(np.mean(out["plain"]) / max(np.mean(out["exact"]), 1e-300))
    return out


def evaluate(bd, cfg: Config, mlp, stats, states, log=print):
    """Coarse plain vs coarse learned against the fine run restricted, at the same time."""
    import torch
    out = []
    for st in states:
        fine, coarse = magnetosphere_pair(st, cfg.n_fine)
        gf = bd.Grid.from_workload(fine).upload()
        gc = bd.Grid.from_workload(coarse).upload()
        Uf = gf.set_state(torch.from_numpy(fine.W).cuda())
        dtf = gf.reduce_dt(Uf, 0.8)
        Uc0 = gf.remap(Uf, gc)
        U1 = torch.empty_like(Uf)
        gf.advance(Uf, U1, dtf, 2 * cfg.eval_fine_steps, flux="hlle", powell=True, recompute_dt=False)
        ref = gf.remap(Uf, gc)
        del U1
        dtc = dtf * 2.0
        res = {}
        fb = torch.zeros(1, dtype=torch.int32, device="cuda")
        for name, learned in (("plain", None),
                              ("learned", gc.learned(mlp, stats, fallback=fb, floor_rel=cfg.floor_rel))):
            U = Uc0.clone()
            Ub = torch.empty_like(U)
            dt = dtc.clone()
            faults = torch.zeros(1, dtype=torch.int32, device="cuda")
            gc.advance(U, Ub, dt, cfg.eval_fine_steps, flux="hlle", powell=True, recompute_dt=False, learned=learned,
                       faults=faults)
            torch.cuda.synchronize()
            l1 = [float((U[v] - ref[v]).abs().sum() / ref[v].abs().sum()) for v in range(8)]
            res[name] = {"l1_rel_mean": float(np.mean(l1)), "l1_rel": l1, "faults": int(faults.item())}
        res["learned"]["flagged_share"] = int(fb.item()) / (float(cfg.eval_fine_steps) * coarse.n_cells)  # per stage
        res["gain"] = res["plain"]["l1_rel_mean"] / max(res["learned"]["l1_rel_mean"], 1e-300)
        res["one_step"] = one_step_gain(bd, cfg, mlp, stats, st)
        res["one_step_exact_target"] = exact_target_one_step(bd, cfg, st)
        log(f"held-out {st}: plain L1 {res['plain']['l1_rel_mean']:.4e}, learned {res['learned']['l1_rel_mean']:.4e}, "
            f"gain {res['gain']:.3f}; one-step gain {res['one_step']['gain']:.3f} (exact target: "
            f"{res['one_step_exact_target']['gain']:.3f})")
        out.append(res)
    return out


def equal_cost(bd, cfg: Config, mlp, stats, st, coarse_steps=100, n_ref=384):
    """The learned coarse run beside a plain run on a finer grid of about the same cost. Plain and learned
    at 128^3 and plain at 192^3 ((3/2)^4 = 5.06 times the plain 128^3 work per unit of simulated time)
    advance from the n_ref^3 initial state restricted, to the time of `coarse_steps` coarse steps, with
    the n_ref^3 run's CFL-0.8 step scaled by the cell size (the dt of every run is that run's CFL 0.8);
    each is compared with the n_ref^3 run restricted to its grid. Returns per run: relative L1 error
    (mean over the 8 conserved variables) and wall time."""
    import time
    import torch
    ref_wl = wk.magnetosphere(n_ref, **st)
    nbr = n_ref // 8
    gr = bd.Grid.from_workload(ref_wl).upload()
    Ur = gr.set_state(torch.from_numpy(ref_wl.W).cuda())
    dtr = gr.reduce_dt(Ur, 0.8)
    runs = {}
    for name, n, learned in (("plain_128", 128, False), ("learned_128", 128, True), ("plain_192", 192, False)):
        k = n_ref // n
        assert k * n == n_ref
        sim = wk.magnetosphere_sim(n, **st)
        lv, ijk, sid = wk.uniform_blocks(sim.nroot)
        wl = wk.Workload(f"coarse_{n}", lv, ijk, sid, [sim], None, flux="hlle", powell=True, cfl=0.8)
        runs[name] = dict(n=n, k=k, learned=learned, grid=bd.Grid.from_workload(wl).upload(),
                          U=restrict_by(Ur, nbr, k), steps=coarse_steps * (n_ref // 128) // k)
    Ub = torch.empty_like(Ur)
    gr.advance(Ur, Ub, dtr, 2 * coarse_steps * (n_ref // 128), flux="hlle", powell=True, recompute_dt=False)
    del Ub
    out = {}
    for name, r in runs.items():
        g, U = r["grid"], r["U"]
        Ub = torch.empty_like(U)
        fb = torch.zeros(1, dtype=torch.int32, device="cuda")
        L = g.learned(mlp, stats, fallback=fb, floor_rel=cfg.floor_rel) if r["learned"] else None
        dt = dtr * float(r["k"])
        g.advance(U.clone(), Ub, dt, 2, flux="hlle", powell=True, recompute_dt=False, learned=L)  # warm-up
        fb.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.advance(U, Ub, dt, 2 * r["steps"], flux="hlle", powell=True, recompute_dt=False, learned=L)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ref = restrict_by(Ur, nbr, r["k"])
        l1 = [float((U[v] - ref[v]).abs().sum() / ref[v].abs().sum()) for v in range(8)]
        out[name] = {"cells": r["n"] ** 3, "steps": r["steps"], "wall_s": wall, "l1_rel_mean": float(np.mean(l1))}
        if r["learned"]:
            out[name]["flagged_share"] = int(fb.item()) / (2.0 * r["steps"] * r["n"] ** 3)
        del Ub
    out["reference"] = f"{n_ref}^3 FP64 run restricted, same time"
    return out


def with_strength(stats, k):
    """Output statistics scaled so that the stage applies k times the network's correction."""
    out = stats.clone()
    out[64:80] *= k
    return out


def save(path, mlp, stats, cfg: Config, summary=None):
    """A trained network as a plain .npz (no pickled objects): FP32 parameters, the 80 normalisation
    values as the stage uses them (strength folded in), the hidden width and the training summary."""
    np.savez(path, params=mlp.p.detach().cpu().numpy().astype(np.float32),
             stats=stats.detach().cpu().numpy().astype(np.float32), hidden=np.int32(cfg.hidden),
             strength=np.float64(cfg.strength), summary=np.str_(json.dumps(summary or {})))


def load(path, device="cuda"):
    """(Mlp, stats tensor, metadata) of a network written by save()."""
    import torch
    from . import binding as bd
    d = np.load(path, allow_pickle=False)
    mlp = bd.Mlp(int(d["hidden"]), torch.from_numpy(d["params"]), device=device)
    meta = {"hidden": int(d["hidden"]), "strength": float(d["strength"]), "summary": json.loads(str(d["summary"]))}
    return mlp, torch.from_numpy(d["stats"]), meta


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-fine", type=int, default=256)
    ap.add_argument("--train-states", type=int, default=32)
    ap.add_argument("--heldout-states", type=int, default=2)
    ap.add_argument("--fine-steps", type=int, default=200, help="fine steps per training state")
    ap.add_argument("--eval-fine-steps", type=int, default=400, help="evaluation horizon in fine steps")
    ap.add_argument("--epochs", type=int, default=24)
    ap.add_argument("--strength", type=float, default=0.25,
                    help="fraction of the network's correction applied (folded into the output statistics)")
    ap.add_argument("--samples", type=int, default=16384)
    ap.add_argument("--top-frac", type=float, default=0.0)
    ap.add_argument("--pair", type=float, default=0.0,
                    help="train on face pairs with this weight on the error of the pair's difference")
    ap.add_argument("--out", default=None)
    ap.add_argument("--init", default=None, help="start from the parameters of a saved network")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=5, help="seed of the training states, sampling and initial weights")
    a = ap.parse_args()
    import torch
    from . import binding as bd
    cfg = Config(n_fine=a.n_fine, train_states=a.train_states, heldout_states=a.heldout_states,
                 fine_steps=a.fine_steps, eval_fine_steps=a.eval_fine_steps, epochs=a.epochs, samples_per_dir=a.samples, top_frac=a.top_frac,
                 pair=a.pair, strength=a.strength, lr=a.lr, seed_train=a.seed)
    log = lambda *m: print(*m, file=sys.stderr, flush=True)
    t0 = time.time()
    X, T = generate(bd, cfg, solar_wind_states(cfg.train_states, cfg.seed_train), log)
    log(f"{X.shape[0]} samples in {time.time() - t0:.1f} s")
    t1 = time.time()
    mlp, stats, hist = train(bd, cfg, X, T, log, init=a.init)
    log(f"training {time.time() - t1:.1f} s")
    stats = with_strength(stats, cfg.strength)
    ev = evaluate(bd, cfg, mlp, stats, solar_wind_states(cfg.heldout_states, cfg.seed_heldout), log)
    summary = {"samples": int(X.shape[0]), "loss": hist, "heldout": ev,
               "gain_mean": float(np.mean([e["gain"] for e in ev])),
               "one_step_gain_mean": float(np.mean([e["one_step"]["gain"] for e in ev])),
               "one_step_exact_target_gain_mean": float(np.mean([e["one_step_exact_target"]["gain"] for e in ev])),
               "config": dataclasses.asdict(cfg)}
    if a.out:
        save(a.out, mlp, stats, cfg, summary)
    print(json.dumps(summary))


if __name__ == "__main__":
    main()
