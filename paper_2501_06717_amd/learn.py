"""Learned flux correction for coarse magnetosphere grids: data, training and evaluation.

The network corrects the plain HLLE flux of a coarse grid (128^3 cells, dx = 2) toward the flux a grid
twice as fine would put through the same face. Training data come from plain FP64 runs on the fine
grid (256^3, dx = 1) of solar-wind states drawn at random:

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

Training and inference run in the library's kernels (BF16 matrix cores, FP32 master weights, Adam).
Data preparation (restriction, face averaging, sampling, statistics) uses torch tensor operations on
the GPU.
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
    """Fine (n_fine^3, dx = 1) and coarse (n_fine/2)^3 (dx = 2) workloads of one solar-wind state."""
    fine = wk.magnetosphere(n_fine, M=M, **state)
    sim_c = wk.magnetosphere_sim(n_fine // 2, **state)
    lv, ijk, sid = wk.uniform_blocks(sim_c.nroot)
    coarse = wk.Workload(f"coarse_{n_fine // 2}", lv, ijk, sid, [sim_c], wk.magnetosphere_state(sim_c, lv, ijk, M),
                         flux="hlle", powell=True, cfl=0.8)
    return fine, coarse


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


def restrict(Uf, nbf):
    """Mean of the 8 fine cells of each coarse cell (conserved variables)."""
    return restrict_by(Uf, nbf, 2)


def restrict_by(Uf, nbf, k):
    """Mean of the k^3 fine cells of each coarse cell (conserved variables); nbf^3 fine blocks of 8^3."""
    G = to_global(Uf, nbf)
    n = G.shape[1] // k
    Gc = G.reshape(8, n, k, n, k, n, k).mean(dim=(2, 4, 6))
    return from_global(Gc, nbf // k)


def faces_global(F, nb, d, c):
    """Per-block face data [nb^3 * 3 * 576, c] -> global faces of direction d: [c, Nz', Ny', Nx'] with
    N + 1 positions along d."""
    import torch
    N = nb * 8
    t = F.reshape(nb, nb, nb, 3, 576, c)[:, :, :, d]        # (bz, by, bx, f, c)
    if d == 0:
        t = t.reshape(nb, nb, nb, 8, 8, 9, c)               # (bz, by, bx, z, y, x)
        body = t[..., :8, :].permute(6, 0, 3, 1, 4, 2, 5).reshape(c, N, N, N)
        last = t[:, :, -1, :, :, 8, :].permute(4, 0, 2, 1, 3).reshape(c, N, N, 1)
        return torch.cat([body, last], dim=3)
    if d == 1:
        t = t.reshape(nb, nb, nb, 8, 9, 8, c)
        body = t[:, :, :, :, :8].permute(6, 0, 3, 1, 4, 2, 5).reshape(c, N, N, N)
        last = t[:, -1, :, :, 8, :, :].permute(4, 0, 2, 1, 3).reshape(c, N, 1, N)
        return torch.cat([body, last], dim=2)
    t = t.reshape(nb, nb, nb, 9, 8, 8, c)
    body = t[:, :, :, :8].permute(6, 0, 3, 1, 4, 2, 5).reshape(c, N, N, N)
    last = t[-1, :, :, 8].permute(4, 0, 2, 1, 3).reshape(c, 1, N, N)
    return torch.cat([body, last], dim=1)


def coarse_face_mean(Ff, d):
    """Mean of the 4 fine faces covering each coarse face: fine global faces [c, ...] of direction d."""
    c = Ff.shape[0]
    if d == 0:
        t = Ff[:, :, :, ::2]
        nz, ny, nx = t.shape[1] // 2, t.shape[2] // 2, t.shape[3]
        return t.reshape(c, nz, 2, ny, 2, nx).mean(dim=(2, 4))
    if d == 1:
        t = Ff[:, :, ::2, :]
        nz, ny, nx = t.shape[1] // 2, t.shape[2], t.shape[3] // 2
        return t.reshape(c, nz, 2, ny, nx, 2).mean(dim=(2, 5))
    t = Ff[:, ::2, :, :]
    nz, ny, nx = t.shape[1], t.shape[2] // 2, t.shape[3] // 2
    return t.reshape(c, nz, ny, 2, nx, 2).mean(dim=(3, 5))


# --------------------------------------------------------------------------------------------------
# data generation

@dataclasses.dataclass
class Config:
    n_fine: int = 256
    train_states: int = 32
    heldout_states: int = 2
    fine_steps: int = 200
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


def snapshot_data(bd, gf, gc, Uf, nbf, gen):
    """(X, T) samples of one fine snapshot: coarse stencil features and flux corrections."""
    import torch
    Uc = restrict(Uf, nbf)
    Xc, Fc = gc.face_data(Uc, flux="hlle")
    _, Ff = gf.face_data(Uf, flux="hlle", want_x=False)
    nbc = nbf // 2
    xs, ts = [], []
    for d in range(3):
        Fg = faces_global(Ff, nbf, d, 8)
        target = coarse_face_mean(Fg, d) - faces_global(Fc, nbc, d, 8)
        Xg = faces_global(Xc, nbc, d, 32)
        T = target.reshape(8, -1).t()
        X = Xg.reshape(32, -1).t()
        n = T.shape[0]
        kt = int(round(gen["samples"] * gen["top_frac"]))
        ku = gen["samples"] - kt
        mag = (T / (T.std(dim=0) + 1e-30)).norm(dim=1)
        top = torch.topk(mag, max(n // 10, kt)).indices
        pick_top = top[torch.randint(0, top.numel(), (kt,), generator=gen["g"], device=top.device)]
        pick_uni = torch.randint(0, n, (ku,), generator=gen["g"], device=top.device)
        idx = torch.cat([pick_uni, pick_top])
        xs.append(X[idx])
        ts.append(T[idx])
        del Fg, target, Xg
    return torch.cat(xs), torch.cat(ts)


def snapshot_pairs(bd, gf, gc, Uf, nbf, gen):
    """Samples of one fine snapshot as face pairs: the low and high face of a coarse cell along each
    direction, X [n, 2, 32] (coarse stencil features) and T [n, 2, 8] (flux corrections). Half of them are
    uniform, `top_frac` from the top decile of the difference of the two corrections."""
    import torch
    Uc = restrict(Uf, nbf)
    Xc, Fc = gc.face_data(Uc, flux="hlle")
    _, Ff = gf.face_data(Uf, flux="hlle", want_x=False)
    nbc = nbf // 2
    xs, ts = [], []
    for d in range(3):
        Fg = faces_global(Ff, nbf, d, 8)
        target = coarse_face_mean(Fg, d) - faces_global(Fc, nbc, d, 8)
        Xg = faces_global(Xc, nbc, d, 32)
        ax = 3 - d                                   # global face arrays are [c, z, y, x]
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        Ta, Tb = target[tuple(lo)].reshape(8, -1).t(), target[tuple(hi)].reshape(8, -1).t()
        Xa, Xb = Xg[tuple(lo)].reshape(32, -1).t(), Xg[tuple(hi)].reshape(32, -1).t()
        n = Ta.shape[0]
        kt = int(round(gen["samples"] * gen["top_frac"]))
        ku = gen["samples"] - kt
        dT = Tb - Ta
        mag = (dT / (dT.std(dim=0) + 1e-30)).norm(dim=1)
        top = torch.topk(mag, max(n // 10, kt)).indices
        pick_top = top[torch.randint(0, top.numel(), (kt,), generator=gen["g"], device=top.device)]
        pick_uni = torch.randint(0, n, (ku,), generator=gen["g"], device=top.device)
        idx = torch.cat([pick_uni, pick_top])
        xs.append(torch.stack([Xa[idx], Xb[idx]], dim=1))
        ts.append(torch.stack([Ta[idx], Tb[idx]], dim=1))
        del Fg, target, Xg
    return torch.cat(xs), torch.cat(ts)


def generate(bd, cfg: Config, states, log=print):
    """Training samples from fine plain FP64 runs of the given solar-wind states."""
    import torch
    gen = {"g": torch.Generator(device="cuda"), "samples": cfg.samples_per_dir, "top_frac": cfg.top_frac}
    gen["g"].manual_seed(cfg.seed_train)
    X, T = [], []
    nbf = cfg.n_fine // 8
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
            x, t = (snapshot_pairs if cfg.pair > 0 else snapshot_data)(bd, gf, gc, U0, nbf, gen)
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
    nbf = n_fine // 8
    fine, coarse = magnetosphere_pair(st, n_fine)
    gf = bd.Grid.from_workload(fine).upload()
    gc = bd.Grid.from_workload(coarse).upload()
    Uf = gf.set_state(torch.from_numpy(fine.W).cuda())
    U1 = torch.empty_like(Uf)
    dtf = torch.zeros(1, dtype=torch.float64, device="cuda")
    gf.advance(Uf, U1, dtf, 2 * warm_steps, flux="hlle", powell=True, cfl=0.8)
    dtf = gf.reduce_dt(Uf, 0.8)
    return gf, gc, coarse, Uf, dtf, restrict(Uf, nbf)


def one_step_gain(bd, cfg: Config, mlp, stats, st, warm_steps=100):
    """Local (one coarse step) error: from the restricted fine state after `warm_steps` fine steps, one
    coarse step (dt = 2 fine dt) plain and learned against the fine run advanced two steps and restricted.
    L1 of the change of state, per variable, relative to the fine change; and the flagged share of the
    learned step's cell-stages."""
    import torch
    nbf = cfg.n_fine // 8
    gf, gc, coarse, Uf, dtf, Uc0 = developed_state(bd, st, cfg.n_fine, warm_steps)
    U1 = torch.empty_like(Uf)
    gf.advance(Uf, U1, dtf, 4, flux="hlle", powell=True, recompute_dt=False)
    dref = restrict(Uf, nbf) - Uc0
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


def faces_to_blocks(G, nb, d):
    """Inverse of faces_global: global faces of direction d [c, ...] -> per-block faces [nb^3, 576, c] in
    the face order of bmhd_face_data."""
    import torch
    ar = lambda n: torch.arange(n, device=G.device)
    bz, by, bx = torch.meshgrid(ar(nb), ar(nb), ar(nb), indexing="ij")
    dims = {0: (8, 8, 9), 1: (8, 9, 8), 2: (9, 8, 8)}[d]
    z, y, x = torch.meshgrid(ar(dims[0]), ar(dims[1]), ar(dims[2]), indexing="ij")
    Z = bz.reshape(-1, 1) * 8 + z.reshape(1, -1)
    Y = by.reshape(-1, 1) * 8 + y.reshape(1, -1)
    X = bx.reshape(-1, 1) * 8 + x.reshape(1, -1)
    return G[:, Z, Y, X].permute(1, 2, 0)


def exact_target_one_step(bd, cfg: Config, st, warm_steps=100):
    """The one_step_gain test with the exact a-priori target (from the fine state, not a network) given to
    the learned stage as its correction: the best a correction of this form can do from this state."""
    import torch
    nbf, nbc = cfg.n_fine // 8, cfg.n_fine // 16
    gf, gc, coarse, Uf, dtf, Uc0 = developed_state(bd, st, cfg.n_fine, warm_steps)
    U1 = torch.empty_like(Uf)
    _, Fc = gc.face_data(Uc0, flux="hlle", want_x=False)
    _, Ff = gf.face_data(Uf, flux="hlle", want_x=False)
    ys = []
    for d in range(3):
        T = coarse_face_mean(faces_global(Ff, nbf, d, 8), d) - faces_global(Fc, nbc, d, 8)
        ys.append(faces_to_blocks(T, nbc, d))
    y = torch.stack(ys, dim=1).reshape(-1, 8).float().contiguous()
    del Ff, Fc, ys
    gf.advance(Uf, U1, dtf, 4, flux="hlle", powell=True, recompute_dt=False)
    dref = restrict(Uf, nbf) - Uc0
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
    nbf = cfg.n_fine // 8
    for st in states:
        fine, coarse = magnetosphere_pair(st, cfg.n_fine)
        gf = bd.Grid.from_workload(fine).upload()
        gc = bd.Grid.from_workload(coarse).upload()
        Uf = gf.set_state(torch.from_numpy(fine.W).cuda())
        dtf = gf.reduce_dt(Uf, 0.8)
        Uc0 = restrict(Uf, nbf)
        U1 = torch.empty_like(Uf)
        gf.advance(Uf, U1, dtf, 2 * cfg.fine_steps, flux="hlle", powell=True, recompute_dt=False)
        ref = restrict(Uf, nbf)
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
            gc.advance(U, Ub, dt, cfg.fine_steps, flux="hlle", powell=True, recompute_dt=False, learned=learned,
                       faults=faults)
            torch.cuda.synchronize()
            l1 = [float((U[v] - ref[v]).abs().sum() / ref[v].abs().sum()) for v in range(8)]
            res[name] = {"l1_rel_mean": float(np.mean(l1)), "l1_rel": l1, "faults": int(faults.item())}
        res["learned"]["flagged_share"] = int(fb.item()) / (float(cfg.fine_steps) * coarse.n_cells)  # per stage
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
    ap.add_argument("--fine-steps", type=int, default=200)
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
    a = ap.parse_args()
    import torch
    from . import binding as bd
    cfg = Config(n_fine=a.n_fine, train_states=a.train_states, heldout_states=a.heldout_states,
                 fine_steps=a.fine_steps, epochs=a.epochs, samples_per_dir=a.samples, top_frac=a.top_frac,
                 pair=a.pair, strength=a.strength, lr=a.lr)
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
