"""Seeded synthetic inputs: block lists, per-simulation domain descriptions and initial primitive states.

This module is the only code that both the HIP path and the CPU oracle consume. It holds none of the
solver's arithmetic: no conversion to conserved variables, no fluxes, no ghost filling, no time step. It
only lays out blocks and evaluates analytic initial conditions at cell centres.

Conventions shared by every consumer (stated here because they define the inputs):

* Blocks hold 8x8x8 cells; a block is (level, block index ijk at its level, simulation id). Level 0 has
  cell size ``dx0``; level 1 has ``dx0 / 2``. Cell (i, j, k) of a block has its centre at
  ``origin + (8 * ijk + (i, j, k) + 0.5) * dx_level``.
* State arrays are variable-major: ``W[8][n_blocks][8][8][8]`` (k, j, i with i fastest), float64.
  Primitive order is (rho, ux, uy, uz, Bx, By, Bz, p), the order of the paper's state vector in the
  fast-wave setup (Sec. 5.1, Eq. 6).
* Boundary codes per face (xlo, xhi, ylo, yhi, zlo, zhi): 0 periodic, 1 outflow (zero gradient),
  2 inflow (fixed primitive state ``inflow_W``).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BC_PERIODIC, BC_OUTFLOW, BC_INFLOW = 0, 1, 2
NX = 8                      # cells per block per axis
GAMMA = 5.0 / 3.0           # only used by the Mach-number rule that sets input pressures


@dataclasses.dataclass
class Sim:
    nroot: tuple            # root blocks per axis (level-0 blocks)
    origin: tuple           # lower domain corner
    dx0: float              # level-0 cell size
    bc: tuple = (0, 0, 0, 0, 0, 0)
    inflow_W: tuple = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0)
    body_c: tuple = (0.0, 0.0, 0.0)
    body_r: float = 0.0     # <= 0: no body


@dataclasses.dataclass
class Workload:
    name: str
    level: np.ndarray       # int32 [nB]
    ijk: np.ndarray         # int32 [nB, 3]
    sim: np.ndarray         # int32 [nB]
    sims: List[Sim]
    W: np.ndarray           # float64 [8, nB, 8, 8, 8]
    flux: str = "rusanov"   # "rusanov" | "hlle"
    powell: bool = False
    cfl: float = 0.8
    n_steps: int = 10

    @property
    def n_blocks(self) -> int:
        return int(self.level.shape[0])

    @property
    def n_cells(self) -> int:
        return self.n_blocks * NX ** 3


# --------------------------------------------------------------------------------------------------
# block lists

def uniform_blocks(nroot, sim_id=0):
    """All level-0 blocks of an nroot box, listed with i fastest."""
    nx, ny, nz = nroot
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.int32)
    n = ijk.shape[0]
    return np.zeros(n, np.int32), ijk, np.full(n, sim_id, np.int32)


def two_level_blocks(nroot, refine_mask, sim_id=0):
    """Unrefined roots (i fastest), then the 8 children of every refined root (roots in i-fastest
    order; children with the x offset fastest, then y, then z)."""
    nx, ny, nz = nroot
    lv, ijk = [], []
    roots = [(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]
    for (i, j, k) in roots:
        if not refine_mask[k, j, i]:
            lv.append(0); ijk.append((i, j, k))
    for (i, j, k) in roots:
        if refine_mask[k, j, i]:
            for c in range(8):
                cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
                lv.append(1); ijk.append((2 * i + cx, 2 * j + cy, 2 * k + cz))
    n = len(lv)
    return np.array(lv, np.int32), np.array(ijk, np.int32).reshape(n, 3), np.full(n, sim_id, np.int32)


def cell_centres(sim: Sim, level, ijk):
    """Cell-centre coordinates, each [nB, 8, 8, 8] (k, j, i order)."""
    dx = sim.dx0 / (2.0 ** np.asarray(level, np.float64))
    idx = np.arange(NX, dtype=np.float64) + 0.5
    out = []
    for a in range(3):
        g = ijk[:, a].astype(np.float64) * NX
        shape = [1, 1, 1]
        shape[2 - a] = NX
        c = sim.origin[a] + (g[:, None, None, None] + idx.reshape(shape)[None]) * dx[:, None, None, None]
        out.append(np.broadcast_to(c, (len(level), NX, NX, NX)))
    return out


def _empty_W(nb):
    return np.zeros((8, nb, NX, NX, NX), np.float64)


# --------------------------------------------------------------------------------------------------
# analytic initial states

def uniform_state(nroot=(2, 2, 2), W0=(1.0, 0.1, -0.2, 0.3, 0.5, -0.4, 0.3, 0.7), bc=(0,) * 6,
                  body_r=0.0, levels=None, flux="rusanov", powell=False):
    """A constant primitive state. With ``levels`` (a refine mask) the grid has two levels."""
    sim = Sim(tuple(nroot), (0.0, 0.0, 0.0), 1.0, tuple(bc), tuple(W0),
              tuple(0.5 * n * NX for n in nroot), body_r)
    if levels is None:
        lv, ijk, sid = uniform_blocks(nroot)
    else:
        lv, ijk, sid = two_level_blocks(nroot, levels)
    W = _empty_W(len(lv))
    for v in range(8):
        W[v] = W0[v]
    return Workload("uniform", lv, ijk, sid, [sim], W, flux=flux, powell=powell)


def cp_alfven(n=32, amp=0.1, p=0.1, flux="rusanov", n_steps=10, cfl=0.8):
    """Circularly polarised Alfven wave along the (1,1,0) diagonal of the periodic unit cube: rho = 1,
    p = 0.1, |B0| = 1 along n = (1,1,0)/sqrt2, perturbation amp * (sin(phi) e1 + cos(phi) e2) in B and
    -amp * (same) in u, phi = 2 pi (x + y), e1 = (-1,1,0)/sqrt2, e2 = z. The exact solution translates
    phi by -2 pi sqrt2 t; the period is 1/sqrt2."""
    assert n % NX == 0
    nb = n // NX
    sim = Sim((nb, nb, nb), (0.0, 0.0, 0.0), 1.0 / n)
    lv, ijk, sid = uniform_blocks(sim.nroot)
    W = cp_alfven_field(sim, lv, ijk, 0.0, amp, p)
    return Workload(f"cp_alfven_{n}", lv, ijk, sid, [sim], W, flux=flux, powell=False, cfl=cfl,
                    n_steps=n_steps)


def cp_alfven_field(sim, lv, ijk, t, amp=0.1, p=0.1):
    x, y, _ = cell_centres(sim, lv, ijk)
    phi = 2.0 * math.pi * (x + y) - 2.0 * math.pi * math.sqrt(2.0) * t
    s2 = 1.0 / math.sqrt(2.0)
    n = (s2, s2, 0.0)
    e1 = (-s2, s2, 0.0)
    e2 = (0.0, 0.0, 1.0)
    W = _empty_W(len(lv))
    W[0] = 1.0
    W[7] = p
    for a in range(3):
        pert = amp * (np.sin(phi) * e1[a] + np.cos(phi) * e2[a])
        W[1 + a] = -pert
        W[4 + a] = n[a] + pert
    return W


def dipole_B(x, y, z, M):
    """Field of a point dipole of moment m = (0, 0, -M) at the origin: B = (3 (m.rhat) rhat - m) / r^3."""
    r2 = x * x + y * y + z * z
    r = np.sqrt(r2)
    r5 = r2 * r2 * r
    mz = -M
    mdotr = mz * z
    Bx = 3.0 * mdotr * x / r5
    By = 3.0 * mdotr * y / r5
    Bz = (3.0 * mdotr * z - mz * r2) / r5
    return Bx, By, Bz


def magnetosphere_sim(n=256, rho=5.0, ux=-400.0, bz=-5.0, body_cells=2.5, mach=8.0, dx0=None):
    """Domain [-n/2, n/2]^3 in units of the level-0 cell at 256^3 (dx = 256/n), body at the origin,
    solar wind entering through x-max (the upstream face for ux < 0), outflow on the other faces.
    Pressure from the sonic Mach number: p = rho |u|^2 / (mach^2 gamma)."""
    assert n % NX == 0
    half = 128.0
    dx = (2.0 * half / n) if dx0 is None else dx0
    nb = n // NX
    p = rho * ux * ux / (mach * mach * GAMMA)
    W_sw = (rho, ux, 0.0, 0.0, 0.0, 0.0, bz, p)
    bc = (BC_OUTFLOW, BC_INFLOW, BC_OUTFLOW, BC_OUTFLOW, BC_OUTFLOW, BC_OUTFLOW)
    return Sim((nb, nb, nb), (-half, -half, -half), dx, bc, W_sw, (0.0, 0.0, 0.0), body_cells)


def magnetosphere_state(sim: Sim, lv, ijk, M=7.9e4):
    """Solar wind everywhere plus the dipole field at cell centres; inside the body sphere u = 0."""
    x, y, z = cell_centres(sim, lv, ijk)
    Bx, By, Bz = dipole_B(x, y, z, M)
    W = _empty_W(len(lv))
    for v in range(8):
        W[v] = sim.inflow_W[v]
    W[4] += Bx
    W[5] += By
    W[6] += Bz
    r2 = (x - sim.body_c[0]) ** 2 + (y - sim.body_c[1]) ** 2 + (z - sim.body_c[2]) ** 2
    inside = r2 < sim.body_r ** 2
    for v in (1, 2, 3):
        W[v][inside] = 0.0
    return W


def magnetosphere(n=256, n_steps=100, M=7.9e4, **kw):
    """Magnetosphere-shaped uniform grid: dipole (moment along -z) plus solar-wind inflow, reflecting
    body of radius 2.5 level-0 cells of the 256^3 grid, HLLE flux with the Powell source."""
    sim = magnetosphere_sim(n, **kw)
    lv, ijk, sid = uniform_blocks(sim.nroot)
    W = magnetosphere_state(sim, lv, ijk, M)
    return Workload(f"magnetosphere_{n}", lv, ijk, sid, [sim], W, flux="hlle", powell=True,
                    cfl=0.8, n_steps=n_steps)


def magnetosphere_cut(n=64, n_steps=10, M=7.9e4):
    """The magnetosphere physics on a smaller box of the same cell size: [-n/2, n/2]^3, dx = 1."""
    sim = magnetosphere_sim(n, dx0=1.0)
    half = n / 2.0
    sim = dataclasses.replace(sim, origin=(-half, -half, -half))
    lv, ijk, sid = uniform_blocks(sim.nroot)
    W = magnetosphere_state(sim, lv, ijk, M)
    return Workload(f"magnetosphere_cut_{n}", lv, ijk, sid, [sim], W, flux="hlle", powell=True,
                    cfl=0.8, n_steps=n_steps)


def refine_shell_mask(sim: Sim, r_in, r_out):
    """Root blocks with any cell centre at r_in <= |x - body_c| <= r_out."""
    nx, ny, nz = sim.nroot
    mask = np.zeros((nz, ny, nx), bool)
    idx = np.arange(NX) + 0.5
    for k in range(nz):
        zc = sim.origin[2] + (k * NX + idx) * sim.dx0 - sim.body_c[2]
        for j in range(ny):
            yc = sim.origin[1] + (j * NX + idx) * sim.dx0 - sim.body_c[1]
            for i in range(nx):
                xc = sim.origin[0] + (i * NX + idx) * sim.dx0 - sim.body_c[0]
                r = np.sqrt(zc[:, None, None] ** 2 + yc[None, :, None] ** 2 + xc[None, None, :] ** 2)
                mask[k, j, i] = bool(np.any((r >= r_in) & (r <= r_out)))
    return mask


def two_level_magnetosphere(nbase=144, n_steps=200, M=7.9e4, r_body=2.5):
    """Two-level grid: level-0 base of nbase^3 cells (dx0 = 1, domain [-nbase/2, nbase/2]^3), a root
    block refined once when any of its cell centres lies 3..10 body radii from the dipole. Same physics
    as the uniform magnetosphere."""
    half = nbase / 2.0
    sim = magnetosphere_sim(nbase, dx0=1.0)
    sim = dataclasses.replace(sim, origin=(-half, -half, -half), body_r=r_body)
    mask = refine_shell_mask(sim, 3.0 * r_body, 10.0 * r_body)
    lv, ijk, sid = two_level_blocks(sim.nroot, mask)
    W = magnetosphere_state(sim, lv, ijk, M)
    return Workload(f"two_level_{nbase}", lv, ijk, sid, [sim], W, flux="hlle", powell=True, cfl=0.8,
                    n_steps=n_steps)


def fast_wave(nroot=(2, 2, 2), refine_octant=False, nx_domain=64.0):
    """The paper's fast magnetosonic wave (Sec. 5.1, Eq. 6): background rho=1, u=(0,0,0.005),
    B=(0,0.04,0), p=0.00054; amplitude (0.1, 0.005, 0, 0, 0, 0.004, 0, 0.00009); k = (pi/16, 0, 0) on
    the periodic domain [-32, 32]^3. Block size here is 8^3 (the paper's is 10^3)."""
    V0 = np.array([1.0, 0.0, 0.0, 0.005, 0.0, 0.04, 0.0, 0.00054])
    V1 = np.array([0.1, 0.005, 0.0, 0.0, 0.0, 0.004, 0.0, 0.00009])
    dx0 = nx_domain / (nroot[0] * NX)
    sim = Sim(tuple(nroot), (-32.0, -32.0, -32.0), dx0)
    if refine_octant:
        mask = np.zeros(nroot[::-1], bool)
        mask[: nroot[2] // 2, : nroot[1] // 2, : nroot[0] // 2] = True
        lv, ijk, sid = two_level_blocks(sim.nroot, mask)
    else:
        lv, ijk, sid = uniform_blocks(sim.nroot)
    x, _, _ = cell_centres(sim, lv, ijk)
    W = _empty_W(len(lv))
    c = np.cos(math.pi / 16.0 * x)
    for v in range(8):
        W[v] = V0[v] + V1[v] * c
    return Workload("fast_wave", lv, ijk, sid, [sim], W, flux="hlle", powell=True, cfl=0.8, n_steps=500)


# --------------------------------------------------------------------------------------------------
# test fields

def unique_id_field(wl: Workload):
    """Integer-valued field U[v, b, c] = 16 * (global cell id) + v + 1 (exact in FP64). Used as a
    conserved field for ghost-fill tests: copy, pairwise-mean restriction and minmod prolongation are
    exact on it."""
    nb = wl.n_blocks
    gid = np.arange(nb * NX ** 3, dtype=np.float64).reshape(nb, NX, NX, NX)
    U = np.empty((8, nb, NX, NX, NX))
    for v in range(8):
        U[v] = 16.0 * gid + v + 1
    return U


def random_positive_state(wl: Workload, seed=0, amp=0.2):
    """A smooth-ish random primitive state with rho, p > 0 (for parity tests on random data)."""
    rng = np.random.default_rng(seed)
    nb = wl.n_blocks
    W = np.empty((8, nb, NX, NX, NX))
    W[0] = 1.0 + amp * rng.uniform(-1, 1, (nb, NX, NX, NX))
    for v in (1, 2, 3):
        W[v] = 0.5 * amp * rng.uniform(-1, 1, (nb, NX, NX, NX))
    for v in (4, 5, 6):
        W[v] = 0.5 + amp * rng.uniform(-1, 1, (nb, NX, NX, NX))
    W[7] = 1.0 + amp * rng.uniform(-1, 1, (nb, NX, NX, NX))
    return W


def with_state(wl: Workload, W, name=None) -> Workload:
    return dataclasses.replace(wl, W=W, name=name or wl.name)


def odd_box(nroot=(3, 2, 5), bc=(1, 1, 0, 0, 2, 1), seed=3):
    """A ragged box of blocks with mixed boundary types and a random positive state."""
    sim = Sim(tuple(nroot), (0.0, 0.0, 0.0), 1.0, tuple(bc), (1.1, -0.2, 0.1, 0.05, 0.3, 0.6, -0.2, 0.9))
    lv, ijk, sid = uniform_blocks(nroot)
    wl = Workload("odd_box", lv, ijk, sid, [sim], _empty_W(len(lv)), flux="hlle", powell=True)
    return with_state(wl, random_positive_state(wl, seed))


def two_level_box(nroot=(4, 3, 2), refine=((1, 1, 0), (2, 1, 0), (1, 0, 1)), bc=(0,) * 6, seed=5,
                  body=False):
    """A small two-level grid with a few refined roots and a random positive state. With ``body`` a small
    body sits on the coarse side of a level face: centred on the level-0 cell two cells below the x-lo face
    of the first refined root whose x-lo neighbour is a level-0 block, radius 1.2 cells, so the coarse cell
    next to that face is a body cell while every fine cell stays fluid."""
    mask = np.zeros(nroot[::-1], bool)
    for (i, j, k) in refine:
        mask[k, j, i] = True
    body_c, body_r = (0.0, 0.0, 0.0), 0.0
    if body:
        for (i, j, k) in refine:
            if i > 0 and not mask[k, j, i - 1]:
                body_c, body_r = (8.0 * i - 1.5, 8.0 * j + 3.5, 8.0 * k + 3.5), 1.2
                break
        else:
            raise ValueError("two_level_box(body=True) needs a refined root with a level-0 x-lo neighbour")
    sim = Sim(tuple(nroot), (0.0, 0.0, 0.0), 1.0, tuple(bc), (1.1, -0.2, 0.1, 0.05, 0.3, 0.6, -0.2, 0.9),
              body_c, body_r)
    lv, ijk, sid = two_level_blocks(nroot, mask)
    wl = Workload("two_level_box", lv, ijk, sid, [sim], _empty_W(len(lv)), flux="hlle", powell=True)
    return with_state(wl, random_positive_state(wl, seed))


def uniform_bound_state(wl: Workload, seed=0, rho=1.0, p=0.6, u0=0.3, b0=0.8):
    """A state whose CFL bound is the same in every cell although the state is not uniform: density and
    pressure uniform, velocity (0, +-u0, 0) and field (0, 0, +-b0) with independent random signs per cell.
    Every cell then has the same |u_d| and the same fast speed along each axis."""
    rng = np.random.default_rng(seed)
    W = _empty_W(wl.n_blocks)
    W[0] = rho
    W[7] = p
    W[2] = u0 * rng.choice([-1.0, 1.0], size=W[2].shape)
    W[6] = b0 * rng.choice([-1.0, 1.0], size=W[6].shape)
    return W


# --------------------------------------------------------------------------------------------------
# batched simulations of superposed linear MHD waves

def _primitive_jacobian(rho, p, B, n):
    """Matrix A of the linearised primitive ideal-MHD system W_t + A W_s = 0 along unit vector n, about
    rest (u = 0) with density rho, pressure p and field B. Used only to shape initial perturbations."""
    A = np.zeros((8, 8))
    bn = float(np.dot(B, n))
    for d in range(3):
        A[0, 1 + d] = rho * n[d]
        A[7, 1 + d] = GAMMA * p * n[d]
        A[1 + d, 7] = n[d] / rho
        for m in range(3):
            A[1 + d, 4 + m] = (n[d] * B[m] - (bn if d == m else 0.0)) / rho
            A[4 + d, 1 + m] = B[d] * n[m] - (bn if d == m else 0.0)
    return A


WAVE_FAMILIES = ("fast-", "alfven-", "slow-", "entropy", "slow+", "alfven+", "fast+")


def wave_eigenvector(rho, p, B, n, family):
    """Right eigenvector of the linearised system for one wave family, normalised to max-norm 1."""
    A = _primitive_jacobian(rho, p, np.asarray(B, float), np.asarray(n, float))
    lam, R = np.linalg.eig(A)
    lam, R = lam.real, R.real
    if family == "entropy":
        r = np.zeros(8); r[0] = 1.0
        return r
    order = np.argsort(lam)           # -cf, -ca, -cs, 0, 0, cs, ca, cf
    pick = {"fast-": 0, "alfven-": 1, "slow-": 2, "slow+": 5, "alfven+": 6, "fast+": 7}[family]
    r = R[:, order[pick]]
    return r / np.abs(r).max()


def batched_waves(n_sims=64, seed=4, n_waves=8, amp_max=0.05, n_lo=64, n_hi=4096, n_steps=100):
    """Many independent periodic simulations on one grid. Block counts are drawn log-uniformly in
    [n_lo, n_hi] and factorised into a box (bz = floor(N^(1/3)), by = floor(sqrt(N / bz)),
    bx = floor(N / (bz by))); cell size 1. Background rho = 1, p = 1, u = 0, |B| = 1 along a random
    direction; each simulation superposes n_waves linear waves (family uniform, integer wave-number
    vector in [-2, 2]^3 without 0, amplitude uniform in [0, amp_max], phase uniform)."""
    rng = np.random.default_rng(seed)
    counts = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), n_sims))).astype(int)
    sims, lv, ijk, sid = [], [], [], []
    for s, N in enumerate(counts):
        bz = int(math.floor(N ** (1.0 / 3.0) + 1e-9))
        by = int(math.floor(math.sqrt(N / bz) + 1e-9))
        bx = int(N // (bz * by))
        sims.append(Sim((bx, by, bz), (0.0, 0.0, 0.0), 1.0))
        l, c, _ = uniform_blocks((bx, by, bz))
        lv.append(l); ijk.append(c); sid.append(np.full(len(l), s, np.int32))
    level = np.concatenate(lv); ijk = np.concatenate(ijk); sim = np.concatenate(sid)
    W = _empty_W(len(level))
    W[0] = 1.0
    W[7] = 1.0
    for s, sd in enumerate(sims):
        sel = sim == s
        v = rng.normal(size=3); Bhat = v / np.linalg.norm(v)
        x, y, z = cell_centres(sd, level[sel], ijk[sel])
        L = np.array(sd.nroot) * NX * sd.dx0
        Ws = np.zeros((8,) + x.shape)
        Ws[0] = 1.0; Ws[7] = 1.0
        for m in range(3):
            Ws[4 + m] = Bhat[m]
        for _ in range(n_waves):
            fam = WAVE_FAMILIES[rng.integers(len(WAVE_FAMILIES))]
            while True:
                nv = rng.integers(-2, 3, size=3)
                if np.any(nv != 0):
                    break
            a = rng.uniform(0.0, amp_max)
            ph = rng.uniform(0.0, 2 * math.pi)
            kvec = 2 * math.pi * nv / L
            khat = kvec / np.linalg.norm(kvec)
            r = wave_eigenvector(1.0, 1.0, Bhat, khat, fam)
            cph = np.cos(kvec[0] * x + kvec[1] * y + kvec[2] * z + ph)
            for q in range(8):
                Ws[q] += a * r[q] * cph
        W[:, sel] = Ws
    return Workload(f"batched_{n_sims}", level, ijk, sim, sims, W, flux="rusanov", powell=False, cfl=0.8,
                    n_steps=n_steps)


# --------------------------------------------------------------------------------------------------
# per-face inputs of the learned flux correction

def face_slots():
    """(d, f, t1, t2) of the 576 faces of each axis of a block, in the face order of the learned form:
    face f of axis d lies between cells f-1 and f along d, slot (t2*8 + t1)*9 + f for d = 0 (t1 = y,
    t2 = z), (t2*9 + f)*8 + t1 for d = 1 (t1 = x, t2 = z), (f*8 + t2)*8 + t1 for d = 2 (t1 = x, t2 = y).
    Returns int arrays f, t1, t2 of shape [3, 576] indexed by (d, slot)."""
    f = np.empty((3, 576), np.int64)
    t1 = np.empty((3, 576), np.int64)
    t2 = np.empty((3, 576), np.int64)
    for d in range(3):
        a, b_, c = np.meshgrid(np.arange(9), np.arange(8), np.arange(8), indexing="ij")  # f, t1, t2
        a, b_, c = a.ravel(), b_.ravel(), c.ravel()
        slot = (c * 8 + b_) * 9 + a if d == 0 else ((c * 9 + a) * 8 + b_ if d == 1 else (a * 8 + c) * 8 + b_)
        f[d, slot], t1[d, slot], t2[d, slot] = a, b_, c
    return f, t1, t2


def face_corrections(wl: Workload, seed=0, scale=1.0):
    """Seeded normalised flux corrections y [n_blocks * 1728, 8] for a single-level grid, drawn per global
    face (standard normal times ``scale``), so that the two blocks that own a face hold the same value
    (across periodic boundaries too). Pure indexing: no arithmetic of the method."""
    assert np.all(wl.level == 0) and wl.sims and len(wl.sims) == 1
    sim = wl.sims[0]
    n = [int(v) * NX for v in sim.nroot]
    rng = np.random.default_rng(seed)
    tables = [rng.standard_normal((n[2] + (d == 2), n[1] + (d == 1), n[0] + (d == 0), 8)) * scale
              for d in range(3)]
    f, t1, t2 = face_slots()
    y = np.empty((wl.n_blocks, 3, 576, 8))
    for d in range(3):
        a1, a2 = (1, 2) if d == 0 else ((0, 2) if d == 1 else (0, 1))
        periodic = sim.bc[2 * d] == BC_PERIODIC and sim.bc[2 * d + 1] == BC_PERIODIC
        g = np.empty((wl.n_blocks, 3, 576), np.int64)
        g[:, d] = wl.ijk[:, d, None] * NX + f[d][None]
        g[:, a1] = wl.ijk[:, a1, None] * NX + t1[d][None]
        g[:, a2] = wl.ijk[:, a2, None] * NX + t2[d][None]
        if periodic:
            g[:, d] %= n[d]
        y[:, d] = tables[d][g[:, 2], g[:, 1], g[:, 0]]
    return np.ascontiguousarray(y.reshape(wl.n_blocks * 1728, 8))
