"""ctypes wrapper around the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the package smoke check and the benchmark's
CPU-baseline leg, never by the product path. It takes numpy arrays and plain Python values; it does not
import the HIP package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["oracle.c", "mlp.c"]

FLUX = {"rusanov": 0, "hlle": 1, "linde": 2}


def build(verbose=False):
    """Compile the oracle with gcc: no FMA contraction, no fast-math, OpenMP over blocks."""
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall",
           "-shared", "-fPIC", *srcs, "-o", LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Sim(ctypes.Structure):
    _fields_ = [("nroot", ctypes.c_int32 * 3), ("origin", ctypes.c_double * 3), ("dx0", ctypes.c_double),
                ("bc", ctypes.c_int32 * 6), ("inflow_w", ctypes.c_double * 8),
                ("body_c", ctypes.c_double * 3), ("body_r", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("flux", ctypes.c_int32), ("powell", ctypes.c_int32), ("n_table", ctypes.c_int32),
                ("recompute_dt", ctypes.c_int32), ("alpha", ctypes.c_double * 2),
                ("beta", ctypes.c_double * 2), ("cfl", ctypes.c_double), ("local_dt", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER
        dp, ip = P(ctypes.c_double), P(ctypes.c_int32)
        L.or_grid_create.restype = ctypes.c_void_p
        L.or_grid_create.argtypes = [ctypes.c_int, ip, ip, ip, ctypes.c_int, P(_Sim)]
        L.or_grid_free.argtypes = [ctypes.c_void_p]
        L.or_neighbors.argtypes = [ctypes.c_void_p, ip]
        L.or_set_state.argtypes = [ctypes.c_void_p, dp, dp]
        L.or_fill_ghosts.argtypes = [ctypes.c_void_p, dp, dp]
        L.or_dt.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, dp]
        L.or_remap.argtypes = [ctypes.c_void_p, dp, ctypes.c_void_p, dp]
        L.or_remap.restype = ctypes.c_int
        L.or_advance.argtypes = [ctypes.c_void_p, dp, dp, dp, ctypes.c_int, P(_Opts), P(ctypes.c_long)]
        L.or_advance.restype = ctypes.c_int
        L.or_prim_to_cons.argtypes = [dp, dp]
        L.or_cons_to_prim.argtypes = [dp, dp]
        L.or_phys_flux.argtypes = [dp, ctypes.c_int, dp]
        L.or_fast_speed.argtypes = [dp, ctypes.c_int]
        L.or_fast_speed.restype = ctypes.c_double
        L.or_num_flux.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp]
        L.or_mc_slope.argtypes = [ctypes.c_double] * 3
        L.or_mc_slope.restype = ctypes.c_double
        L.or_restrict8.argtypes = [dp]
        L.or_restrict8.restype = ctypes.c_double
        L.or_prolong1.argtypes = [ctypes.c_double, dp, dp, ip]
        L.or_prolong1.restype = ctypes.c_double
        L.or_face_features.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.or_block_indicator.argtypes = [ctypes.c_void_p, dp, dp]
        L.or_adapt.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_double, ip, ip, ip, ctypes.c_long]
        L.or_adapt.restype = ctypes.c_long
        L.or_advance_learned.argtypes = [ctypes.c_void_p, dp, dp, dp, ctypes.c_int, P(_Opts), dp, dp,
                                         ctypes.c_double, ctypes.c_double, P(ctypes.c_long), P(ctypes.c_long)]
        L.or_advance_learned.restype = ctypes.c_int
        L.or_xchg_messages.argtypes = [ctypes.c_void_p, ip, ctypes.c_int, P(ctypes.c_int64), ctypes.c_long]
        L.or_xchg_messages.restype = ctypes.c_long
        L.or_xchg_run.argtypes = [ctypes.c_void_p, ip, ctypes.c_int, dp, dp]
        L.or_xchg_run.restype = ctypes.c_int
        L.mlp_n_params.argtypes = [ctypes.c_int]
        L.mlp_n_params.restype = ctypes.c_long
        L.mlp_forward.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, dp]
        L.mlp_loss_grad.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.mlp_loss_grad.restype = ctypes.c_double
        L.mlp_adam.argtypes = [dp, dp, dp, dp, ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


# ------------------------------------------------------------------------------------------------
# point functions (used by the pins)

def prim_to_cons(w):
    w = np.ascontiguousarray(w, np.float64); u = np.empty(8)
    lib().or_prim_to_cons(_dp(w), _dp(u)); return u


def cons_to_prim(u):
    u = np.ascontiguousarray(u, np.float64); w = np.empty(8)
    lib().or_cons_to_prim(_dp(u), _dp(w)); return w


def phys_flux(w, d):
    w = np.ascontiguousarray(w, np.float64); f = np.empty(8)
    lib().or_phys_flux(_dp(w), d, _dp(f)); return f


def fast_speed(w, d):
    w = np.ascontiguousarray(w, np.float64)
    return lib().or_fast_speed(_dp(w), d)


def num_flux(wl, wr, d, kind="rusanov"):
    wl = np.ascontiguousarray(wl, np.float64); wr = np.ascontiguousarray(wr, np.float64); f = np.empty(8)
    lib().or_num_flux(_dp(wl), _dp(wr), d, FLUX[kind], _dp(f)); return f


def mc_slope(wm, w0, wp):
    return lib().or_mc_slope(float(wm), float(w0), float(wp))


def restrict8(c):
    c = np.ascontiguousarray(c, np.float64)
    return lib().or_restrict8(_dp(c))


def prolong1(uc, cm, cp, s):
    cm = np.ascontiguousarray(cm, np.float64); cp = np.ascontiguousarray(cp, np.float64)
    s = np.ascontiguousarray(s, np.int32)
    return lib().or_prolong1(float(uc), _dp(cm), _dp(cp), _ip(s))


# ------------------------------------------------------------------------------------------------
# grid-level driver

class Grid:
    """An oracle grid built from a block list (level, ijk, sim) and per-simulation descriptions
    (objects with nroot, origin, dx0, bc, inflow_W, body_c, body_r attributes)."""

    def __init__(self, level, ijk, sim, sims):
        self.level = np.ascontiguousarray(level, np.int32)
        self.ijk = np.ascontiguousarray(ijk, np.int32).reshape(-1, 3)
        self.sim = np.ascontiguousarray(sim, np.int32)
        self.nb = int(self.level.shape[0])
        self.ns = len(sims)
        arr = (_Sim * self.ns)()
        for i, s in enumerate(sims):
            arr[i].nroot[:] = [int(v) for v in s.nroot]
            arr[i].origin[:] = [float(v) for v in s.origin]
            arr[i].dx0 = float(s.dx0)
            arr[i].bc[:] = [int(v) for v in s.bc]
            arr[i].inflow_w[:] = [float(v) for v in s.inflow_W]
            arr[i].body_c[:] = [float(v) for v in s.body_c]
            arr[i].body_r = float(s.body_r)
        self._sims = arr
        h = lib().or_grid_create(self.nb, _ip(self.level), _ip(self.ijk), _ip(self.sim), self.ns, arr)
        if not h:
            raise ValueError("oracle: invalid grid")
        self.h = h

    @classmethod
    def from_workload(cls, wl):
        return cls(wl.level, wl.ijk, wl.sim, wl.sims)

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_grid_free(self.h)
            self.h = None

    def neighbors(self):
        out = np.empty((self.nb, 26, 5), np.int32)
        lib().or_neighbors(self.h, _ip(out))
        return out

    def set_state(self, W):
        W = np.ascontiguousarray(W, np.float64)
        U = np.empty_like(W)
        lib().or_set_state(self.h, _dp(W), _dp(U))
        return U

    def fill_ghosts(self, U):
        U = np.ascontiguousarray(U, np.float64)
        view = np.empty((8, self.nb, 12, 12, 12))
        lib().or_fill_ghosts(self.h, _dp(U), _dp(view))
        return view

    def dt(self, U, cfl):
        U = np.ascontiguousarray(U, np.float64)
        out = np.empty(self.ns)
        lib().or_dt(self.h, _dp(U), float(cfl), _dp(out))
        return out

    def remap(self, U, to):
        """The state U of this grid moved onto grid `to` (same simulations, blocks refined or coarsened):
        copy, prolongation or restriction per cell (or_remap)."""
        U = np.ascontiguousarray(U, np.float64)
        out = np.empty((8, to.nb, 8, 8, 8))
        if lib().or_remap(self.h, _dp(U), to.h, _dp(out)) != 0:
            raise ValueError("remap: the grids differ in their simulations or a block of `to` cannot be supplied")
        return out

    def block_indicator(self, U):
        """Refinement indicator per block (or_block_indicator)."""
        U = np.ascontiguousarray(U, np.float64)
        ind = np.empty(self.nb)
        lib().or_block_indicator(self.h, _dp(U), _dp(ind))
        return ind

    def adapt(self, ind, r_refine, r_coarsen):
        """The adapted block list (levels, ijk [n, 3], sims) for indicators ind (or_adapt)."""
        ind = np.ascontiguousarray(ind, np.float64)
        cap = 8 * self.nb + 8
        lv, ijk, sim = np.empty(cap, np.int32), np.empty(3 * cap, np.int32), np.empty(cap, np.int32)
        n = lib().or_adapt(self.h, _dp(ind), float(r_refine), float(r_coarsen), _ip(lv), _ip(ijk), _ip(sim), cap)
        if n < 0:
            raise RuntimeError("adapt: output too small")
        return lv[:n].copy(), ijk[:3 * n].reshape(n, 3).copy(), sim[:n].copy()

    def advance(self, U0, U1, dt, n_stages, flux="rusanov", powell=False, cfl=0.8, recompute_dt=True,
                alpha=(0.0, 0.5), beta=(1.0, 0.5), local_dt=False):
        """Advance in place (U0, U1 updated; returns (dt, faults)). Heun by default. With local_dt (local
        time stepping) dt is one value per cell, shape (nB, 8, 8, 8), instead of one per simulation."""
        assert U0.flags.c_contiguous and U1.flags.c_contiguous
        shape = (self.nb, 8, 8, 8) if local_dt else (self.ns,)
        dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, np.float64), shape)).copy()
        o = _Opts(FLUX[flux], int(bool(powell)), 2, int(bool(recompute_dt)),
                  (ctypes.c_double * 2)(*alpha), (ctypes.c_double * 2)(*beta), float(cfl), int(bool(local_dt)))
        faults = ctypes.c_long(0)
        rc = lib().or_advance(self.h, _dp(U0), _dp(U1), _dp(dt), int(n_stages), ctypes.byref(o),
                              ctypes.byref(faults))
        if rc != 0:
            raise RuntimeError(f"oracle advance failed ({rc})")
        return dt, int(faults.value)

    def face_features(self, U, stats=None):
        """Stencil features of every face, [n_blocks * 1728, 32] (or_face_features); z-scored with
        stats[0:64] = (mean[32], std[32]) when given."""
        U = np.ascontiguousarray(U, np.float64)
        X = np.empty((self.nb * 1728, 32))
        st = None if stats is None else np.ascontiguousarray(np.asarray(stats, np.float64)[:64])
        lib().or_face_features(self.h, _dp(U), _dp(st) if st is not None else None, _dp(X))
        return X

    def advance_learned(self, U0, U1, dt, n_stages, y, ystats, tau=0.1, floor_rel=0.0, flux="hlle",
                        powell=True, cfl=0.8, recompute_dt=True, alpha=(0.0, 0.5), beta=(1.0, 0.5)):
        """Advance in place with the learned correction given as normalised per-face corrections
        y [n_blocks * 1728, 8] (face-normal frame) and ystats = (out_mean[8], out_std[8]); returns
        (dt, faults, flagged cells summed over the stages)."""
        assert U0.flags.c_contiguous and U1.flags.c_contiguous
        dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, np.float64), (self.ns,))).copy()
        y = np.ascontiguousarray(y, np.float64)
        assert y.shape == (self.nb * 1728, 8)
        ys = np.ascontiguousarray(np.asarray(ystats, np.float64).reshape(16))
        o = _Opts(FLUX[flux], int(bool(powell)), 2, int(bool(recompute_dt)),
                  (ctypes.c_double * 2)(*alpha), (ctypes.c_double * 2)(*beta), float(cfl), 0)
        faults, flagged = ctypes.c_long(0), ctypes.c_long(0)
        rc = lib().or_advance_learned(self.h, _dp(U0), _dp(U1), _dp(dt), int(n_stages), ctypes.byref(o), _dp(y),
                                      _dp(ys), float(tau), float(floor_rel), ctypes.byref(faults),
                                      ctypes.byref(flagged))
        if rc != 0:
            raise RuntimeError("oracle learned advance failed: it needs a single-level grid")
        return dt, int(faults.value), int(flagged.value)

    def xchg_messages(self, rank, n_ranks):
        """Every message of the exchange between processes for the block-to-process map `rank`, one row of
        16 int64 per message (see or_xchg_messages)."""
        rank = np.ascontiguousarray(rank, np.int32)
        cap = self.nb * 26 * 4 + 1
        out = np.empty((cap, 16), np.int64)
        n = lib().or_xchg_messages(self.h, _ip(rank), int(n_ranks), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   cap)
        if n < 0:
            raise RuntimeError("xchg_messages: too many messages")
        return out[:n].copy()

    def xchg_run(self, U, rank, n_ranks):
        """The padded views [8, nB, 12, 12, 12] after the exchange between simulated processes."""
        U = np.ascontiguousarray(U, np.float64)
        rank = np.ascontiguousarray(rank, np.int32)
        view = np.empty((8, self.nb, 12, 12, 12))
        lib().or_xchg_run(self.h, _ip(rank), int(n_ranks), _dp(U), _dp(view))
        return view

    def run(self, W, n_steps, **kw):
        """Convenience: conserved state after n_steps full steps from primitive W."""
        U0 = self.set_state(W)
        U1 = np.zeros_like(U0)
        dt, faults = self.advance(U0, U1, np.zeros(self.ns), 2 * n_steps, **kw)
        return U0, dt, faults


# ------------------------------------------------------------------------------------------------
# MLP of the learned flux correction (32 inputs, three SiLU hidden layers of width H, 8 outputs)

def mlp_n_params(H):
    return int(lib().mlp_n_params(int(H)))


def mlp_forward(params, H, x):
    params = np.ascontiguousarray(params, np.float64); x = np.ascontiguousarray(x, np.float64)
    N = x.shape[0]
    y = np.empty((N, 8))
    lib().mlp_forward(_dp(params), int(H), N, _dp(x), _dp(y))
    return y


def mlp_loss_grad(params, H, x, t):
    params = np.ascontiguousarray(params, np.float64); x = np.ascontiguousarray(x, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    g = np.empty_like(params)
    loss = lib().mlp_loss_grad(_dp(params), int(H), x.shape[0], _dp(x), _dp(t), _dp(g))
    return loss, g


def mlp_adam(p, m, v, g, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """In place on float64 arrays p, m, v."""
    lib().mlp_adam(_dp(p), _dp(m), _dp(v), _dp(np.ascontiguousarray(g, np.float64)), p.size, lr, b1, b2, eps, int(t))


# ------------------------------------------------------------------------------------------------
# training targets of the learned flux correction (the library's own form, not the paper's)

def _face_slot(d, x, y, z):
    """Index of face (x, y, z) of direction d in a block's face-data layout (576 faces per direction)."""
    return ((z * 8 + y) * 9 + x) if d == 0 else (((z * 9 + y) * 8 + x) if d == 1 else ((z * 8 + y) * 8 + x))


def _face_coords(d, f):
    """Face coordinates (x, y, z) of slot f of direction d (the coordinate along d in 0..8)."""
    if d == 0:
        return f % 9, (f // 9) % 8, f // 72
    if d == 1:
        return f % 8, (f // 8) % 9, f // 72
    return f % 8, (f // 8) % 8, f // 64


def face_targets(Ff, fine_ijk, Fc, coarse_ijk):
    """For every face of a level-0 grid (blocks coarse_ijk), the mean of the 4 faces of the fine grid (the
    same domain refined once: blocks fine_ijk at level 1) covering it, minus the coarse face value, per
    component. Ff [n_fine * 1728, 8] and Fc [n_coarse * 1728, 8] are float32 face data in the layout
    [block][direction][576 faces][8]; the result is float32 in the coarse layout.

    In global fine coordinates the coarse face at position a along its normal d (block ic) is the fine
    face plane 16 ic + 2 a, and a coarse tangential position t covers the fine rows 16 ic + 2 t and + 1.
    A fine face at normal position P belongs to the fine block P // 8 at local position P % 8, except a
    coarse block's high face (a = 8), which is read as local position 8 of the fine block below it, so that
    every fine face read lies in one of the coarse block's children. The mean is taken in float64 as
    ((f00 + f10) + (f01 + f11)) / 4 with the first tangential axis (x before y before z) fastest, the
    difference rounded to float32 once."""
    Ff = np.asarray(Ff, np.float32).reshape(-1, 3, 576, 8).astype(np.float64)
    Fc = np.asarray(Fc, np.float32).reshape(-1, 3, 576, 8).astype(np.float64)
    coarse_ijk = np.asarray(coarse_ijk).reshape(-1, 3)
    where = {tuple(int(v) for v in ijk): b for b, ijk in enumerate(np.asarray(fine_ijk).reshape(-1, 3))}
    out = np.empty(Fc.shape, np.float32)
    for d in range(3):
        t1, t2 = [a for a in range(3) if a != d]
        for f in range(576):
            q = _face_coords(d, f)
            for c in range(coarse_ijk.shape[0]):
                parts = []
                for e2 in (0, 1):
                    for e1 in (0, 1):
                        g = [16 * int(coarse_ijk[c, a]) + 2 * q[a] for a in range(3)]
                        g[t1] += e1
                        g[t2] += e2
                        n = [g[a] // 8 for a in range(3)]
                        loc = [g[a] % 8 for a in range(3)]
                        if q[d] == 8:
                            n[d] -= 1
                            loc[d] = 8
                        parts.append(Ff[where[tuple(n)], d, _face_slot(d, *loc)])
                mean = ((parts[0] + parts[1]) + (parts[2] + parts[3])) * 0.25
                out[c, d, f] = (mean - Fc[c, d, f]).astype(np.float32)
    return out.reshape(-1, 8)
