"""Thin ctypes binding of libbmhd.so (include/bmhd.h). Argument marshalling only: every step of the
solver runs in the library's HIP kernels. Device buffers are torch tensors on the current HIP device;
every call is enqueued on torch's current stream.

The binding fails loudly when the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbmhd.so")

BC_PERIODIC, BC_OUTFLOW, BC_INFLOW = 0, 1, 2
FLUX = {"rusanov": 0, "hlle": 1, "linde": 2}
PRECISION = {"fp64": 0, "fp32_flux": 1}
SCHEME = {"default": 0, "face": 1, "plane": 2, "block": 3}

EXPORTS = ["bmhd_version", "bmhd_last_error", "bmhd_grid_create", "bmhd_grid_destroy", "bmhd_grid_info_get",
           "bmhd_grid_neighbors", "bmhd_grid_upload", "bmhd_set_state", "bmhd_fill_ghosts", "bmhd_remap",
           "bmhd_reduce_dt", "bmhd_advance", "bmhd_autotune", "bmhd_mlp_last_error", "bmhd_mlp_n_params", "bmhd_mlp_work_bytes",
           "bmhd_mlp_forward", "bmhd_mlp_backward", "bmhd_mlp_backward_noalloc", "bmhd_mlp_adam", "bmhd_mlp_to_bf16", "bmhd_face_data",
           "bmhd_block_indicator", "bmhd_adapt", "bmhd_xchg_create", "bmhd_xchg_destroy", "bmhd_xchg_sizes", "bmhd_xchg_messages", "bmhd_xchg_upload",
           "bmhd_xchg_interior", "bmhd_xchg_pack", "bmhd_xchg_unpack", "bmhd_xchg_stage", "bmhd_xchg_flux_correct",
           "bmhd_face_targets", "bmhd_xchg_create_for_stage"]


class SimDesc(ctypes.Structure):
    _fields_ = [("nroot", ctypes.c_int32 * 3), ("origin", ctypes.c_double * 3), ("dx0", ctypes.c_double),
                ("bc", ctypes.c_int32 * 6), ("inflow_W", ctypes.c_double * 8), ("body_c", ctypes.c_double * 3),
                ("body_r", ctypes.c_double)]


class GridDesc(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int32), ("level", ctypes.POINTER(ctypes.c_int32)),
                ("ijk", ctypes.POINTER(ctypes.c_int32)), ("sim", ctypes.POINTER(ctypes.c_int32)),
                ("n_sims", ctypes.c_int32), ("sims", ctypes.POINTER(SimDesc))]


class Learned(ctypes.Structure):
    _fields_ = [("hidden", ctypes.c_int32), ("mode", ctypes.c_int32), ("params", ctypes.c_void_p),
                ("params_bf16", ctypes.c_void_p), ("stats", ctypes.c_void_p), ("x_buf", ctypes.c_void_p),
                ("y_buf", ctypes.c_void_p), ("flags", ctypes.c_void_p), ("fallback_cells", ctypes.c_void_p),
                ("tau", ctypes.c_double), ("floor_rel", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("flux", ctypes.c_int32), ("powell", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("recompute_dt", ctypes.c_int32), ("cfl", ctypes.c_double), ("alpha", ctypes.c_double * 2),
                ("beta", ctypes.c_double * 2), ("slab", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("persist_wgs", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("learned", ctypes.POINTER(Learned)), ("n_events", ctypes.c_int32),
                ("events", ctypes.POINTER(ctypes.c_void_p)), ("local_dt", ctypes.c_int32)]


class GridInfo(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int32), ("n_sims", ctypes.c_int32), ("n_level_faces", ctypes.c_int32),
                ("n_flux_faces", ctypes.c_int32), ("work_bytes", ctypes.c_size_t)]


class BmhdError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libbmhd.so (built by paper_2501_06717_amd.build). Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise BmhdError(f"{LIB_PATH} is missing: build it with `python -m paper_2501_06717_amd.build` "
                        "(there is no fallback path)")
    L = ctypes.CDLL(LIB_PATH)
    P, vp, i32 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32
    L.bmhd_version.restype = i32
    L.bmhd_last_error.restype = ctypes.c_char_p
    L.bmhd_grid_create.argtypes = [P(GridDesc), P(vp)]
    L.bmhd_grid_create.restype = i32
    L.bmhd_grid_destroy.argtypes = [vp]
    L.bmhd_grid_destroy.restype = None
    L.bmhd_grid_info_get.argtypes = [vp, P(GridInfo)]
    L.bmhd_grid_info_get.restype = i32
    L.bmhd_grid_neighbors.argtypes = [vp, P(i32)]
    L.bmhd_grid_neighbors.restype = i32
    L.bmhd_grid_upload.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.bmhd_grid_upload.restype = i32
    L.bmhd_set_state.argtypes = [vp, vp, vp, vp]
    L.bmhd_set_state.restype = i32
    L.bmhd_fill_ghosts.argtypes = [vp, vp, vp, vp]
    L.bmhd_fill_ghosts.restype = i32
    L.bmhd_remap.argtypes = [vp, vp, vp, vp, vp]
    L.bmhd_remap.restype = i32
    L.bmhd_reduce_dt.argtypes = [vp, vp, ctypes.c_double, vp, vp]
    L.bmhd_reduce_dt.restype = i32
    L.bmhd_advance.argtypes = [vp, vp, vp, vp, i32, P(Opts), vp, vp]
    L.bmhd_advance.restype = i32
    L.bmhd_autotune.argtypes = [vp, vp, vp, vp, P(Opts), i32, P(Opts), P(ctypes.c_float), vp]
    L.bmhd_autotune.restype = i32
    L.bmhd_face_data.argtypes = [vp, vp, i32, vp, vp, vp, vp]
    L.bmhd_face_data.restype = i32
    L.bmhd_mlp_last_error.restype = ctypes.c_char_p
    L.bmhd_mlp_n_params.argtypes = [i32]
    L.bmhd_mlp_n_params.restype = ctypes.c_int64
    L.bmhd_mlp_work_bytes.argtypes = [i32, i32]
    L.bmhd_mlp_work_bytes.restype = ctypes.c_size_t
    L.bmhd_mlp_forward.argtypes = [vp, vp, i32, i32, vp, vp, vp, i32, vp]
    L.bmhd_mlp_forward.restype = i32
    L.bmhd_mlp_backward.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, vp, i32, vp]
    L.bmhd_mlp_backward.restype = i32
    L.bmhd_mlp_backward_noalloc.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, i32, vp]
    L.bmhd_mlp_backward_noalloc.restype = i32
    L.bmhd_mlp_adam.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, i32, vp]
    L.bmhd_mlp_adam.restype = i32
    L.bmhd_mlp_to_bf16.argtypes = [vp, vp, ctypes.c_int64, vp]
    L.bmhd_mlp_to_bf16.restype = i32
    L.bmhd_block_indicator.argtypes = [vp, vp, vp, vp]
    L.bmhd_block_indicator.restype = i32
    L.bmhd_adapt.argtypes = [vp, P(ctypes.c_double), ctypes.c_double, ctypes.c_double, P(i32), P(i32), P(i32), i32,
                             P(i32)]
    L.bmhd_adapt.restype = i32
    L.bmhd_xchg_create.argtypes = [vp, P(i32), i32, P(vp)]
    L.bmhd_xchg_create.restype = i32
    L.bmhd_xchg_destroy.argtypes = [vp]
    L.bmhd_xchg_destroy.restype = None
    L.bmhd_xchg_sizes.argtypes = [vp, P(i32), P(ctypes.c_int64), P(ctypes.c_size_t)]
    L.bmhd_xchg_sizes.restype = i32
    L.bmhd_xchg_messages.argtypes = [vp, P(ctypes.c_int64), ctypes.c_int64]
    L.bmhd_xchg_messages.restype = ctypes.c_int64
    L.bmhd_xchg_upload.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.bmhd_xchg_upload.restype = i32
    L.bmhd_xchg_interior.argtypes = [vp, i32, vp, vp, vp]
    L.bmhd_xchg_interior.restype = i32
    L.bmhd_xchg_pack.argtypes = [vp, i32, i32, vp, vp, vp]
    L.bmhd_xchg_pack.restype = i32
    L.bmhd_xchg_unpack.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    L.bmhd_xchg_unpack.restype = i32
    L.bmhd_xchg_create_for_stage.argtypes = L.bmhd_xchg_create.argtypes
    L.bmhd_xchg_create_for_stage.restype = i32
    L.bmhd_face_targets.argtypes = [vp, vp, vp, vp, vp, vp]
    L.bmhd_face_targets.restype = i32
    L.bmhd_xchg_stage.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, P(Opts), vp, vp]
    L.bmhd_xchg_stage.restype = i32
    L.bmhd_xchg_flux_correct.argtypes = [vp, i32, i32, vp, vp, P(Opts), vp, vp]
    L.bmhd_xchg_flux_correct.restype = i32
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        msg = lib().bmhd_last_error().decode()
        raise BmhdError(f"bmhd error {rc}: {msg}")


def make_opts(flux="rusanov", powell=False, precision="fp64", recompute_dt=True, cfl=0.8,
              alpha=(0.0, 0.5), beta=(1.0, 0.5), slab=0, scheme=0, persist_wgs=0, use_graph=False,
              events=None, learned=None, local_dt=False) -> Opts:
    """Options for bmhd_advance. `events`: optional list of torch.cuda.Event (enable_timing=True), two per
    stage, recorded by the library around each stage kernel. `local_dt`: local time stepping (dt is then
    one float64 per cell, shape (n_blocks, 8, 8, 8))."""
    o = Opts()
    o.flux = FLUX[flux]
    o.powell = int(bool(powell))
    o.precision = PRECISION[precision]
    o.recompute_dt = int(bool(recompute_dt))
    o.cfl = float(cfl)
    o.alpha[:] = [float(a) for a in alpha]
    o.beta[:] = [float(b) for b in beta]
    o.slab = int(slab)
    o.scheme = SCHEME[scheme] if isinstance(scheme, str) else int(scheme)
    o.persist_wgs = int(persist_wgs)
    o.use_graph = int(bool(use_graph))
    o.local_dt = int(bool(local_dt))
    if learned is not None:
        o._learned_keepalive = learned
        o.learned = ctypes.pointer(learned)
    else:
        o.learned = None
    if events:
        arr = (ctypes.c_void_p * len(events))(*[ctypes.c_void_p(e.cuda_event) for e in events])
        o._events_keepalive = arr
        o.n_events = len(events)
        o.events = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    else:
        o.n_events = 0
        o.events = None
    return o


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype=None):
    import torch
    if not t.is_cuda:
        raise BmhdError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise BmhdError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise BmhdError(f"tensor dtype must be {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


class Grid:
    """A grid handle: host tables built by the library, plus (after `upload`) a torch-owned device
    workspace holding them."""

    def __init__(self, level: Sequence[int], ijk, sim, sims):
        L = lib()
        self.level = np.ascontiguousarray(level, np.int32)
        self.ijk = np.ascontiguousarray(ijk, np.int32).reshape(-1, 3)
        self.sim = np.ascontiguousarray(sim, np.int32)
        self.nb = int(self.level.shape[0])
        self.ns = len(sims)
        self.sims = list(sims)
        arr = (SimDesc * self.ns)()
        for i, s in enumerate(sims):
            arr[i].nroot[:] = [int(v) for v in s.nroot]
            arr[i].origin[:] = [float(v) for v in s.origin]
            arr[i].dx0 = float(s.dx0)
            arr[i].bc[:] = [int(v) for v in s.bc]
            arr[i].inflow_W[:] = [float(v) for v in s.inflow_W]
            arr[i].body_c[:] = [float(v) for v in s.body_c]
            arr[i].body_r = float(s.body_r)
        d = GridDesc()
        d.n_blocks = self.nb
        d.level = self.level.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.ijk = self.ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.sim = self.sim.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.n_sims = self.ns
        d.sims = arr
        h = ctypes.c_void_p()
        _check(L.bmhd_grid_create(ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.work = None
        info = GridInfo()
        _check(L.bmhd_grid_info_get(self.h, ctypes.byref(info)))
        self.info = info

    @classmethod
    def from_workload(cls, wl):
        return cls(wl.level, wl.ijk, wl.sim, wl.sims)

    def __del__(self):
        # at interpreter exit the module's globals may already be gone: the process frees the grid then
        h = getattr(self, "h", None)
        L = globals().get("_lib")
        if h is not None and h.value and L is not None:
            L.bmhd_grid_destroy(h)
            self.h = None

    @property
    def n_cells(self):
        return self.nb * 512

    def neighbors(self) -> np.ndarray:
        out = np.empty((self.nb, 26, 5), np.int32)
        _check(lib().bmhd_grid_neighbors(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def upload(self, device="cuda", stream=None):
        import torch
        n = int(self.info.work_bytes)
        self.work = torch.empty(n + 256, dtype=torch.uint8, device=device)
        base = self.work.data_ptr()
        aligned = (base + 255) & ~255
        _check(lib().bmhd_grid_upload(self.h, ctypes.c_void_p(aligned), ctypes.c_size_t(n), _stream_ptr(stream)))
        return self

    def _need(self, t, n, what):
        """Size check before a pointer crosses the boundary (the library cannot see tensor sizes)."""
        if t.numel() != n:
            raise BmhdError(f"{what} holds {t.numel()} values; this grid needs {n}")

    def set_state(self, W, U=None, stream=None):
        import torch
        self._need(W, 8 * self.nb * 512, "W")
        if U is None:
            U = torch.empty_like(W)
        self._need(U, 8 * self.nb * 512, "U")
        _check(lib().bmhd_set_state(self.h, _dev_ptr(W, torch.float64), _dev_ptr(U, torch.float64),
                                    _stream_ptr(stream)))
        return U

    def fill_ghosts(self, U, view=None, stream=None):
        import torch
        self._need(U, 8 * self.nb * 512, "U")
        if view is None:
            view = torch.empty((8, self.nb, 12, 12, 12), dtype=torch.float64, device=U.device)
        self._need(view, 8 * self.nb * 1728, "view")
        _check(lib().bmhd_fill_ghosts(self.h, _dev_ptr(U, torch.float64), _dev_ptr(view, torch.float64),
                                      _stream_ptr(stream)))
        return view

    def remap(self, U, to, out=None, stream=None):
        """The state U of this grid moved onto grid `to` (same simulations; blocks refined or coarsened):
        copy, prolongation or restriction per cell, on the device."""
        import torch
        self._need(U, 8 * self.nb * 512, "U")
        if out is None:
            out = torch.empty((8, to.nb, 8, 8, 8), dtype=torch.float64, device=U.device)
        to._need(out, 8 * to.nb * 512, "out")
        _check(lib().bmhd_remap(self.h, _dev_ptr(U, torch.float64), to.h, _dev_ptr(out, torch.float64),
                                _stream_ptr(stream)))
        return out

    def face_targets(self, Ff, coarse, Fc, out=None, stream=None):
        """Flux-correction targets of grid `coarse`'s faces from this grid (the same simulations refined
        everywhere): mean of the 4 fine face fluxes minus the coarse one, [coarse.nb * 1728, 8] float32."""
        import torch
        if tuple(Ff.shape) != (self.nb * 1728, 8) or tuple(Fc.shape) != (coarse.nb * 1728, 8):
            raise BmhdError("face data must be [n_blocks * 1728, 8] of the fine and the coarse grid")
        if out is None:
            out = torch.empty((coarse.nb * 1728, 8), dtype=torch.float32, device=Ff.device)
        if tuple(out.shape) != (coarse.nb * 1728, 8):
            raise BmhdError("targets must be [coarse n_blocks * 1728, 8]")
        _check(lib().bmhd_face_targets(self.h, _dev_ptr(Ff, torch.float32), coarse.h, _dev_ptr(Fc, torch.float32),
                                       _dev_ptr(out, torch.float32), _stream_ptr(stream)))
        return out

    def block_indicator(self, U, out=None, stream=None):
        """Refinement indicator per block (device tensor [n_blocks])."""
        import torch
        self._need(U, 8 * self.nb * 512, "U")
        if out is None:
            out = torch.empty(self.nb, dtype=torch.float64, device=U.device)
        self._need(out, self.nb, "indicator")
        _check(lib().bmhd_block_indicator(self.h, _dev_ptr(U, torch.float64), _dev_ptr(out, torch.float64),
                                          _stream_ptr(stream)))
        return out

    def adapt_blocks(self, ind, r_refine, r_coarsen):
        """The adapted block list (levels, ijk [n, 3], sims) for host indicators `ind`."""
        ind = np.ascontiguousarray(ind, np.float64)
        if ind.size != self.nb:
            raise BmhdError(f"one indicator per block: {ind.size} given, {self.nb} blocks")
        P = ctypes.POINTER
        n = ctypes.c_int32()
        _check(lib().bmhd_adapt(self.h, ind.ctypes.data_as(P(ctypes.c_double)), float(r_refine), float(r_coarsen),
                                None, None, None, 0, ctypes.byref(n)))
        cap = int(n.value)
        lv, ijk, sim = np.empty(cap, np.int32), np.empty(3 * cap, np.int32), np.empty(cap, np.int32)
        _check(lib().bmhd_adapt(self.h, ind.ctypes.data_as(P(ctypes.c_double)), float(r_refine), float(r_coarsen),
                                lv.ctypes.data_as(P(ctypes.c_int32)), ijk.ctypes.data_as(P(ctypes.c_int32)),
                                sim.ctypes.data_as(P(ctypes.c_int32)), cap, ctypes.byref(n)))
        return lv, ijk.reshape(-1, 3), sim

    def adapt(self, U, r_refine, r_coarsen, stream=None):
        """One adaptation between steps: indicator on the device, new block list on the host, a new grid
        (tables uploaded) and the state remapped onto it. Returns (new grid, new state)."""
        ind = self.block_indicator(U, stream=stream).cpu().numpy()
        lv, ijk, sim = self.adapt_blocks(ind, r_refine, r_coarsen)
        new = Grid(lv, ijk, sim, self.sims).upload(device=U.device, stream=stream)
        return new, self.remap(U, new, stream=stream)

    def reduce_dt(self, U, cfl, dt=None, stream=None):
        import torch
        self._need(U, 8 * self.nb * 512, "U")
        if dt is None:
            dt = torch.empty(self.ns, dtype=torch.float64, device=U.device)
        if dt.numel() < self.ns:
            raise BmhdError("dt needs one value per simulation")
        _check(lib().bmhd_reduce_dt(self.h, _dev_ptr(U, torch.float64), float(cfl), _dev_ptr(dt, torch.float64),
                                    _stream_ptr(stream)))
        return dt

    def advance(self, U0, U1, dt, n_stages, opts: Optional[Opts] = None, faults=None, stream=None, **kw):
        import torch
        o = opts if opts is not None else make_opts(**kw)
        self._need(U0, 8 * self.nb * 512, "U0")
        self._need(U1, 8 * self.nb * 512, "U1")
        need = self.nb * 512 if o.local_dt else self.ns
        if dt.numel() < need:
            raise BmhdError(f"dt holds {dt.numel()} values; this grid and local_dt={o.local_dt} need {need}")
        fp = _dev_ptr(faults, torch.int32) if faults is not None else ctypes.c_void_p(0)
        _check(lib().bmhd_advance(self.h, _dev_ptr(U0, torch.float64), _dev_ptr(U1, torch.float64),
                                  _dev_ptr(dt, torch.float64), int(n_stages), ctypes.byref(o), fp,
                                  _stream_ptr(stream)))

    def face_data(self, U, flux="hlle", stats=None, want_x=True, want_f=True, stream=None):
        """Per-face stencil features [nB*1728][32] and plain fluxes [nB*1728][8] (face-normal frame)."""
        import torch
        self._need(U, 8 * self.nb * 512, "U")
        if stats is not None and stats.numel() < 64:
            raise BmhdError("stats needs the 32 input means and 32 deviations")
        nf = self.nb * 1728
        X = torch.empty((nf, 32), dtype=torch.float32, device=U.device) if want_x else None
        F = torch.empty((nf, 8), dtype=torch.float32, device=U.device) if want_f else None
        _check(lib().bmhd_face_data(self.h, _dev_ptr(U, torch.float64), FLUX[flux],
                                    _dev_ptr(stats, torch.float32) if stats is not None else None,
                                    _dev_ptr(X) if want_x else None, _dev_ptr(F) if want_f else None,
                                    _stream_ptr(stream)))
        return X, F

    def learned(self, mlp, stats, mode="bf16", tau=0.1, fallback=None, floor_rel=0.0):
        """Scratch buffers and the options struct of the learned correction for this grid."""
        import torch
        nf = self.nb * 1728
        dev = mlp.p.device
        self._lx = torch.empty((nf, 32), dtype=torch.float32, device=dev)
        self._ly = torch.empty((nf, 8), dtype=torch.float32, device=dev)
        self._lf = torch.zeros(self.nb * 512, dtype=torch.uint8, device=dev)
        if stats.numel() != 80:
            raise BmhdError("stats must hold the 80 normalisation values")
        self._lstats = stats.to(dev, torch.float32).contiguous()
        L = Learned()
        L.hidden = mlp.H
        L.mode = MLP_MODE[mode]
        L.params = mlp.p.data_ptr()
        L.params_bf16 = mlp.pb.data_ptr()
        L.stats = self._lstats.data_ptr()
        L.x_buf = self._lx.data_ptr()
        L.y_buf = self._ly.data_ptr()
        L.flags = self._lf.data_ptr()
        L.fallback_cells = fallback.data_ptr() if fallback is not None else None
        L.tau = float(tau)
        L.floor_rel = float(floor_rel)
        return L

    def given_corrections(self, y, stats, tau=0.1, fallback=None, floor_rel=0.0):
        """Options of the learned form with the normalised flux corrections y [n_blocks * 1728, 8] float32
        (face-normal frame, the face order of bmhd_face_data) given instead of a network's outputs."""
        import torch
        if tuple(y.shape) != (self.nb * 1728, 8) or y.dtype != torch.float32 or not y.is_contiguous():
            raise BmhdError("given corrections must be a contiguous float32 tensor [n_blocks * 1728, 8]")
        self._ly = y
        self._lf = torch.zeros(self.nb * 512, dtype=torch.uint8, device=y.device)
        self._lstats = stats.to(y.device, torch.float32).contiguous()
        L = Learned()
        L.hidden = 32
        L.mode = 2
        L.stats = self._lstats.data_ptr()
        L.y_buf = y.data_ptr()
        L.flags = self._lf.data_ptr()
        L.fallback_cells = fallback.data_ptr() if fallback is not None else None
        L.tau = float(tau)
        L.floor_rel = float(floor_rel)
        return L

    def autotune(self, U0, U1, dt, n_steps=3, stream=None, **kw):
        """Time the stage kernel's launch shapes on (scratch) buffers; returns (best Opts, {shape: ms})."""
        import torch
        self._need(U0, 8 * self.nb * 512, "U0")
        self._need(U1, 8 * self.nb * 512, "U1")
        base = make_opts(**kw)
        if dt.numel() < self.ns:
            raise BmhdError("dt needs one value per simulation")
        best = Opts()
        ms = (ctypes.c_float * 13)()
        _check(lib().bmhd_autotune(self.h, _dev_ptr(U0, torch.float64), _dev_ptr(U1, torch.float64),
                                   _dev_ptr(dt, torch.float64), ctypes.byref(base), int(n_steps), ctypes.byref(best),
                                   ms, _stream_ptr(stream)))
        names = [f"{s}_slab{k}{p}" for s in ("face", "plane") for k in (4, 8) for p in ("", "_persist2", "_persist4")]
        names.append("block")
        return best, dict(zip(names, list(ms)))


class Xchg:
    """Ghost exchange between (virtual) processes for a block-to-process assignment: message maps built by
    the library on the host, pack / unpack kernels on the device. Views and buffers are torch tensors."""

    def __init__(self, grid: "Grid", rank, n_ranks, for_stage=False):
        """for_stage: maps for the sharded stage (views hold only what the stage and the packs read)."""
        L = lib()
        self.grid = grid
        self.rank = np.ascontiguousarray(rank, np.int32)
        if self.rank.size != grid.nb:
            raise BmhdError("one process index per block")
        self.nr = int(n_ranks)
        self.for_stage = bool(for_stage)
        h = ctypes.c_void_p()
        create = L.bmhd_xchg_create_for_stage if for_stage else L.bmhd_xchg_create
        _check(create(grid.h, self.rank.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), self.nr, ctypes.byref(h)))
        self.h = h
        self.nloc = np.zeros(self.nr, np.int32)
        self.len = np.zeros((2, self.nr, self.nr), np.int64)
        wb = ctypes.c_size_t()
        _check(L.bmhd_xchg_sizes(self.h, self.nloc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 self.len.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(wb)))
        self.work_bytes = int(wb.value)
        self.work = None

    def __del__(self):
        h = getattr(self, "h", None)
        L = globals().get("_lib")
        if h is not None and h.value and L is not None:
            L.bmhd_xchg_destroy(h)
            self.h = None

    def messages(self) -> np.ndarray:
        L = lib()
        n = int(L.bmhd_xchg_messages(self.h, None, 0))
        out = np.zeros((max(n, 1), 16), np.int64)
        got = int(L.bmhd_xchg_messages(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n))
        if got < 0:
            _check(got)
        return out[:n]

    def upload(self, device="cuda", stream=None):
        import torch
        self.work = torch.empty(self.work_bytes + 256, dtype=torch.uint8, device=device)
        aligned = (self.work.data_ptr() + 255) & ~255
        _check(lib().bmhd_xchg_upload(self.h, ctypes.c_void_p(aligned), ctypes.c_size_t(self.work_bytes),
                                      _stream_ptr(stream)))
        return self

    def new_view(self, r, device="cuda"):
        import torch
        return torch.zeros((8, int(self.nloc[r]), 12, 12, 12), dtype=torch.float64, device=device)

    def send_len(self, p, s):
        return int(self.len[p - 1, s].sum())

    def recv_len(self, p, r):
        return int(self.len[p - 1, :, r].sum())

    def _need_view(self, r, view):
        if tuple(view.shape) != (8, int(self.nloc[r]), 12, 12, 12):
            raise BmhdError("the view must be [8][blocks of the process][12][12][12]")

    def interior(self, r, U, view, stream=None):
        import torch
        if tuple(U.shape) != (8, self.grid.nb, 8, 8, 8):
            raise BmhdError("the state must be [8][n_blocks][8][8][8]")
        self._need_view(r, view)
        _check(lib().bmhd_xchg_interior(self.h, int(r), _dev_ptr(U, torch.float64),
                                        _dev_ptr(view, torch.float64) if view.numel() else None, _stream_ptr(stream)))

    def pack(self, p, s, view, send, stream=None):
        import torch
        self._need_view(s, view)
        if send.numel() < self.send_len(p, s):
            raise BmhdError("send buffer too small")
        _check(lib().bmhd_xchg_pack(self.h, int(p), int(s), _dev_ptr(view, torch.float64) if view.numel() else None,
                                    _dev_ptr(send, torch.float64) if send.numel() else None, _stream_ptr(stream)))

    def unpack(self, p, r, recv, view, bad=None, stream=None):
        import torch
        self._need_view(r, view)
        if recv.numel() < self.recv_len(p, r):
            raise BmhdError("receive buffer too small")
        _check(lib().bmhd_xchg_unpack(self.h, int(p), int(r), _dev_ptr(recv, torch.float64) if recv.numel() else None,
                                      _dev_ptr(view, torch.float64) if view.numel() else None,
                                      _dev_ptr(bad, torch.int32) if bad is not None else None,
                                      _stream_ptr(stream)))

    def transfer(self, p, sends, recvs):
        """The point-to-point transfers of pass p, as device copies: the segment for r in s's send buffer
        to the segment from s in r's receive buffer."""
        for s in range(self.nr):
            so = 0
            for r in range(self.nr):
                n = int(self.len[p - 1, s, r])
                if n:
                    ro = int(self.len[p - 1, :s, r].sum())
                    recvs[r][ro:ro + n].copy_(sends[s][so:so + n])
                so += n

    def run(self, U, bad=None):
        """Both passes of the exchange for every process: returns the views (bad: optional int32 device
        counter of skipped messages)."""
        import torch
        # complete views: every cell is written below (interior, 26 directions of ghost cells), no clearing;
        # stage-mode views hold only what the stage reads from them
        views = [torch.empty((8, int(self.nloc[r]), 12, 12, 12), dtype=torch.float64, device=U.device)
                 for r in range(self.nr)]
        for r in range(self.nr):
            self.interior(r, U, views[r])
        for p in (1, 2):
            sends = [torch.empty(self.send_len(p, s), dtype=torch.float64, device=U.device) for s in range(self.nr)]
            recvs = [torch.empty(self.recv_len(p, r), dtype=torch.float64, device=U.device) for r in range(self.nr)]
            for s in range(self.nr):
                self.pack(p, s, views[s], sends[s])
            self.transfer(p, sends, recvs)
            for r in range(self.nr):
                self.unpack(p, r, recvs[r], views[r], bad=bad)
        return views

    def stage(self, r, e, view, U0, Uin, Uout, dt, opts: Optional[Opts] = None, faults=None, stream=None, **kw):
        """Stage e (0 or 1) of process r's blocks, ghost cells from its exchanged view."""
        import torch
        o = opts if opts is not None else make_opts(**kw)
        state = (8, self.grid.nb, 8, 8, 8)
        if any(tuple(t.shape) != state for t in (U0, Uin, Uout)):
            raise BmhdError(f"states must be {state}")
        self._need_view(r, view)
        if dt.numel() < self.grid.ns:
            raise BmhdError("dt needs one value per simulation")
        fp = _dev_ptr(faults, torch.int32) if faults is not None else ctypes.c_void_p(0)
        _check(lib().bmhd_xchg_stage(self.h, int(r), int(e), _dev_ptr(view, torch.float64) if view.numel() else None,
                                     _dev_ptr(U0, torch.float64), _dev_ptr(Uin, torch.float64),
                                     _dev_ptr(Uout, torch.float64), _dev_ptr(dt, torch.float64), ctypes.byref(o), fp,
                                     _stream_ptr(stream)))

    def flux_correct(self, r, e, Uout, dt, opts: Optional[Opts] = None, faults=None, stream=None, **kw):
        import torch
        o = opts if opts is not None else make_opts(**kw)
        if tuple(Uout.shape) != (8, self.grid.nb, 8, 8, 8) or dt.numel() < self.grid.ns:
            raise BmhdError("state or dt of the wrong size")
        fp = _dev_ptr(faults, torch.int32) if faults is not None else ctypes.c_void_p(0)
        _check(lib().bmhd_xchg_flux_correct(self.h, int(r), int(e), _dev_ptr(Uout, torch.float64),
                                            _dev_ptr(dt, torch.float64), ctypes.byref(o), fp, _stream_ptr(stream)))

    def advance(self, U0, U1, n_steps, cfl=0.8, faults=None, **kw):
        """n_steps steps of the two-stage scheme with the processes' blocks advanced separately: per stage,
        both exchange passes into every process's view, each process's stage from its view, then the flux
        corrections. dt per step: the CFL minimum over all blocks (bmhd_reduce_dt, the stand-in for the
        reduction over processes). Returns the last step's dt."""
        o = make_opts(recompute_dt=False, cfl=cfl, **kw)
        dt = None
        for _ in range(n_steps):
            dt = self.grid.reduce_dt(U0, cfl)
            for e, (Uin, Uout) in enumerate(((U0, U1), (U1, U0))):
                views = self.run(Uin)
                for r in range(self.nr):
                    self.stage(r, e, views[r], U0, Uin, Uout, dt, opts=o, faults=faults)
                for r in range(self.nr):
                    self.flux_correct(r, e, Uout, dt, opts=o, faults=faults)
        return dt


# ------------------------------------------------------------------------------------------------
# learned flux correction: MLP on matrix cores

MLP_MODE = {"bf16": 0, "fp32": 1}


def _mcheck(rc):
    if rc != 0:
        raise BmhdError(f"bmhd mlp error {rc}: {lib().bmhd_mlp_last_error().decode()}")


class Mlp:
    """Parameters (FP32 master + BF16 copy) and Adam moments of the flux-correction MLP, all torch
    tensors on the GPU."""

    def __init__(self, hidden=128, params=None, device="cuda"):
        import torch
        self.H = int(hidden)
        self.n = int(lib().bmhd_mlp_n_params(self.H))
        if params is None:
            params = torch.zeros(self.n, dtype=torch.float32)
        self.p = torch.as_tensor(params, dtype=torch.float32).to(device).contiguous()
        assert self.p.numel() == self.n
        self.pb = torch.empty(self.n, dtype=torch.int16, device=device)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.t = 0
        self.refresh()

    def refresh(self, stream=None):
        _mcheck(lib().bmhd_mlp_to_bf16(_dev_ptr(self.p), _dev_ptr(self.pb), self.n, _stream_ptr(stream)))

    def forward(self, x, save=False, mode="bf16", stream=None):
        import torch
        n = x.shape[0]
        y = torch.empty((n, 8), dtype=torch.float32, device=x.device)
        z = torch.empty((3, n, self.H), dtype=torch.float32, device=x.device) if save else None
        _mcheck(lib().bmhd_mlp_forward(_dev_ptr(self.p), _dev_ptr(self.pb), self.H, n, _dev_ptr(x, torch.float32),
                                       _dev_ptr(y), _dev_ptr(z) if save else None, MLP_MODE[mode],
                                       _stream_ptr(stream)))
        return (y, z) if save else y

    def loss_grad(self, x, t, mode="bf16", stream=None, noalloc=False):
        """Returns (loss tensor, gradient tensor) for targets t[n][8]. With noalloc the backward pass
        runs on the library's static work area (bmhd_mlp_backward_noalloc) instead of a work tensor."""
        import torch
        n = x.shape[0]
        y, z = self.forward(x, save=True, mode=mode, stream=stream)
        g = torch.empty_like(self.p)
        sq = torch.empty((n, 8), dtype=torch.float32, device=x.device)
        if noalloc:
            _mcheck(lib().bmhd_mlp_backward_noalloc(_dev_ptr(self.p), self.H, n, _dev_ptr(x),
                                                    _dev_ptr(t, torch.float32), _dev_ptr(z), _dev_ptr(y), _dev_ptr(g),
                                                    _dev_ptr(sq), MLP_MODE[mode], _stream_ptr(stream)))
            return sq.mean(), g
        work = torch.empty(int(lib().bmhd_mlp_work_bytes(self.H, n)) // 4, dtype=torch.float32, device=x.device)
        _mcheck(lib().bmhd_mlp_backward(_dev_ptr(self.p), self.H, n, _dev_ptr(x), _dev_ptr(t, torch.float32),
                                        _dev_ptr(z), _dev_ptr(y), _dev_ptr(g), _dev_ptr(sq), _dev_ptr(work),
                                        MLP_MODE[mode], _stream_ptr(stream)))
        return sq.mean(), g

    def adam(self, g, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        self.t += 1
        _mcheck(lib().bmhd_mlp_adam(_dev_ptr(self.p), _dev_ptr(self.pb), _dev_ptr(self.m), _dev_ptr(self.v),
                                    _dev_ptr(g), self.n, lr, b1, b2, eps, self.t, _stream_ptr(stream)))
