"""Python binding of libgwlike (the C ABI in include/gwlike.h): argument marshalling only.

Every computation runs in the HIP library; this module checks tensor placement, dtype and
shape, passes device pointers and the current HIP stream, and raises on a non-zero status.
It fails loudly if the compiled library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import collections
import ctypes
import os
import weakref
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgwlike.so")

GWL_FP64 = 0
GWL_MIXED = 1
GWL_F_ISCO_CUTOFF = 1
NPARAM = 11
MAX_DET = 4

_c_double_p = ctypes.POINTER(ctypes.c_double)


class Detector(ctypes.Structure):
    """An L-shaped detector: latitude, longitude, x- and y-arm azimuths (rad, clockwise from North)."""
    _fields_ = [("lat", ctypes.c_double), ("lon", ctypes.c_double),
                ("xarm_az", ctypes.c_double), ("yarm_az", ctypes.c_double)]


class GWLError(RuntimeError):
    def __init__(self, func: str, status: int, msg: str):
        super().__init__(f"{func} returned {status}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libgwlike.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first (python -c "
                           f"'import __graft_entry__ as g; g.build()'); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, cint = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    sig = {
        "gwl_last_error": ([], ctypes.c_char_p),
        "gwl_version": ([], ctypes.c_char_p),
        "gwl_event_create": ([vp, vp, ctypes.POINTER(Detector), cint, vp, i64, dbl, dbl, ctypes.c_uint, vp,
                              ctypes.POINTER(vp)], cint),
        "gwl_event_destroy": ([vp], cint),
        "gwl_event_create_rb": ([vp, vp, ctypes.POINTER(Detector), cint, vp, i64, dbl, dbl, _c_double_p, dbl,
                                 ctypes.c_uint, vp, ctypes.POINTER(vp)], cint),
        "gwl_event_rb_info": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64)], cint),
        "gwl_event_create_cal": ([vp, vp, ctypes.POINTER(Detector), cint, vp, i64, dbl, dbl, cint, ctypes.c_uint, vp,
                                  ctypes.POINTER(vp)], cint),
        "gwl_event_create_rb_cal": ([vp, vp, ctypes.POINTER(Detector), cint, vp, i64, dbl, dbl, _c_double_p, dbl, cint,
                                     ctypes.c_uint, vp, ctypes.POINTER(vp)], cint),
        "gwl_event_info": ([vp, ctypes.POINTER(cint), ctypes.POINTER(i64), ctypes.POINTER(dbl)], cint),
        "gwl_logl_batch": ([vp, vp, i64, cint, vp, vp], cint),
        "gwl_logl_grad": ([vp, vp, i64, cint, vp, vp, vp], cint),
        "gwl_waveform": ([vp, i64, ctypes.POINTER(Detector), cint, vp, i64, dbl, vp, vp], cint),
        "gwl_multi_plan_create": ([ctypes.POINTER(vp), cint, ctypes.POINTER(i64), cint, cint, ctypes.POINTER(vp)],
                                  cint),
        "gwl_multi_plan_create_order": ([ctypes.POINTER(vp), cint, ctypes.POINTER(i64), cint, cint, cint,
                                         ctypes.POINTER(vp)], cint),
        "gwl_multi_launch": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), _c_double_p, vp],
                             cint),
        "gwl_plan_destroy": ([vp], cint),
        "gwl_plan_info": ([vp, ctypes.POINTER(cint), ctypes.POINTER(cint), ctypes.POINTER(i64)], cint),
        "gwl_multi_autotune": ([ctypes.c_char_p, ctypes.POINTER(vp), cint, ctypes.POINTER(i64), cint, cint], cint),
        "gwl_autotune": ([ctypes.c_char_p, vp, i64, cint, cint], cint),
        "gwl_autotune_load": ([ctypes.c_char_p], cint),
        "gwl_launch_shape": ([vp, i64, cint, cint, ctypes.POINTER(cint), ctypes.POINTER(cint)], cint),
        "gwl_event_reserve": ([vp, i64, cint, cint, vp], cint),
        "gwl_launch_layout": ([vp, i64, cint, cint, ctypes.POINTER(cint), ctypes.POINTER(cint), ctypes.POINTER(cint)],
                              cint),
        "gwl_logl_batch_noalloc": ([vp, vp, i64, cint, vp, vp], cint),
        "gwl_profile_enable": ([cint], cint),
        "gwl_profile_read": ([ctypes.POINTER(i64), ctypes.POINTER(dbl)], cint),
        "gwl_logl_batch_live": ([vp, vp, i64, vp, cint, vp, vp], cint),
        "gwl_slice_ends": ([i64, cint, cint] + [vp] * 9 + [vp], cint),
        "gwl_slice_ends_select": ([i64, cint, cint] + [vp] * 7 + [vp], cint),
        "gwl_slice_list_init": ([i64, vp, vp, vp], cint),
        "gwl_slice_move_begin": ([i64, cint] + [vp] * 5 + [vp], cint),
        "gwl_slice_move_end": ([i64, cint] + [vp] * 4 + [vp], cint),
        "gwl_slice_draws": ([i64, cint, cint] + [vp] * 14 + [vp], cint),
        "gwl_slice_select": ([i64, cint, cint] + [vp] * 15 + [vp], cint),
        "gwl_prior_transform": ([i64, cint] + [vp] * 5 + [vp], cint),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(func: str, status: int) -> None:
    if status != 0:
        raise GWLError(func, status, lib().gwl_last_error().decode(errors="replace"))


def _prec(precision) -> int:
    if precision in ("mixed", GWL_MIXED):
        return GWL_MIXED
    if precision in ("fp64", "f64", "double", GWL_FP64):
        return GWL_FP64
    raise ValueError(f"precision must be 'mixed' or 'fp64', not {precision!r}")


def _stream(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dev(t: torch.Tensor, name: str, dtype: torch.dtype) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return t.contiguous()


def _dets(dets) -> "ctypes.Array[Detector]":
    rows = [tuple(float(v) for v in d) for d in dets]
    arr = (Detector * max(1, len(rows)))()
    for i, r in enumerate(rows):
        if len(r) != 4:
            raise ValueError("each detector is (lat, lon, xarm_az, yarm_az) in radians")
        arr[i] = Detector(*r)
    return arr, len(rows)


class Event:
    """One segment seen by several detectors: the library's prepared per-bin tables.

    data  complex128 CUDA tensor [ndet, M];  psd float64 CUDA [ndet, M];  fgrid float64 CUDA [M];
    dets  [ndet] x (lat, lon, xarm_az, yarm_az) radians;  df = 1/T;  gmst in radians.
    fiducial  optional 11 parameters: relative binning against that waveform, with edges spaced
              rb_eps radians of the phase bound apart (see gwl_event_create_rb).
    calibration_nodes  optional n >= 4: a calibration model per detector (see gwl_event_create_cal);
              theta then has 11 + 2 n ndet columns.
    isco_cutoff  the model is zero above each point's ISCO frequency (GWL_F_ISCO_CUTOFF).
    """

    def __init__(self, data: torch.Tensor, psd: torch.Tensor, dets: Sequence, fgrid: torch.Tensor, df: float,
                 gmst: float = 0.0, fiducial=None, rb_eps: float = 0.1, calibration_nodes: int = 0,
                 isco_cutoff: bool = False):
        data = _dev(data, "data", torch.complex128)
        psd = _dev(psd, "psd", torch.float64)
        fgrid = _dev(fgrid, "fgrid", torch.float64)
        darr, nd = _dets(dets)
        if data.dim() != 2 or psd.shape != data.shape or fgrid.shape != (data.shape[1],) or data.shape[0] != nd:
            raise ValueError("shapes must be data [ndet, M], psd [ndet, M], fgrid [M] with ndet = len(dets)")
        self.ndet, self.M, self.df, self.gmst = nd, int(data.shape[1]), float(df), float(gmst)
        self.device = data.device
        h = ctypes.c_void_p()
        self.ncal = int(calibration_nodes)
        if isco_cutoff and (self.ncal or fiducial is not None):
            raise ValueError("the ISCO cut-off is available on plain events only")
        if self.ncal and fiducial is not None:
            fid = [float(x) for x in fiducial]
            if len(fid) != NPARAM:
                raise ValueError("fiducial must have 11 parameters")
            fid = (ctypes.c_double * NPARAM)(*fid)
            _check("gwl_event_create_rb_cal", lib().gwl_event_create_rb_cal(
                ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(psd.data_ptr()), darr, nd,
                ctypes.c_void_p(fgrid.data_ptr()), self.M, self.df, self.gmst, fid, float(rb_eps), self.ncal, 0,
                _stream(data), ctypes.byref(h)))
        elif self.ncal:
            _check("gwl_event_create_cal", lib().gwl_event_create_cal(
                ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(psd.data_ptr()), darr, nd,
                ctypes.c_void_p(fgrid.data_ptr()), self.M, self.df, self.gmst, self.ncal, 0, _stream(data),
                ctypes.byref(h)))
        elif fiducial is None:
            _check("gwl_event_create", lib().gwl_event_create(
                ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(psd.data_ptr()), darr, nd,
                ctypes.c_void_p(fgrid.data_ptr()), self.M, self.df, self.gmst, GWL_F_ISCO_CUTOFF if isco_cutoff else 0,
                _stream(data), ctypes.byref(h)))
        else:
            fid = [float(x) for x in fiducial]
            if len(fid) != NPARAM:
                raise ValueError("fiducial must have 11 parameters")
            fid = (ctypes.c_double * NPARAM)(*fid)
            _check("gwl_event_create_rb", lib().gwl_event_create_rb(
                ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(psd.data_ptr()), darr, nd,
                ctypes.c_void_p(fgrid.data_ptr()), self.M, self.df, self.gmst, fid, float(rb_eps), 0, _stream(data),
                ctypes.byref(h)))
        self._h = h
        self.rb_edges = self.rb_info()[0]

    def rb_info(self):
        """(number of relative-binning edges or 0, number of grid bins)."""
        ne, nb = ctypes.c_int64(), ctypes.c_int64()
        _check("gwl_event_rb_info", lib().gwl_event_rb_info(self.handle, ctypes.byref(ne), ctypes.byref(nb)))
        return ne.value, nb.value

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise ValueError("event is closed")
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().gwl_event_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _theta(theta: torch.Tensor, ev: Optional["Event"] = None) -> torch.Tensor:
    theta = _dev(theta, "theta", torch.float64)
    width = NPARAM + (2 * ev.ncal * ev.ndet if ev is not None else 0)
    if theta.dim() != 2 or theta.shape[1] != width:
        raise ValueError(f"theta must be [B, {width}]")
    return theta


def logl(theta: torch.Tensor, ev: Event, precision="mixed") -> torch.Tensor:
    """logL[B] for theta[B, 11] (float64 CUDA; 11 + 2 n ndet columns on a calibrated event)."""
    theta = _theta(theta, ev)
    out = torch.empty(theta.shape[0], dtype=torch.float64, device=theta.device)
    _check("gwl_logl_batch", lib().gwl_logl_batch(ev.handle, ctypes.c_void_p(theta.data_ptr()), theta.shape[0],
                                                  _prec(precision), ctypes.c_void_p(out.data_ptr()), _stream(theta)))
    return out


def logl_live(theta: torch.Tensor, live: torch.Tensor, ev: Event, precision="mixed",
              out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """logL of the first `live` rows of theta[B, 11], live a device int64 scalar read when the
    kernels run (gwl_logl_batch_live); the other entries of the result are left as they were."""
    theta = _theta(theta, ev)
    if not (isinstance(live, torch.Tensor) and live.is_cuda and live.dtype == torch.int64 and live.numel() == 1):
        raise ValueError("live must be a CUDA int64 tensor with one element")
    if out is None:
        out = torch.empty(theta.shape[0], dtype=torch.float64, device=theta.device)
    _check("gwl_logl_batch_live", lib().gwl_logl_batch_live(ev.handle, _ptr(theta), theta.shape[0], _ptr(live),
                                                            _prec(precision), _ptr(out), _stream(theta)))
    return out


def logl_grad(theta: torch.Tensor, ev: Event, precision="mixed"):
    """(logL[B], dlogL/dtheta[B, P]), P the width of theta."""
    theta = _theta(theta, ev)
    out = torch.empty(theta.shape[0], dtype=torch.float64, device=theta.device)
    grad = torch.empty_like(theta)
    _check("gwl_logl_grad", lib().gwl_logl_grad(ev.handle, ctypes.c_void_p(theta.data_ptr()), theta.shape[0],
                                                _prec(precision), ctypes.c_void_p(out.data_ptr()),
                                                ctypes.c_void_p(grad.data_ptr()), _stream(theta)))
    return out, grad


# one-shot calls: events built on first use and kept for the same (live) input tensors
_EVENT_CACHE: "collections.OrderedDict" = collections.OrderedDict()
_EVENT_CACHE_MAX = 8


def _cached_event(data, psd, dets, fgrid, df, gmst) -> Event:
    dets_key = tuple(tuple(float(x) for x in d) for d in dets)
    key = (data.data_ptr(), data._version, psd.data_ptr(), psd._version, fgrid.data_ptr(), fgrid._version,
           dets_key, float(df) if df is not None else None, float(gmst))
    hit = _EVENT_CACHE.get(key)
    if hit is not None:
        refs, ev = hit
        if all(r() is t for r, t in zip(refs, (data, psd, fgrid))):   # the same tensors, still alive
            _EVENT_CACHE.move_to_end(key)
            return ev
        del _EVENT_CACHE[key]
    if df is None:
        df = float(fgrid[1] - fgrid[0]) if fgrid.numel() > 1 else 1.0
    ev = Event(data, psd, dets, fgrid, df, gmst)
    _EVENT_CACHE[key] = ((weakref.ref(data), weakref.ref(psd), weakref.ref(fgrid)), ev)
    while len(_EVENT_CACHE) > _EVENT_CACHE_MAX:
        _EVENT_CACHE.popitem(last=False)[1][1].close()
    return ev


def logl_batch(theta: torch.Tensor, data: torch.Tensor, psd: torch.Tensor, dets: Sequence, fgrid: torch.Tensor,
               df: Optional[float] = None, precision="mixed", gmst: float = 0.0) -> torch.Tensor:
    """One-shot logL[B]: the event tables are built on the first call for these data, PSD and
    grid tensors and reused while the same tensors are passed again (df defaults to the grid step)."""
    return logl(theta, _cached_event(data, psd, dets, fgrid, df, gmst), precision)


def logl_grad_batch(theta: torch.Tensor, data: torch.Tensor, psd: torch.Tensor, dets: Sequence,
                    fgrid: torch.Tensor, df: Optional[float] = None, precision="mixed", gmst: float = 0.0):
    """One-shot (logL[B], dlogL/dtheta[B, 11]), with the same event reuse as logl_batch."""
    return logl_grad(theta, _cached_event(data, psd, dets, fgrid, df, gmst), precision)


class LogL(torch.autograd.Function):
    """logL as a differentiable function of theta; the adjoint is computed in the forward pass."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, ev: Event, precision="mixed"):
        if ctx.needs_input_grad[0]:
            val, g = logl_grad(theta.detach(), ev, precision)
            ctx.save_for_backward(g)
        else:
            val = logl(theta.detach(), ev, precision)
        return val

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out[:, None] * g, None, None


def waveform(theta: torch.Tensor, dets: Sequence, fgrid: torch.Tensor, gmst: float = 0.0) -> torch.Tensor:
    """Model strain h_det(f_k): complex128 [B, ndet, M] on the theta's device."""
    theta = _theta(theta)
    fgrid = _dev(fgrid, "fgrid", torch.float64)
    darr, nd = _dets(dets)
    M = int(fgrid.shape[0])
    out = torch.empty(theta.shape[0], nd, M, dtype=torch.complex128, device=theta.device)
    _check("gwl_waveform", lib().gwl_waveform(ctypes.c_void_p(theta.data_ptr()), theta.shape[0], darr, nd,
                                              ctypes.c_void_p(fgrid.data_ptr()), M, float(gmst),
                                              ctypes.c_void_p(out.data_ptr()), _stream(theta)))
    return out


class MultiPlan:
    """Many events of uneven size evaluated by one persistent launch captured in a HIP graph.

    events   list of Event (same detector count, same device); batches: points per event.
    launch(thetas) takes one float64 CUDA tensor [B_e, P_e] per event (P_e = 11, or 11 + 2 n ndet
    on a calibrated event, whose own kernels run after the persistent launch) and returns
    (logls, grads or None, latency_us or None). order: "tuned" (the autotuner's queue order),
    "ascending" (small events first) or "descending" (large events first).
    """

    ORDERS = {"tuned": 0, "ascending": 1, "descending": 2}

    def __init__(self, events: Sequence[Event], batches: Sequence[int], precision="mixed", with_grad: bool = False,
                 order: str = "tuned"):
        if order not in self.ORDERS:
            raise ValueError(f"order must be one of {sorted(self.ORDERS)}")
        self.events = list(events)
        self.batches = [int(b) for b in batches]
        if len(self.events) != len(self.batches) or not self.events:
            raise ValueError("one batch size per event is required")
        self.with_grad = bool(with_grad)
        E = len(self.events)
        evs = (ctypes.c_void_p * E)(*[ev.handle.value for ev in self.events])
        bs = (ctypes.c_int64 * E)(*self.batches)
        h = ctypes.c_void_p()
        _check("gwl_multi_plan_create_order", lib().gwl_multi_plan_create_order(evs, E, bs, _prec(precision),
                                                                                int(self.with_grad),
                                                                                self.ORDERS[order], ctypes.byref(h)))
        self._h = h

    def launch(self, thetas: Sequence[torch.Tensor], latency: bool = False):
        E = len(self.events)
        if len(thetas) != E:
            raise ValueError("one theta tensor per event is required")
        thetas = [_theta(t, ev) for t, ev in zip(thetas, self.events)]
        for t, b in zip(thetas, self.batches):
            if t.shape[0] != b:
                raise ValueError("theta batch sizes must match the plan")
        dev = thetas[0].device
        logls = [torch.empty(b, dtype=torch.float64, device=dev) for b in self.batches]
        grads = [torch.empty_like(t) for t in thetas] if self.with_grad else None
        tp = (ctypes.c_void_p * E)(*[t.data_ptr() for t in thetas])
        lp = (ctypes.c_void_p * E)(*[t.data_ptr() for t in logls])
        gp = (ctypes.c_void_p * E)(*[t.data_ptr() for t in grads]) if grads is not None else None
        lat = (ctypes.c_double * E)() if latency else None
        _check("gwl_multi_launch", lib().gwl_multi_launch(self._h, tp, lp, gp, lat, _stream(thetas[0])))
        # keep the inputs alive until the stream has consumed them
        self._last = (thetas, logls, grads)
        return logls, grads, (list(lat) if latency else None)

    def info(self):
        """(chunk length in bins, queued by descending work, number of work items)."""
        c, d, n = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        _check("gwl_plan_info", lib().gwl_plan_info(self._h, ctypes.byref(c), ctypes.byref(d), ctypes.byref(n)))
        return c.value, bool(d.value), n.value

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().gwl_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(ev: Event, batch: int, precision="mixed", with_grad: bool = False,
             cache_path: Optional[str] = None) -> None:
    """Time tile shapes for this event and batch size; record the best (in memory and in cache_path)."""
    path = cache_path.encode() if cache_path else None
    _check("gwl_autotune", lib().gwl_autotune(path, ev.handle, int(batch), _prec(precision), int(bool(with_grad))))


def multi_autotune(events: Sequence[Event], batches: Sequence[int], precision="mixed", with_grad: bool = False,
                   cache_path: Optional[str] = None) -> None:
    """Time multi-event plan shapes for this workload; MultiPlan then uses the fastest."""
    E = len(events)
    if E == 0 or len(batches) != E:
        raise ValueError("one batch size per event is required")
    evs = (ctypes.c_void_p * E)(*[ev.handle.value for ev in events])
    bs = (ctypes.c_int64 * E)(*[int(b) for b in batches])
    path = cache_path.encode() if cache_path else None
    _check("gwl_multi_autotune", lib().gwl_multi_autotune(path, evs, E, bs, _prec(precision), int(bool(with_grad))))


def launch_shape(ev: Event, batch: int, precision="mixed", with_grad: bool = False):
    """(number of bin chunks, chunk length in bins) that a call with these arguments would use."""
    n, c = ctypes.c_int(), ctypes.c_int()
    _check("gwl_launch_shape", lib().gwl_launch_shape(ev.handle, int(batch), _prec(precision), int(bool(with_grad)),
                                                      ctypes.byref(n), ctypes.byref(c)))
    return n.value, c.value


def reserve(ev: Event, batch: int, precision="mixed", with_grad: bool = False, stream=None) -> None:
    """Grow the event's workspace on `stream` (default: the current stream) for calls of this size,
    so that they allocate nothing, also under graph capture (gwl_event_reserve)."""
    if stream is None:
        stream = torch.cuda.current_stream(ev.device)
    _check("gwl_event_reserve", lib().gwl_event_reserve(ev.handle, int(batch), _prec(precision), int(bool(with_grad)),
                                                        ctypes.c_void_p(stream.cuda_stream)))


def launch_layout(ev: Event, batch: int, precision="mixed", with_grad: bool = False):
    """(wavefronts per workgroup, workgroups per point group, set-up inside the kernel) of a call."""
    w, g, st = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check("gwl_launch_layout", lib().gwl_launch_layout(ev.handle, int(batch), _prec(precision), int(bool(with_grad)),
                                                        ctypes.byref(w), ctypes.byref(g), ctypes.byref(st)))
    return w.value, g.value, bool(st.value)


def autotune_load(cache_path: str) -> None:
    _check("gwl_autotune_load", lib().gwl_autotune_load(cache_path.encode()))


def profile_enable(on: bool = True) -> None:
    """Bracket every bin-loop launch with HIP events on its stream (measurement aid)."""
    _check("gwl_profile_enable", lib().gwl_profile_enable(int(bool(on))))


def profile_read():
    """(launches, total_ms) of the bin-loop launches bracketed since the previous read."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check("gwl_profile_read", lib().gwl_profile_read(ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def version() -> str:
    return lib().gwl_version().decode()


# ---- slice-sampling bookkeeping (gwl_slice_*): n chains in d dimensions -----------------------
def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _f64(t: torch.Tensor, name: str, shape) -> torch.Tensor:
    t = _dev(t, name, torch.float64)
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, not {tuple(t.shape)}")
    return t


def slice_ends(x: torch.Tensor, dirn: torch.Tensor, u0: torch.Tensor, u1: torch.Tensor, m: int):
    """(pts[(m - 1) n, d], lo, hi, jl, jr): the initial interval of every chain and the m - 1 ends
    its stepping out may examine (slot s of chain i at row s n + i)."""
    n, d = x.shape
    x, dirn = _f64(x, "x", (n, d)), _f64(dirn, "dirn", (n, d))
    u0, u1 = _f64(u0, "u0", (n,)), _f64(u1, "u1", (n,))
    pts = torch.empty(max(m - 1, 0) * n, d, dtype=torch.float64, device=x.device)
    lo, hi, jl, jr = (torch.empty(n, dtype=torch.float64, device=x.device) for _ in range(4))
    _check("gwl_slice_ends", lib().gwl_slice_ends(n, d, m, _ptr(x), _ptr(dirn), _ptr(u0), _ptr(u1), _ptr(pts),
                                                  _ptr(lo), _ptr(hi), _ptr(jl), _ptr(jr), _stream(x)))
    return pts, lo, hi, jl, jr


def slice_ends_select(pts, logl, lmin, lo, hi, jl, jr, m: int) -> None:
    """Steps the interval ends out (in place on lo, hi) given ln L at the m - 1 slots."""
    n = lo.shape[0]
    d = pts.shape[1]
    for t, name in ((lo, "lo"), (hi, "hi")):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.shape == (n,)):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape ({n},)")
    pts, logl = _f64(pts, "pts", ((m - 1) * n, d)), _f64(logl, "logl", ((m - 1) * n,))
    lmin, jl, jr = _f64(lmin, "lmin", ()), _f64(jl, "jl", (n,)), _f64(jr, "jr", (n,))
    _check("gwl_slice_ends_select", lib().gwl_slice_ends_select(n, d, m, _ptr(pts), _ptr(logl), _ptr(lmin), _ptr(lo),
                                                                _ptr(hi), _ptr(jl), _ptr(jr), _stream(pts)))


def _list(lst, nact, n):
    if not (isinstance(lst, torch.Tensor) and lst.is_cuda and lst.dtype == torch.int32 and lst.is_contiguous()
            and tuple(lst.shape) == (n,)):
        raise ValueError(f"a chain list must be a contiguous int32 CUDA tensor of shape ({n},)")
    if not (isinstance(nact, torch.Tensor) and nact.is_cuda and nact.dtype == torch.int64 and nact.numel() == 1):
        raise ValueError("a list length must be a CUDA int64 tensor with one element")


def slice_list_init(n: int, device, lst: Optional[torch.Tensor] = None, nact: Optional[torch.Tensor] = None):
    """(list, nact): the list of all n chains (int32) and its length (int64 device scalar)."""
    lst = torch.empty(n, dtype=torch.int32, device=device) if lst is None else lst
    nact = torch.empty((), dtype=torch.int64, device=device) if nact is None else nact
    _list(lst, nact, n)
    _check("gwl_slice_list_init", lib().gwl_slice_list_init(n, _ptr(lst), _ptr(nact), _stream(lst)))
    return lst, nact


def _flags(t, name, n):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.bool and t.is_contiguous()
            and tuple(t.shape) == (n,)):
        raise ValueError(f"{name} must be a contiguous bool CUDA tensor of shape ({n},)")


def slice_move_begin(x, xn, done, lst: Optional[torch.Tensor] = None, nact: Optional[torch.Tensor] = None):
    """The start of a move in one launch: xn = x, done = False, and the list of all chains.
    Returns (list, nact)."""
    n, d = x.shape
    x, xn = _f64(x, "x", (n, d)), _f64(xn, "xn", (n, d))
    _flags(done, "done", n)
    lst = torch.empty(n, dtype=torch.int32, device=x.device) if lst is None else lst
    nact = torch.empty((), dtype=torch.int64, device=x.device) if nact is None else nact
    _list(lst, nact, n)
    _check("gwl_slice_move_begin", lib().gwl_slice_move_begin(n, d, _ptr(x), _ptr(xn), _ptr(done), _ptr(lst),
                                                              _ptr(nact), _stream(x)))
    return lst, nact


def slice_move_end(done, moved, xn, x) -> None:
    """The end of a move in one launch: moved |= done, x = xn."""
    n, d = x.shape
    x, xn = _f64(x, "x", (n, d)), _f64(xn, "xn", (n, d))
    _flags(done, "done", n)
    _flags(moved, "moved", n)
    _check("gwl_slice_move_end", lib().gwl_slice_move_end(n, d, _ptr(done), _ptr(moved), _ptr(xn), _ptr(x),
                                                          _stream(x)))


def slice_draws(x, dirn, lo, hi, u, lst, nact, calls: Optional[torch.Tensor] = None):
    """(t[n G], pts[G n, d], a, b, live, nact_next): G shrinkage draws for each listed chain
    (list entry j's draw k at row j G + k), each taken as if the earlier ones had fallen outside;
    live = nact G (device), added to `calls` if given; nact_next is cleared for the selection."""
    n, d = x.shape
    G = u.shape[0]
    x, dirn = _f64(x, "x", (n, d)), _f64(dirn, "dirn", (n, d))
    lo, hi, u = _f64(lo, "lo", (n,)), _f64(hi, "hi", (n,)), _f64(u, "u", (G, n))
    _list(lst, nact, n)
    if calls is not None and not (calls.is_cuda and calls.dtype == torch.int64 and calls.numel() == 1):
        raise ValueError("calls must be a CUDA int64 tensor with one element")
    t = torch.empty(n * G, dtype=torch.float64, device=x.device)
    pts = torch.empty(G * n, d, dtype=torch.float64, device=x.device)
    a, b = torch.empty_like(lo), torch.empty_like(lo)
    live, nact_next = (torch.empty((), dtype=torch.int64, device=x.device) for _ in range(2))
    _check("gwl_slice_draws", lib().gwl_slice_draws(n, d, G, _ptr(lst), _ptr(nact), _ptr(x), _ptr(dirn), _ptr(lo),
                                                    _ptr(hi), _ptr(u), _ptr(t), _ptr(pts), _ptr(a), _ptr(b),
                                                    _ptr(live), _ptr(nact_next),
                                                    _ptr(calls) if calls is not None else None, _stream(x)))
    return t, pts, a, b, live, nact_next


def slice_select(x, dirn, t, logl, lmin, a, b, xn, done, lo, hi, lst, nact, nact_next,
                 list_next: Optional[torch.Tensor] = None):
    """For every listed chain not done: the first draw inside the region becomes its point (xn,
    done); otherwise its interval becomes (a, b) and it joins the next list. In place on xn, done,
    lo, hi; returns the next list (its length in nact_next, which slice_draws cleared)."""
    n, d = x.shape
    G = t.shape[0] // n
    for v, name, shape, dt in ((xn, "xn", (n, d), torch.float64), (done, "done", (n,), torch.bool),
                               (lo, "lo", (n,), torch.float64), (hi, "hi", (n,), torch.float64)):
        if not (v.is_cuda and v.dtype == dt and v.is_contiguous() and tuple(v.shape) == shape):
            raise ValueError(f"{name} must be a contiguous {dt} CUDA tensor of shape {shape}")
    x, dirn, t = _f64(x, "x", (n, d)), _f64(dirn, "dirn", (n, d)), _f64(t, "t", (n * G,))
    lmin = _f64(lmin, "lmin", ())
    if logl.dtype != torch.float64 or not logl.is_cuda or logl.dim() != 1 or logl.shape[0] > G * n \
            or not logl.is_contiguous():
        raise ValueError(f"logl must be a contiguous float64 CUDA tensor of at most {G * n} values")
    a, b = _f64(a, "a", (n,)), _f64(b, "b", (n,))
    _list(lst, nact, n)
    list_next = torch.empty(n, dtype=torch.int32, device=x.device) if list_next is None else list_next
    _list(list_next, nact_next, n)
    _check("gwl_slice_select", lib().gwl_slice_select(n, d, G, _ptr(lst), _ptr(nact), _ptr(x), _ptr(dirn), _ptr(t),
                                                      _ptr(logl), _ptr(lmin), _ptr(a), _ptr(b), _ptr(xn), _ptr(done),
                                                      _ptr(lo), _ptr(hi), _ptr(list_next), _ptr(nact_next),
                                                      _stream(x)))
    return list_next


MAP_LINEAR, MAP_CBRT, MAP_ASIN, MAP_ACOS = 0, 1, 2, 3


class PriorColumns:
    """The per-column maps and coefficients of gwl_prior_transform, held as the host arrays the
    call copies (built once, reused by every call)."""

    def __init__(self, maps, c0, c1):
        d = len(maps)
        if not (len(c0) == len(c1) == d) or not 1 <= d <= 64:
            raise ValueError("maps, c0 and c1 must have the same length, 1 to 64")
        if any(int(m) not in (MAP_LINEAR, MAP_CBRT, MAP_ASIN, MAP_ACOS) for m in maps):
            raise ValueError(f"unknown map code in {list(maps)}")
        self.d = d
        self.maps = (ctypes.c_int * d)(*[int(m) for m in maps])
        self.c0 = (ctypes.c_double * d)(*[float(x) for x in c0])
        self.c1 = (ctypes.c_double * d)(*[float(x) for x in c1])
        self.ptrs = tuple(ctypes.cast(a, ctypes.c_void_p) for a in (self.maps, self.c0, self.c1))


def prior_transform(u: torch.Tensor, cols: PriorColumns) -> torch.Tensor:
    """theta[n, d] = g_j(c0_j + c1_j clamp(u, 0, 1)) column by column (gwl_prior_transform)."""
    if u.dim() != 2 or u.shape[1] != cols.d:
        raise ValueError(f"u must have shape (n, {cols.d}), not {tuple(u.shape)}")
    u = _dev(u, "u", torch.float64)
    theta = torch.empty_like(u)
    _check("gwl_prior_transform", lib().gwl_prior_transform(u.shape[0], cols.d, *cols.ptrs, _ptr(u), _ptr(theta),
                                                            _stream(u)))
    return theta
