"""glmrec: point-process GLM connectivity reconstruction on one AMD MI355X.

Python binding of the C ABI in include/glmrec.h (libglmrec.so, HIP for
gfx950).  The functions below keep the C names (`glmr_create`, `glmr_eval`,
...) and only marshal arguments; `Context` wraps them for convenience.
Arrays may be NumPy arrays (host memory) or torch CUDA tensors (device
memory, GLMR_DEVICE); torch is used for device memory and streams only.
"""
from __future__ import annotations

import ctypes
import sys
from typing import Optional

import numpy as np

from . import _lib as L
from ._lib import (GLMR_BF16, GLMR_DEVICE, GLMR_FP8, GLMR_FP32, GLMR_FP64, GLMR_HOST, GLMR_OK,
                   GLMR_NOT_CONVERGED, GlmrError, PRECISIONS)

__all__ = ["Context", "Batch", "GlmrError", "glmr_create", "glmr_destroy", "glmr_set_spikes",
           "glmr_event_slots", "glmr_set_spike_times", "glmr_ei_interval", "glmr_ei_interval_f32", "glmr_set_delays",
           "glmr_get_state", "glmr_set_state",
           "glmr_set_kernel", "glmr_set_kernel_noalloc", "glmr_set_precision", "glmr_set_params", "glmr_get_params", "glmr_eval", "glmr_fit",
           "glmr_fit_defaults", "glmr_status_string", "glmr_last_error", "glmr_query",
           "glmr_batch_create", "glmr_batch_destroy", "glmr_batch_eval", "glmr_batch_get_grad",
           "glmr_batch_fit", "glmr_prof_enable", "glmr_prof_get", "glmr_prof_reset"]


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, where) of a NumPy array or a torch tensor of the given dtype."""
    if x is None:
        return None, None
    if _is_torch(x):
        import torch
        tdt = {np.float64: torch.float64, np.int64: torch.int64, np.int32: torch.int32}[dtype]
        if x.dtype != tdt or not x.is_contiguous():
            raise TypeError(f"tensor must be contiguous {tdt}")
        return ctypes.c_void_p(x.data_ptr()), (GLMR_DEVICE if x.is_cuda else GLMR_HOST)
    a = np.asarray(x)
    if a.dtype != dtype or not a.flags.c_contiguous:
        raise TypeError(f"array must be C-contiguous {np.dtype(dtype)}")
    return ctypes.c_void_p(a.ctypes.data), GLMR_HOST


def _check(status: int, ctx=None):
    if status < 0:
        lib = L.load()
        msg = lib.glmr_status_string(status).decode()
        if ctx is not None:
            detail = lib.glmr_last_error(ctx)
            if detail:
                msg += ": " + detail.decode()
        raise GlmrError(status, msg)
    return status


# ---------------------------------------------------------------- C names

def glmr_create(n_neurons, n_bins, dt, precision="fp32", device=0, stream=None, chunk_bins=0,
                tile_n=0, trace="auto", time_mode="grid"):
    lib = L.load()
    cfg = L.glmr_config(n_neurons, n_bins, dt, chunk_bins, PRECISIONS[precision], device,
                        ctypes.c_void_p(stream) if stream else None, tile_n, L.TRACE_MODES[trace],
                        L.TIME_MODES[time_mode])
    out = ctypes.c_void_p()
    _check(lib.glmr_create(ctypes.byref(cfg), ctypes.byref(out)))
    return out


def glmr_destroy(ctx):
    L.load().glmr_destroy(ctx)


def glmr_set_spikes(ctx, bins, neurons):
    pb, wb = _ptr(bins, np.int64)
    pn, wn = _ptr(neurons, np.int32)
    if wb != wn:
        raise ValueError("bins and neurons must both be host or both be device arrays")
    n = int(bins.shape[0])
    if neurons.shape[0] != n:
        raise ValueError("bins and neurons differ in length")
    _sync_torch(bins)
    return _check(L.load().glmr_set_spikes(ctx, pb, pn, n, wb), ctx)


def glmr_event_slots(times, T0, T1, max_gap=0.0):
    """Slot count of the event grid of the (host) spike times."""
    t = np.ascontiguousarray(times, dtype=np.float64)
    out = ctypes.c_int64()
    _check(L.load().glmr_event_slots(ctypes.c_void_p(t.ctypes.data), int(t.shape[0]), float(T0), float(T1),
                                     float(max_gap), ctypes.byref(out)))
    return out.value


def glmr_set_spike_times(ctx, times, neurons, T0, T1, max_gap=0.0):
    pt, wt = _ptr(times, np.float64)
    pn, wn = _ptr(neurons, np.int32)
    if wt != wn:
        raise ValueError("times and neurons must both be host or both be device arrays")
    n = int(times.shape[0])
    if neurons.shape[0] != n:
        raise ValueError("times and neurons differ in length")
    _sync_torch(times)
    return _check(L.load().glmr_set_spike_times(ctx, pt, pn, n, float(T0), float(T1), float(max_gap), wt), ctx)


def glmr_ei_interval(D, delta):
    """(F, H) of one event-grid interval, by the library's own code on the host."""
    F, H = ctypes.c_double(), ctypes.c_double()
    L.load().glmr_ei_interval(float(D), float(delta), ctypes.byref(F), ctypes.byref(H))
    return F.value, H.value


def glmr_ei_interval_f32(D, delta):
    """(F, H) of one event-grid interval in FP32, as the resident BF16 kernels take it."""
    F, H = ctypes.c_float(), ctypes.c_float()
    L.load().glmr_ei_interval_f32(float(D), float(delta), ctypes.byref(F), ctypes.byref(H))
    return F.value, H.value


def glmr_set_delays(ctx, d_bins, d_self_bins):
    return _check(L.load().glmr_set_delays(ctx, int(d_bins), int(d_self_bins)), ctx)


def glmr_set_kernel(ctx, tau):
    return _check(L.load().glmr_set_kernel(ctx, float(tau)), ctx)


def glmr_set_kernel_noalloc(ctx, tau):
    return _check(L.load().glmr_set_kernel_noalloc(ctx, float(tau)), ctx)


def glmr_set_precision(ctx, precision):
    return _check(L.load().glmr_set_precision(ctx, PRECISIONS[precision]), ctx)


def glmr_set_params(ctx, J, mu):
    pj, wj = _ptr(J, np.float64)
    pm, wm = _ptr(mu, np.float64)
    if wj != wm:
        raise ValueError("J and mu must both be host or both be device arrays")
    _sync_torch(J)
    return _check(L.load().glmr_set_params(ctx, pj, pm, wj), ctx)


def glmr_get_params(ctx, J=None, mu=None):
    """Fill J [N,N] and mu [N] (NumPy or torch float64); returns tau."""
    tau = ctypes.c_double()
    pj, wj = _ptr(J, np.float64)
    pm, wm = _ptr(mu, np.float64)
    where = wj if wj is not None else (wm if wm is not None else GLMR_HOST)
    _check(L.load().glmr_get_params(ctx, pj, pm, ctypes.byref(tau), where), ctx)
    return tau.value


def glmr_eval(ctx, ll_rows=None, grad_J=None, grad_mu=None, want_tau=False):
    """Evaluate into the given output arrays; returns (ll, dll_dtau or None)."""
    ll = ctypes.c_double()
    gt = ctypes.c_double()
    outs = [o for o in (ll_rows, grad_J, grad_mu) if o is not None]
    wheres = {(_ptr(o, np.float64)[1]) for o in outs}
    if len(wheres) > 1:
        raise ValueError("outputs must all be host or all be device arrays")
    where = wheres.pop() if wheres else GLMR_HOST
    st = L.load().glmr_eval(ctx, ctypes.byref(ll), _ptr(ll_rows, np.float64)[0],
                            _ptr(grad_J, np.float64)[0], _ptr(grad_mu, np.float64)[0],
                            ctypes.byref(gt) if want_tau else None, where)
    _check(st, ctx)
    return ll.value, (gt.value if want_tau else None)


def glmr_fit_defaults():
    o = L.glmr_fit_opts()
    L.load().glmr_fit_defaults(ctypes.byref(o))
    return o


def glmr_fit(ctx, opts=None):
    o = opts if opts is not None else glmr_fit_defaults()
    rep = L.glmr_fit_report()
    st = _check(L.load().glmr_fit(ctx, ctypes.byref(o), ctypes.byref(rep)), ctx)
    return st, rep


def glmr_get_state(ctx):
    """The context's checkpoint (parameters, tau, delays, precision, ascent) as bytes."""
    n = ctypes.c_size_t(0)
    _check(L.load().glmr_get_state(ctx, None, ctypes.byref(n)), ctx)
    buf = ctypes.create_string_buffer(n.value)
    _check(L.load().glmr_get_state(ctx, buf, ctypes.byref(n)), ctx)
    return buf.raw[:n.value]


def glmr_set_state(ctx, state: bytes):
    return _check(L.load().glmr_set_state(ctx, bytes(state), len(state)), ctx)


def glmr_status_string(status):
    return L.load().glmr_status_string(status).decode()


def glmr_last_error(ctx):
    return L.load().glmr_last_error(ctx).decode()


def glmr_query(ctx):
    n_pad, b_pad, chunk = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    planes, tile, resident = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(L.load().glmr_query(ctx, ctypes.byref(n_pad), ctypes.byref(b_pad), ctypes.byref(chunk),
                               ctypes.byref(planes), ctypes.byref(tile), ctypes.byref(resident)), ctx)
    return dict(n_pad=n_pad.value, b_pad=b_pad.value, chunk_bins=chunk.value, planes=planes.value,
                tile_n=tile.value, trace_resident=bool(resident.value), trace_frag=resident.value == 2)


def glmr_autotune(ctx, cache_path=None):
    u, g = ctypes.c_int32(), ctypes.c_int32()
    _check(L.load().glmr_autotune(ctx, cache_path.encode() if cache_path else None, ctypes.byref(u),
                                  ctypes.byref(g)), ctx)
    return u.value, g.value


def glmr_prof_enable(ctx, on=True):
    return _check(L.load().glmr_prof_enable(ctx, 1 if on else 0), ctx)


def glmr_prof_reset(ctx):
    L.load().glmr_prof_reset(ctx)


def glmr_prof_get(ctx):
    cap = 32
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_double * cap)()
    n = (ctypes.c_int64 * cap)()
    k = L.load().glmr_prof_get(ctx, names, ms, n, cap)
    return {names[i].decode(): (ms[i], n[i]) for i in range(min(k, cap))}


def glmr_batch_create(ctxs):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs])
    out = ctypes.c_void_p()
    _check(L.load().glmr_batch_create(arr, len(ctxs), ctypes.byref(out)))
    return out


def glmr_batch_destroy(b):
    L.load().glmr_batch_destroy(b)


def glmr_batch_eval(b, n):
    ll = (ctypes.c_double * n)()
    _check(L.load().glmr_batch_eval(b, ll))
    return np.array(ll[:])


def glmr_batch_get_grad(b, r, grad_J=None, grad_mu=None):
    pj, wj = _ptr(grad_J, np.float64)
    pm, wm = _ptr(grad_mu, np.float64)
    where = wj if wj is not None else (wm if wm is not None else GLMR_HOST)
    return _check(L.load().glmr_batch_get_grad(b, r, pj, pm, where))


def glmr_batch_autotune(b, cache_path=None):
    u, g = ctypes.c_int32(), ctypes.c_int32()
    _check(L.load().glmr_batch_autotune(b, cache_path.encode() if cache_path else None, ctypes.byref(u),
                                        ctypes.byref(g)))
    return u.value, g.value


def glmr_batch_fit(b, n, opts=None):
    o = opts if opts is not None else glmr_fit_defaults()
    reps = (L.glmr_fit_report * n)()
    st = _check(L.load().glmr_batch_fit(b, ctypes.byref(o), reps))
    return st, list(reps)


def _sync_torch(x):
    """Device inputs are produced on torch's stream; make them visible to the
    library's stream."""
    if _is_torch(x) and x.is_cuda:
        import torch
        torch.cuda.current_stream(x.device).synchronize()


# -------------------------------------------------------------- convenience

class Context:
    """One recording: N neurons, B bins of width dt, one precision.  With
    time_mode="events" the bins are the slots of the event grid (continuous
    time; see from_events)."""

    def __init__(self, n_neurons: int, n_bins: int, dt: float, precision: str = "fp32",
                 device: int = 0, stream=None, chunk_bins: int = 0, tile_n: int = 0,
                 trace: str = "auto", time_mode: str = "grid"):
        self.N, self.B, self.dt, self.precision = int(n_neurons), int(n_bins), float(dt), precision
        self.time_mode = time_mode
        self._c = glmr_create(self.N, self.B, self.dt, precision, device, stream, chunk_bins, tile_n,
                              trace, time_mode)

    @classmethod
    def from_events(cls, n_neurons: int, times, neurons, T0: float, T1: float, precision: str = "fp64",
                    max_gap: float = 0.0, device: int = 0, stream=None, chunk_bins: int = 0, tile_n: int = 0,
                    trace: str = "auto"):
        """Continuous-time context of spike times (seconds, host arrays sorted by
        (time, neuron)) on [T0, T1); the spikes are set, the kernel is not.
        trace: "auto" keeps the BF16 trace resident when it fits, "recompute"
        rebuilds it inside the contractions."""
        times = np.ascontiguousarray(times, dtype=np.float64)
        neurons = np.ascontiguousarray(neurons, dtype=np.int32)
        slots = glmr_event_slots(times, T0, T1, max_gap)
        c = cls(n_neurons, slots, (T1 - T0) / slots, precision, device, stream, chunk_bins, tile_n,
                trace=trace, time_mode="events")
        c.T0, c.T1, c.max_gap = float(T0), float(T1), float(max_gap)
        c.set_spike_times(times, neurons, T0, T1, max_gap)
        return c

    def set_spike_times(self, times, neurons, T0, T1, max_gap=0.0):
        return glmr_set_spike_times(self._c, times, neurons, T0, T1, max_gap)

    def close(self):
        if self._c is not None and self._c.value:
            glmr_destroy(self._c)
        self._c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._c

    def set_spikes(self, bins, neurons):
        """Returns GLMR_OK or GLMR_ENOSPIKES is raised as GlmrError unless allow_silent."""
        return glmr_set_spikes(self._c, bins, neurons)

    def set_spikes_allow_silent(self, bins, neurons):
        try:
            return glmr_set_spikes(self._c, bins, neurons)
        except GlmrError as e:
            if e.status == L.GLMR_ENOSPIKES:
                return e.status
            raise

    def set_kernel(self, tau: float):
        return glmr_set_kernel(self._c, tau)

    def set_kernel_noalloc(self, tau: float):
        """set_kernel without device allocation (the library's static scratch);
        needs one set_kernel on this context first."""
        return glmr_set_kernel_noalloc(self._c, tau)

    def set_delays(self, d_bins: int, d_self_bins: int):
        """Transmission delays in bins: d on every connection j -> i (j != i),
        d_self on the self-connection (Sec. 2.4, Eq. (15))."""
        return glmr_set_delays(self._c, d_bins, d_self_bins)

    def set_params(self, J, mu):
        return glmr_set_params(self._c, J, mu)

    def set_precision(self, precision: str):
        glmr_set_precision(self._c, precision)
        self.precision = precision

    def get_params(self):
        J = np.zeros((self.N, self.N))
        mu = np.zeros(self.N)
        tau = glmr_get_params(self._c, J, mu)
        return J, mu, tau

    def eval(self, grad: bool = True, rows: bool = True, want_tau: bool = False):
        """Host evaluation: dict(ll, ll_rows, gJ, gmu, gtau)."""
        ll_rows = np.zeros(self.N) if rows else None
        gJ = np.zeros((self.N, self.N)) if grad else None
        gmu = np.zeros(self.N) if grad else None
        ll, gt = glmr_eval(self._c, ll_rows, gJ, gmu, want_tau)
        return dict(ll=ll, ll_rows=ll_rows, gJ=gJ, gmu=gmu, gtau=gt)

    def fit(self, max_iter=500, ftol=0.0, lbfgs_m=40, max_backtracks=30, warm_start_mu=False,
            from_zero=False, polish=None, polish_iter=200, l1_alpha=0.0, l1_eps=0.0, j_max=0.0,
            rate_min=0.0, rate_max=0.0, resume=False, keep_history=False):
        """Per-row L-BFGS ascent.  polish="bf16j2" (BF16 with a two-term J, the
        trace kept) or "fp32" continues a BF16 ascent from the BF16 optimum to
        the exact one (then switches back), starting from the BF16 ascent's
        curvature pairs.  l1_alpha /
        l1_eps: the smooth epsilon-l1 penalty; j_max, rate_min, rate_max: bounds.
        resume=True continues the ascent the context holds (an earlier fit's, or
        one restored by set_state); keep_history=True starts a new ascent from
        the last one's L-BFGS pairs (e.g. after set_precision)."""
        o = glmr_fit_defaults()
        o.max_iter, o.ftol, o.lbfgs_m, o.max_backtracks = max_iter, ftol, lbfgs_m, max_backtracks
        o.warm_start_mu, o.from_zero, o.resume = int(warm_start_mu), int(from_zero), int(resume)
        o.keep_history = int(keep_history)
        o.l1_alpha, o.l1_eps, o.j_max, o.rate_min, o.rate_max = l1_alpha, l1_eps, j_max, rate_min, rate_max
        st, rep = glmr_fit(self._c, o)
        out = dict(status=st, converged=(st == GLMR_OK), iters=rep.iters, evals=rep.evals,
                   ll=rep.ll, max_eta=rep.max_eta, rows_converged=rep.rows_converged,
                   seconds=rep.seconds)
        if polish and polish != self.precision:
            prec0 = self.precision
            self.set_precision(polish)
            o.max_iter, o.from_zero, o.warm_start_mu, o.ftol = polish_iter, 0, 0, 0.0
            o.resume, o.keep_history = 0, 1
            st2, rep2 = glmr_fit(self._c, o)
            self.set_precision(prec0)
            out.update(status=st2, converged=(st2 == GLMR_OK), polish_iters=rep2.iters,
                       polish_evals=rep2.evals, ll=rep2.ll, max_eta=rep2.max_eta,
                       rows_converged=rep2.rows_converged, seconds=out["seconds"] + rep2.seconds)
        return out

    def get_state(self) -> bytes:
        """Checkpoint: parameters, tau, delays, precision and the ascent's state."""
        return glmr_get_state(self._c)

    def set_state(self, state: bytes):
        """Restore a checkpoint of this recording; fit(resume=True) then continues it."""
        glmr_set_state(self._c, state)
        # the head's precision field (after magic, N, time mode, n_bins, dt, tau, d, d_self)
        code = int.from_bytes(bytes(state[56:60]), sys.byteorder, signed=True)
        self.precision = {v: k for k, v in PRECISIONS.items()}[code]

    def query(self):
        return glmr_query(self._c)

    def autotune(self, cache_path=None):
        """Pick the fastest tile shapes for this context's sizes (see glmr_autotune)."""
        return glmr_autotune(self._c, cache_path)

    def prof(self, on=True):
        glmr_prof_enable(self._c, on)

    def prof_get(self):
        return glmr_prof_get(self._c)

    def prof_reset(self):
        glmr_prof_reset(self._c)


class Batch:
    """Several contexts evaluated and fitted together."""

    def __init__(self, ctxs):
        self.ctxs = list(ctxs)
        self._b = glmr_batch_create([c.handle for c in self.ctxs])

    def close(self):
        if self._b is not None and self._b.value:
            glmr_batch_destroy(self._b)
        self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval(self):
        return glmr_batch_eval(self._b, len(self.ctxs))

    def autotune(self, cache_path=None):
        """Pick the fastest tile shapes of the grouped launches (see glmr_batch_autotune)."""
        return glmr_batch_autotune(self._b, cache_path)

    def grad(self, r):
        c = self.ctxs[r]
        gJ = np.zeros((c.N, c.N))
        gmu = np.zeros(c.N)
        glmr_batch_get_grad(self._b, r, gJ, gmu)
        return gJ, gmu

    def fit(self, max_iter=500, ftol=0.0, lbfgs_m=40, max_backtracks=30, warm_start_mu=False,
            from_zero=False, l1_alpha=0.0, l1_eps=0.0, j_max=0.0, rate_min=0.0, rate_max=0.0,
            resume=False):
        o = glmr_fit_defaults()
        o.max_iter, o.ftol, o.lbfgs_m, o.max_backtracks = max_iter, ftol, lbfgs_m, max_backtracks
        o.warm_start_mu, o.from_zero, o.resume = int(warm_start_mu), int(from_zero), int(resume)
        o.l1_alpha, o.l1_eps, o.j_max, o.rate_min, o.rate_max = l1_alpha, l1_eps, j_max, rate_min, rate_max
        st, reps = glmr_batch_fit(self._b, len(self.ctxs), o)
        return st, [dict(iters=r.iters, evals=r.evals, ll=r.ll, max_eta=r.max_eta,
                         rows_converged=r.rows_converged, seconds=r.seconds) for r in reps]
