"""ctypes binding over libumi.so (include/umi.h).

Argument marshalling only: every step of the estimate runs in the HIP
kernels.  torch supplies device memory and the current HIP stream.  If the
library has not been built, importing this module raises immediately.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libumi.so")

UMI_OK = 0
UMI_ERR_INVALID_ARG = 1
UMI_ERR_NO_MEMORY = 2
UMI_ERR_DEVICE = 3
UMI_ERR_UNSUPPORTED = 4
STATUS_NAMES = {0: "UMI_OK", 1: "UMI_ERR_INVALID_ARG", 2: "UMI_ERR_NO_MEMORY",
                3: "UMI_ERR_DEVICE", 4: "UMI_ERR_UNSUPPORTED"}
MODE_PERSISTENT = 0
MODE_PER_CURVE = 1
MAX_WINDOW = 2047
SCALES = {"upper_rms": 0, "mad": 1}  # umi_scale
# Table 4 use-case settings (alpha, c)
PRESETS = {"tess": (2.0, 5.0), "kepler": (3.0, 5.0), "variable": (1.0, 5.0),
           "max_sensitivity": (10.0, 2.5)}


class UmiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status
        self.message = message


class Launch(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("groups_per_cu", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("main_start", ctypes.c_void_p), ("main_stop", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_void_p), ("c", ctypes.c_void_p), ("scale", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("detrended", ctypes.c_void_p),
                ("window_days", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("max_step_samples", ctypes.c_int64),
                ("staging_bytes", ctypes.c_int64), ("max_curves", ctypes.c_int32),
                ("max_W", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("copy_threads", ctypes.c_int32), ("device", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ServerCompletion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("admitted", ctypes.c_double), ("launched", ctypes.c_double),
                ("done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "submitted", "completed", "failed", "rejected", "steps", "step_curves", "samples",
        "largest_step_samples", "arena_capacity", "arena_used", "arena_high_water",
        "staging_fallbacks")] + [
        ("loop_s", ctypes.c_double * 4), ("longest_iteration_s", ctypes.c_double),
        ("longest_iteration_loop_s", ctypes.c_double * 4), ("exec_s", ctypes.c_double * 4)]


_vp = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def _load():
    # torch first: libumi.so needs libamdhip64.so.7, and loading it after torch
    # binds it to torch's HIP runtime (same soname), so the device pointers and
    # streams torch hands over belong to the runtime the library launches on.
    # Loaded the other way round a process would hold two HIP runtimes.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libumi.so is not built (%s); run `python paper_2604_06602_amd/build.py` "
                          "or __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    lib.umi_detrend.restype = ctypes.c_int
    lib.umi_detrend.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_float,
                                ctypes.c_float, ctypes.c_int32, _vp, _vp, _vp]
    lib.umi_detrend_batch.restype = ctypes.c_int
    lib.umi_detrend_batch.argtypes = [_vp, _vp, _i64p, ctypes.c_int64, _i32p, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_int32, _vp, _vp,
                                      ctypes.POINTER(Launch), _vp]
    lib.umi_detrend_batch_noalloc.restype = ctypes.c_int
    lib.umi_detrend_batch_noalloc.argtypes = [_vp, _vp, _i64p, ctypes.c_int64, _i32p,
                                              ctypes.c_float, ctypes.c_float, ctypes.c_int32,
                                              _vp, _vp, ctypes.POINTER(Launch), _vp]
    lib.umi_detrend_gather.restype = ctypes.c_int
    lib.umi_detrend_gather.argtypes = [_vp, _vp, _i64p, _i64p, ctypes.c_int64, _i32p,
                                       ctypes.c_float, ctypes.c_float, ctypes.c_int32, _vp, _vp,
                                       ctypes.POINTER(Launch), _vp]
    lib.umi_detrend_gather_ex.restype = ctypes.c_int
    lib.umi_detrend_gather_ex.argtypes = [_vp, _vp, _i64p, _i64p, ctypes.c_int64, _i32p,
                                          ctypes.c_float, ctypes.c_float, ctypes.c_int32, _vp,
                                          _vp, ctypes.POINTER(Options), ctypes.POINTER(Launch),
                                          _vp]
    lib.umi_plan_run_ex.restype = ctypes.c_int
    lib.umi_plan_run_ex.argtypes = [_vp, _i64p, _i64p, _i32p, ctypes.c_int64, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_int32, ctypes.POINTER(Options)]
    lib.umi_plan_create.restype = ctypes.c_int
    lib.umi_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int64,
                                    ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp]
    lib.umi_plan_run.restype = ctypes.c_int
    lib.umi_plan_run.argtypes = [_vp, _i64p, _i64p, _i32p, ctypes.c_int64, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_int32]
    lib.umi_plan_destroy.restype = ctypes.c_int
    lib.umi_plan_destroy.argtypes = [_vp]
    lib.umi_window_from_cadence.restype = ctypes.c_int32
    lib.umi_window_from_cadence.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.umi_set_tuning.restype = ctypes.c_int
    lib.umi_set_tuning.argtypes = [ctypes.c_char_p]
    lib.umi_last_error.restype = ctypes.c_char_p
    lib.umi_last_error.argtypes = []
    lib.umi_release.restype = None
    lib.umi_release.argtypes = []
    lib.umi_version.restype = ctypes.c_char_p
    lib.umi_version.argtypes = []
    lib.umi_debug_inject_error.restype = None
    lib.umi_debug_inject_error.argtypes = [ctypes.c_int]
    lib.umi_host_copy_many.restype = ctypes.c_int
    lib.umi_host_copy_many.argtypes = [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32]
    lib.umi_copy_async.restype = ctypes.c_int
    lib.umi_copy_async.argtypes = [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp]
    lib.umi_server_create.restype = ctypes.c_int
    lib.umi_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]
    lib.umi_server_submit.restype = ctypes.c_int
    lib.umi_server_submit.argtypes = [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_int32,
                                      ctypes.c_double, _vp, ctypes.c_uint64]
    lib.umi_server_poll.restype = ctypes.c_int
    lib.umi_server_poll.argtypes = [_vp, ctypes.POINTER(ServerCompletion), ctypes.c_int32,
                                    ctypes.c_double, ctypes.POINTER(ctypes.c_int32)]
    lib.umi_server_stats_get.restype = ctypes.c_int
    lib.umi_server_stats_get.argtypes = [_vp, ctypes.POINTER(ServerStats)]
    for name in ("umi_server_reset_stats", "umi_server_shutdown", "umi_server_destroy"):
        getattr(lib, name).restype = ctypes.c_int
        getattr(lib, name).argtypes = [_vp]
    return lib


lib = _load()


def _check(status: int):
    if status != UMI_OK:
        raise UmiError(status, lib.umi_last_error().decode(errors="replace"))


def host_copy_many(dst_ptrs, src_ptrs, nbytes, threads: int = 1):
    """Host-to-host copies nbytes[i] from src_ptrs[i] to dst_ptrs[i] (int64
    arrays of addresses and sizes) in one native call, which runs without the
    interpreter lock and splits the work over `threads` native threads."""
    d = np.ascontiguousarray(dst_ptrs, np.uint64)
    s = np.ascontiguousarray(src_ptrs, np.uint64)
    b = np.ascontiguousarray(nbytes, np.int64)
    if not (d.shape == s.shape == b.shape and b.ndim == 1):
        raise ValueError("host_copy_many: three 1-D arrays of equal length")
    _check(lib.umi_host_copy_many(d.ctypes.data, s.ctypes.data, b.ctypes.data, b.size,
                                  int(threads)))


COPY_H2D, COPY_D2H, COPY_KERNEL = 1, 2, 4


def copy_async(dst_ptrs, src_ptrs, nbytes, kind: int, stream=None):
    """Enqueue host<->device copies (kind COPY_H2D or COPY_D2H) of nbytes[i]
    from src_ptrs[i] to dst_ptrs[i] on `stream` (a torch stream, a raw
    hipStream_t address, or None for the current stream) in one native call.
    With COPY_KERNEL or-ed into kind the copies run as a kernel that reaches
    the (pinned) host buffers directly instead of through the copy engines."""
    d = np.ascontiguousarray(dst_ptrs, np.uint64)
    s = np.ascontiguousarray(src_ptrs, np.uint64)
    b = np.ascontiguousarray(nbytes, np.int64)
    if not (d.shape == s.shape == b.shape and b.ndim == 1):
        raise ValueError("copy_async: three 1-D arrays of equal length")
    st = ctypes.c_void_p(stream) if isinstance(stream, int) else _stream_handle(stream)
    _check(lib.umi_copy_async(d.ctypes.data, s.ctypes.data, b.ctypes.data, b.size, int(kind), st))


def last_error() -> str:
    return lib.umi_last_error().decode(errors="replace")


def version() -> str:
    return lib.umi_version().decode()


def window_from_cadence(cadence_days: float, window_days: float = 0.5) -> int:
    """Window-size rule of Section 2: round(window / cadence) | 1 (-1 if invalid)."""
    return int(lib.umi_window_from_cadence(float(cadence_days), float(window_days)))


def set_tuning(table_text: str | None):
    _check(lib.umi_set_tuning(None if table_text is None else table_text.encode()))


def release():
    lib.umi_release()


def debug_inject_error(status: int):
    lib.umi_debug_inject_error(int(status))


# ---------------------------------------------------------------------------
# tensor-facing calls


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _dev_ptr(t, dtype, name, n):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class LaunchOptions:
    mode: int = MODE_PERSISTENT
    tile: int = 0
    groups_per_cu: int = 0
    main_start: object = None  # torch.cuda.Event recorded before the main kernel
    main_stop: object = None   # torch.cuda.Event recorded after it

    def as_struct(self) -> Launch:
        def ev(e):
            return None if e is None else ctypes.c_void_p(int(e.cuda_event))
        return Launch(int(self.mode), int(self.tile), int(self.groups_per_cu), 0,
                      ev(self.main_start), ev(self.main_stop))


def _options(n_curves, alpha, c, scale, detrended_ptr, window_days=None):
    """(umi_options or None, scalar alpha, scalar c, arrays to keep alive).
    ``alpha`` and ``c`` are scalars or one value per curve; ``scale`` is a key
    of SCALES; ``window_days`` is None, a scalar or one value per curve (time
    windows where > 0).  None means the plain call suffices."""
    if scale not in SCALES:
        raise ValueError("scale must be one of %s" % sorted(SCALES))
    a_arr = c_arr = None
    a0 = c0 = None
    if np.ndim(alpha) == 0:
        a0 = float(alpha)
    else:
        a_arr = np.ascontiguousarray(alpha, dtype=np.float32)
        if a_arr.shape != (n_curves,):
            raise ValueError("per-curve alpha needs %d values" % n_curves)
        a0 = 2.0
    if np.ndim(c) == 0:
        c0 = float(c)
    else:
        c_arr = np.ascontiguousarray(c, dtype=np.float32)
        if c_arr.shape != (n_curves,):
            raise ValueError("per-curve c needs %d values" % n_curves)
        c0 = 5.0
    w_arr = None
    if window_days is not None:
        w_arr = np.ascontiguousarray(np.broadcast_to(np.asarray(window_days, np.float64),
                                                     (n_curves,)))
    if (a_arr is None and c_arr is None and scale == "upper_rms" and detrended_ptr is None
            and w_arr is None):
        return None, a0, c0, ()
    o = Options(None if a_arr is None else a_arr.ctypes.data,
                None if c_arr is None else c_arr.ctypes.data, SCALES[scale], 0, detrended_ptr,
                None if w_arr is None else w_arr.ctypes.data)
    return o, a0, c0, (a_arr, c_arr, w_arr)


def detrend_batch_into(flux, time, lengths, W, trend, median=None, alpha=2.0, c=5.0, iters=5,
                       launch: LaunchOptions | None = None, stream=None, scale="upper_rms",
                       detrended=None, window_days=None):
    """Raw batch call on preallocated device tensors (packed ragged layout).
    ``alpha``/``c`` may hold one value per curve; ``detrended`` receives
    flux / trend; ``window_days`` (> 0) selects time windows."""
    torch = _torch()
    lengths = np.ascontiguousarray(lengths, dtype=np.int64)
    Wa = np.ascontiguousarray(np.broadcast_to(np.asarray(W, dtype=np.int32), lengths.shape))
    n = int(lengths.sum()) if lengths.size else 0
    fp = _dev_ptr(flux, torch.float32, "flux", n)
    tp = _dev_ptr(time, torch.float64, "time", n)
    op = _dev_ptr(trend, torch.float32, "trend", n)
    mp = _dev_ptr(median, torch.float32, "median", n)
    dp = _dev_ptr(detrended, torch.float32, "detrended", n)
    opts, a0, c0, keep = _options(lengths.size, alpha, c, scale, dp, window_days)
    lp = None
    if launch is not None:
        lp = ctypes.byref(launch.as_struct())
    if opts is None:
        st = lib.umi_detrend_batch(fp, tp, lengths.ctypes.data_as(_i64p), lengths.size,
                                   Wa.ctypes.data_as(_i32p), a0, c0, int(iters),
                                   op, mp, lp, _stream_handle(stream))
    else:
        st = lib.umi_detrend_gather_ex(fp, tp, None, lengths.ctypes.data_as(_i64p),
                                       lengths.size, Wa.ctypes.data_as(_i32p), a0, c0,
                                       int(iters), op, mp, ctypes.byref(opts), lp,
                                       _stream_handle(stream))
    del keep
    _check(st)


NOALLOC_MAX_SAMPLES = 1 << 24
NOALLOC_MAX_CURVES = 8192
NOALLOC_MAX_TILES = 1 << 20


def detrend_batch_noalloc_into(flux, time, lengths, W, trend, median=None, alpha=2.0, c=5.0,
                               iters=5, launch: LaunchOptions | None = None, stream=None):
    """umi_detrend_batch_noalloc on preallocated device tensors: the packed
    batch call whose workspace is the library's static device array (at most
    NOALLOC_MAX_SAMPLES samples and NOALLOC_MAX_CURVES curves per call)."""
    torch = _torch()
    lengths = np.ascontiguousarray(lengths, dtype=np.int64)
    Wa = np.ascontiguousarray(np.broadcast_to(np.asarray(W, dtype=np.int32), lengths.shape))
    n = int(lengths.sum()) if lengths.size else 0
    lp = ctypes.byref(launch.as_struct()) if launch is not None else None
    st = lib.umi_detrend_batch_noalloc(_dev_ptr(flux, torch.float32, "flux", n),
                                       _dev_ptr(time, torch.float64, "time", n),
                                       lengths.ctypes.data_as(_i64p), lengths.size,
                                       Wa.ctypes.data_as(_i32p), float(alpha), float(c),
                                       int(iters), _dev_ptr(trend, torch.float32, "trend", n),
                                       _dev_ptr(median, torch.float32, "median", n), lp,
                                       _stream_handle(stream))
    _check(st)


def detrend_batch(flux, time, lengths, W, alpha=2.0, c=5.0, iters=5, with_median=False,
                  launch: LaunchOptions | None = None, stream=None, scale="upper_rms",
                  with_detrended=False, window_days=None):
    """Packed ragged batch: returns (trend, median or None) as device tensors,
    plus the detrended flux when ``with_detrended``."""
    torch = _torch()
    trend = torch.empty_like(flux)
    median = torch.empty_like(flux) if with_median else None
    det = torch.empty_like(flux) if with_detrended else None
    detrend_batch_into(flux, time, lengths, W, trend, median, alpha, c, iters, launch, stream,
                       scale, det, window_days)
    return (trend, median, det) if with_detrended else (trend, median)


def detrend(flux, time=None, W=361, alpha=2.0, c=5.0, iters=5, with_median=False, stream=None,
            scale="upper_rms", with_detrended=False, window_days=None):
    """One curve: returns (trend, median or None) as device tensors, plus the
    detrended flux when ``with_detrended``."""
    torch = _torch()
    n = flux.numel()
    if scale != "upper_rms" or with_detrended or window_days is not None:
        return detrend_batch(flux, time, [n], W, alpha, c, iters, with_median, None, stream,
                             scale, with_detrended, window_days)
    trend = torch.empty_like(flux)
    median = torch.empty_like(flux) if with_median else None
    st = lib.umi_detrend(_dev_ptr(flux, torch.float32, "flux", n),
                         _dev_ptr(time, torch.float64, "time", n), n, int(W), float(alpha),
                         float(c), int(iters), _dev_ptr(trend, torch.float32, "trend", n),
                         _dev_ptr(median, torch.float32, "median", n), _stream_handle(stream))
    _check(st)
    return trend, median


def _host_arrays(offsets, lengths, W):
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    lengths = np.ascontiguousarray(lengths, dtype=np.int64)
    Wa = np.ascontiguousarray(np.broadcast_to(np.asarray(W, dtype=np.int32), lengths.shape))
    if offsets.shape != lengths.shape:
        raise ValueError("offsets and lengths differ in size")
    return offsets, lengths, Wa


def _span_ptr(t, dtype, name, span):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s tensor" % (name, dtype))
    if t.numel() < span:
        raise ValueError("%s holds %d samples, curves reach %d" % (name, t.numel(), span))
    return ctypes.c_void_p(t.data_ptr())


def detrend_gather_into(flux, time, offsets, lengths, W, trend, median=None, alpha=2.0, c=5.0,
                        iters=5, launch: LaunchOptions | None = None, stream=None,
                        scale="upper_rms", detrended=None, window_days=None):
    """Curves at explicit sample offsets of the device arrays (no packing)."""
    torch = _torch()
    offsets, lengths, Wa = _host_arrays(offsets, lengths, W)
    span = int((offsets + np.maximum(lengths, 0)).max()) if lengths.size else 0
    lp = ctypes.byref(launch.as_struct()) if launch is not None else None
    dp = _span_ptr(detrended, torch.float32, "detrended", span)
    opts, a0, c0, keep = _options(lengths.size, alpha, c, scale, dp, window_days)
    args = (_span_ptr(flux, torch.float32, "flux", span),
            _span_ptr(time, torch.float64, "time", span),
            offsets.ctypes.data_as(_i64p), lengths.ctypes.data_as(_i64p),
            lengths.size, Wa.ctypes.data_as(_i32p), a0, c0,
            int(iters), _span_ptr(trend, torch.float32, "trend", span),
            _span_ptr(median, torch.float32, "median", span))
    if opts is None:
        st = lib.umi_detrend_gather(*args, lp, _stream_handle(stream))
    else:
        st = lib.umi_detrend_gather_ex(*args, ctypes.byref(opts), lp, _stream_handle(stream))
    del keep
    _check(st)


class Plan:
    """A replayable launch (hipGraph per staging slot) over fixed device arrays."""

    def __init__(self, flux, time, trend, median=None, max_curves=1024, max_W=MAX_WINDOW,
                 stream=None):
        torch = _torch()
        cap = flux.numel()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if int(self.stream.cuda_stream) == 0:
            raise ValueError("a plan needs a non-default stream")
        self._keep = (flux, time, trend, median)  # the plan holds their pointers
        h = ctypes.c_void_p()
        st = lib.umi_plan_create(ctypes.byref(h), cap, int(max_curves), int(max_W),
                                 _span_ptr(flux, torch.float32, "flux", cap),
                                 _span_ptr(time, torch.float64, "time", cap),
                                 _span_ptr(trend, torch.float32, "trend", cap),
                                 _span_ptr(median, torch.float32, "median", cap),
                                 ctypes.c_void_p(int(self.stream.cuda_stream)))
        _check(st)
        self._h = h
        self.capacity = cap
        self.max_curves = int(max_curves)
        self.max_W = int(max_W)

    def run(self, offsets, lengths, W, alpha=2.0, c=5.0, iters=5, scale="upper_rms",
            detrended=None, window_days=None):
        """Stage and replay one batch; ``alpha``/``c`` may hold one value per
        curve; ``detrended`` (capacity samples) receives flux / trend."""
        if self._h is None:
            raise RuntimeError("plan destroyed")
        torch = _torch()
        offsets, lengths, Wa = _host_arrays(offsets, lengths, W)
        dp = _span_ptr(detrended, torch.float32, "detrended", self.capacity)
        opts, a0, c0, keep = _options(lengths.size, alpha, c, scale, dp, window_days)
        if opts is None:
            st = lib.umi_plan_run(self._h, offsets.ctypes.data_as(_i64p),
                                  lengths.ctypes.data_as(_i64p), Wa.ctypes.data_as(_i32p),
                                  lengths.size, a0, c0, int(iters))
        else:
            st = lib.umi_plan_run_ex(self._h, offsets.ctypes.data_as(_i64p),
                                     lengths.ctypes.data_as(_i64p), Wa.ctypes.data_as(_i32p),
                                     lengths.size, a0, c0, int(iters), ctypes.byref(opts))
        del keep
        _check(st)

    def destroy(self):
        if self._h is not None:
            st = lib.umi_plan_destroy(self._h)
            self._h = None
            self._keep = None
            _check(st)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
