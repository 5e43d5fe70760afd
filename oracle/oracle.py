"""ctypes shim over the C oracle (``umi_oracle.c``) -- TEST INFRASTRUCTURE ONLY.

Every function here marshals numpy arrays into the C oracle and back; none
holds any of the method's arithmetic.  Section references are to arXiv
2604.06602.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "umi_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libumi_oracle.so")
_lock = threading.Lock()
_lib = None

_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def compile_oracle(src: str, out: str) -> str:
    """gcc, plain -O2, no fast-math."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-Wall",
           "-Wextra", "-o", tmp, src, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/libumi_oracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        compile_oracle(_SRC, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        path = os.environ.get("UMI_ORACLE_LIB")  # a test may point at a mutated build
        if not path:
            if not os.path.exists(_LIB_PATH):
                build(force=True)
            path = _LIB_PATH
        lib = ctypes.CDLL(path)
        lib.umi_oracle_window_from_cadence.restype = ctypes.c_int
        lib.umi_oracle_window_from_cadence.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.umi_oracle_weight.restype = ctypes.c_double
        lib.umi_oracle_weight.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.umi_oracle_median.restype = ctypes.c_float
        lib.umi_oracle_median.argtypes = [_f32p, ctypes.c_int]
        lib.umi_oracle_upper_scale.restype = ctypes.c_double
        lib.umi_oracle_upper_scale.argtypes = [_f32p, ctypes.c_int, ctypes.c_double]
        lib.umi_oracle_window.restype = ctypes.c_double
        lib.umi_oracle_window.argtypes = [_f32p, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int, _f32p, _f64p]
        lib.umi_oracle_segments.restype = ctypes.c_int64
        lib.umi_oracle_segments.argtypes = [_f32p, _f64p, ctypes.c_int64, ctypes.c_int,
                                            _i64p, _i64p]
        lib.umi_oracle_detrend.restype = ctypes.c_int
        lib.umi_oracle_detrend.argtypes = [_f32p, _f64p, ctypes.c_int64, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                           _f64p, _f32p]
        lib.umi_oracle_detrend_at.restype = ctypes.c_int
        lib.umi_oracle_detrend_at.argtypes = [_f32p, _f64p, ctypes.c_int64, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              _i64p, ctypes.c_int64, _f64p, _f32p]
        lib.umi_oracle_mad_scale.restype = ctypes.c_double
        lib.umi_oracle_mad_scale.argtypes = [_f32p, ctypes.c_int, ctypes.c_double]
        lib.umi_oracle_window_ex.restype = ctypes.c_double
        lib.umi_oracle_window_ex.argtypes = [_f32p, ctypes.c_int, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                             _f32p, _f64p]
        lib.umi_oracle_detrend_ex.restype = ctypes.c_int
        lib.umi_oracle_detrend_ex.argtypes = [_f32p, _f64p, ctypes.c_int64, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_double, _f64p, _f32p]
        lib.umi_oracle_detrend_at_ex.restype = ctypes.c_int
        lib.umi_oracle_detrend_at_ex.argtypes = [_f32p, _f64p, ctypes.c_int64, ctypes.c_int,
                                                 ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                 ctypes.c_int, ctypes.c_double, _i64p,
                                                 ctypes.c_int64, _f64p, _f32p]
        lib.umi_oracle_detrend_batch_ex.restype = ctypes.c_int
        lib.umi_oracle_detrend_batch_ex.argtypes = [_f32p, _f64p, _i64p, ctypes.c_int64, _i32p,
                                                    _f64p, _f64p, _f64p, ctypes.c_int,
                                                    ctypes.c_int, _f64p, _f32p, ctypes.c_int]
        lib.umi_oracle_normalise.restype = None
        lib.umi_oracle_normalise.argtypes = [_f32p, _f64p, ctypes.c_int64, _f64p]
        lib.umi_oracle_detrend_batch.restype = ctypes.c_int
        lib.umi_oracle_detrend_batch.argtypes = [_f32p, _f64p, _i64p, ctypes.c_int64, _i32p,
                                                 ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                 _f64p, _f32p, ctypes.c_int]
        _lib = lib
        return lib


SCALES = {"upper_rms": 0, "mad": 1}  # Section 2.2 / the MAD ablation


def _scale(scale) -> int:
    if scale not in SCALES:
        raise ValueError("scale must be one of %s" % sorted(SCALES))
    return SCALES[scale]


def _ptr(a, typ):
    return None if a is None else a.ctypes.data_as(typ)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def window_from_cadence(cadence_days: float, window_days: float = 0.5) -> int:
    """Window-size rule of Section 2: round(window / cadence) | 1."""
    return int(_load().umi_oracle_window_from_cadence(cadence_days, window_days))


def weight(u: float, alpha: float) -> float:
    """Asymmetric bisquare weight, Section 2.3 Eqs. 2-3."""
    return float(_load().umi_oracle_weight(float(u), float(alpha)))


def median(x) -> np.float32:
    """Lower median by IEEE totalOrder of the float32 bits (Section 2.1)."""
    x = _f32(x)
    return np.float32(_load().umi_oracle_median(_ptr(x, _f32p), int(x.size)))


def upper_scale(x, m: float) -> float:
    """Upper-RMS scale 0.6745*sigma_upper about m (Section 2.2, Eq. 1)."""
    x = _f32(x)
    return float(_load().umi_oracle_upper_scale(_ptr(x, _f32p), int(x.size), float(m)))


def mad_scale(x, m: float) -> float:
    """The MAD ablation's scale: lower median of |x - m| (no 0.6745 factor)."""
    x = _f32(x)
    return float(_load().umi_oracle_mad_scale(_ptr(x, _f32p), int(x.size), float(m)))


def window(x, alpha=2.0, c=5.0, iters=5, scale="upper_rms"):
    """One window's estimate: returns (trend, median, scale)."""
    x = _f32(x)
    med = ctypes.c_float()
    sc = ctypes.c_double()
    t = _load().umi_oracle_window_ex(_ptr(x, _f32p), int(x.size), float(alpha), float(c),
                                     int(iters), _scale(scale), ctypes.byref(med),
                                     ctypes.byref(sc))
    return float(t), np.float32(med.value), float(sc.value)


def segments(flux, time, W):
    """Per-sample segment bounds (first, last valid index; -1 if none)."""
    flux = _f32(flux)
    time = _f64(time)
    n = flux.size
    lo = np.empty(n, np.int64)
    hi = np.empty(n, np.int64)
    _load().umi_oracle_segments(_ptr(flux, _f32p), _ptr(time, _f64p), n, int(W),
                                _ptr(lo, _i64p), _ptr(hi, _i64p))
    return lo, hi


def detrend(flux, time, W, alpha=2.0, c=5.0, iters=5, scale="upper_rms", window_days=0.0):
    """Whole curve: returns (trend float64, median float32).  ``window_days``
    > 0 selects time windows of that length (W still bounds them)."""
    flux = _f32(flux)
    time = _f64(time)
    if time is not None and time.size != flux.size:
        raise ValueError("time and flux differ in length")
    n = flux.size
    trend = np.empty(n, np.float64)
    med = np.empty(n, np.float32)
    rc = _load().umi_oracle_detrend_ex(_ptr(flux, _f32p), _ptr(time, _f64p), n, int(W),
                                       float(alpha), float(c), int(iters), _scale(scale),
                                       float(window_days), _ptr(trend, _f64p),
                                       _ptr(med, _f32p))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return trend, med


def detrend_at(flux, time, W, idx, alpha=2.0, c=5.0, iters=5, scale="upper_rms",
               window_days=0.0):
    """Estimates only at positions ``idx`` of one curve."""
    flux = _f32(flux)
    time = _f64(time)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    trend = np.empty(idx.size, np.float64)
    med = np.empty(idx.size, np.float32)
    rc = _load().umi_oracle_detrend_at_ex(_ptr(flux, _f32p), _ptr(time, _f64p), flux.size,
                                          int(W), float(alpha), float(c), int(iters),
                                          _scale(scale), float(window_days), _ptr(idx, _i64p),
                                          idx.size, _ptr(trend, _f64p), _ptr(med, _f32p))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return trend, med


def detrend_batch(flux, time, lengths, W, alpha=2.0, c=5.0, iters=5, n_threads=None,
                  scale="upper_rms", window_days=None):
    """Packed ragged batch; curves spread over ``n_threads`` host threads.
    ``W``, ``alpha``, ``c`` and ``window_days`` (time windows where > 0) are
    scalars or one value per curve."""
    flux = _f32(flux)
    time = _f64(time)
    lengths = np.ascontiguousarray(lengths, dtype=np.int64)
    Wa = np.ascontiguousarray(np.broadcast_to(np.asarray(W), lengths.shape), dtype=np.int32)
    if int(lengths.sum()) != flux.size:
        raise ValueError("lengths do not add up to the packed size")
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    trend = np.empty(flux.size, np.float64)
    med = np.empty(flux.size, np.float32)
    al = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha, np.float64), lengths.shape))
    ca = np.ascontiguousarray(np.broadcast_to(np.asarray(c, np.float64), lengths.shape))
    wd = None
    if window_days is not None:
        wd = np.ascontiguousarray(np.broadcast_to(np.asarray(window_days, np.float64),
                                                  lengths.shape))
    rc = _load().umi_oracle_detrend_batch_ex(_ptr(flux, _f32p), _ptr(time, _f64p),
                                             _ptr(lengths, _i64p), lengths.size,
                                             _ptr(Wa, _i32p), _ptr(al, _f64p), _ptr(ca, _f64p),
                                             _ptr(wd, _f64p), int(iters), _scale(scale),
                                             _ptr(trend, _f64p), _ptr(med, _f32p),
                                             int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return trend, med


def normalise(flux, trend):
    """Detrended flux: flux / trend, NaN where the trend is NaN."""
    flux = _f32(flux)
    trend = np.ascontiguousarray(trend, dtype=np.float64)
    if trend.size != flux.size:
        raise ValueError("flux and trend differ in length")
    out = np.empty(flux.size, np.float64)
    _load().umi_oracle_normalise(_ptr(flux, _f32p), _ptr(trend, _f64p), flux.size,
                                 _ptr(out, _f64p))
    return out
