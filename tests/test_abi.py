"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "umi.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2604_06602_amd import _lib
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(umi_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["umi_detrend", "umi_detrend_batch", "umi_window_from_cadence", "umi_last_error",
              "umi_release", "umi_set_tuning", "umi_version", "umi_debug_inject_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib.lib, name), name


def test_library_is_the_in_tree_hip_build(lib):
    assert os.path.dirname(lib.LIB_PATH) == os.path.join(ROOT, "paper_2604_06602_amd")
    assert lib.version().startswith("umi-mi355x")


def test_window_rule(lib):
    assert lib.window_from_cadence(2 / 1440) == 361
    assert lib.window_from_cadence(29.4 / 1440) == 25
    assert lib.window_from_cadence(30 / 1440) == 25
    assert lib.window_from_cadence(2 / 1440, 1.5) == 1081
    assert lib.window_from_cadence(0.0) == -1
    assert lib.window_from_cadence(float("nan")) == -1
    assert lib.window_from_cadence(2 / 1440, -1) == -1


def test_window_rule_agrees_with_oracle(lib, oracle_lib):
    for cad in [0.5, 1, 2, 10, 20, 29.4, 30, 60]:
        for wd in [0.25, 0.5, 1.0, 1.5]:
            assert lib.window_from_cadence(cad / 1440, wd) == oracle_lib.window_from_cadence(cad / 1440, wd)


def _raw_batch(lib, lengths, W, alpha=2.0, c=5.0, iters=5, flux=1, trend=1, launch=None):
    lengths = np.asarray(lengths, np.int64)
    Wa = np.asarray(W, np.int32)
    lp = ctypes.byref(launch) if launch is not None else None
    return lib.lib.umi_detrend_batch(
        ctypes.c_void_p(flux) if flux else None, None,
        lengths.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), lengths.size,
        Wa.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), alpha, c, iters,
        ctypes.c_void_p(trend) if trend else None, None, lp, None)


@pytest.mark.parametrize("W,alpha,c,iters,status", [
    (4, 2.0, 5.0, 5, 1), (0, 2.0, 5.0, 5, 1), (-3, 2.0, 5.0, 5, 1),
    (361, 0.0, 5.0, 5, 1), (361, -1.0, 5.0, 5, 1), (361, float("nan"), 5.0, 5, 1),
    (361, float("inf"), 5.0, 5, 1), (361, 2.0, 0.0, 5, 1), (361, 2.0, float("nan"), 5, 1),
    (361, 2.0, 5.0, -1, 1), (2049, 2.0, 5.0, 5, 4),
])
def test_invalid_arguments_rejected_before_launch(lib, W, alpha, c, iters, status):
    st = _raw_batch(lib, [10], [W], alpha, c, iters)
    assert st == status
    assert lib.last_error()


def test_other_invalid_arguments(lib):
    assert _raw_batch(lib, [-1], [5]) == 1
    assert _raw_batch(lib, [10], [5], flux=0) == 1
    assert _raw_batch(lib, [10], [5], trend=0) == 1
    bad_mode = lib.Launch(7, 0, 0, 0, None, None)
    assert _raw_batch(lib, [10], [5], launch=bad_mode) == 1
    assert _raw_batch(lib, [10], [5], launch=lib.Launch(0, -1, 0, 0, None, None)) == 1
    assert _raw_batch(lib, [10], [5], launch=lib.Launch(0, 0, 0, 3, None, None)) == 1
    assert lib.lib.umi_detrend(None, None, -5, 5, 2.0, 5.0, 5, None, None, None) == 1
    # a batch whose second curve is bad is rejected as a whole
    assert _raw_batch(lib, [10, 10], [5, 6]) == 1


def test_empty_batches_are_noops(lib):
    assert _raw_batch(lib, [], []) == 0
    assert _raw_batch(lib, [0, 0], [5, 7], flux=0, trend=0) == 0
    assert lib.lib.umi_detrend(None, None, 0, 5, 2.0, 5.0, 5, None, None, None) == 0


def test_injected_error_propagates_once(lib):
    lib.debug_inject_error(lib.UMI_ERR_DEVICE)
    assert _raw_batch(lib, [0], [5]) == lib.UMI_ERR_DEVICE
    assert "injected" in lib.last_error()
    assert _raw_batch(lib, [0], [5]) == 0
    with pytest.raises(lib.UmiError) as ei:
        lib.debug_inject_error(lib.UMI_ERR_NO_MEMORY)
        lib._check(_raw_batch(lib, [0], [5]))
    assert ei.value.status == lib.UMI_ERR_NO_MEMORY


def test_tuning_table_parsing(lib):
    lib.set_tuning("# W_max tile groups\n31 2000 4\n127 1500 3\n\n2047 0 0\n")
    # batch-size rows precede a bucket's row for any size, smallest first
    lib.set_tuning("31 64 4 40000\n31 512 4 160000\n31 1536 4\n127 128 4 40000\n127 1536 4 0\n")
    lib.set_tuning(None)
    for bad in ["31 2000", "31 2000 4 9 1", "127 10 2\n31 10 2", "x 1 2", "31 -1 2", "31 10 99",
                "31 10 2 -5", "31 10 2 x", "31 10 2\n31 10 2 50", "31 10 2 50\n31 10 2 50",
                "31 10 2 50\n31 10 2 40"]:
        with pytest.raises(lib.UmiError):
            lib.set_tuning(bad)
    lib.set_tuning(None)


def test_gather_validation_without_device(lib):
    i64 = ctypes.POINTER(ctypes.c_int64)
    i32 = ctypes.POINTER(ctypes.c_int32)

    def gather(offs, lens, Ws):
        o = np.asarray(offs, np.int64)
        L = np.asarray(lens, np.int64)
        w = np.asarray(Ws, np.int32)
        return lib.lib.umi_detrend_gather(ctypes.c_void_p(1), None, o.ctypes.data_as(i64),
                                          L.ctypes.data_as(i64), L.size, w.ctypes.data_as(i32),
                                          2.0, 5.0, 5, ctypes.c_void_p(1), None, None, None)
    assert gather([0, 50], [100, 100], [5, 5]) == 1          # overlapping ranges
    assert gather([-1], [10], [5]) == 1                      # negative offset
    assert gather([0, 100], [100, 0], [5, 4]) == 1           # even W even on an empty curve
    assert gather([0, 100], [0, 0], [5, 5]) == 0             # nothing to do
    assert lib.lib.umi_detrend_gather(None, None, None, None, 0, None, 2.0, 5.0, 5, None, None,
                                      None, None) == 0


def test_options_validation_without_device(lib):
    """umi_options: per-curve alpha/c must be finite and > 0, the scale known,
    reserved zero; all checked before anything touches the device."""
    i64 = ctypes.POINTER(ctypes.c_int64)
    i32 = ctypes.POINTER(ctypes.c_int32)
    L = np.asarray([10, 20], np.int64)
    w = np.asarray([5, 7], np.int32)

    def call(alpha=None, c=None, scale=0, reserved=0, offsets=None, window_days=None,
             time=None):
        a = None if alpha is None else np.asarray(alpha, np.float32)
        cc = None if c is None else np.asarray(c, np.float32)
        wd = None if window_days is None else np.asarray(window_days, np.float64)
        o = lib.Options(None if a is None else a.ctypes.data, None if cc is None else cc.ctypes.data,
                        scale, reserved, None, None if wd is None else wd.ctypes.data)
        offs = None if offsets is None else np.asarray(offsets, np.int64)
        lib.debug_inject_error(0)
        return lib.lib.umi_detrend_gather_ex(
            ctypes.c_void_p(1), time, None if offs is None else offs.ctypes.data_as(i64),
            L.ctypes.data_as(i64), L.size, w.ctypes.data_as(i32), 2.0, 5.0, 5,
            ctypes.c_void_p(1), None, ctypes.byref(o), None, None)
    assert call(alpha=[2.0, 0.0]) == 1
    assert call(alpha=[2.0, float("nan")]) == 1
    assert call(c=[-5.0, 5.0]) == 1
    assert call(c=[5.0, float("inf")]) == 1
    assert call(scale=2) == 1
    assert call(scale=-1) == 1
    assert call(reserved=1) == 1
    assert call(alpha=[2.0, 3.0], offsets=[0, 5]) == 1    # overlapping explicit offsets
    assert call(window_days=[0.5, -1.0], time=ctypes.c_void_p(8)) == 1
    assert call(window_days=[0.5, float("nan")], time=ctypes.c_void_p(8)) == 1
    assert call(window_days=[0.5, 0.0]) == 1              # time windows need times
    with pytest.raises(ValueError):
        lib._options(2, [2.0], 5.0, "upper_rms", None)    # wrong per-curve count
    with pytest.raises(ValueError):
        lib._options(2, 2.0, 5.0, "iqr", None)
    assert lib._options(2, 2.0, 5.0, "upper_rms", None)[0] is None  # plain call suffices
    assert lib.lib.umi_plan_run_ex(None, None, None, None, 0, 2.0, 5.0, 5, None) == 1


def test_plan_validation_without_device(lib):
    h = ctypes.c_void_p()
    # no stream: graph capture needs a non-default stream
    assert lib.lib.umi_plan_create(ctypes.byref(h), 100, 4, 25, ctypes.c_void_p(1), None,
                                   ctypes.c_void_p(1), None, None) == 1
    assert lib.lib.umi_plan_create(ctypes.byref(h), 0, 4, 25, ctypes.c_void_p(1), None,
                                   ctypes.c_void_p(1), None, ctypes.c_void_p(1)) == 1
    assert lib.lib.umi_plan_create(ctypes.byref(h), 100, 4, 24, ctypes.c_void_p(1), None,
                                   ctypes.c_void_p(1), None, ctypes.c_void_p(1)) == 1
    assert lib.lib.umi_plan_create(None, 100, 4, 25, ctypes.c_void_p(1), None,
                                   ctypes.c_void_p(1), None, ctypes.c_void_p(1)) == 1
    assert lib.lib.umi_plan_run(None, None, None, None, 0, 2.0, 5.0, 5) == 1
    assert lib.lib.umi_plan_destroy(None) == 0


def test_autotune_table_is_loadable(lib, monkeypatch):
    from paper_2604_06602_amd import autotune
    monkeypatch.setattr(autotune, "_arch", lambda: "gfx950")
    table = autotune.load_table()
    assert table is not None, "no committed tuning table for this library version"
    lib.set_tuning(table)          # the library accepts it
    lib.set_tuning(None)
    rows = [(tuple(map(int, l.split())) + (0,))[:4] for l in table.strip().splitlines()]
    general = [r for r in rows if r[3] == 0]
    assert [r[0] for r in general] == [b[0] for b in autotune.BUCKETS]
    sized = {(r[0], r[3]) for r in rows if r[3] > 0}
    assert sized == {(b[0], s) for b in autotune.BUCKETS for _, s in autotune.SMALL_BATCHES}
    for w_max, tile, gpc, _ in rows:
        assert 1 <= tile <= autotune.max_tile(dict(autotune.BUCKETS)[w_max])
        assert 1 <= gpc <= 4


def test_autotune_candidates():
    from paper_2604_06602_amd import autotune
    assert autotune.default_tile(361) == 1536 and autotune.default_tile(25) == 1536
    assert autotune.default_tile(721) == 1328 and autotune.default_tile(2047) == 2
    assert autotune.max_tile(25) == 1536 and autotune.max_tile(1441) == 608
    for W in [25, 121, 361, 721, 1441]:
        c = autotune.tile_candidates(W)
        assert autotune.default_tile(W) in c and max(c) == autotune.max_tile(W)


def test_diag_library_exports_its_header():
    """The measurement aid (include/umi_diag.h) loads and rejects bad
    arguments before launching anything."""
    text = open(os.path.join(ROOT, "include", "umi_diag.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(umi_[a-z_]+)\s*\(", text)))
    assert names == ["umi_diag_fma_peak"]
    diag = ctypes.CDLL(os.path.join(ROOT, "paper_2604_06602_amd", "libumi_diag.so"))
    for n in names:
        assert hasattr(diag, n), n
    f = diag.umi_diag_fma_peak
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_double)]
    assert f(0, 8, ctypes.c_void_p(1), None, None) == 1
    assert f(10, 0, ctypes.c_void_p(1), None, None) == 1
    assert f(10, 8, None, None, None) == 1


def test_serve_header_and_host_copy_many(lib):
    """include/umi_serve.h: its symbol is exported, and the batched host copy
    moves every byte of a ragged list (empty, sub-piece and multi-piece
    copies, 1 and several threads, from two calling threads at once) and
    rejects bad arguments before copying anything."""
    import threading
    text = open(os.path.join(ROOT, "include", "umi_serve.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(umi_[a-z_]+)\s*\(", text)))
    assert names == ["umi_copy_async", "umi_host_copy_many", "umi_server_create",
                     "umi_server_destroy", "umi_server_poll", "umi_server_reset_stats",
                     "umi_server_shutdown", "umi_server_stats_get", "umi_server_submit"]
    for n in names:
        assert hasattr(lib.lib, n), n
    rng = np.random.default_rng(5)
    sizes = [0, 1, 7, 1 << 20, (1 << 20) + 1, 3 * (1 << 20) + 12345, 100, 0, 5 << 20]
    srcs = [rng.integers(0, 256, s, dtype=np.uint8) for s in sizes]
    total = sum(sizes)

    def one(threads):
        dst = np.zeros(total, np.uint8)
        offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
        lib.host_copy_many([dst.ctypes.data + int(o) for o in offs],
                           [s.ctypes.data for s in srcs], sizes, threads)
        assert np.array_equal(dst, np.concatenate(srcs))

    for threads in [1, 2, 4, 8]:
        one(threads)
    errs = []

    def hammer():
        try:
            for _ in range(20):
                one(4)
        except Exception as e:  # pragma: no cover - reported below
            errs.append(e)
    ts = [threading.Thread(target=hammer) for _ in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errs
    a = np.ones(8, np.uint8)
    b = np.zeros(8, np.uint8)
    lib.host_copy_many([], [], [], 4)  # n = 0: no-op
    for bad in [dict(threads=0), dict(threads=65), dict(nbytes=[-1]), dict(dst=[0]),
                dict(src=[0])]:
        args = dict(dst=[b.ctypes.data], src=[a.ctypes.data], nbytes=[8], threads=2)
        args.update(bad)
        with pytest.raises(lib.UmiError):
            lib.host_copy_many(args["dst"], args["src"], args["nbytes"], args["threads"])
    assert not b.any()
    f = lib.lib.umi_host_copy_many
    assert f(None, None, None, 1, 1) == 1 and f(None, None, None, -1, 1) == 1


def test_copy_async_rejects_bad_arguments(lib):
    """umi_copy_async checks everything before enqueueing (no device call is
    made here: every case fails validation, and n = 0 is a no-op)."""
    a = np.ones(8, np.uint8)
    lib.copy_async([], [], [], lib.COPY_H2D, 0)
    for bad in [dict(kind=0), dict(kind=3), dict(kind=lib.COPY_KERNEL), dict(kind=3 | lib.COPY_KERNEL),
                dict(kind=8 | lib.COPY_D2H), dict(nbytes=[-1]), dict(dst=[0]), dict(src=[0]),
                dict(nbytes=[-1], kind=lib.COPY_D2H | lib.COPY_KERNEL)]:
        args = dict(dst=[a.ctypes.data], src=[a.ctypes.data], nbytes=[8], kind=lib.COPY_D2H)
        args.update(bad)
        with pytest.raises(lib.UmiError):
            lib.copy_async(args["dst"], args["src"], args["nbytes"], args["kind"], 0)
    f = lib.lib.umi_copy_async
    assert f(None, None, None, 1, 1, None) == 1 and f(None, None, None, -1, 1, None) == 1


def test_server_validation_without_device(lib):
    """The native server's entry points reject bad arguments before any
    device call: config fields out of range, NULL handles and buffers."""
    import ctypes
    L = lib.lib

    def cfg(**kw):
        base = dict(capacity=1000, max_step_samples=0, staging_bytes=0, max_curves=0, max_W=0,
                    max_inflight=0, copy_threads=0, device=0, reserved=0)
        base.update(kw)
        return lib.ServerConfig(**base)

    for bad in [dict(capacity=0), dict(capacity=-5), dict(max_W=4), dict(max_W=2049),
                dict(max_inflight=9), dict(copy_threads=65), dict(device=-1), dict(reserved=1),
                dict(staging_bytes=1000), dict(max_curves=-1), dict(max_step_samples=-2)]:
        h = ctypes.c_void_p(1234)
        c = cfg(**bad)
        assert L.umi_server_create(ctypes.byref(c), ctypes.byref(h)) == lib.UMI_ERR_INVALID_ARG, bad
        assert h.value is None  # *out cleared
    assert L.umi_server_create(None, None) == lib.UMI_ERR_INVALID_ARG
    x = np.zeros(4, np.float32)
    assert L.umi_server_submit(None, x.ctypes.data, None, 4, 5, 2.0, 5.0, 5, -1.0, x.ctypes.data,
                               0) == lib.UMI_ERR_INVALID_ARG
    n = ctypes.c_int32(7)
    buf = (lib.ServerCompletion * 2)()
    assert L.umi_server_poll(None, buf, 2, 0.0, ctypes.byref(n)) == lib.UMI_ERR_INVALID_ARG
    st = lib.ServerStats()
    assert L.umi_server_stats_get(None, ctypes.byref(st)) == lib.UMI_ERR_INVALID_ARG
    assert L.umi_server_reset_stats(None) == lib.UMI_ERR_INVALID_ARG
    assert L.umi_server_shutdown(None) == lib.UMI_ERR_INVALID_ARG
    assert L.umi_server_destroy(None) == lib.UMI_OK
    assert ctypes.sizeof(lib.ServerConfig) == 48 and ctypes.sizeof(lib.ServerCompletion) == 40


def test_host_copy_many_with_many_small_copies(lib):
    """Tens of thousands of tiny copies (pieces index the copy list by binary
    search): every destination gets its own source's bytes."""
    rng = np.random.default_rng(11)
    n = 20000
    sizes = rng.integers(0, 40, n)
    src = rng.integers(0, 256, int(sizes.sum()), dtype=np.uint8)
    dst = np.zeros_like(src)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    perm = rng.permutation(n)  # scatter the copies in a shuffled order
    lib.host_copy_many(dst.ctypes.data + offs[perm], src.ctypes.data + offs[perm], sizes[perm], 8)
    assert np.array_equal(dst, src)


def _raw_noalloc(lib, lengths, W, flux=1, trend=1):
    lengths = np.asarray(lengths, np.int64)
    Wa = np.asarray(W, np.int32)
    return lib.lib.umi_detrend_batch_noalloc(
        ctypes.c_void_p(flux) if flux else None, None,
        lengths.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), lengths.size,
        Wa.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 2.0, 5.0, 5,
        ctypes.c_void_p(trend) if trend else None, None, None, None)


def test_noalloc_limits_and_validation_without_device(lib):
    """The allocation-free call checks its fixed limits, and the arguments the
    batch call checks, on the host before it touches the device."""
    text = open(HEADER).read()
    consts = dict(re.findall(r"#define (UMI_NOALLOC_\w+) (\d+)", text))
    assert int(consts["UMI_NOALLOC_MAX_SAMPLES"]) == lib.NOALLOC_MAX_SAMPLES
    assert int(consts["UMI_NOALLOC_MAX_CURVES"]) == lib.NOALLOC_MAX_CURVES
    assert int(consts["UMI_NOALLOC_MAX_TILES"]) == lib.NOALLOC_MAX_TILES
    big = lib.NOALLOC_MAX_SAMPLES
    assert _raw_noalloc(lib, [big, 1], [25, 25]) == lib.UMI_ERR_UNSUPPORTED
    assert "UMI_NOALLOC_MAX_SAMPLES" in lib.last_error()
    assert _raw_noalloc(lib, [2**62, 2**62], [25, 25]) == lib.UMI_ERR_UNSUPPORTED  # no overflow
    n = lib.NOALLOC_MAX_CURVES + 1
    assert _raw_noalloc(lib, [1] * n, [25] * n) == lib.UMI_ERR_UNSUPPORTED
    assert "UMI_NOALLOC_MAX_CURVES" in lib.last_error()
    assert _raw_noalloc(lib, [10], [4]) == lib.UMI_ERR_INVALID_ARG
    assert _raw_noalloc(lib, [-1], [5]) == lib.UMI_ERR_INVALID_ARG
    assert _raw_noalloc(lib, [10], [5], flux=0) == lib.UMI_ERR_INVALID_ARG
    assert _raw_noalloc(lib, [10], [5], trend=0) == lib.UMI_ERR_INVALID_ARG
    assert _raw_noalloc(lib, [], []) == lib.UMI_OK
    assert _raw_noalloc(lib, [0, 0], [5, 7], flux=0, trend=0) == lib.UMI_OK
    lib.debug_inject_error(lib.UMI_ERR_DEVICE)
    assert _raw_noalloc(lib, [0], [5]) == lib.UMI_ERR_DEVICE
