"""Serving loop: continuous batching of detrending requests on one GPU.

Requests (one light curve each) arrive at any time through ``Server.submit``.
A scheduler thread

  * admits waiting requests first-in first-out while their samples fit the
    device-memory budget: the budget is one resident arena of device arrays
    (flux, time, trend) plus the plan's per-sample workspace, and every
    admission group (the requests admitted together) gets one contiguous
    range of it: its curves are staged into a pinned ring by one batched
    native copy, then uploaded with one host-to-device copy per array on a
    copy stream;
  * launches steps: all admitted, not yet launched groups that share the
    iteration count go into one batch -- each curve keeps its own alpha and
    c (the Table 4 settings mix freely) -- run through a replayable plan (a
    captured hipGraph of the tile-table copy, the segmentation pre-pass and
    the persistent estimate kernel) on the compute stream.  Up to two steps
    are in flight, so requests that arrive while one step runs are uploaded
    and staged concurrently and run in the next step;
  * completes steps: the trend of each group comes back with one
    device-to-host copy into the pinned ring and one batched native copy
    out of it, requests are resolved, and their arena ranges and budget are
    released.

Latency is measured from the request's arrival time (``submit``'s
``arrival`` argument, defaulting to now: an open-loop driver passes the
scheduled arrival) to the moment its result is in host memory.

The executor interface is small so the scheduler can be exercised on the CPU
with ``FakeExecutor``.
"""
from __future__ import annotations

import atexit
import itertools
import threading
import time as _time
from collections import deque
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

# Device bytes held per resident sample: flux f32, time f64, trend f32, and
# the plan workspace: one i32 segment word per sample plus the tile list
# (8 bytes per tile of at least 512 samples) and the pre-pass chunk records
# (144 bytes per 2,048 samples), together rounded up to 1 byte per sample.
BYTES_PER_SAMPLE = 4 + 8 + 4 + 4 + 1


class Rejected(ValueError):
    """The request can never be admitted (e.g. larger than the whole budget)."""


# ---------------------------------------------------------------------------
# arena: first-fit allocation of sample ranges


class Arena:
    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self._free = [(0, self.capacity)]  # sorted, coalesced (start, length)
        self.used = 0
        self.high_water = 0

    def alloc(self, n: int):
        if n <= 0:
            return 0
        for i, (s, L) in enumerate(self._free):
            if L >= n:
                if L == n:
                    self._free.pop(i)
                else:
                    self._free[i] = (s + n, L - n)
                self.used += n
                self.high_water = max(self.high_water, self.used)
                return s
        return None

    def free(self, start: int, n: int):
        if n <= 0:
            return
        fl = self._free
        lo, hi = 0, len(fl)
        while lo < hi:
            mid = (lo + hi) // 2
            if fl[mid][0] < start:
                lo = mid + 1
            else:
                hi = mid
        fl.insert(lo, (start, n))
        # coalesce with neighbours
        if lo + 1 < len(fl) and fl[lo][0] + fl[lo][1] == fl[lo + 1][0]:
            fl[lo] = (fl[lo][0], fl[lo][1] + fl[lo + 1][1])
            fl.pop(lo + 1)
        if lo > 0 and fl[lo - 1][0] + fl[lo - 1][1] == fl[lo][0]:
            fl[lo - 1] = (fl[lo - 1][0], fl[lo - 1][1] + fl[lo][1])
            fl.pop(lo)
        self.used -= n


# ---------------------------------------------------------------------------
# requests and groups


@dataclass(slots=True)
class Request:
    rid: int
    flux: np.ndarray
    time: np.ndarray | None
    W: int
    alpha: float
    c: float
    iters: int
    arrival: float
    future: Future
    admitted: float = 0.0
    launched: float = 0.0
    done: float = 0.0
    offset: int = -1

    @property
    def n(self) -> int:
        return int(self.flux.size)

    @property
    def key(self):
        # alpha and c travel per curve (Table 4 settings mix in one step);
        # the iteration count is per launch
        return self.iters


@dataclass
class Group:
    key: tuple
    offset: int
    size: int
    requests: list
    upload: object = None     # executor token
    launched: bool = False


@dataclass
class Step:
    groups: list
    handle: object = None
    launched_at: float = 0.0


@dataclass
class Stats:
    latencies: list = field(default_factory=list)
    queued: list = field(default_factory=list)     # arrival -> admitted
    staged: list = field(default_factory=list)     # admitted -> launched
    service: list = field(default_factory=list)    # launched -> result in host memory
    step_curves: list = field(default_factory=list)
    loop_max_s: float = 0.0                          # longest scheduler iteration
    loop_max_phases: dict = field(default_factory=dict)  # and how it was spent
    step_samples_max: int = 0
    phase_s: dict = field(default_factory=lambda: {"finish": 0.0, "admit": 0.0,
                                                   "upload": 0.0, "launch": 0.0})
    submit_lag: list = field(default_factory=list)  # arrival -> submit() called
    completed: int = 0
    failed: int = 0
    rejected: int = 0
    steps: int = 0
    samples: int = 0
    first_arrival: float | None = None
    last_done: float | None = None

    def summary(self, arena: Arena | None = None) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.zeros(0)
        span = (self.last_done - self.first_arrival) if self.completed else 0.0
        out = {
            "completed": self.completed, "failed": self.failed, "rejected": self.rejected,
            "steps": self.steps,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "max_ms": float(lat.max() * 1e3) if lat.size else None,
            "curves_per_s": self.completed / span if span > 0 else None,
            "samples_per_s": self.samples / span if span > 0 else None,
        }
        for name in ("queued", "staged", "service"):
            v = np.array(getattr(self, name)) if getattr(self, name) else np.zeros(0)
            out[name + "_p50_ms"] = float(np.percentile(v, 50) * 1e3) if v.size else None
            out[name + "_p99_ms"] = float(np.percentile(v, 99) * 1e3) if v.size else None
        sc = np.array(self.step_curves) if self.step_curves else np.zeros(0)
        out["mean_curves_per_step"] = float(sc.mean()) if sc.size else None
        lag = np.array(self.submit_lag) if self.submit_lag else np.zeros(0)
        out["submit_lag_p99_ms"] = float(np.percentile(lag, 99) * 1e3) if lag.size else None
        out["scheduler_longest_iteration_ms"] = self.loop_max_s * 1e3
        out["scheduler_longest_iteration_phases_ms"] = {
            k: v * 1e3 for k, v in self.loop_max_phases.items()}
        out["largest_step_samples"] = self.step_samples_max
        out["scheduler_phase_s"] = dict(self.phase_s)
        if arena is not None:
            out["arena_high_water_samples"] = arena.high_water
            out["arena_capacity_samples"] = arena.capacity
        return out


# ---------------------------------------------------------------------------
# executors


def _addr(a: np.ndarray) -> int:
    return a.__array_interface__["data"][0]


def staging_copies_many(groups_parts, bases):
    """The copy list that stages several groups at once: group g's curves
    ((flux, time) pairs of contiguous float32 / float64 arrays) at host
    address bases[g], every time array back to back first (8-byte aligned
    when the base is), then every flux array.  Returns (dst, src, nbytes)
    for one batched native copy."""
    k = [len(p) for p in groups_parts]
    flat = [fp for p in groups_parts for fp in p]
    m = len(flat)
    sizes = np.fromiter((f.size for f, _ in flat), np.int64, m)
    gid = np.repeat(np.arange(len(k)), k)
    first = np.concatenate([[0], np.cumsum(k)[:-1]]).astype(np.int64)
    csum = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = csum[:-1] - csum[first][gid]              # sample position inside its group
    n_g = csum[first + np.asarray(k)] - csum[first]  # samples per group
    base = np.asarray(bases, np.int64)[gid]
    dst = np.concatenate([base + 8 * pos, base + 8 * n_g[gid] + 4 * pos]).astype(np.uint64)
    src = np.fromiter(itertools.chain((_addr(t) for _, t in flat), (_addr(f) for f, _ in flat)),
                      np.uint64, 2 * m)
    return dst, src, np.concatenate([8 * sizes, 4 * sizes])


class PinnedRing:
    """A preallocated pinned host buffer handed out as a ring: blocks are
    allocated at the head and released in any order; space comes back when
    the oldest live blocks are released.  Avoids pinned allocations (which
    are slow and can serialise with the device) on the serving path."""

    ALIGN = 256

    def __init__(self, torch, nbytes: int):
        self.buf = torch.empty(int(nbytes), dtype=torch.uint8, pin_memory=True)
        self.mem = self.buf.numpy()
        self.size = int(nbytes)
        self.head = 0
        self.live = deque()  # [start, end, released] oldest first

    def _reclaim(self):
        while self.live and self.live[0][2]:
            self.live.popleft()

    def alloc(self, nbytes: int):
        """A block of at least nbytes, as (token, start), or None if full."""
        n = -(-int(nbytes) // self.ALIGN) * self.ALIGN
        if n > self.size:
            return None
        self._reclaim()
        tail = self.live[0][0] if self.live else None
        start = self.head
        if tail is None:
            start = 0 if self.head + n > self.size else self.head
        elif self.head >= tail:           # free space: [head, size) and [0, tail)
            if self.head + n > self.size:
                if n >= tail:
                    return None
                start = 0
        elif self.head + n >= tail:       # free space: [head, tail)
            return None
        blk = [start, start + n, False]
        self.live.append(blk)
        self.head = start + n
        return blk, start

    def release(self, token):
        token[2] = True
        self._reclaim()

    def view(self, start: int, dtype, count: int):
        return self.mem[start:start + count * np.dtype(dtype).itemsize].view(dtype)

    def tensor(self, start: int, torch_dtype, count: int, itemsize: int):
        return self.buf[start:start + count * itemsize].view(torch_dtype)


class GpuExecutor:
    """Resident device arrays, a copy stream and a compute stream, pinned
    staging rings, and a replayable plan over the arrays."""

    def __init__(self, capacity: int, max_curves: int = 4096, max_W: int = 721, device=0,
                 staging_bytes: int = 4 << 30, copy_threads: int = 4):
        import torch

        from . import _lib
        self.torch = torch
        self.capacity = int(capacity)
        self.dev = torch.device("cuda", device)
        self.flux = torch.zeros(self.capacity, dtype=torch.float32, device=self.dev)
        self.time = torch.zeros(self.capacity, dtype=torch.float64, device=self.dev)
        self.trend = torch.zeros(self.capacity, dtype=torch.float32, device=self.dev)
        self.copy_stream = torch.cuda.Stream(device=self.dev)
        self.compute_stream = torch.cuda.Stream(device=self.dev)
        self.plan = _lib.Plan(self.flux, self.time, self.trend, None, max_curves=max_curves,
                              max_W=max_W, stream=self.compute_stream)
        self.max_curves = int(max_curves)
        self.max_W = int(max_W)
        self.ring_in = PinnedRing(torch, staging_bytes)        # flux + time of admitted groups
        self.ring_out = PinnedRing(torch, staging_bytes // 3)  # trend of finished steps
        # native threads for the copies into and out of pinned staging; the
        # host<->device copies of a group or a step are one native call each
        self.copy_threads = max(1, int(copy_threads))
        self._copy = _lib.host_copy_many
        self._copy_async = _lib.copy_async
        # the rings are pinned, so the copies run as a kernel that reaches
        # them directly: enqueues through the runtime's copy engines have
        # blocked the scheduler thread for several milliseconds now and then
        self._H2D = _lib.COPY_H2D | _lib.COPY_KERNEL
        self._D2H = _lib.COPY_D2H | _lib.COPY_KERNEL
        self._flux_ptr = self.flux.data_ptr()
        self._time_ptr = self.time.data_ptr()
        self._trend_ptr = self.trend.data_ptr()
        self._copy_stream_ptr = int(self.copy_stream.cuda_stream)
        self.pinned_fallbacks = 0  # one-off pinned blocks taken because a ring was full
        # seconds spent in each part of staging and launching (diagnostics)
        self.phase_s = {"stage_alloc": 0.0, "stage_list": 0.0, "stage_copy": 0.0,
                        "h2d": 0.0, "h2d_enqueue": 0.0, "h2d_event": 0.0, "launch_plan": 0.0,
                        "d2h": 0.0, "results": 0.0}
        self.phase_max_s = dict.fromkeys(self.phase_s, 0.0)  # longest single call of each

    def _phase(self, name, dt):
        self.phase_s[name] += dt
        if dt > self.phase_max_s[name]:
            self.phase_max_s[name] = dt

    def _pinned(self, ring, nbytes):
        got = ring.alloc(nbytes)
        if got is None:  # ring full: a one-off pinned block
            self.pinned_fallbacks += 1
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, pin_memory=True)
            return None, t, t.numpy()
        tok, start = got
        return tok, ring.buf[start:start + int(nbytes)], ring.mem[start:start + int(nbytes)]

    def upload_many(self, groups):
        """Upload several groups ((offset, parts) pairs, parts = the requests'
        (flux, time) arrays): one pinned ring block holds them all (each
        group's times, then its fluxes), one batched native copy fills it, one
        native call enqueues every host-to-device copy, and one event marks
        them done.  Returns one upload handle per group; the first carries the
        ring block, which is released when its step completes (every group's
        copy is done by then: the steps wait on the shared event)."""
        clk = _time.perf_counter
        if not groups:
            return []
        t0 = clk()
        sizes = []
        for offset, parts in groups:
            n = sum(f.size for f, _ in parts)
            if not (0 <= offset and offset + n <= self.capacity):
                raise ValueError("upload range [%d, %d) outside the arena" % (offset, offset + n))
            sizes.append(n)
        align = PinnedRing.ALIGN
        spans = [(12 * n + align - 1) // align * align for n in sizes]
        tok, tbuf, mem = self._pinned(self.ring_in, sum(spans))
        t1 = clk()
        bases = _addr(mem) + np.concatenate([[0], np.cumsum(spans[:-1])]).astype(np.int64)
        dst, src, nbytes = staging_copies_many([parts for _, parts in groups], bases)
        offs = np.fromiter((o for o, _ in groups), np.int64, len(groups))
        ns = np.asarray(sizes, np.int64)
        h_dst = np.concatenate([self._time_ptr + 8 * offs, self._flux_ptr + 4 * offs])
        h_src = np.concatenate([bases, bases + 8 * ns])
        h_nb = np.concatenate([8 * ns, 4 * ns])
        t2 = clk()
        self._copy(dst, src, nbytes, self.copy_threads)
        t3 = clk()
        self._copy_async(h_dst.astype(np.uint64), h_src.astype(np.uint64), h_nb, self._H2D,
                         self._copy_stream_ptr)
        t3b = clk()
        ev = self.torch.cuda.Event()
        ev.record(self.copy_stream)
        t4 = clk()
        self._phase("h2d_enqueue", t3b - t3)
        self._phase("h2d_event", t4 - t3b)
        self._phase("stage_alloc", t1 - t0)
        self._phase("stage_list", t2 - t1)
        self._phase("stage_copy", t3 - t2)
        self._phase("h2d", t4 - t3)
        return [(ev, tok, tbuf)] + [(ev, None, None)] * (len(groups) - 1)

    def stage_upload(self, offset: int, parts):
        """Upload one group (see upload_many)."""
        return self.upload_many([(offset, parts)])[0]

    def upload(self, offset: int, flux: np.ndarray, time: np.ndarray):
        return self.stage_upload(offset, [(flux, time)])

    def launch(self, offsets, lengths, Ws, alphas, cs, iters, uploads, ranges):
        """Run one batch; then copy each (offset, size) range of the trend back."""
        torch = self.torch
        for off, size in ranges:
            if not (0 <= off and off + size <= self.capacity):
                raise ValueError("result range [%d, %d) outside the arena" % (off, off + size))
        t0 = _time.perf_counter()
        seen = set()
        for ev, _, _ in uploads:  # groups uploaded together share one event
            if id(ev) not in seen:
                seen.add(id(ev))
                self.compute_stream.wait_event(ev)
        try:
            self.plan.run(offsets, lengths, Ws, np.asarray(alphas, np.float32),
                          np.asarray(cs, np.float32), iters)
        except Exception:
            # the step never ran: its uploads' staging is free once copied
            for ev, tok, _ in uploads:
                ev.synchronize()
                if tok is not None:
                    self.ring_in.release(tok)
            raise
        computed = torch.cuda.Event()
        computed.record(self.compute_stream)
        t1 = _time.perf_counter()
        self.copy_stream.wait_event(computed)
        outs, dst, src, nbytes = [], [], [], []
        for off, size in ranges:
            tok, tbuf, mem = self._pinned(self.ring_out, 4 * size)
            arr = mem[:4 * size].view(np.float32)
            outs.append((tok, tbuf, arr))
            dst.append(_addr(arr))
            src.append(self._trend_ptr + 4 * off)
            nbytes.append(4 * size)
        self._copy_async(dst, src, nbytes, self._D2H, self._copy_stream_ptr)
        done = torch.cuda.Event()
        done.record(self.copy_stream)
        self._phase("launch_plan", t1 - t0)
        self._phase("d2h", _time.perf_counter() - t1)
        return (done, outs, [u[1] for u in uploads])

    def ready(self, handle) -> bool:
        return handle[0].query()

    def results(self, handle):
        t0 = _time.perf_counter()
        handle[0].synchronize()
        # fresh arrays: the ring blocks are reused right away
        res = [np.empty_like(arr) for _, _, arr in handle[1]]
        if res:
            self._copy([_addr(o) for o in res], [_addr(arr) for _, _, arr in handle[1]],
                       [o.nbytes for o in res], self.copy_threads)
        for tok, _, _ in handle[1]:
            if tok is not None:
                self.ring_out.release(tok)
        for tok in handle[2]:  # the step is done, so its uploads are too
            if tok is not None:
                self.ring_in.release(tok)
        self._phase("results", _time.perf_counter() - t0)
        return res

    def close(self):
        self.plan.destroy()


class FakeExecutor:
    """CPU stand-in with the executor interface: `fn(flux, time, W, alpha, c,
    iters)` computes one curve, `delay` seconds model a step's device time,
    and `fail_when(step_index, curves)` may raise to inject a step failure."""

    def __init__(self, capacity: int, fn=None, delay: float = 0.0, fail_when=None,
                 max_curves: int = 4096):
        self.capacity = int(capacity)
        self.flux = np.zeros(self.capacity, np.float32)
        self.time = np.zeros(self.capacity, np.float64)
        self.fn = fn or (lambda f, t, W, a, c, it: f.astype(np.float32) * np.float32(2.0))
        self.delay = delay
        self.fail_when = fail_when
        self.max_curves = int(max_curves)
        self.max_W = 2047
        self._step = itertools.count()

    def upload(self, offset, flux, time):
        self.flux[offset:offset + flux.size] = flux
        self.time[offset:offset + flux.size] = time
        return None

    def launch(self, offsets, lengths, Ws, alphas, cs, iters, uploads, ranges):
        k = next(self._step)
        if self.fail_when is not None:
            self.fail_when(k, len(offsets))
        trend = np.full(self.capacity, np.nan, np.float32)
        for o, L, W, a, c in zip(offsets, lengths, Ws, alphas, cs):
            trend[o:o + L] = self.fn(self.flux[o:o + L], self.time[o:o + L], W, a, c, iters)
        outs = [trend[o:o + s].copy() for o, s in ranges]
        return (_time.perf_counter() + self.delay, outs)

    def ready(self, handle) -> bool:
        return _time.perf_counter() >= handle[0]

    def results(self, handle):
        while not self.ready(handle):
            _time.sleep(max(0.0, handle[0] - _time.perf_counter()))
        return handle[1]

    def close(self):
        pass


# ---------------------------------------------------------------------------
# server


class Server:
    # Samples per step (and per admission group): bounds the pinned staging a
    # step needs, so the executor's rings always have room (a lone request
    # larger than this still forms a step of its own).
    MAX_STEP_SAMPLES = 1 << 25

    def __init__(self, executor, max_step_curves: int | None = None, max_inflight: int = 2,
                 clock=_time.perf_counter, max_step_samples: int | None = None):
        self.ex = executor
        self.arena = Arena(executor.capacity)
        self.max_step_curves = int(max_step_curves or getattr(executor, "max_curves", 4096))
        self.max_step_samples = int(max_step_samples or self.MAX_STEP_SAMPLES)
        self.max_inflight = max_inflight
        self.max_W = int(getattr(executor, "max_W", 2047))
        self.clock = clock
        self.stats = Stats()
        self._ids = itertools.count()
        self._lock = threading.Condition()
        self._waiting: deque = deque()   # submitted, not admitted
        self._groups: list = []           # admitted and uploaded, not launched
        self._to_upload: deque = deque()  # admitted, upload not started
        self._inflight: deque = deque()   # launched steps, oldest first
        self._closing = False
        self._error: BaseException | None = None
        self._thread = threading.Thread(target=self._loop, name="umi-serve", daemon=True)
        self._thread.start()

    # -- client side -------------------------------------------------------
    def submit(self, flux, time=None, W: int = 361, alpha: float = 2.0, c: float = 5.0,
               iters: int = 5, arrival: float | None = None) -> Future:
        fut: Future = Future()
        flux = np.ascontiguousarray(flux, dtype=np.float32)
        if time is None:
            time_ = np.zeros(flux.size, np.float64)  # no gap information
        else:
            time_ = np.ascontiguousarray(time, dtype=np.float64)
        arrival = self.clock() if arrival is None else arrival
        try:
            if flux.ndim != 1 or time_.shape != flux.shape:
                raise ValueError("flux and time must be 1-D of equal length")
            if W < 1 or W % 2 == 0 or W > self.max_W:
                raise ValueError("W must be odd, 1 <= W <= %d" % self.max_W)
            # the kernels take alpha and c as float32: a value that overflows
            # or flushes there would fail the whole step it shares
            with np.errstate(over="ignore"):
                a32, c32 = np.float32(alpha), np.float32(c)
            if not (np.isfinite(a32) and a32 > 0 and np.isfinite(c32) and c32 > 0):
                raise ValueError("alpha and c must be finite and > 0 as float32")
            if int(iters) != iters or iters < 0:
                raise ValueError("iters must be an integer >= 0")
            if flux.size > self.arena.capacity:
                raise Rejected("curve of %d samples exceeds the device budget of %d samples"
                               % (flux.size, self.arena.capacity))
        except ValueError as e:
            with self._lock:
                self.stats.rejected += 1
            fut.set_exception(e)
            return fut
        if flux.size == 0:  # nothing to compute: resolved at once
            fut.set_result(np.zeros(0, np.float32))
            return fut
        req = Request(next(self._ids), flux, time_, int(W), float(alpha), float(c), int(iters),
                      arrival, fut)
        submitted = self.clock()
        with self._lock:
            self.stats.submit_lag.append(submitted - arrival)
            if self._closing:
                raise RuntimeError("server is closed")
            if self.stats.first_arrival is None or arrival < self.stats.first_arrival:
                self.stats.first_arrival = arrival
            self._waiting.append(req)
            self._lock.notify_all()
        return fut

    def close(self, timeout: float | None = None):
        """Finish everything submitted, then stop."""
        with self._lock:
            self._closing = True
            self._lock.notify_all()
        self._thread.join(timeout)
        self.ex.close()
        if self._error is not None:
            raise RuntimeError("scheduler failed") from self._error

    def summary(self) -> dict:
        with self._lock:
            out = self.stats.summary(self.arena)
            out["pinned_fallbacks"] = getattr(self.ex, "pinned_fallbacks", None)
            ph = getattr(self.ex, "phase_s", None)
            if ph is not None:
                out["executor_phase_s"] = dict(ph)
            pm = getattr(self.ex, "phase_max_s", None)
            if pm is not None:
                out["executor_phase_max_ms"] = {k: v * 1e3 for k, v in pm.items()}
            return out

    def reset_stats(self):
        """Start a new measurement window (e.g. after a warm-up)."""
        with self._lock:
            self.stats = Stats()
            for name in ("phase_s", "phase_max_s"):
                ph = getattr(self.ex, name, None)
                if ph is not None:
                    for k in ph:
                        ph[k] = 0.0
            self.arena.high_water = self.arena.used

    # -- scheduler ---------------------------------------------------------
    def _admit(self):
        """Admit waiting requests FIFO into contiguous arena groups per key."""
        admitted = []
        while self._waiting:
            req = self._waiting[0]
            if req.future.cancelled():
                self._waiting.popleft()
                continue
            off = self.arena.alloc(req.n)
            if off is None:
                break  # head of line waits for memory: FIFO admission
            self._waiting.popleft()
            req.offset = off
            req.admitted = self.clock()
            admitted.append(req)
        # requests admitted together with equal parameters form one group; a
        # group's arena range is contiguous when its requests' ranges are
        groups = []
        for req in admitted:
            g = groups[-1] if groups else None
            if (g is not None and g.key == req.key and g.offset + g.size == req.offset
                    and len(g.requests) < self.max_step_curves
                    and g.size + req.n <= self.max_step_samples):
                g.requests.append(req)
                g.size += req.n
            else:
                groups.append(Group(req.key, req.offset, req.n, [req]))
        return groups

    def _upload(self, groups):
        if hasattr(self.ex, "upload_many"):
            ups = self.ex.upload_many([(g.offset, [(r.flux, r.time) for r in g.requests])
                                       for g in groups])
            for g, up in zip(groups, ups):
                g.upload = up
            return
        for g in groups:
            parts = [(r.flux, r.time) for r in g.requests]
            if hasattr(self.ex, "stage_upload"):
                g.upload = self.ex.stage_upload(g.offset, parts)
            else:
                g.upload = self.ex.upload(g.offset, np.concatenate([p[0] for p in parts]),
                                          np.concatenate([p[1] for p in parts]))

    def _next_step(self):
        """The oldest admitted key's groups, up to the step's curve limit."""
        if not self._groups:
            return None
        key = self._groups[0].key
        chosen, n, samples = [], 0, 0
        for g in self._groups:  # groups respect both limits on their own (see _admit)
            if (g.key == key and n + len(g.requests) <= self.max_step_curves
                    and (not chosen or samples + g.size <= self.max_step_samples)):
                chosen.append(g)
                n += len(g.requests)
                samples += g.size
        for g in chosen:
            self._groups.remove(g)
        return Step(chosen)

    def _launch(self, step: Step):
        reqs = [r for g in step.groups for r in g.requests]
        now = self.clock()
        for r in reqs:
            r.launched = now
        try:
            step.handle = self.ex.launch([r.offset for r in reqs], [r.n for r in reqs],
                                         [r.W for r in reqs], [r.alpha for r in reqs],
                                         [r.c for r in reqs], step.groups[0].key,
                                         [g.upload for g in step.groups if g.upload is not None],
                                         [(g.offset, g.size) for g in step.groups])
            step.launched_at = now
            self.stats.steps += 1
            self.stats.step_curves.append(len(reqs))
            self.stats.step_samples_max = max(self.stats.step_samples_max,
                                              sum(g.size for g in step.groups))
            return True
        except Exception as e:  # a failed step fails only its own requests
            self._finish(step, error=e)
            return False

    def _finish(self, step: Step, error: BaseException | None = None):
        outs = None
        if error is None:
            try:
                outs = self.ex.results(step.handle)
            except Exception as e:
                error = e
        now = self.clock()
        settle = []
        for gi, g in enumerate(step.groups):
            pos = 0
            for r in g.requests:
                r.done = now
                if error is None:
                    settle.append((r, outs[gi][pos:pos + r.n]))
                    self.stats.completed += 1
                    self.stats.samples += r.n
                    self.stats.latencies.append(now - r.arrival)
                    self.stats.queued.append(r.admitted - r.arrival)
                    self.stats.staged.append(r.launched - r.admitted)
                    self.stats.service.append(now - r.launched)
                else:
                    settle.append((r, None))
                    self.stats.failed += 1
                pos += r.n
            self.arena.free(g.offset, g.size)
        self.stats.last_done = now
        for r, res in settle:  # statistics are complete before any caller wakes
            if r.future.cancelled():
                continue
            if error is None:
                r.future.set_result(res)
            else:
                r.future.set_exception(error)

    def _loop(self):
        clk = self.clock
        groups = []
        try:
            while True:
                t0 = clk()
                with self._lock:
                    # completions first: they free memory for admissions
                    while self._inflight and self.ex.ready(self._inflight[0].handle):
                        self._finish(self._inflight.popleft())
                    t1 = clk()
                    self._to_upload.extend(self._admit())
                    # stage uploads ahead of launch, but no more than two
                    # steps' worth: pinned staging stays bounded under backlog
                    staged = sum(g.size for g in self._groups)
                    groups = []
                    while self._to_upload and (not groups and not self._groups
                                               or staged < 2 * self.max_step_samples):
                        g = self._to_upload.popleft()
                        groups.append(g)
                        staged += g.size
                    t2 = clk()
                self._upload(groups)
                t3 = clk()
                with self._lock:
                    self._groups.extend(groups)
                    while self._groups and len(self._inflight) < self.max_inflight:
                        step = self._next_step()
                        if self._launch(step):
                            self._inflight.append(step)
                    t4 = clk()
                    ph = self.stats.phase_s
                    ph["finish"] += t1 - t0
                    ph["admit"] += t2 - t1
                    ph["upload"] += t3 - t2
                    ph["launch"] += t4 - t3
                    if t4 - t0 > self.stats.loop_max_s:
                        self.stats.loop_max_s = t4 - t0
                        self.stats.loop_max_phases = {"finish": t1 - t0, "admit": t2 - t1,
                                                      "upload": t3 - t2, "launch": t4 - t3}
                    idle = not self._inflight and not self._groups and not self._to_upload
                    if idle and not self._waiting and self._closing:
                        return
                    if idle and not self._waiting:
                        self._lock.wait(0.05)
                    elif self._inflight:
                        # poll the oldest step without holding the lock long
                        pass
                if self._inflight:
                    _time.sleep(2e-5)
        except BaseException as e:  # keep the failure visible to close()
            self._error = e
            with self._lock:
                self._fail_all(RuntimeError("scheduler failed: %r" % e), groups)

    def _fail_all(self, err, in_hand=()):
        """Fail every request not yet resolved: waiting, admitted (queued for
        upload, in the groups being uploaded, uploaded) and in flight.  Called
        with the lock held."""
        reqs = list(self._waiting)
        for g in list(self._to_upload) + list(in_hand) + list(self._groups):
            reqs.extend(g.requests)
        for st in self._inflight:
            for g in st.groups:
                reqs.extend(g.requests)
        for r in reqs:
            if not r.future.done():
                r.future.set_exception(err)
        self._waiting.clear()


# ---------------------------------------------------------------------------
# native server


class NativeServer:
    """The library's native serving loop (include/umi_serve.h, umi_server_*)
    behind the same interface as ``Server``: ``submit`` returns a Future,
    ``close``, ``summary`` and ``reset_stats``.  Admission, staging, uploads,
    steps and the copies of results into each request's output run in the
    library's own threads; Python validates a request, keeps its arrays alive
    until it completes, and resolves futures from one completion thread.

    The arena holds ``capacity`` samples (BYTES_PER_SAMPLE of device memory
    each, with the plan workspace).  Times are Python's perf_counter clock,
    which is the clock the library stamps completions with (CLOCK_MONOTONIC)."""

    # smaller than the Python loop's: after a hiccup the backlog then runs in
    # steps whose result copies stay short
    MAX_STEP_SAMPLES = 1 << 22

    def __init__(self, capacity: int, max_curves: int = 4096, max_W: int = 721, device: int = 0,
                 max_step_samples: int | None = None, max_inflight: int = 2,
                 staging_bytes: int = 4 << 30, copy_threads: int = 4):
        import ctypes

        from . import _lib
        self._lib = _lib
        self._ct = ctypes
        self.capacity = int(capacity)
        self.max_W = int(max_W)
        self.clock = _time.perf_counter
        cfg = _lib.ServerConfig(self.capacity, int(max_step_samples or self.MAX_STEP_SAMPLES),
                                int(staging_bytes), int(max_curves), self.max_W,
                                int(max_inflight), int(copy_threads), int(device), 0)
        h = ctypes.c_void_p()
        _lib._check(_lib.lib.umi_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._lock = threading.Lock()
        self._pending: dict = {}  # tag -> (future, flux, time, out, arrival)
        self._tags = itertools.count()
        self.stats = Stats()
        self._stop = False
        self._closed = False
        self._poller = threading.Thread(target=self._poll_loop, name="umi-serve-native",
                                        daemon=True)
        self._poller.start()
        # a server left open is shut down before the interpreter exits, so the
        # library's threads never outlive the process's teardown
        atexit.register(self.close)

    def submit(self, flux, time=None, W: int = 361, alpha: float = 2.0, c: float = 5.0,
               iters: int = 5, arrival: float | None = None) -> Future:
        fut: Future = Future()
        flux = np.ascontiguousarray(flux, dtype=np.float32)
        time_ = None if time is None else np.ascontiguousarray(time, dtype=np.float64)
        arrival = self.clock() if arrival is None else float(arrival)
        try:
            if flux.ndim != 1 or (time_ is not None and time_.shape != flux.shape):
                raise ValueError("flux and time must be 1-D of equal length")
            if W < 1 or W % 2 == 0 or W > self.max_W:
                raise ValueError("W must be odd, 1 <= W <= %d" % self.max_W)
            with np.errstate(over="ignore"):
                a32, c32 = np.float32(alpha), np.float32(c)
            if not (np.isfinite(a32) and a32 > 0 and np.isfinite(c32) and c32 > 0):
                raise ValueError("alpha and c must be finite and > 0 as float32")
            if int(iters) != iters or iters < 0:
                raise ValueError("iters must be an integer >= 0")
            if flux.size > self.capacity:
                raise Rejected("curve of %d samples exceeds the device budget of %d samples"
                               % (flux.size, self.capacity))
        except ValueError as e:
            with self._lock:
                self.stats.rejected += 1
            fut.set_exception(e)
            return fut
        if flux.size == 0:
            fut.set_result(np.zeros(0, np.float32))
            return fut
        out = np.empty(flux.size, np.float32)
        tag = next(self._tags)
        with self._lock:
            if self._closed:
                raise RuntimeError("server is closed")
            self._pending[tag] = (fut, flux, time_, out, arrival)
            st = self.stats
            st.submit_lag.append(self.clock() - arrival)
            if st.first_arrival is None or arrival < st.first_arrival:
                st.first_arrival = arrival
        status = self._lib.lib.umi_server_submit(
            self._h, flux.ctypes.data, None if time_ is None else time_.ctypes.data, flux.size,
            int(W), float(a32), float(c32), int(iters), arrival, out.ctypes.data, tag)
        if status != self._lib.UMI_OK:
            with self._lock:
                self._pending.pop(tag, None)
            raise self._lib.UmiError(status, self._lib.last_error())
        return fut

    def _poll_loop(self):
        ct = self._ct
        lib = self._lib.lib
        buf = (self._lib.ServerCompletion * 512)()
        n = ct.c_int32(0)
        while True:
            lib.umi_server_poll(self._h, buf, 512, 0.05, ct.byref(n))
            k = n.value
            if k == 0:
                if self._stop:
                    return
                continue
            settle = []
            with self._lock:
                st = self.stats
                for j in range(k):
                    cpl = buf[j]
                    fut, flux, _, out, arrival = self._pending.pop(cpl.tag)
                    if cpl.status == 0:
                        st.completed += 1
                        st.samples += flux.size
                        st.latencies.append(cpl.done - arrival)
                        st.queued.append(cpl.admitted - arrival)
                        st.staged.append(cpl.launched - cpl.admitted)
                        st.service.append(cpl.done - cpl.launched)
                        if st.last_done is None or cpl.done > st.last_done:
                            st.last_done = cpl.done
                        settle.append((fut, out, None))
                    else:
                        st.failed += 1
                        settle.append((fut, None, self._lib.UmiError(
                            cpl.status, "the step this request ran in failed")))
            for fut, out, err in settle:  # statistics are complete before any caller wakes
                if fut.cancelled():
                    continue
                if err is None:
                    fut.set_result(out)
                else:
                    fut.set_exception(err)

    def close(self, timeout: float | None = None):
        """Finish everything submitted, then stop and free the server."""
        with self._lock:
            if self._closed:
                return
            self._closed = True
        atexit.unregister(self.close)
        self._lib.lib.umi_server_shutdown(self._h)
        self._stop = True
        self._poller.join(timeout)
        self._lib.lib.umi_server_destroy(self._h)
        self._h = None

    def native_stats(self) -> dict:
        ns = self._lib.ServerStats()
        self._lib._check(self._lib.lib.umi_server_stats_get(self._h, self._ct.byref(ns)))
        return {name: (list(getattr(ns, name)) if name.endswith("_s") and name != "longest_iteration_s"
                       else getattr(ns, name)) for name, _ in ns._fields_}

    def summary(self) -> dict:
        ns = self.native_stats()
        with self._lock:
            out = self.stats.summary()
        phases = ("finish", "admit", "upload", "launch")
        out["steps"] = ns["steps"]
        out["mean_curves_per_step"] = ns["step_curves"] / ns["steps"] if ns["steps"] else None
        out["largest_step_samples"] = ns["largest_step_samples"]
        out["scheduler_phase_s"] = dict(zip(phases, ns["loop_s"]))
        out["scheduler_longest_iteration_ms"] = ns["longest_iteration_s"] * 1e3
        out["scheduler_longest_iteration_phases_ms"] = {
            k: v * 1e3 for k, v in zip(phases, ns["longest_iteration_loop_s"])}
        out["executor_phase_s"] = dict(zip(("stage_copy", "upload_enqueue", "launch_plan",
                                            "results"), ns["exec_s"]))
        out["arena_high_water_samples"] = ns["arena_high_water"]
        out["arena_capacity_samples"] = ns["arena_capacity"]
        out["pinned_fallbacks"] = ns["staging_fallbacks"]
        out["scheduler"] = "native"
        return out

    def reset_stats(self):
        """Start a new measurement window (e.g. after a warm-up)."""
        with self._lock:
            self.stats = Stats()
        self._lib._check(self._lib.lib.umi_server_reset_stats(self._h))


# ---------------------------------------------------------------------------
# open-loop driver


def run_open_loop(server: Server, curves, arrivals, keep_results=None, pause_gc=True,
                  progress=None, progress_every: float = 10.0):
    """Submit ``curves[i % len(curves)]`` at times ``arrivals`` (seconds from
    the start) regardless of completions, then wait for all of them.
    ``keep_results(i)`` selects the requests whose results are returned;
    ``progress(submitted, seconds)``, if given, is called about every
    ``progress_every`` seconds while requests are being submitted.
    With ``pause_gc`` the cyclic garbage collector is frozen and paused for
    the measured window (its full sweeps over ~1e5 live requests otherwise
    stall both the scheduler and the arrival generator for tens of ms).
    Returns (summary, {i: (curve index, result)})."""
    import gc
    if pause_gc:
        gc.collect()
        gc.freeze()
        gc.disable()
    try:
        return _open_loop(server, curves, arrivals, keep_results, progress, progress_every)
    finally:
        if pause_gc:
            gc.enable()
            gc.unfreeze()


def _open_loop(server, curves, arrivals, keep_results, progress=None, progress_every=10.0):
    # Results are taken as they complete and dropped unless kept, as a client
    # would: holding every result of a minute at 20,000 curves/s would pin
    # about 100 GB of host memory and stall both threads in page faults.
    t0 = server.clock()
    pending = deque()
    kept = {}

    def drain(wait):
        while pending and (wait or pending[0][1].done()):
            i, fu = pending.popleft()
            res = fu.result()
            if keep_results is not None and keep_results(i):
                # a copy: the result is a view of its whole group's array
                kept[i] = (i % len(curves), np.array(res))

    next_report = t0 + progress_every
    for i, at in enumerate(arrivals):
        target = t0 + float(at)
        drain(False)
        if progress is not None and target >= next_report:
            progress(i, target - t0)
            next_report += progress_every
        while True:
            now = server.clock()
            if now >= target:
                break
            _time.sleep(min(target - now, 0.001))
        f, t, W = curves[i % len(curves)]
        pending.append((i, server.submit(f, t, W, arrival=target)))
    drain(True)
    return server.summary(), kept
