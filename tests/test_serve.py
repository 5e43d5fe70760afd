"""Serving scheduler on the CPU: a fake executor stands in for the GPU.

Covers the arena allocator, continuous batching (results identical alone and
in a mix), admission by budget, rejection, cancellation, a failed step
failing only its own requests, and parameter grouping.
"""
from __future__ import annotations

import threading
import time

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

from paper_2604_06602_amd.serve import Arena, FakeExecutor, Rejected, Server


def running_mean(f, t, W, a, c, it):
    k = np.ones(W) / W
    return (np.convolve(f.astype(np.float64), k, mode="same") * a + c + it).astype(np.float32)


@settings(max_examples=60, deadline=None)
@given(st.lists(st.tuples(st.booleans(), st.integers(1, 40)), max_size=60))
def test_arena_matches_a_bitmap(ops):
    cap = 200
    a = Arena(cap)
    used = np.zeros(cap, bool)
    live = []
    for is_alloc, n in ops:
        if is_alloc or not live:
            off = a.alloc(n)
            if off is None:
                # first fit failed: no run of n free slots may exist
                assert all(r < n for r in _free_runs(used))
                continue
            assert not used[off:off + n].any() and off + n <= cap
            used[off:off + n] = True
            live.append((off, n))
        else:
            off, n = live.pop(len(live) // 2)
            a.free(off, n)
            used[off:off + n] = False
        assert a.used == used.sum()
        # free list is sorted, disjoint, coalesced, and matches the bitmap
        prev_end = -1
        for s, L in a._free:
            assert s > prev_end and not used[s:s + L].any()
            prev_end = s + L
        assert sum(L for _, L in a._free) == cap - used.sum()


def _free_runs(used):
    runs, n = [], 0
    for u in used:
        if u:
            if n:
                runs.append(n)
            n = 0
        else:
            n += 1
    if n:
        runs.append(n)
    return runs


def _curves(n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        L = int(rng.integers(50, 400))
        out.append((rng.normal(1, 1e-3, L).astype(np.float32), np.arange(L) * 0.01,
                    int(rng.choice([5, 11, 25]))))
    return out


def test_results_identical_alone_and_in_a_mix():
    curves = _curves(40)
    alone = []
    srv = Server(FakeExecutor(100000, fn=running_mean))
    for f, t, W in curves:
        alone.append(srv.submit(f, t, W).result(timeout=10))
    srv.close()
    srv = Server(FakeExecutor(100000, fn=running_mean, delay=0.002))
    futs = [srv.submit(f, t, W) for f, t, W in curves]
    mixed = [fu.result(timeout=10) for fu in futs]
    s = srv.summary()
    srv.close()
    for x, y in zip(alone, mixed):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
    assert s["completed"] == 40 and s["steps"] < 40  # requests shared steps


def test_budget_forces_queueing_and_everything_completes():
    curves = [(np.ones(400, np.float32), None, 5) for _ in range(30)]
    ex = FakeExecutor(1000, delay=0.001)
    srv = Server(ex)
    futs = [srv.submit(f, t, W) for f, t, W in curves]
    for fu in futs:
        assert np.array_equal(fu.result(timeout=10), np.full(400, 2.0, np.float32))
    s = srv.summary()
    srv.close()
    assert s["arena_high_water_samples"] <= 1000 and s["completed"] == 30


def test_oversize_and_invalid_requests_are_rejected():
    srv = Server(FakeExecutor(1000))
    with pytest.raises(Rejected):
        srv.submit(np.ones(1001, np.float32)).result(timeout=5)
    with pytest.raises(ValueError):
        srv.submit(np.ones(10, np.float32), W=4).result(timeout=5)
    with pytest.raises(ValueError):
        srv.submit(np.ones(10, np.float32), alpha=0.0).result(timeout=5)
    ok = srv.submit(np.ones(1000, np.float32), W=5)
    assert ok.result(timeout=5).size == 1000
    s = srv.summary()
    srv.close()
    assert s["rejected"] == 3


def test_parameters_that_break_float32_fail_only_their_request():
    """alpha or c that are infinite, or overflow or flush to zero as float32
    (the kernels' type), are rejected at submit; a step that the C ABI would
    reject as a whole never forms, so valid requests of the same burst run."""
    class CheckingExecutor(FakeExecutor):
        def launch(self, offsets, lengths, Ws, alphas, cs, iters, uploads, ranges):
            for a, c in zip(alphas, cs):  # the C ABI's finite_pos on float32
                a32, c32 = np.float32(a), np.float32(c)
                if not (np.isfinite(a32) and a32 > 0 and np.isfinite(c32) and c32 > 0):
                    raise RuntimeError("UMI_ERR_INVALID_ARG: per-curve alpha/c")
            return super().launch(offsets, lengths, Ws, alphas, cs, iters, uploads, ranges)
    srv = Server(CheckingExecutor(100000, delay=0.02))
    bad = [dict(alpha=float("inf")), dict(c=float("inf")), dict(alpha=1e39), dict(c=1e-50),
           dict(alpha=float("nan")), dict(iters=-1), dict(iters=2.5)]
    futs = []
    for i in range(len(bad)):
        futs.append(("ok", srv.submit(np.ones(100, np.float32), W=5)))
        futs.append(("bad", srv.submit(np.ones(100, np.float32), W=5, **bad[i])))
    for kind, fu in futs:
        if kind == "ok":
            assert fu.result(timeout=5)[0] == 2.0
        else:
            with pytest.raises(ValueError):
                fu.result(timeout=5)
    s = srv.summary()
    srv.close()
    assert s["rejected"] == len(bad) and s["completed"] == len(bad) and s["failed"] == 0


def test_cancelled_request_never_runs():
    gate = threading.Event()

    def slow(f, t, W, a, c, it):
        gate.wait(5)
        return f.copy()
    srv = Server(FakeExecutor(500, fn=slow))
    first = srv.submit(np.ones(500, np.float32), W=5)   # fills the whole budget
    time.sleep(0.05)
    second = srv.submit(np.ones(100, np.float32), W=5)  # must wait for memory
    assert second.cancel()
    gate.set()
    first.result(timeout=5)
    srv.close()
    assert second.cancelled()
    assert srv.summary()["completed"] == 1


def test_failed_step_fails_only_its_requests():
    def fail_second(step, n):
        if step == 1:
            raise RuntimeError("injected device fault")
    ex = FakeExecutor(100000, delay=0.01, fail_when=fail_second)
    srv = Server(ex, max_inflight=1)
    a = srv.submit(np.ones(100, np.float32), W=5)
    a.result(timeout=5)
    b = srv.submit(np.ones(100, np.float32), W=5)
    with pytest.raises(RuntimeError, match="injected"):
        b.result(timeout=5)
    c = srv.submit(np.ones(100, np.float32), W=5)
    assert c.result(timeout=5)[0] == 2.0
    s = srv.summary()
    srv.close()
    assert s["failed"] == 1 and s["completed"] == 2


def test_presets_share_steps_iteration_counts_do_not():
    """Per-curve alpha and c (Table 4) mix in one step and each curve gets its
    own pair; requests with another iteration count run in other steps."""
    seen = []

    def record(f, t, W, a, c, it):
        seen.append((a, c, it))
        return f * np.float32(a) + np.float32(c)

    class Recording(FakeExecutor):
        def launch(self, offsets, lengths, Ws, alphas, cs, iters, uploads, ranges):
            steps.append((len(offsets), iters))
            return super().launch(offsets, lengths, Ws, alphas, cs, iters, uploads, ranges)
    steps = []
    srv = Server(Recording(100000, fn=record, delay=0.02), max_inflight=1)
    first = srv.submit(np.ones(50, np.float32), W=5)          # occupies the device
    time.sleep(0.005)
    presets = [(2.0, 5.0), (3.0, 5.0), (1.0, 5.0), (10.0, 2.5)]
    futs = [srv.submit(np.ones(50, np.float32), W=5, alpha=a, c=c) for a, c in presets]
    other = srv.submit(np.ones(50, np.float32), W=5, iters=3)
    first.result(timeout=5)
    for (a, c), fu in zip(presets, futs):
        assert (fu.result(timeout=5) == np.float32(a) + np.float32(c)).all()
    other.result(timeout=5)
    srv.close()
    assert (4, 5) in steps or any(n >= 2 and it == 5 for n, it in steps[1:])
    assert all(it in (3, 5) for _, it in steps)
    assert sorted(set(seen)) == sorted(set([(a, c, 5) for a, c in presets] + [(2.0, 5.0, 3)]))


def test_latency_is_measured_from_scheduled_arrival():
    srv = Server(FakeExecutor(10000, delay=0.01))
    t0 = time.perf_counter()
    fu = srv.submit(np.ones(10, np.float32), W=5, arrival=t0 - 0.5)
    fu.result(timeout=5)
    s = srv.summary()
    srv.close()
    assert s["p50_ms"] >= 500


def test_admission_groups_respect_the_step_limit():
    class Checking(FakeExecutor):
        def launch(self, offsets, lengths, Ws, alphas, cs, iters, uploads, ranges):
            assert len(offsets) <= 7
            return super().launch(offsets, lengths, Ws, alphas, cs, iters, uploads, ranges)
    gate = threading.Event()
    srv = Server(Checking(100000, delay=0.001), max_step_curves=7)
    futs = [srv.submit(np.ones(20, np.float32), W=5) for _ in range(50)]
    for fu in futs:
        fu.result(timeout=10)
    s = srv.summary()
    srv.close()
    assert s["completed"] == 50 and s["steps"] >= 8


class _FakeTorch:
    """Enough of torch for PinnedRing on the CPU (no pinned memory here)."""
    uint8 = np.uint8

    class _T:
        def __init__(self, n):
            self.a = np.zeros(n, np.uint8)

        def numpy(self):
            return self.a

    @classmethod
    def empty(cls, n, dtype=None, pin_memory=False):
        return cls._T(n)


@settings(max_examples=80, deadline=None)
@given(st.lists(st.tuples(st.booleans(), st.integers(1, 3000)), max_size=80))
def test_pinned_ring_blocks_never_overlap(ops):
    from paper_2604_06602_amd.serve import PinnedRing
    ring = PinnedRing(_FakeTorch, 8192)
    live = []
    for is_alloc, n in ops:
        if is_alloc or not live:
            got = ring.alloc(n)
            if got is None:
                continue
            tok, start = got
            assert 0 <= start and start + n <= ring.size
            for t2, s2, n2 in live:
                assert start + n <= s2 or s2 + n2 <= start, "overlapping live blocks"
            live.append((tok, start, n))
        else:
            tok, _, _ = live.pop(len(live) // 3)
            ring.release(tok)
    for tok, _, _ in live:
        ring.release(tok)
    assert not ring.live
    assert ring.alloc(8192) is not None  # everything came back


def test_steps_respect_the_sample_limit_and_big_requests_still_run():
    """Groups and steps stay within max_step_samples, except a lone request
    larger than the limit, which forms a step of its own."""
    seen = []

    class Checking(FakeExecutor):
        def launch(self, offsets, lengths, Ws, alphas, cs, iters, uploads, ranges):
            seen.append(sum(lengths))
            return super().launch(offsets, lengths, Ws, alphas, cs, iters, uploads, ranges)
    srv = Server(Checking(100000, delay=0.002), max_step_samples=1000)
    futs = [srv.submit(np.ones(300, np.float32), W=5) for _ in range(20)]
    big = srv.submit(np.ones(2500, np.float32), W=5)
    futs += [srv.submit(np.ones(300, np.float32), W=5) for _ in range(10)]
    for fu in futs + [big]:
        fu.result(timeout=10)
    srv.close()
    assert 2500 in seen
    assert all(s <= 1000 for s in seen if s != 2500)
    assert sum(seen) == 30 * 300 + 2500


def test_upload_failure_fails_every_request_and_close_reports_it():
    """An exception in the uploader thread stops serving: every request ever
    submitted resolves (none hangs), those not finished with an error, and
    close() reports the failure."""
    class Failing(FakeExecutor):
        n = 0

        def upload(self, offset, flux, time):
            Failing.n += 1
            if Failing.n == 3:
                raise OSError("staging failed")
            return super().upload(offset, flux, time)
    srv = Server(Failing(100000, delay=0.002), max_step_curves=2)
    futs = [srv.submit(np.ones(100, np.float32), W=5) for _ in range(12)]
    done = [fu.exception(timeout=10) is None for fu in futs]
    assert not all(done) and any(isinstance(fu.exception(), RuntimeError) for fu in futs)
    with pytest.raises(RuntimeError):
        srv.close(timeout=10)


def test_staging_copies_many_lays_out_each_group_at_its_base():
    """Several groups staged at once: group g's times then fluxes at its own
    base address, each sample written once, nothing between the groups."""
    from paper_2604_06602_amd import host_copy_many
    from paper_2604_06602_amd.serve import staging_copies_many
    rng = np.random.default_rng(3)
    for trial in range(10):
        groups = []
        for _ in range(int(rng.integers(1, 6))):
            parts = []
            for _ in range(int(rng.integers(1, 8))):
                L = int(rng.integers(0, 5000))
                parts.append((rng.random(L).astype(np.float32), rng.random(L) * 27.0))
            groups.append(parts)
        spans = [(12 * sum(f.size for f, _ in g) + 255) // 256 * 256 for g in groups]
        buf = np.zeros(sum(spans) + 256, np.uint8)
        base0 = (buf.ctypes.data + 255) // 256 * 256
        off0 = base0 - buf.ctypes.data
        bases = base0 + np.concatenate([[0], np.cumsum(spans[:-1])]).astype(np.int64)
        dst, src, nbytes = staging_copies_many(groups, bases)
        host_copy_many(dst, src, nbytes, threads=1 + trial % 4)
        at = off0
        for g, span in zip(groups, spans):
            n = sum(f.size for f, _ in g)
            t = buf[at:at + 8 * n].view(np.float64)
            f = buf[at + 8 * n:at + 12 * n].view(np.float32)
            assert np.array_equal(t, np.concatenate([p[1] for p in g]))
            assert np.array_equal(f, np.concatenate([p[0] for p in g]))
            assert not buf[at + 12 * n:at + span].any()
            at += span


def test_empty_request_resolves_without_a_step():
    srv = Server(FakeExecutor(1000, delay=0.001))
    fu = srv.submit(np.zeros(0, np.float32), W=5)
    res = fu.result(timeout=10)
    assert res.dtype == np.float32 and res.size == 0
    assert srv.summary()["steps"] == 0
    srv.close()


def test_open_loop_reports_progress():
    from paper_2604_06602_amd.serve import run_open_loop
    srv = Server(FakeExecutor(100000, delay=0.0005))
    curves = [(np.ones(200, np.float32), np.arange(200) * 0.01, 5)]
    arrivals = np.linspace(0.0, 0.35, 60)
    seen = []
    summary, _ = run_open_loop(srv, curves, arrivals, progress=lambda n, s: seen.append((n, s)),
                               progress_every=0.1)
    srv.close()
    assert summary["completed"] == 60
    assert len(seen) >= 3 and all(b[0] > a[0] for a, b in zip(seen, seen[1:]))
