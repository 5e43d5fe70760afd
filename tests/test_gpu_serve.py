"""GPU serving: continuous batching through the replayable plan.

Curves drawn like the mixed workload arrive while earlier ones run, each
with one of the Table 4 (alpha, c) settings, so steps mix them; every result
must equal the same curve run alone through the C ABI with its own setting
within the trend tolerance (1e-5 relative; a lone curve may split its
windows over several lanes, which orders the sums differently), and sampled
positions must match the FP64 oracle (trend at 1e-5 relative).
"""
from __future__ import annotations

import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.mark.parametrize("scheduler", ["python", "native"])
def test_serving_results_equal_alone_and_oracle(torch, oracle_lib, scheduler):
    import paper_2604_06602_amd as umi
    from paper_2604_06602_amd.serve import GpuExecutor, NativeServer, Server

    rng = np.random.default_rng(4)
    presets = [(2.0, 5.0), (3.0, 5.0), (1.0, 5.0), (10.0, 2.5)]
    curves = []
    for i in range(60):
        f, t, W = synth.curve_for(4, i)
        L = min(f.size, 30000)
        curves.append((f[:L], t[:L], W) + presets[i % 4])
    total = sum(cv[0].size for cv in curves)
    print("serving test: %s scheduler, %d curves" % (scheduler, len(curves)), flush=True)
    if scheduler == "native":  # the library's own loop; small staging rings
        srv = NativeServer(total // 2, max_curves=64, max_W=721, staging_bytes=16 << 20,
                           max_step_samples=40000)
    else:
        ex = GpuExecutor(capacity=total // 2, max_curves=64, max_W=721)  # budget forces queueing
        srv = Server(ex)
    futs = []
    for i, (f, t, W, a, c) in enumerate(curves):
        futs.append(srv.submit(f, t, W, alpha=a, c=c))
        if i % 10 == 9:  # bursts of ten: later arrivals find earlier ones on the GPU
            time.sleep(float(rng.exponential(0.002)))
    results = [fu.result(timeout=120) for fu in futs]
    summary = srv.summary()
    srv.close()
    assert summary["completed"] == len(curves) and summary["steps"] < len(curves)
    for (f, t, W, a, c), res in zip(curves, results):
        fd = torch.from_numpy(f).cuda()
        td = torch.from_numpy(t).cuda()
        alone, _ = umi.detrend(fd, td, W, alpha=a, c=c)
        torch.cuda.synchronize()
        alone = alone.cpu().numpy()
        # a lone curve takes split tiles (several lanes per window), a crowded
        # step may not: the same within the trend tolerance, NaNs identical
        assert np.array_equal(np.isnan(alone), np.isnan(res))
        ok = ~np.isnan(res)
        if ok.any():
            rel = np.abs(alone[ok].astype(np.float64) - res[ok]) / np.abs(res[ok])
            assert rel.max() <= 1e-5
    for (f, t, W, a, c), res in list(zip(curves, results))[:8]:
        idx = np.unique(rng.integers(0, f.size, 40))
        o_tr, _ = oracle_lib.detrend_at(f, t, W, idx, alpha=a, c=c)
        ok = ~np.isnan(o_tr)
        assert np.array_equal(np.isnan(res[idx]), ~ok)
        rel = np.abs(res[idx][ok] - o_tr[ok]) / np.abs(o_tr[ok])
        assert rel.max() <= 1e-5


@pytest.mark.parametrize("by_kernel", [False, True], ids=["copy_engine", "copy_kernel"])
def test_copy_async_round_trip(torch, by_kernel):
    """The serving loop's batched host<->device copies: a ragged list of
    pinned-host ranges up to the device and back on one stream, every byte
    where it belongs and nothing written past the ranges -- through the
    runtime's copy engines, and as the copy kernel (odd sizes and offsets take
    its byte path, aligned ones its 16-byte path, and more than 64 copies
    take several launches)."""
    import paper_2604_06602_amd as umi
    rng = np.random.default_rng(9)
    sizes = [0, 1, 4096, 1 << 20, 3 * (1 << 20) + 5]
    if by_kernel:
        sizes = sizes + [int(v) for v in rng.integers(0, 70000, 90)] + [16, 32768, 32769]
    flag = umi.COPY_KERNEL if by_kernel else 0
    total = sum(sizes)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    host = torch.empty(total, dtype=torch.uint8, pin_memory=True)
    host.numpy()[:] = rng.integers(0, 256, total, dtype=np.uint8)
    back = torch.zeros(total, dtype=torch.uint8, pin_memory=True)
    dev = torch.zeros(total + 64, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    umi.copy_async([dev.data_ptr() + int(o) for o in offs], [host.data_ptr() + int(o) for o in offs],
                   sizes, umi.COPY_H2D | flag, s)
    umi.copy_async([back.data_ptr() + int(o) for o in offs], [dev.data_ptr() + int(o) for o in offs],
                   sizes, umi.COPY_D2H | flag, s)
    s.synchronize()
    assert torch.equal(back, host)
    assert not dev[total:].any().item()


def test_executor_device_memory_stays_within_its_budget(torch):
    """The serving executor's arrays plus the plan workspace that
    umi_plan_create allocates hold at most BYTES_PER_SAMPLE per sample of the
    arena (measured as the drop in free device memory; torch's allocator
    rounds each array up to 2 MiB)."""
    from paper_2604_06602_amd.serve import BYTES_PER_SAMPLE, GpuExecutor
    budget = 2 << 30
    capacity = budget // BYTES_PER_SAMPLE
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info()
    ex = GpuExecutor(capacity, max_curves=4096, max_W=721, staging_bytes=64 << 20)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    used = free0 - free1
    ex.close()
    del ex
    assert used <= budget + 3 * (2 << 20) + (1 << 20), (used, budget)
    assert used >= capacity * (BYTES_PER_SAMPLE - 1)  # the estimate is not loose either


def test_native_server_steps_iterations_and_memory(torch, oracle_lib):
    """The native scheduler: requests larger than a step (each a step of its
    own), two iteration counts (never mixed in a step), curves without times
    (no gap breaks), empty requests and an arena smaller than the whole load
    (admission waits for memory); every result equals the curve run alone
    through the C ABI with its settings (trend tolerance, NaN pattern
    identical), a sample matches the FP64 oracle, and the server's device
    memory stays within BYTES_PER_SAMPLE per arena sample (plus staging-free
    slack: the rings are host memory)."""
    import paper_2604_06602_amd as umi
    from paper_2604_06602_amd.serve import BYTES_PER_SAMPLE, NativeServer

    rng = np.random.default_rng(11)
    reqs = []
    for i in range(40):
        f, t, W = synth.curve_for(4, 100 + i)
        L = min(f.size, 50000 if i % 9 == 0 else 20000)
        iters = 3 if i % 2 else 5
        tt = None if i % 5 == 3 else t[:L]
        reqs.append((f[:L], tt, W, iters))
    reqs.append((np.zeros(0, np.float32), None, 361, 5))
    biggest = max(r[0].size for r in reqs)
    capacity = max(biggest, sum(r[0].size for r in reqs) // 3)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info()
    srv = NativeServer(capacity, max_curves=32, max_W=721, staging_bytes=32 << 20,
                       max_step_samples=30000)
    torch.cuda.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    print("native server test: %d requests, arena %d samples, %d bytes of device memory"
          % (len(reqs), capacity, used), flush=True)
    futs = [srv.submit(f, t, W, iters=it) for f, t, W, it in reqs]
    results = [fu.result(timeout=120) for fu in futs]
    summary = srv.summary()
    srv.close()
    assert used <= capacity * BYTES_PER_SAMPLE + 8 * (2 << 20), (used, capacity)
    assert summary["completed"] == len(reqs) - 1 and summary["failed"] == 0
    assert biggest > 30000  # at least one request is larger than a step
    assert summary["largest_step_samples"] >= biggest  # it ran as a step of its own
    for (f, t, W, it), res in zip(reqs, results):
        assert res.shape == f.shape and res.dtype == np.float32
        if f.size == 0:
            continue
        fd = torch.from_numpy(f).cuda()
        td = None if t is None else torch.from_numpy(t).cuda()
        alone, _ = umi.detrend(fd, td, W, iters=it)
        torch.cuda.synchronize()
        alone = alone.cpu().numpy()
        assert np.array_equal(np.isnan(alone), np.isnan(res))
        ok = ~np.isnan(res)
        if ok.any():
            rel = np.abs(alone[ok].astype(np.float64) - res[ok]) / np.abs(res[ok])
            assert rel.max() <= 1e-5
    for (f, t, W, it), res in list(zip(reqs, results))[:6]:
        idx = np.unique(rng.integers(0, f.size, 40))
        tt = np.zeros(f.size) if t is None else t
        o_tr, _ = oracle_lib.detrend_at(f, tt, W, idx, iters=it)
        ok = ~np.isnan(o_tr)
        assert np.array_equal(np.isnan(res[idx]), ~ok)
        rel = np.abs(res[idx][ok] - o_tr[ok]) / np.abs(o_tr[ok])
        assert rel.max() <= 1e-5
