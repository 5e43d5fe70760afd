"""GPU: curves at explicit offsets (gather) and replayed plans (hipGraph).

Every replay of a captured plan is compared bit-for-bit with an eager batch
call on the same curves, with eager work and synchronisation between the
replays; samples outside the batch's ranges must stay untouched.
"""
from __future__ import annotations

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


@pytest.fixture(scope="module")
def umi(torch):
    import paper_2604_06602_amd as _u
    return _u


def eager(torch, umi, curves, alpha=2.0, c=5.0, iters=5):
    b = synth.lightcurves.pack(curves)
    f = torch.from_numpy(b.flux).cuda()
    t = torch.from_numpy(b.time).cuda()
    tr, md = umi.detrend_batch(f, t, b.lengths, b.W, alpha, c, iters, with_median=True)
    torch.cuda.synchronize()
    return b, tr.cpu().numpy(), md.cpu().numpy()


def place(rng, curves, capacity):
    """Scatter curves at random non-overlapping offsets of an arena."""
    offs, pos = [], int(rng.integers(0, 50))
    for f, _, _ in curves:
        offs.append(pos)
        pos += f.size + int(rng.integers(0, 300))
    assert pos <= capacity
    return np.array(offs, np.int64)


def test_gather_equals_packed_batch(torch, umi):
    rng = np.random.default_rng(1)
    curves = [synth.curve_for(3, i) for i in range(8)]
    curves = [(f[:20000], t[:20000], W) for f, t, W in curves]
    b, ref_tr, ref_md = eager(torch, umi, curves)
    cap = b.n_samples + 8 * 400
    offs = place(rng, curves, cap)
    flux = torch.full((cap,), float("nan"), dtype=torch.float32, device="cuda")
    time = torch.zeros(cap, dtype=torch.float64, device="cuda")
    for o, (f, t, _) in zip(offs, curves):
        flux[o:o + f.size] = torch.from_numpy(f).cuda()
        time[o:o + f.size] = torch.from_numpy(t).cuda()
    trend = torch.full((cap,), 123.0, dtype=torch.float32, device="cuda")
    median = torch.full((cap,), 456.0, dtype=torch.float32, device="cuda")
    umi.detrend_gather_into(flux, time, offs, [f.size for f, _, _ in curves],
                            [W for _, _, W in curves], trend, median)
    torch.cuda.synchronize()
    tr = trend.cpu().numpy()
    md = median.cpu().numpy()
    inside = np.zeros(cap, bool)
    for i, (o, (f, _, _)) in enumerate(zip(offs, curves)):
        sl = slice(o, o + f.size)
        inside[sl] = True
        ref = slice(b.offsets[i], b.offsets[i] + f.size)
        assert np.array_equal(tr[sl].view(np.uint32), ref_tr[ref].view(np.uint32))
        assert np.array_equal(md[sl].view(np.uint32), ref_md[ref].view(np.uint32))
    assert (tr[~inside] == 123.0).all() and (md[~inside] == 456.0).all()


def test_gather_rejects_overlap(torch, umi):
    flux = torch.ones(1000, dtype=torch.float32, device="cuda")
    trend = torch.empty_like(flux)
    with pytest.raises(umi.UmiError):
        umi.detrend_gather_into(flux, None, [0, 50], [100, 100], [5, 5], trend)


def test_plan_replays_match_eager(torch, umi):
    rng = np.random.default_rng(2)
    cap = 400000
    flux = torch.full((cap,), float("nan"), dtype=torch.float32, device="cuda")
    time = torch.zeros(cap, dtype=torch.float64, device="cuda")
    trend = torch.full((cap,), 7.0, dtype=torch.float32, device="cuda")
    median = torch.full((cap,), 7.0, dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    plan = umi.Plan(flux, time, trend, median, max_curves=64, max_W=721, stream=s)
    batches = []
    for k in range(7):
        n = [5, 1, 12, 0, 3, 9, 4][k]
        ids = rng.choice(400, n, replace=False)
        curves = [synth.curve_for(3, int(i)) for i in ids]
        curves = [(f[:25000], t[:25000], W) for f, t, W in curves]
        batches.append(curves)
    params = [(2.0, 5.0, 5), (1.0, 5.0, 5), (10.0, 2.5, 5), (2.0, 5.0, 5), (3.0, 5.0, 2),
              (2.0, 5.0, 0), (2.0, 5.0, 5)]
    for k, curves in enumerate(batches):
        a, c, it = params[k]
        offs = place(rng, curves, cap) if curves else np.zeros(0, np.int64)
        lengths = [f.size for f, _, _ in curves]
        Ws = [W for _, _, W in curves]
        with torch.cuda.stream(s):
            trend.fill_(7.0)
            median.fill_(7.0)
            for o, (f, t, _) in zip(offs, curves):
                flux[o:o + f.size].copy_(torch.from_numpy(f), non_blocking=False)
                time[o:o + f.size].copy_(torch.from_numpy(t), non_blocking=False)
        plan.run(offs, lengths, Ws, a, c, it)
        s.synchronize()
        tr = trend.cpu().numpy()
        md = median.cpu().numpy()
        if curves:
            b, ref_tr, ref_md = eager(torch, umi, curves, a, c, it)  # eager work between replays
            for i, o in enumerate(offs):
                sl = slice(o, o + lengths[i])
                ref = slice(b.offsets[i], b.offsets[i] + lengths[i])
                assert np.array_equal(tr[sl].view(np.uint32), ref_tr[ref].view(np.uint32)), (k, i)
                assert np.array_equal(md[sl].view(np.uint32), ref_md[ref].view(np.uint32)), (k, i)
            inside = np.zeros(cap, bool)
            for o, L in zip(offs, lengths):
                inside[o:o + L] = True
            assert (tr[~inside] == 7.0).all()
        else:
            assert (tr == 7.0).all()
    plan.destroy()


def test_plan_rejects_oversized_batches(torch, umi):
    cap = 10000
    flux = torch.ones(cap, dtype=torch.float32, device="cuda")
    trend = torch.empty_like(flux)
    s = torch.cuda.Stream()
    plan = umi.Plan(flux, None, trend, None, max_curves=2, max_W=121, stream=s)
    with pytest.raises(umi.UmiError):
        plan.run([0, 100, 200], [10, 10, 10], [5, 5, 5])   # too many curves
    with pytest.raises(umi.UmiError):
        plan.run([9995], [10], [5])                          # beyond capacity
    with pytest.raises(umi.UmiError):
        plan.run([0], [100], [361])                          # W above max_W
    plan.run([0, 5000], [3000, 3000], [121, 25])
    s.synchronize()
    assert np.isfinite(trend[:3000].cpu().numpy()).all()
    plan.destroy()


def test_plan_small_batch_tiles_stay_within_its_capacity(torch, umi):
    """A plan sized for exactly one 20,000-sample curve: the small-batch tile
    rule may not cut that curve into more tiles than the plan holds, and the
    replay equals the direct call (whose tiles the rule does cut) bit for
    bit, on the first replay and after eager work on the second."""
    f, t, W = synth.curve_config0()
    cap = f.size
    flux = torch.from_numpy(f).cuda()
    time = torch.from_numpy(t).cuda()
    trend = torch.empty_like(flux)
    s = torch.cuda.Stream()
    plan = umi.Plan(flux, time, trend, None, max_curves=1, max_W=W, stream=s)
    ref, _ = umi.detrend(flux, time, W)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    for rep in range(2):
        trend.fill_(7.0)
        torch.cuda.synchronize()
        plan.run([0], [cap], [W])
        s.synchronize()
        assert np.array_equal(trend.cpu().numpy().view(np.uint32), ref.view(np.uint32)), rep
        umi.detrend(flux, time, W)  # eager work between the replays
        torch.cuda.synchronize()
    plan.destroy()
