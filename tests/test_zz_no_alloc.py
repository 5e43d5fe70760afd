"""The allocation-free batch call (umi_detrend_batch_noalloc) against the
allocating one (umi_detrend_batch) and the FP64 oracle.

Both calls run the same kernels on the same tiles, so trend and median must
agree bit for bit; the second of two calls in a row takes a smaller batch than
the first, whose contents the shared static workspace still holds.  Against
the oracle: median bit-exact, trend within 1e-5 relative, NaN at the same
samples.  Every call goes through the C ABI.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5


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


def _batch(ids):
    return synth.lightcurves.pack([synth.curve_for(3, i) for i in ids])


def _short_ids(n, limit=15000, start=0):
    out = []
    i = start
    while len(out) < n:
        if synth.curve_for(3, i)[0].size < limit:
            out.append(i)
        i += 1
    return out


def _run(torch, umi, b, noalloc, launch=None):
    f = torch.from_numpy(b.flux).cuda()
    t = torch.from_numpy(b.time).cuda()
    tr = torch.full_like(f, 12345.0)  # anything left unwritten shows
    md = torch.full_like(f, 12345.0)
    if noalloc:
        umi.detrend_batch_noalloc_into(f, t, b.lengths, b.W, tr, md, launch=launch)
    else:
        umi.detrend_batch_into(f, t, b.lengths, b.W, tr, md, launch=launch)
    torch.cuda.synchronize()
    return tr.cpu().numpy(), md.cpu().numpy()


def _same_bits(a, b, what):
    assert a.shape == b.shape, what
    diff = np.flatnonzero(a.view(np.uint32) != b.view(np.uint32))
    assert diff.size == 0, "%s: %d samples differ, first %s" % (what, diff.size, diff[:5])


def _oracle_parity(g_tr, g_md, o_tr, o_md, what):
    o_nan = np.isnan(o_tr)
    assert np.array_equal(np.isnan(g_tr), o_nan), what + ": NaN pattern"
    ok = ~o_nan
    _same_bits(g_md[ok], o_md[ok], what + " median")
    rel = np.abs(g_tr[ok].astype(np.float64) - o_tr[ok]) / np.abs(o_tr[ok])
    assert rel.max() <= REL_TOL, "%s: max rel err %.3e" % (what, rel.max())


def test_noalloc_matches_batch_call_twice_in_a_row(torch, umi, oracle_lib):
    big = _batch(_short_ids(10))          # every W of the mixed workload, NaN gaps
    small = _batch(_short_ids(3, start=200))
    assert small.n_samples < big.n_samples
    for b, what in ((big, "first call"), (small, "second, smaller call")):
        g_tr, g_md = _run(torch, umi, b, noalloc=True)
        d_tr, d_md = _run(torch, umi, b, noalloc=False)
        _same_bits(g_tr, d_tr, what + " trend vs umi_detrend_batch")
        _same_bits(g_md, d_md, what + " median vs umi_detrend_batch")
        o_tr, o_md = oracle_lib.detrend_batch(b.flux, b.time, b.lengths, b.W)
        _oracle_parity(g_tr, g_md, o_tr, o_md, what + " vs oracle")


def test_noalloc_small_batch_split_tiles_and_per_curve_mode(torch, umi, oracle_lib):
    # one curve: the small-batch rule cuts it into split tiles (several lanes
    # per window); then the per-curve launch mode over two curves
    one = synth.lightcurves.pack([synth.curve_config0()])
    g_tr, g_md = _run(torch, umi, one, noalloc=True)
    d_tr, d_md = _run(torch, umi, one, noalloc=False)
    _same_bits(g_tr, d_tr, "one curve trend")
    _same_bits(g_md, d_md, "one curve median")
    o_tr, o_md = oracle_lib.detrend_batch(one.flux, one.time, one.lengths, one.W)
    _oracle_parity(g_tr, g_md, o_tr, o_md, "one curve vs oracle")

    two = _batch(_short_ids(2, start=400))
    per = umi.LaunchOptions(mode=umi.MODE_PER_CURVE)
    g_tr, g_md = _run(torch, umi, two, noalloc=True, launch=per)
    d_tr, d_md = _run(torch, umi, two, noalloc=False, launch=per)
    _same_bits(g_tr, d_tr, "per-curve trend")
    _same_bits(g_md, d_md, "per-curve median")


def test_noalloc_leaves_device_memory_alone(torch, umi):
    b = _batch(_short_ids(4, start=600))
    f = torch.from_numpy(b.flux).cuda()
    t = torch.from_numpy(b.time).cuda()
    tr = torch.empty_like(f)
    umi.detrend_batch_noalloc_into(f, t, b.lengths, b.W, tr)  # first call on this device
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for k in (4, 2, 3):
        umi.detrend_batch_noalloc_into(f[:int(b.lengths[:k].sum())], t[:int(b.lengths[:k].sum())],
                                       b.lengths[:k], b.W[:k], tr[:int(b.lengths[:k].sum())])
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
