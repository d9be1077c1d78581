"""Time binning on the device: dd_downfactor, dd_time_binning and one plan per run of DM
trials at 2^k t_samp, against the FP64 oracle (run on an MI355X with -m gpu)."""
import sys

import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import assert_rows_close, assert_stats_close, compare_candidates, cuda

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    return cuda()


@pytest.fixture(scope="module")
def dd():
    import paper_1401_8258_amd as dd
    dd.load_library()
    return dd


def _stored(x32, dt):
    return {"f32": x32, "u8": fbsynth.to_u8(x32), "f16": fbsynth.to_f16(x32)}[dt]


@pytest.mark.parametrize("nchan,nsamp,stride,dt", [
    (64, 16384, 16384, "f32"), (3, 1001, 1013, "f32"), (5, 2, 2, "u8"), (7, 4099, 4099, "u8"),
    (4, 3000, 3001, "f16"), (2, 2049, 2051, "f16"), (1, (1 << 20) + 3, (1 << 20) + 3, "f32"),
    (9, 777, 781, "u8")])
def test_downfactor_exact(torch, dd, nchan, nsamp, stride, dt):
    """One FP32 add per output: u8 and FP16 sums are exact and an FP32 sum is the rounded
    exact sum, so the result equals the oracle's FP64 sum rounded to FP32, bit for bit
    (also for ragged lengths, odd strides and unaligned rows)."""
    _say(f"case: downfactor {nchan}x{nsamp} stride {stride} {dt}")
    x = _stored(np.random.default_rng(nchan * 7919 + nsamp).standard_normal((nchan, stride)).astype(np.float32), dt)
    dev = torch.from_numpy(np.ascontiguousarray(x)).cuda()[:, :nsamp]
    got = dd.downfactor(dev)
    want = orc.downfactor(x[:, :nsamp]).astype(np.float32)
    np.testing.assert_array_equal(got.cpu().numpy(), want)
    if nsamp >= 4:  # twice: each level rounds its own sums to FP32
        got2 = dd.downfactor(got).cpu().numpy()
        np.testing.assert_array_equal(got2, orc.downfactor(want).astype(np.float32))


@pytest.mark.parametrize("dt", ["f32", "u8", "f16"])
def test_binned_plan_config1(torch, dd, dt):
    """The 64-channel workload spans five binning runs (DM_diag = 1.34): each run's series,
    statistics and 6-sigma candidates against the oracle; u8 codes stay exact through the
    downfactored FP32 sums. The injected pulse (4 sigma per sample at full resolution) is
    detected in the factor-4 run near its DM trial."""
    _say(f"case: binned config1 {dt}")
    b = fbsynth.config1()
    x = _stored(b.data, dt)
    bp = dd.BinnedPlan(b.freq_mhz, b.tsamp_s, b.dm, dtype=dt, max_log2=4)
    assert abs(bp.dm_diag - orc.diagonal_dm(b.freq_mhz, b.tsamp_s)) == 0.0
    res = bp.dedisperse(torch.from_numpy(np.ascontiguousarray(x)).cuda(), k_sigma=6.0)
    torch.cuda.synchronize()
    want = orc.dedisperse_binned(x, b.freq_mhz, b.tsamp_s, b.dm, 4)
    assert [(s.log2, s.d0, s.d1) for s, _ in res.segments] == [w[:3] for w in want]
    assert bp.nout(b.nsamp) == [w[3].shape[1] for w in want]
    for (seg, r), (k, d0, d1, s) in zip(res.segments, want):
        got = r.out.cpu().numpy()
        mean, rms = orc.series_stats(s)
        if dt == "u8":
            np.testing.assert_array_equal(got, s.astype(np.float32))
        else:
            assert_rows_close(got, s, rms, what=f"{dt} run {k}")
        assert_stats_close(r.mean.cpu().numpy(), r.rms.cpu().numpy(), mean, rms)
        compare_candidates(r.candidates(), s, mean, rms, 6.0)
    c = res.candidates()
    best = c[np.argmax(c["snr"])]
    assert abs(int(best["dm_index"]) - 50) <= 2 and abs(int(best["t"]) - 8192) <= 8 and best["snr"] > 7.0


def test_binned_cap_and_single_run(torch, dd):
    """max_log2 = 0 is the plain plan; a DM range under the diagonal is one factor-1 run."""
    b = fbsynth.config1()
    x = torch.from_numpy(b.data).cuda()
    plain = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm).dedisperse(x).out.cpu().numpy()
    for bp in (dd.BinnedPlan(b.freq_mhz, b.tsamp_s, b.dm, max_log2=0),
               dd.BinnedPlan(b.freq_mhz, b.tsamp_s, b.dm[:13], max_log2=6)):
        assert len(bp.segments) == 1 and bp.segments[0].log2 == 0
        r = bp.dedisperse(x).segments[0][1]
        # fewer trials can mean a smaller maximum delay and a longer series: same leading columns
        np.testing.assert_array_equal(r.out.cpu().numpy()[:, :plain.shape[1]], plain[:bp.dm.size])


def test_config2_binned_full_size(torch, dd):
    """The full 1024 x 2^20 x 2048 FP32 workload with time binning up to factor 16 (the
    benchmark's binned pass): the first and last trial of every run against whole oracle
    rows, with their statistics and candidates."""
    _say("case: config2 binned full size, generating input")
    b = fbsynth.config2()
    bp = dd.BinnedPlan(b.freq_mhz, b.tsamp_s, b.dm, max_log2=4)
    assert [s.log2 for s in bp.segments] == [0, 1, 2, 3, 4]
    x = torch.from_numpy(b.data).cuda()
    _say("case: config2 binned full size, running")
    res = bp.dedisperse(x, k_sigma=6.0, cand_cap=1 << 20)
    torch.cuda.synchronize()
    del x
    level, cur = b.data, 0
    for seg, r in res.segments:
        while cur < seg.log2:
            _say(f"case: config2 binned, oracle downfactor to level {cur + 1}")
            level = orc.downfactor(level)
            cur += 1
        tab = orc.delay_table(b.freq_mhz, b.dm[seg.d0:seg.d1], b.tsamp_s * 2 ** seg.log2)
        np.testing.assert_array_equal(seg.plan.delays(), tab)
        cands = r.candidates()
        for i in sorted({0, seg.d1 - seg.d0 - 1}):
            _say(f"case: config2 binned run {seg.log2} row {seg.d0 + i}")
            want = orc.dedisperse(level, tab, rows=[i])
            mean, rms = orc.series_stats(want)
            assert_rows_close(r.out[i:i + 1].cpu().numpy(), want, rms, what=f"run {seg.log2} row {i}")
            assert_stats_close(r.mean[i:i + 1].cpu().numpy(), r.rms[i:i + 1].cpu().numpy(), mean, rms)
            compare_candidates(cands[cands["dm_index"] == i], want, mean, rms, 6.0, row_ids=[i])


@pytest.mark.parametrize("dt", ["f32", "u8"])
def test_binned_batched_equals_per_run(torch, dd, dt):
    """The runs in one persistent launch equal one launch per run, bit for bit (for u8 the
    factor-1 run keeps its own launch: the batch needs one input type)."""
    b = fbsynth.config1()
    x = torch.from_numpy(np.ascontiguousarray(_stored(b.data, dt))).cuda()
    bp = dd.BinnedPlan(b.freq_mhz, b.tsamp_s, b.dm, dtype=dt, max_log2=4)
    a = bp.dedisperse(x, k_sigma=4.0)
    c = bp.dedisperse(x, k_sigma=4.0, batched=True)
    torch.cuda.synchronize()
    for (_, r1), (_, r2) in zip(a.segments, c.segments):
        assert torch.equal(r1.out, r2.out) and torch.equal(r1.mean, r2.mean) and torch.equal(r1.rms, r2.rms)
        np.testing.assert_array_equal(r1.candidates(), r2.candidates())
