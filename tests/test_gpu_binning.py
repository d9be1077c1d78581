"""Time binning on the device: dd_downfactor, dd_time_binning and one plan per run of DM
trials at 2^k t_samp, against the FP64 oracle (run on an MI355X with -m gpu)."""
import sys

import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import GUARD, assert_rows_close, assert_stats_close, compare_candidates, cuda

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
    """The runs in one batched call equal one launch per run, bit for bit (for u8 the factor-1
    run is a direct-read item beside the FP32 LDS-form runs of the same call)."""
    b = fbsynth.config1()
    x = torch.from_numpy(np.ascontiguousarray(_stored(b.data, dt))).cuda()
    bp = dd.BinnedPlan(b.freq_mhz, b.tsamp_s, b.dm, dtype=dt, max_log2=4)
    a = bp.dedisperse(x, k_sigma=4.0)
    c = bp.dedisperse(x, k_sigma=4.0, batched=True)
    torch.cuda.synchronize()
    for (_, r1), (_, r2) in zip(a.segments, c.segments):
        assert torch.equal(r1.out, r2.out) and torch.equal(r1.mean, r2.mean) and torch.equal(r1.rms, r2.rms)
        np.testing.assert_array_equal(r1.candidates(), r2.candidates())


def _binned_stream_case(dt, sizes, k_sigma, gap=None):
    """A seed whose stream windows (every run, every push) keep their candidates a margin
    from the threshold; returns (freq, tsamp, dm, stored input, per-run oracle series of the
    input with zeros in place of the lost block, push results expected as run windows)."""
    freq = fbsynth.channel_freqs(428.0, 0.3125, 64)
    tsamp = 51.2e-6
    dm = fbsynth.dm_trials(0.0, 0.1, 128)
    for seed in range(300, 340):
        x32 = np.random.default_rng(seed).standard_normal((64, sum(sizes))).astype(np.float32)
        x = np.ascontiguousarray(_stored(x32, dt))
        xz = x.copy()
        if gap is not None:
            a = sum(sizes[:gap])
            xz[:, a:a + sizes[gap]] = 0
        runs = orc.dedisperse_binned(xz, freq, tsamp, dm, 4)
        if gap is not None:  # outputs only are compared
            return freq, tsamp, dm, x, xz, runs
        ok = True
        for k, d0, d1, s in runs:
            maxdelay = (sum(sizes) >> k) - s.shape[1]
            received = emitted = 0
            for n in sizes:  # the windows a stream emits: outputs made computable by each block
                received += n >> k
                t1 = received - maxdelay
                if t1 > emitted:
                    w = s[:, emitted:t1]
                    ok = ok and orc.threshold_margin(w, *orc.series_stats(w), k_sigma) > 4 * GUARD
                    emitted = t1
        if ok:
            return freq, tsamp, dm, x, xz, runs
    raise AssertionError("no well-conditioned seed in 40")


@pytest.mark.parametrize("dt,batched", [("f32", False), ("f32", True), ("u8", False), ("u8", True),
                                        ("f16", False)])
def test_binned_stream_equals_one_shot(torch, dd, dt, batched):
    """A time-binned stream over 1024-sample blocks and a ragged last block of 336 (each a
    multiple of 16, the largest factor): every run emits, per push, the outputs its own ring
    made computable, equal bit for bit to the one-shot binned call over the concatenated
    input at the same run times; each window's statistics and the merged 4-sigma candidates
    against the oracle; all outputs of every run emitted once. Each run holds its own ring at
    its binned sampling time."""
    _say(f"case: binned stream {dt} batched={batched}")
    sizes = [1024] * 13 + [336]
    freq, tsamp, dm, x, _, runs = _binned_stream_case(dt, sizes, 4.0)
    bp = dd.BinnedPlan(freq, tsamp, dm, dtype=dt, max_log2=4)
    assert [s.log2 for s in bp.segments] == [0, 1, 2, 3, 4]
    one = bp.dedisperse(torch.from_numpy(x).cuda())
    one = [r.out.cpu().numpy() for _, r in one.segments]
    st = dd.BinnedStream(bp, 1024)
    emitted = [0] * len(runs)
    pos = 0
    for j, n in enumerate(sizes):
        blk = torch.from_numpy(np.ascontiguousarray(x[:, pos:pos + n])).cuda()
        pos += n
        res = st.push(blk, k_sigma=4.0, batched=batched)
        if res is None:  # only while every run fills
            assert all(e == 0 for e in emitted)
            continue
        merged = res.candidates()
        total = 0
        for i, ((seg, t0, r), (k, d0, d1, s)) in enumerate(zip(res.segments, runs)):
            if r is None:
                continue
            nk = r.out.shape[1]
            assert t0 == emitted[i], (k, t0, emitted[i])
            emitted[i] = t0 + nk
            np.testing.assert_array_equal(r.out.cpu().numpy(), one[i][:, t0:t0 + nk])
            w = s[:, t0:t0 + nk]
            mean, rms = orc.series_stats(w)
            assert_stats_close(r.mean.cpu().numpy(), r.rms.cpu().numpy(), mean, rms)
            c = r.candidates()
            compare_candidates(c, w, mean, rms, 4.0, t_offset=t0)
            total += c.size
        assert merged.size == total
        assert np.all(np.diff(merged["dm_index"].astype(np.int64) * (1 << 40) + merged["t"]) > 0)
    assert emitted == [o.shape[1] for o in one]
    assert emitted == [(sum(sizes) >> s.log2) - s.plan.maxdelay for s in bp.segments]


def test_binned_stream_gap_fill_and_refusals(torch, dd):
    """A lost block with gap fill on: every run's outputs equal the one-shot binned call over
    the input with zeros in place of the lost block, at the same run times. A block that is
    not a multiple of 16 samples, a wrong seq (gap fill off) and a batched push of
    register-window runs (a form that is not batched) are refused before anything changes,
    and the stream continues. An FP16 factor-1 run beside FP32 runs (different kernels and
    tiles) pushes batched, equal to the unbatched push."""
    _say("case: binned stream gap fill")
    sizes = [1024] * 12
    freq, tsamp, dm, x, xz, runs = _binned_stream_case("f32", sizes, 4.0, gap=7)
    bp = dd.BinnedPlan(freq, tsamp, dm, max_log2=4)
    one = [r.out.cpu().numpy() for _, r in bp.dedisperse(torch.from_numpy(xz).cuda()).segments]
    st = dd.BinnedStream(bp, 1024, gap_fill=True)
    seen = 0
    for j in range(len(sizes)):
        if j == 7:
            continue
        blk = torch.from_numpy(np.ascontiguousarray(x[:, 1024 * j:1024 * (j + 1)])).cuda()
        res = st.push(blk, seq=j, k_sigma=4.0)
        if res is None:
            continue
        for i, (seg, t0, r) in enumerate(res.segments):
            if r is not None:
                np.testing.assert_array_equal(r.out.cpu().numpy(), one[i][:, t0:t0 + r.out.shape[1]])
                seen += 1
    assert seen > 20
    plain = dd.BinnedStream(bp, 1024)
    blk = torch.from_numpy(np.ascontiguousarray(x[:, :1024])).cuda()
    with pytest.raises(dd.DedispError):
        plain.push(blk[:, :1000])
    with pytest.raises(dd.DedispError):
        plain.push(blk, seq=1)
    plain.push(blk, seq=0)
    assert plain.seq == 1
    brw = dd.BinnedPlan(freq, tsamp, dm, max_log2=4, form="regwin")
    assert not brw.batchable
    srw = dd.BinnedStream(brw, 1024)
    with pytest.raises(dd.DedispError):
        srw.push(blk, batched=True)
    assert srw.seq == 0
    bp16 = dd.BinnedPlan(freq, tsamp, dm, dtype="f16", max_log2=4)
    assert bp16.batchable and bp16.segments[0].plan.tiles != bp16.segments[1].plan.tiles
    s16, u16 = dd.BinnedStream(bp16, 1024), dd.BinnedStream(bp16, 1024)
    for j in range(len(sizes)):
        b16 = torch.from_numpy(fbsynth.to_f16(x[:, 1024 * j:1024 * (j + 1)])).cuda()
        rb = s16.push(b16, k_sigma=4.0, batched=True)
        ru = u16.push(b16, k_sigma=4.0)
        assert (rb is None) == (ru is None)
        if rb is None:
            continue
        for (_, tb, b), (_, tu, u) in zip(rb.segments, ru.segments):
            assert tb == tu and (b is None) == (u is None)
            if b is not None:
                np.testing.assert_array_equal(b.out.cpu().numpy(), u.out.cpu().numpy())
        np.testing.assert_array_equal(rb.candidates(), ru.candidates())
    assert s16.seq == u16.seq == len(sizes)
    srw.push(blk)
    assert srw.seq == 1
