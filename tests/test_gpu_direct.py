"""The direct-read kernel form (DD_FORM_DIRECT, 8-bit input) against the oracle and the LDS form.

8-bit codes sum exactly in FP32 (at most 255 x 4096 < 2^24), so every output must equal the
FP64 oracle's value of Eq. bruteEquation bit for bit, and equal the LDS form's; the
statistics partials are sums of exact integers, so mean and rms equal the LDS form's too.
The cases cover the form's own geometry: 1024-sample tiles of 16 samples per lane, a
ragged last tile, the 16-bit pair fold every 256 channels, the four shifted copies of the
input (workspace for a plain call, the ring for a stream, including a ring shorter than a
tile), the batched launch beside LDS-form items, and the 4096-channel 120-180 MHz beams
whose delays grow by ~100 samples per DM trial. Each case prints its shape before it runs.
"""
import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import GUARD, assert_stats_close, compare_candidates, cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return cuda()


@pytest.fixture(scope="module")
def dd():
    import paper_1401_8258_amd as dd
    dd.load_library()
    return dd


def _say(msg):
    print(msg, flush=True)


def _codes(rng, nchan, nsamp, pad=0):
    """u8 codes of N(0,1) noise as fbsynth stores them (mean 128, sigma 16), rows padded."""
    full = np.zeros((nchan, nsamp + pad), np.uint8)
    full[:, :nsamp] = fbsynth.to_u8(fbsynth.noise(rng, nchan, nsamp))
    return full


def test_default_form_for_u8_and_config3_bit_exact(torch, dd):
    """Config 3's u8 input: the default plan is the direct-read form; outputs equal the
    oracle bit for bit, statistics and candidates equal the oracle's and the LDS form's."""
    _say("case: direct form, config 3 u8")
    b, u8, _ = fbsynth.config3()
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    want = orc.dedisperse(u8, tab)
    mean, rms = orc.series_stats(want)
    k = 4.0
    assert orc.threshold_margin(want, mean, rms, k) > GUARD
    p = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm, dtype="u8")
    q = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm, dtype="u8", form="lds")
    assert p.form == "direct" and q.form == "lds"
    x = torch.from_numpy(u8).cuda()
    r1 = p.dedisperse(x, k_sigma=k)
    r2 = q.dedisperse(x, k_sigma=k)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r1.out.cpu().numpy().astype(np.float64), want)
    assert torch.equal(r1.out, r2.out)
    assert torch.equal(r1.mean, r2.mean) and torch.equal(r1.rms, r2.rms)
    assert_stats_close(r1.mean.cpu().numpy(), r1.rms.cpu().numpy(), mean, rms)
    compare_candidates(r1.candidates(), want, mean, rms, k)
    np.testing.assert_array_equal(r1.candidates(), r2.candidates())


# nchan, f_top, channel width (MHz), tsamp, ndm, DM step, nsamp, input row padding,
# output row padding, (dms_per_wave, waves[, samples_per_lane]) or None
EDGES = [
    (1, 428.0, 0.3125, 51.2e-6, 1, 0.1, 300, 0, 0, None),        # one channel, one trial
    (64, 428.0, 0.3125, 51.2e-6, 128, 0.1, 556, 0, 0, None),     # nout = 1
    (64, 428.0, 0.3125, 51.2e-6, 128, 0.1, 1500, 3, 1, (1, 8)),  # nout < one tile, odd paddings
    (37, 428.0, 0.5, 51.2e-6, 33, 0.1, 3000, 1, 0, (4, 2)),      # odd channels, partial group
    (300, 428.0, 0.06, 51.2e-6, 70, 0.1, 5001, 0, 4, (2, 8)),    # one pair fold, ragged tail
    (300, 428.0, 0.06, 51.2e-6, 70, 0.1, 5001, 0, 4, (2, 8, 32)),  # the same, 2048-sample tiles
    (64, 428.0, 0.3125, 51.2e-6, 50, 0.1, 3100, 3, 1, (1, 4, 32)),  # ragged second sub-tile
    (513, 428.0, 20.0 / 513, 51.2e-6, 40, 0.1, 4097, 0, 0, (4, 1)),  # folds at 256 and 512
    (257, 180.0, 60.0 / 257, 81.92e-6, 24, 0.05, 26000, 0, 0, None),  # low band, large shifts
]


@pytest.mark.parametrize("nchan,ftop,df,tsamp,ndm,step,nsamp,pad,opad,tun", EDGES)
def test_edges_bit_exact(torch, dd, nchan, ftop, df, tsamp, ndm, step, nsamp, pad, opad, tun):
    _say(f"case: direct nchan={nchan} ndm={ndm} step={step} nsamp={nsamp} pad={pad} opad={opad} tun={tun}")
    freq = fbsynth.channel_freqs(ftop, df, nchan)
    dm = fbsynth.dm_trials(0.0, step, ndm)
    tab = orc.delay_table(freq, dm, tsamp)
    assert nsamp > int(tab.max())
    nout = nsamp - int(tab.max())
    k = 3.0 if ndm * nout < 500_000 else 4.5
    # the first seed whose oracle values all keep a clear margin from their thresholds
    for seed in range(nchan * 13 + ndm, nchan * 13 + ndm + 50):
        full = _codes(np.random.default_rng(seed), nchan, nsamp, pad)
        data = np.ascontiguousarray(full[:, :nsamp])
        want = orc.dedisperse(data, tab)
        mean, rms = orc.series_stats(want)
        if orc.threshold_margin(want, mean, rms, k) > 4 * GUARD:
            break
    else:
        pytest.fail("no well-conditioned seed in 50")
    p = dd.Plan(freq, tsamp, dm, dtype="u8", form="direct", tuning=tun)
    q = dd.Plan(freq, tsamp, dm, dtype="u8", form="lds")
    if tun is not None:
        assert p.tiles[:len(tun)] == tuple(tun)
    xt = torch.from_numpy(full).cuda()[:, :nsamp]
    o1 = torch.full((ndm, nout + opad), -7.0, device="cuda")
    r1 = p.dedisperse(xt, k_sigma=k, out=o1)
    r2 = q.dedisperse(xt, k_sigma=k)
    torch.cuda.synchronize()
    if opad:
        assert torch.all(o1[:, nout:] == -7.0), "write past nout"
    np.testing.assert_array_equal(r1.out.cpu().numpy().astype(np.float64), want)
    assert torch.equal(r1.out, r2.out)
    assert torch.equal(r1.mean, r2.mean) and torch.equal(r1.rms, r2.rms)
    compare_candidates(r1.candidates(), want, mean, rms, k)


@pytest.mark.parametrize("tun", [None, (1, 4, 32)])
def test_stream_ragged_blocks_equal_one_shot_and_oracle(torch, dd, tun):
    """A stream of ragged blocks on a low-band beam: each window equals the one-shot result
    and the oracle's definition of a stream (the ring holds the shifted copies)."""
    _say(f"case: direct stream, low band, tun={tun}")
    freq = fbsynth.channel_freqs(180.0, 60.0 / 512, 512)
    dm = fbsynth.dm_trials(0.0, 0.05, 40)
    tsamp = 81.92e-6
    tab = orc.delay_table(freq, dm, tsamp)
    block = 5000
    sizes = [block, block, 1111, block, 1, block, 2500, block, block, block]
    x = _codes(np.random.default_rng(77), 512, sum(sizes))
    expected = orc.stream_expected(np.split(x, np.cumsum(sizes)[:-1], axis=1), tab)
    plan = dd.Plan(freq, tsamp, dm, dtype="u8", form="direct", tuning=tun)
    assert plan.form == "direct"
    one = plan.dedisperse(torch.from_numpy(x).cuda()).out
    s = dd.Stream(plan, block)
    pos = 0
    emitted = 0
    for j, n in enumerate(sizes):
        r = s.push(torch.from_numpy(np.ascontiguousarray(x[:, pos:pos + n])).cuda())
        pos += n
        t0, t1, want = expected[j]
        if t1 == t0:
            assert r is None
            continue
        assert r is not None and r.t0 == t0 and r.out.shape[1] == t1 - t0
        assert torch.equal(r.out, one[:, t0:t1]), f"window at {t0}"
        np.testing.assert_array_equal(r.out.cpu().numpy().astype(np.float64), want)
        emitted = t1
    assert emitted == sum(sizes) - int(tab.max())


@pytest.mark.parametrize("tun", [None, (2, 4, 32)])
def test_stream_ring_shorter_than_a_tile(torch, dd, tun):
    """Blocks of 40 samples and a maximum delay of 8: the ring (64 samples) is shorter than
    the 1024- or 2048-sample tile, so every window reads the copies' mirror, many times over."""
    _say(f"case: direct stream, tiny ring, tun={tun}")
    freq = fbsynth.channel_freqs(428.0, 0.3125, 16)
    dm = fbsynth.dm_trials(0.0, 0.1, 9)
    x = _codes(np.random.default_rng(3), 16, 3000)
    plan = dd.Plan(freq, 51.2e-6, dm, dtype="u8", form="direct", tuning=tun)
    one = plan.dedisperse(torch.from_numpy(x).cuda()).out
    s = dd.Stream(plan, 40)
    pos = seen = 0
    while pos < x.shape[1]:
        n = min(40, x.shape[1] - pos)
        r = s.push(torch.from_numpy(np.ascontiguousarray(x[:, pos:pos + n])).cuda())
        pos += n
        if r is None:
            continue
        assert r.t0 == seen
        assert torch.equal(r.out, one[:, seen:seen + r.out.shape[1]])
        seen += r.out.shape[1]
    assert seen == one.shape[1]


def test_batch_mixes_direct_and_lds_items(torch, dd):
    """One batch call: direct-read items of different channel counts, DM ranges and tiles
    (one of them a stream window) and an LDS-form item; each equals its own single call,
    statistics and candidates included (those run once for the whole batch)."""
    _say("case: direct batch with an LDS item")
    rng = np.random.default_rng(11)
    # different channel counts, DM ranges and tiles (trials per wavefront, wavefronts)
    shapes = [(256, 428.0, 20.0, 51.2e-6, 300, 0.1, 12000, None),
              (1024, 180.0, 60.0, 81.92e-6, 100, 0.05, 30000, (1, 8)),
              (64, 428.0, 20.0, 51.2e-6, 77, 0.2, 4000, (4, 2)),
              (200, 428.0, 20.0, 51.2e-6, 130, 0.1, 9000, (2, 7)),
              (512, 180.0, 60.0, 81.92e-6, 60, 0.05, 20000, (2, 4, 32)),
              (128, 428.0, 20.0, 51.2e-6, 40, 0.1, 7000, (1, 2, 32))]
    jobs, singles = [], []
    for nchan, ftop, bw, ts, ndm, step, nsamp, tun in shapes:
        freq = fbsynth.channel_freqs(ftop, bw / nchan, nchan)
        dm = fbsynth.dm_trials(0.0, step, ndm)
        p = dd.Plan(freq, ts, dm, dtype="u8", form="direct", tuning=tun)
        assert p.form == "direct"
        x = torch.from_numpy(_codes(rng, nchan, nsamp)).cuda()
        jobs.append((p, x))
        singles.append(p.dedisperse(x, k_sigma=5.0))
    freq = fbsynth.channel_freqs(428.0, 20.0 / 128, 128)
    q = dd.Plan(freq, 51.2e-6, fbsynth.dm_trials(0.0, 0.1, 64), dtype="u8", form="lds")
    xq = torch.from_numpy(_codes(rng, 128, 6000)).cuda()
    jobs.append((q, xq))
    singles.append(q.dedisperse(xq, k_sigma=5.0))
    # a stream item: its pending window against the same window of a fresh stream pushed alone
    sp = dd.Plan(fbsynth.channel_freqs(180.0, 60.0 / 256, 256), 81.92e-6, fbsynth.dm_trials(0.0, 0.05, 50), dtype="u8")
    blocks = [torch.from_numpy(_codes(rng, 256, 3000)).cuda() for _ in range(5)]
    alone, batched = dd.Stream(sp, 3000), dd.Stream(sp, 3000)
    ref = None
    for blk in blocks:
        ref = alone.push(blk, k_sigma=5.0) or ref
    win = None
    for blk in blocks[:-1]:
        batched.push(blk)
    win = batched.append(blocks[-1])
    assert win is not None
    jobs.append((batched, win))
    res = dd.batch_dedisperse(jobs, k_sigma=5.0)
    torch.cuda.synchronize()
    for one, got in zip(singles, res[:-1]):
        assert torch.equal(one.out, got.out)
        assert torch.equal(one.mean, got.mean) and torch.equal(one.rms, got.rms)
        np.testing.assert_array_equal(one.candidates(), got.candidates())
    assert res[-1].t0 == ref.t0 and torch.equal(res[-1].out, ref.out)


def test_tilings_equal(torch, dd):
    """Every (dms_per_wave, waves[, samples_per_lane]) tiling of the direct-read form gives the
    same bits."""
    _say("case: direct tilings")
    freq = fbsynth.channel_freqs(180.0, 60.0 / 300, 300)
    dm = fbsynth.dm_trials(0.0, 0.1, 53)
    x = torch.from_numpy(_codes(np.random.default_rng(8), 300, 30000)).cuda()
    base = dd.Plan(freq, 81.92e-6, dm, dtype="u8").dedisperse(x)
    for tun in [(1, 1), (1, 8), (2, 2), (4, 4), (4, 8), (2, 5), (1, 8, 32), (2, 4, 32), (2, 3, 32)]:
        r = dd.Plan(freq, 81.92e-6, dm, dtype="u8", form="direct", tuning=tun).dedisperse(x)
        assert torch.equal(r.out, base.out), tun
        assert torch.equal(r.mean, base.mean) and torch.equal(r.rms, base.rms), tun


def test_full_size_4096ch_beam_sampled_rows(torch, dd):
    """A config-4 4096-channel beam (120-180 MHz, 81.92 us, u8 with injected pulses) at full
    size in the default plan: the brightest pulses' trials and both ends equal the oracle
    bit for bit, and every output equals the LDS form's."""
    specs = [sp for sp in fbsynth.config4_specs() if sp["nchan"] == 4096]
    sp = min(specs, key=lambda s: s["ndm"] * s["nsamp"])
    _say(f"case: direct full-size 4096-ch beam ndm={sp['ndm']} nsamp={sp['nsamp']} step={sp['step']}")
    rng = np.random.default_rng(sp["seed"])
    b = fbsynth.make_beam(sp["name"], sp["nchan"], sp["f_top"], sp["bw"], sp["tsamp"], sp["dm0"], sp["step"],
                          sp["ndm"], sp["nsamp"], rng, sp["npulse"], storage="u8")
    p = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm, dtype="u8")
    q = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm, dtype="u8", form="lds")
    assert p.form == "direct"
    x = torch.from_numpy(b.data).cuda()
    r1 = p.dedisperse(x, k_sigma=6.0)
    r2 = q.dedisperse(x, k_sigma=6.0)
    torch.cuda.synchronize()
    assert torch.equal(r1.out, r2.out)
    assert torch.equal(r1.mean, r2.mean) and torch.equal(r1.rms, r2.rms)
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    bright = sorted(b.pulses, key=lambda pl: -pl.amp * pl.width)[:2]
    rows = sorted({0, b.ndm - 1} | {int(np.argmin(np.abs(b.dm - pl.dm))) for pl in bright})
    want = orc.dedisperse(b.data, tab, rows=rows)
    np.testing.assert_array_equal(r1.out[rows].cpu().numpy().astype(np.float64), want)
