"""HIP path against the FP64 oracle, through the C ABI (run on an MI355X with -m gpu)."""
import sys

import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import (GUARD, RMS_TOL, assert_rows_close, assert_stats_close, compare_candidates, cuda)

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


def _run(torch, dd, beam_freq, tsamp, dm, data, k=0.0, tuning=None, cap=1 << 16):
    plan = dd.Plan(beam_freq, tsamp, dm, dtype=torch.from_numpy(data[:1, :1]).dtype, tuning=tuning)
    x = torch.from_numpy(np.ascontiguousarray(data)).cuda()
    r = plan.dedisperse(x, k_sigma=k, cand_cap=cap)
    torch.cuda.synchronize()
    return plan, r


def test_config1_full_parity(torch, dd):
    _say("case: config1 full parity")
    b = fbsynth.config1()
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    want = orc.dedisperse(b.data, tab)
    mean, rms = orc.series_stats(want)
    plan, r = _run(torch, dd, b.freq_mhz, b.tsamp_s, b.dm, b.data, k=4.0)
    np.testing.assert_array_equal(plan.delays(), tab)
    got = r.out.cpu().numpy()
    assert_rows_close(got, want, rms, what="config1")
    assert_stats_close(r.mean.cpu().numpy(), r.rms.cpu().numpy(), mean, rms)
    compare_candidates(r.candidates(), want, mean, rms, 4.0)
    # the injected pulse (DM 5.0 = trial 50, width 8) is recovered at its DM
    p = b.pulses[0]
    box = got[:, int(p.t0):int(p.t0) + p.width].sum(axis=1)
    assert abs(int(np.argmax(box)) - 50) <= 1


EDGE = [
    # nchan, ndm, nsamp, tuning, step
    (1, 1, 300, None, 0.1),
    (1, 5, 64, (8, 1), 0.1),
    (37, 33, 2000, None, 0.3),          # ragged channel block, ragged DM group, ragged tile
    (64, 70, 1501, (8, 2, 3), 0.2),
    (64, 128, 556, None, 0.1),          # nout = 1
    (96, 17, 5000, (8, 4, 1), 0.5),
    (33, 64, 3000, (8, 8), 0.1),
    (200, 40, 4097, (8, 8, 5), 0.2),    # large in-group delay spread
]


def _well_conditioned(shape, k, seed0, make, delays):
    """The first of 50 seeds whose oracle series keep every value at least 4 GUARD rms away
    from its threshold, so the candidate comparison always runs (FP32 rounding cannot move a
    value across)."""
    for seed in range(seed0, seed0 + 50):
        data = make(np.random.default_rng(seed), shape)
        want = orc.dedisperse(data, delays)
        mean, rms = orc.series_stats(want)
        if orc.threshold_margin(want, mean, rms, k) > 4 * GUARD:
            return data, want, mean, rms
    raise AssertionError("no well-conditioned seed in 50")


@pytest.mark.parametrize("nchan,ndm,nsamp,tuning,step", EDGE)
def test_edge_shapes(torch, dd, nchan, ndm, nsamp, tuning, step):
    _say(f"case: edge nchan={nchan} ndm={ndm} nsamp={nsamp} tuning={tuning}")
    freq = fbsynth.channel_freqs(428.0, 20.0 / 64, nchan)
    dm = fbsynth.dm_trials(0.0, step, ndm)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    if tab.max() >= nsamp:
        pytest.skip("shape leaves no output")
    data, want, mean, rms = _well_conditioned(
        (nchan, nsamp), 3.0, nchan * 1000 + ndm, lambda rng, sh: rng.standard_normal(sh).astype(np.float32), tab)
    plan, r = _run(torch, dd, freq, 51.2e-6, dm, data, k=3.0, tuning=tuning)
    assert_rows_close(r.out.cpu().numpy(), want, rms, what="edge")
    assert_stats_close(r.mean.cpu().numpy(), r.rms.cpu().numpy(), mean, rms)
    compare_candidates(r.candidates(), want, mean, rms, 3.0)


def test_integer_inputs_bit_exact_and_tuning_invariant(torch, dd):
    """u8 codes sum exactly in FP32, so every tiling must equal the oracle bit for bit."""
    _, u8, _ = fbsynth.config3()
    b = fbsynth.config1()
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    want = orc.dedisperse(u8, tab)
    for tuning in [None, (8, 1), (8, 2), (8, 8, 2), (8, 4, 7)]:
        _say(f"case: u8 bit-exact tuning={tuning}")
        _, r = _run(torch, dd, b.freq_mhz, b.tsamp_s, b.dm, u8, tuning=tuning)
        np.testing.assert_array_equal(r.out.cpu().numpy().astype(np.float64), want)


def test_fp32_tiling_invariance(torch, dd):
    """The channel summation order is fixed, so FP32 results do not depend on the tiles."""
    b = fbsynth.config1()
    outs = []
    for tuning in [None, (8, 1), (8, 2, 3), (8, 8), (8, 4, 8)]:
        _say(f"case: fp32 tiling {tuning}")
        _, r = _run(torch, dd, b.freq_mhz, b.tsamp_s, b.dm, b.data, tuning=tuning)
        outs.append(r.out.cpu().numpy())
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_f16_and_u8_against_oracle_on_the_stored_input(torch, dd):
    """Config 3: FP16 storage within 1e-5 rms of the FP64 oracle on the same FP16 values, u8
    storage equal to it bit for bit (integer codes sum exactly); candidates identical to the
    oracle's on each stored input. The error table against the FP32 original is in
    test_gpu_precision.py."""
    _say("case: precision variants against the oracle")
    b, u8, f16 = fbsynth.config3()
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    for name, x, k in (("f16", f16, 4.0), ("u8", u8, 4.0)):
        want = orc.dedisperse(x, tab)
        mean, rms = orc.series_stats(want)
        assert orc.threshold_margin(want, mean, rms, k) > GUARD
        _, r = _run(torch, dd, b.freq_mhz, b.tsamp_s, b.dm, x, k=k)
        got = r.out.cpu().numpy()
        if name == "u8":
            np.testing.assert_array_equal(got.astype(np.float64), want)
        else:
            assert_rows_close(got, want, rms, what=name)
        assert_stats_close(r.mean.cpu().numpy(), r.rms.cpu().numpy(), mean, rms)
        compare_candidates(r.candidates(), want, mean, rms, k)


def test_zero_dm_and_impulse(torch, dd):
    _say("case: zero DM / impulse")
    freq = fbsynth.channel_freqs(428.0, 0.3125, 64)
    dm = fbsynth.dm_trials(0.0, 0.1, 128)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    a = np.zeros((64, 3000), np.float32)
    a[63, 1700] = 1.0
    _, r = _run(torch, dd, freq, 51.2e-6, dm, a)
    got = r.out.cpu().numpy()
    for d in range(128):
        assert list(np.flatnonzero(got[d])) == [1700 - tab[63, d]]
    rng = np.random.default_rng(1)
    x = rng.integers(0, 256, size=(64, 3000)).astype(np.float32)
    _, r = _run(torch, dd, freq, 51.2e-6, np.zeros(3), x)
    np.testing.assert_array_equal(r.out.cpu().numpy()[0], x.astype(np.float64).sum(axis=0))


def test_stream_equals_one_shot(torch, dd):
    _say("case: stream vs one shot")
    freq = fbsynth.channel_freqs(428.0, 20.0 / 128, 128)
    dm = fbsynth.dm_trials(0.0, 0.1, 96)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    m = int(tab.max())
    block = 700
    sizes = [block] * 6 + [333, block]
    # a seed for which every block's outputs keep a margin from their thresholds
    for seed in range(21, 71):
        x = np.random.default_rng(seed).standard_normal((128, sum(sizes))).astype(np.float32)
        expected = orc.stream_expected(np.split(x, np.cumsum(sizes)[:-1], axis=1), tab)
        margins = [orc.threshold_margin(w, *orc.series_stats(w), 3.0) for t0, t1, w in expected if t1 > t0]
        if min(margins) > 4 * GUARD:
            break
    else:
        raise AssertionError("no well-conditioned seed in 50")
    plan = dd.Plan(freq, 51.2e-6, dm)
    s = dd.Stream(plan, block)
    one = plan.dedisperse(torch.from_numpy(x).cuda()).out.cpu().numpy()
    pos = 0
    produced = 0
    for j, n in enumerate(sizes):
        blk = torch.from_numpy(np.ascontiguousarray(x[:, pos:pos + n])).cuda()
        pos += n
        r = s.push(blk, k_sigma=3.0)
        t0, t1, want = expected[j]
        if t1 == t0:
            assert r is None
            continue
        assert r is not None and r.t0 == t0 and r.out.shape[1] == t1 - t0
        got = r.out.cpu().numpy()
        np.testing.assert_array_equal(got, one[:, t0:t1])
        mean, rms = orc.series_stats(want)
        assert_stats_close(r.mean.cpu().numpy(), r.rms.cpu().numpy(), mean, rms)
        compare_candidates(r.candidates(), want, mean, rms, 3.0, t_offset=t0)
        produced = t1
    assert produced == sum(sizes) - m


def test_stream_gap_fill(torch, dd):
    """Lost blocks (a seq jump) with gap fill on: the ring receives zeros for them, and every
    output the stream then emits equals the one-shot result on the input with zeros in place
    of the lost blocks, at the same global times; without gap fill the jump is refused."""
    _say("case: stream gap fill")
    freq = fbsynth.channel_freqs(428.0, 20.0 / 128, 128)
    dm = fbsynth.dm_trials(0.0, 0.1, 96)
    block = 700
    nblk = 9
    lost = {3, 4}
    x = np.random.default_rng(5).standard_normal((128, block * nblk)).astype(np.float32)
    for dtype in ("f32", "u8"):
        xs = fbsynth.to_u8(x) if dtype == "u8" else x
        fs = xs.copy()
        for j in lost:
            fs[:, j * block:(j + 1) * block] = 0
        plan = dd.Plan(freq, 51.2e-6, dm, dtype=dtype)
        one = plan.dedisperse(torch.from_numpy(fs).cuda()).out.cpu().numpy()
        s = dd.Stream(plan, block, gap_fill=True)
        strict = dd.Stream(plan, block)
        seen = []
        for j in range(nblk):
            if j in lost:
                continue
            blk = torch.from_numpy(np.ascontiguousarray(xs[:, j * block:(j + 1) * block])).cuda()
            r = s.push(blk, seq=j)
            if j == min(lost) + len(lost):  # the first block after the gap
                with pytest.raises(dd.DedispError) as e:
                    strict.push(blk, seq=j)
                assert e.value.code == -3
            elif j < min(lost):
                strict.push(blk, seq=j)
            if r is None:
                continue
            got = r.out.cpu().numpy()
            np.testing.assert_array_equal(got, one[:, r.t0:r.t0 + got.shape[1]])
            seen.append((r.t0, got.shape[1]))
        # the window after the gap starts past outputs that only the zeros made computable
        starts = [t for t, n in seen]
        assert starts == sorted(starts) and seen[-1][0] + seen[-1][1] == nblk * block - plan.maxdelay


def test_candidate_overflow(torch, dd):
    _say("case: candidate overflow")
    b = fbsynth.config1()
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    want = orc.dedisperse(b.data, tab)
    mean, rms = orc.series_stats(want)
    full = orc.candidates(want, mean, rms, 2.5)
    n = full["t"].size
    assert n > 100
    _, r = _run(torch, dd, b.freq_mhz, b.tsamp_s, b.dm, b.data, k=2.5, cap=37)
    assert r.ncand() == n
    # the synchronising check reports the overflow (DD_WARN_CAND_OVERFLOW) and the true count
    import ctypes as C
    from paper_1401_8258_amd import _lib
    cnt = C.c_int64()
    rc = _lib.load().dd_candidates_check(C.c_void_p(r._ncand.data_ptr()), 37,
                                         C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(cnt))
    assert rc == _lib.DD_WARN_CAND_OVERFLOW and cnt.value == n
    assert _lib.load().dd_candidates_check(C.c_void_p(r._ncand.data_ptr()), n, None, C.byref(cnt)) == _lib.DD_OK
    with pytest.warns(dd.CandidateOverflow):
        got = r.candidates()
    assert got.size == 37
    np.testing.assert_array_equal(got["dm_index"], full["dm_index"][:37])
    np.testing.assert_array_equal(got["t"], full["t"][:37])


def test_error_paths(torch, dd):
    _say("case: error paths")
    from paper_1401_8258_amd import _lib
    import ctypes as C
    b = fbsynth.config1()
    plan = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm)
    x = torch.zeros((64, 1000), device="cuda")
    out = torch.empty((128, 1000), device="cuda")
    ws = plan.workspace(1000)
    lib = _lib.load()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.dd_dedisperse(plan.handle, C.c_void_p(x.data_ptr()), 1000, 1000, C.c_void_p(out.data_ptr()), 1000,
                           None, None, 0.0, None, 0, None, C.c_void_p(ws.data_ptr()), 16, st)
    assert rc == _lib.DD_ERR_WORKSPACE
    rc = lib.dd_dedisperse(plan.handle, C.c_void_p(x.data_ptr()), 500, 1000, C.c_void_p(out.data_ptr()), 1000,
                           None, None, 0.0, None, 0, None, C.c_void_p(ws.data_ptr()), ws.numel(), st)
    assert rc == _lib.DD_ERR_TOO_SHORT
    s = dd.Stream(plan, 256)
    s.seq = 3
    with pytest.raises(dd.DedispError) as e:
        s.push(torch.zeros((64, 256), device="cuda"))
    assert e.value.code == _lib.DD_ERR_SEQUENCE


def test_config2_full_size_sampled(torch, dd):
    """Full 1024 x 2^20 x 2048 workload in the benchmark's launch configuration; the oracle
    recomputes whole sampled rows (and their statistics and candidates): both ends, a middle
    row, and the trials nearest the four brightest injected pulses, where the series reach
    their largest values and FP32 accumulation error peaks."""
    _say("case: config2 full size, generating input")
    b = fbsynth.config2()
    bright = sorted(b.pulses, key=lambda p: -p.amp)[:4]
    rows = sorted({0, 777, 2047} | {int(np.argmin(np.abs(b.dm - p.dm))) for p in bright})
    _say(f"case: config2 rows {rows}")
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    plan = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm)
    np.testing.assert_array_equal(plan.delays(), tab)
    x = torch.from_numpy(b.data).cuda()
    _say("case: config2 full size, running")
    r = plan.dedisperse(x, k_sigma=6.0, cand_cap=1 << 20)
    torch.cuda.synchronize()
    del x
    got_mean, got_rms = r.mean.cpu().numpy(), r.rms.cpu().numpy()
    cands = r.candidates()
    for d in rows:
        _say(f"case: config2 oracle row {d}")
        want = orc.dedisperse(b.data, tab, rows=[d])
        mean, rms = orc.series_stats(want)
        got = r.out[d:d + 1].cpu().numpy()
        assert_rows_close(got, want, rms, what=f"config2 row {d}")
        assert_stats_close(got_mean[d:d + 1], got_rms[d:d + 1], mean, rms)
        sel = cands[cands["dm_index"] == d]
        compare_candidates(sel, want, mean, rms, 6.0, row_ids=[d])
    # bright, resolved pulses show up near their DM in the candidate list
    for p in b.pulses:
        if p.amp * 32.0 < 10.0 or p.width < 4:
            continue
        near = cands[np.abs(b.dm[cands["dm_index"]] - p.dm) < 2.0]
        assert near.size > 0, p
