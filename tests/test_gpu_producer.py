"""FP32 with producer wavefronts (the default for FP32 input, two of them; here also one,
three and four):
these wavefronts issue every LDS DMA while the others only compute. Results must equal the oracle to the FP32 tolerance on
the edge shapes, on ragged stream pushes (ring input), and in a batched launch, where they
must also equal the plan's own single calls bit for bit. Each case prints its shape first.
"""
import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from paper_1401_8258_amd._lib import DedispError
from tests.gpu_util import GUARD, assert_rows_close, assert_stats_close, compare_candidates, cuda
from tests.test_gpu_edges_narrow import NARROW

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return cuda()


@pytest.fixture(scope="module")
def dd():
    import paper_1401_8258_amd as dd
    dd.load_library()
    return dd


@pytest.mark.parametrize("pw", [1, 2])
@pytest.mark.parametrize("nchan,df,ndm,step,nsamp,tuning,pad", NARROW)
def test_producer_edges(torch, dd, pw, nchan, df, ndm, step, nsamp, tuning, pad):
    print(f"case: f32 producers={pw} nchan={nchan} ndm={ndm} step={step} nsamp={nsamp} pad={pad}", flush=True)
    freq = fbsynth.channel_freqs(428.0, df, nchan)
    dm = fbsynth.dm_trials(0.0, step, ndm)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    if nsamp <= int(tab.max()):
        pytest.skip("shape shorter than the delay spread")
    try:
        plan = dd.Plan(freq, 51.2e-6, dm, tuning=(8, 0, 0, pw))
    except DedispError:
        # only the wide-band shape has windows beyond the producers' 1024-word limit
        assert df > 1.0
        return
    assert plan.producer_waves == pw
    for seed in range(nchan * 5 + ndm, nchan * 5 + ndm + 50):
        rng = np.random.default_rng(seed)
        full = np.zeros((nchan, nsamp + pad), np.float32)
        full[:, :nsamp] = fbsynth.noise(rng, nchan, nsamp)
        data = np.ascontiguousarray(full[:, :nsamp])
        want = orc.dedisperse(data, tab)
        mean, rms = orc.series_stats(want)
        if orc.threshold_margin(want, mean, rms, 3.0) > 4 * GUARD:
            break
    xt = torch.from_numpy(full).cuda()[:, :nsamp]
    res = plan.dedisperse(xt, k_sigma=3.0)
    torch.cuda.synchronize()
    assert_rows_close(res.out.cpu().numpy(), want, rms, what=f"f32 producers={pw}")
    assert_stats_close(res.mean.cpu().numpy(), res.rms.cpu().numpy(), mean, rms)
    compare_candidates(res.candidates(), want, mean, rms, 3.0)
    # the same sums as the all-wavefront form with the same DM group size
    base = dd.Plan(freq, 51.2e-6, dm, tuning=(8, plan.tiles[1], 0, -1))
    if base.tiles[1] == plan.tiles[1]:
        ref = base.dedisperse(xt, k_sigma=3.0)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(res.out.cpu().numpy(), ref.out.cpu().numpy())


@pytest.mark.parametrize("pw,tun", [(1, (8, 5, 2, 1)), (2, (8, 6, 4, 2))])
def test_producer_stream_ragged(torch, dd, pw, tun):
    print(f"case: f32 stream, producers={pw}, ragged blocks", flush=True)
    freq = fbsynth.channel_freqs(428.0, 20.0 / 128, 128)
    dm = fbsynth.dm_trials(0.0, 0.1, 96)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    sizes = [700, 700, 333, 700, 1, 700, 650, 700]
    x = fbsynth.noise(np.random.default_rng(41), 128, sum(sizes))
    plan = dd.Plan(freq, 51.2e-6, dm, tuning=tun)
    assert plan.producer_waves == pw
    st = dd.Stream(plan, 700)
    expected = orc.stream_expected(np.split(x, np.cumsum(sizes)[:-1], axis=1), tab)
    pos = 0
    for n, (t0, t1, want) in zip(sizes, expected):
        r = st.push(torch.from_numpy(np.ascontiguousarray(x[:, pos:pos + n])).cuda())
        pos += n
        if t1 <= t0:
            assert r is None
            continue
        assert r.t0 == t0 and r.out.shape[1] == t1 - t0
        _, rms = orc.series_stats(want) if want.shape[1] > 1 else (None, np.ones(want.shape[0]))
        assert_rows_close(r.out.cpu().numpy(), want, np.maximum(rms, 1.0), what="f32 producer stream")


def test_producer_batch_equals_single_calls(torch, dd):
    print("case: batch of f32 beams with two producer wavefronts", flush=True)
    rng = np.random.default_rng(12)
    jobs, refs = [], []
    for nchan, ndm, nsamp, step in [(64, 100, 6000, 0.1), (128, 40, 9000, 0.3), (32, 300, 4000, 0.05)]:
        freq = fbsynth.channel_freqs(428.0, 20.0 / nchan, nchan)
        dm = fbsynth.dm_trials(0.0, step, ndm)
        x = rng.standard_normal((nchan, nsamp)).astype(np.float32)
        p = dd.Plan(freq, 51.2e-6, dm, tuning=(8, 4, 0, 2))
        jobs.append((p, torch.from_numpy(x).cuda()))
        refs.append((freq, dm, x))
    res = dd.batch_dedisperse(jobs, k_sigma=4.0)
    torch.cuda.synchronize()
    for (p, x), r, (freq, dm, xh) in zip(jobs, res, refs):
        s = p.dedisperse(x, k_sigma=4.0)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(s.out.cpu().numpy(), r.out.cpu().numpy())
        want = orc.dedisperse(xh, orc.delay_table(freq, dm, 51.2e-6))
        _, rms = orc.series_stats(want)
        assert_rows_close(r.out.cpu().numpy(), want, rms, what="batch f32 producers")


@pytest.mark.parametrize("waves", [0, 5])
@pytest.mark.parametrize("nchan,df,ndm,step,nsamp,tuning,pad", NARROW)
def test_four_trial_form_edges(torch, dd, waves, nchan, df, ndm, step, nsamp, tuning, pad):
    """4 trials per computing wavefront (up to 14 of them beside 2 producers, 1024 threads):
    the oracle to the FP32 tolerance, and the 8-trial producer form bit for bit (series,
    mean and rms: every trial's sums and statistics partials are formed the same way)."""
    print(f"case: f32 4-trial form waves={waves} nchan={nchan} ndm={ndm} step={step} nsamp={nsamp} pad={pad}",
          flush=True)
    freq = fbsynth.channel_freqs(428.0, df, nchan)
    dm = fbsynth.dm_trials(0.0, step, ndm)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    if nsamp <= int(tab.max()):
        pytest.skip("shape shorter than the delay spread")
    try:
        plan = dd.Plan(freq, 51.2e-6, dm, tuning=(4, waves, 0, 2))
        ref_plan = dd.Plan(freq, 51.2e-6, dm, tuning=(8, 0, 0, 2))
    except DedispError:
        assert df > 1.0  # windows beyond the producers' 1024-word limit
        return
    assert plan.tiles[0] == 4 and plan.producer_waves == 2 and 1 <= plan.tiles[1] <= 14
    for seed in range(nchan * 7 + ndm, nchan * 7 + ndm + 50):
        rng = np.random.default_rng(seed)
        full = np.zeros((nchan, nsamp + pad), np.float32)
        full[:, :nsamp] = fbsynth.noise(rng, nchan, nsamp)
        data = np.ascontiguousarray(full[:, :nsamp])
        want = orc.dedisperse(data, tab)
        mean, rms = orc.series_stats(want)
        if orc.threshold_margin(want, mean, rms, 3.0) > 4 * GUARD:
            break
    xt = torch.from_numpy(full).cuda()[:, :nsamp]
    res = plan.dedisperse(xt, k_sigma=3.0)
    ref = ref_plan.dedisperse(xt, k_sigma=3.0)
    torch.cuda.synchronize()
    assert_rows_close(res.out.cpu().numpy(), want, rms, what="f32 4-trial form")
    assert_stats_close(res.mean.cpu().numpy(), res.rms.cpu().numpy(), mean, rms)
    compare_candidates(res.candidates(), want, mean, rms, 3.0)
    np.testing.assert_array_equal(res.out.cpu().numpy(), ref.out.cpu().numpy())
    np.testing.assert_array_equal(res.mean.cpu().numpy(), ref.mean.cpu().numpy())
    np.testing.assert_array_equal(res.rms.cpu().numpy(), ref.rms.cpu().numpy())


@pytest.mark.parametrize("tun", [(4, 14, 0, 2), (4, 7, 3, 1)])
def test_four_trial_form_stream_and_batch(torch, dd, tun):
    """Ragged stream pushes (ring input) equal the oracle; a batch of 4-trial plans equals
    their single calls bit for bit."""
    print(f"case: f32 4-trial form {tun}, stream and batch", flush=True)
    freq = fbsynth.channel_freqs(428.0, 20.0 / 128, 128)
    dm = fbsynth.dm_trials(0.0, 0.1, 96)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    sizes = [700, 700, 333, 700, 1, 700, 650, 700]
    x = fbsynth.noise(np.random.default_rng(43), 128, sum(sizes))
    plan = dd.Plan(freq, 51.2e-6, dm, tuning=tun)
    assert plan.tiles[:2] == (4, tun[1]) and plan.producer_waves == tun[3]
    st = dd.Stream(plan, 700)
    expected = orc.stream_expected(np.split(x, np.cumsum(sizes)[:-1], axis=1), tab)
    pos = 0
    for n, (t0, t1, want) in zip(sizes, expected):
        r = st.push(torch.from_numpy(np.ascontiguousarray(x[:, pos:pos + n])).cuda())
        pos += n
        if t1 <= t0:
            assert r is None
            continue
        assert r.t0 == t0 and r.out.shape[1] == t1 - t0
        _, rms = orc.series_stats(want) if want.shape[1] > 1 else (None, np.ones(want.shape[0]))
        assert_rows_close(r.out.cpu().numpy(), want, np.maximum(rms, 1.0), what="f32 4-trial stream")
    rng = np.random.default_rng(13)
    jobs = []
    # uneven beams whose 56-trial groups fit the producers' 1024-word windows
    for nchan, ndm, nsamp, step in [(64, 100, 6000, 0.1), (128, 40, 9000, 0.1), (32, 300, 4000, 0.05)]:
        f = fbsynth.channel_freqs(428.0, 20.0 / nchan, nchan)
        p = dd.Plan(f, 51.2e-6, fbsynth.dm_trials(0.0, step, ndm), tuning=tun)
        jobs.append((p, torch.from_numpy(rng.standard_normal((nchan, nsamp)).astype(np.float32)).cuda()))
    res = dd.batch_dedisperse(jobs, k_sigma=4.0)
    torch.cuda.synchronize()
    for (p, xd), r in zip(jobs, res):
        s = p.dedisperse(xd, k_sigma=4.0)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(s.out.cpu().numpy(), r.out.cpu().numpy())
        np.testing.assert_array_equal(s.mean.cpu().numpy(), r.mean.cpu().numpy())
        np.testing.assert_array_equal(s.candidates(), r.candidates())


def test_four_trial_form_full_size_equals_default(torch, dd):
    """The full 1024 x 2^20 x 2048 FP32 workload in the 4-trial form (14 computing
    wavefronts) equals the 8-trial producer form bit for bit: series, statistics and
    6-sigma candidates."""
    print("case: f32 4-trial form, full size, generating input", flush=True)
    b = fbsynth.config2()
    x = torch.from_numpy(b.data).cuda()
    p4 = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm, tuning=(4, 14, 0, 2))
    p8 = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm, tuning=(8, 6, 0, 2))
    print("case: f32 4-trial form, full size, running both", flush=True)
    r4 = p4.dedisperse(x, k_sigma=6.0, cand_cap=1 << 20)
    r8 = p8.dedisperse(x, k_sigma=6.0, cand_cap=1 << 20)
    torch.cuda.synchronize()
    assert torch.equal(r4.out, r8.out)
    assert torch.equal(r4.mean, r8.mean) and torch.equal(r4.rms, r8.rms)
    np.testing.assert_array_equal(r4.candidates(), r8.candidates())


@pytest.mark.parametrize("tun", [(4, 13, 0, 3), (4, 12, 0, 4), (8, 5, 0, 3), (8, 4, 0, 4)])
@pytest.mark.parametrize("nchan,df,ndm,step,nsamp,tuning,pad", NARROW)
def test_three_and_four_producers_edges(torch, dd, tun, nchan, df, ndm, step, nsamp, tuning, pad):
    """3 or 4 producer wavefronts, each taking whole channels of a stage (stage widths a
    multiple of the producer count, channels past the last one repeating it): the oracle to
    the FP32 tolerance, and the same trials with 2 producers bit for bit."""
    print(f"case: f32 producers tuning={tun} nchan={nchan} ndm={ndm} step={step} nsamp={nsamp} pad={pad}",
          flush=True)
    freq = fbsynth.channel_freqs(428.0, df, nchan)
    dm = fbsynth.dm_trials(0.0, step, ndm)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    if nsamp <= int(tab.max()):
        pytest.skip("shape shorter than the delay spread")
    try:
        plan = dd.Plan(freq, 51.2e-6, dm, tuning=tun)
    except DedispError as e:
        # a group of this many trials spans windows beyond the producers' 1024-word limit
        assert "do not fit" in str(e)
        return
    ref_plan = dd.Plan(freq, 51.2e-6, dm, tuning=(tun[0], 0, 0, 2))
    assert plan.producer_waves == tun[3] and plan.tiles[0] == tun[0]
    for seed in range(nchan * 11 + ndm, nchan * 11 + ndm + 50):
        rng = np.random.default_rng(seed)
        full = np.zeros((nchan, nsamp + pad), np.float32)
        full[:, :nsamp] = fbsynth.noise(rng, nchan, nsamp)
        data = np.ascontiguousarray(full[:, :nsamp])
        want = orc.dedisperse(data, tab)
        mean, rms = orc.series_stats(want)
        if orc.threshold_margin(want, mean, rms, 3.0) > 4 * GUARD:
            break
    xt = torch.from_numpy(full).cuda()[:, :nsamp]
    res = plan.dedisperse(xt, k_sigma=3.0)
    ref = ref_plan.dedisperse(xt, k_sigma=3.0)
    torch.cuda.synchronize()
    assert_rows_close(res.out.cpu().numpy(), want, rms, what=f"f32 producers {tun}")
    assert_stats_close(res.mean.cpu().numpy(), res.rms.cpu().numpy(), mean, rms)
    compare_candidates(res.candidates(), want, mean, rms, 3.0)
    np.testing.assert_array_equal(res.out.cpu().numpy(), ref.out.cpu().numpy())
    np.testing.assert_array_equal(res.mean.cpu().numpy(), ref.mean.cpu().numpy())
    np.testing.assert_array_equal(res.rms.cpu().numpy(), ref.rms.cpu().numpy())
