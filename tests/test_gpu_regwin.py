"""The register-window kernel form (DD_FORM_REGWIN) against the LDS form and the oracle.

Both forms sum each output over the channels in the same fixed order (FP32 inside blocks of
32 channels, block sums in order), so their series must agree bit for bit; the oracle bounds
both within 1e-5 series RMS (Eq. bruteEquation). Each case prints its shape before it runs.
"""
import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import GUARD, assert_rows_close, assert_stats_close, compare_candidates, cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return cuda()


@pytest.fixture(scope="module")
def dd():
    import paper_1401_8258_amd as dd
    dd.load_library()
    return dd


def _both(dd, freq, tsamp, dm):
    a = dd.Plan(freq, tsamp, dm, form="regwin")
    b = dd.Plan(freq, tsamp, dm, form="lds")
    assert a.form == "regwin" and b.form == "lds"
    return a, b


def test_config1_equals_lds_form_and_oracle(torch, dd):
    print("case: config 1, register-window form", flush=True)
    b = fbsynth.config1()
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    want = orc.dedisperse(b.data, tab)
    mean, rms = orc.series_stats(want)
    rw, lds = _both(dd, b.freq_mhz, b.tsamp_s, b.dm)
    np.testing.assert_array_equal(rw.delays(), tab)
    x = torch.from_numpy(b.data).cuda()
    k = 4.0
    assert orc.threshold_margin(want, mean, rms, k) > GUARD
    r1 = rw.dedisperse(x, k_sigma=k)
    r2 = lds.dedisperse(x, k_sigma=k)
    torch.cuda.synchronize()
    assert torch.equal(r1.out, r2.out), "register-window and LDS forms differ"
    got = r1.out.cpu().numpy()
    assert_rows_close(got, want, rms, what="regwin config 1")
    assert_stats_close(r1.mean.cpu().numpy(), r1.rms.cpu().numpy(), mean, rms)
    compare_candidates(r1.candidates(), want, mean, rms, k)


# nchan, channel width (MHz), ndm, DM step, nsamp, input row padding, output row padding
EDGES = [
    (1, 0.3125, 1, 0.1, 300, 0, 0),          # one channel, one trial
    (64, 0.3125, 128, 0.1, 556, 0, 0),       # nout = 1
    (64, 0.3125, 128, 0.1, 1000, 3, 1),      # nout < one tile; odd paddings (no float4 stores)
    (37, 0.5, 33, 0.1, 2000, 0, 0),          # odd channel count, partial stage and group
    (13, 0.3125, 70, 0.1, 5001, 1, 0),       # fewer channels than a stage, 2 groups
    (200, 0.1, 130, 0.1, 4097, 0, 4),        # 25 stages, 3 groups, ragged tail tile
    (512, 20.0 / 512, 300, 0.1, 20000, 0, 0),  # the full band at 512 channels
]


@pytest.mark.parametrize("nchan,df,ndm,step,nsamp,pad,opad", EDGES)
def test_edges_equal_lds_form_and_oracle(torch, dd, nchan, df, ndm, step, nsamp, pad, opad):
    print(f"case: regwin nchan={nchan} ndm={ndm} step={step} nsamp={nsamp} pad={pad} opad={opad}", flush=True)
    freq = fbsynth.channel_freqs(428.0, df, nchan)
    dm = fbsynth.dm_trials(0.0, step, ndm)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    if nsamp <= int(tab.max()):
        pytest.skip("shape shorter than the delay spread")
    # at 3 sigma a few million outputs almost always put some value near its threshold
    k = 3.0 if ndm * (nsamp - int(tab.max())) < 500_000 else 4.5
    # the first seed whose oracle values all keep a clear margin from their thresholds
    for seed in range(nchan * 11 + ndm, nchan * 11 + ndm + 50):
        rng = np.random.default_rng(seed)
        full = np.zeros((nchan, nsamp + pad), np.float32)
        full[:, :nsamp] = fbsynth.noise(rng, nchan, nsamp)
        data = np.ascontiguousarray(full[:, :nsamp])
        want = orc.dedisperse(data, tab)
        mean, rms = orc.series_stats(want)
        if orc.threshold_margin(want, mean, rms, k) > 4 * GUARD:
            break
    else:
        pytest.fail("no well-conditioned seed in 50")
    rw, lds = _both(dd, freq, 51.2e-6, dm)
    xt = torch.from_numpy(full).cuda()[:, :nsamp]
    nout = nsamp - int(tab.max())
    o1 = torch.full((ndm, nout + opad), -7.0, device="cuda")
    o2 = torch.full((ndm, nout + opad), -7.0, device="cuda")
    r1 = rw.dedisperse(xt, k_sigma=k, out=o1)
    r2 = lds.dedisperse(xt, k_sigma=k, out=o2)
    torch.cuda.synchronize()
    assert torch.equal(r1.out, r2.out), "register-window and LDS forms differ"
    if opad:
        assert torch.all(o1[:, nout:] == -7.0), "write past nout"
    assert_rows_close(r1.out.cpu().numpy(), want, rms, what="regwin edge")
    assert_stats_close(r1.mean.cpu().numpy(), r1.rms.cpu().numpy(), mean, rms)
    compare_candidates(r1.candidates(), want, mean, rms, k)


def test_stream_equals_one_shot(torch, dd):
    print("case: regwin stream, ragged blocks", flush=True)
    freq = fbsynth.channel_freqs(428.0, 20.0 / 256, 256)
    dm = fbsynth.dm_trials(0.0, 0.1, 200)
    sizes = [3000, 3000, 1111, 3000, 1, 3000, 2500, 3000]
    rng = np.random.default_rng(5150)
    x = fbsynth.noise(rng, 256, sum(sizes))
    plan = dd.Plan(freq, 51.2e-6, dm, form="regwin")
    assert plan.form == "regwin"
    whole = plan.dedisperse(torch.from_numpy(x).cuda()).out
    st = dd.Stream(plan, 3000)
    pos = 0
    seen = 0
    for n in sizes:
        r = st.push(torch.from_numpy(np.ascontiguousarray(x[:, pos:pos + n])).cuda())
        pos += n
        if r is None:
            continue
        n_out = r.out.shape[1]
        assert r.t0 == seen
        assert torch.equal(r.out, whole[:, seen:seen + n_out]), f"stream block at t0={r.t0} differs"
        seen += n_out
    assert seen == whole.shape[1]


def test_full_size_equals_lds_form(torch, dd):
    """The full FP32 workload (1024 channels, 2^20 samples, 2048 trials): every output of the
    register-window form equals the LDS form's, and sampled rows (the brightest pulses' trials
    and both ends) equal the oracle."""
    print("case: regwin full size 1024 ch x 2^20 x 2048 DMs", flush=True)
    b = fbsynth.config2()
    rw, lds = _both(dd, b.freq_mhz, b.tsamp_s, b.dm)
    x = torch.from_numpy(b.data).cuda()
    r1 = rw.dedisperse(x, k_sigma=6.0)
    torch.cuda.synchronize()
    r2 = lds.dedisperse(x, k_sigma=6.0)
    torch.cuda.synchronize()
    assert torch.equal(r1.out, r2.out), "register-window and LDS forms differ"
    del r2
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    rows = [0, 329, 1508, 2047]
    want = orc.dedisperse(b.data, tab, rows=rows)
    mean, rms = orc.series_stats(want)
    got = r1.out[rows].cpu().numpy()
    assert_rows_close(got, want, rms, what="regwin full size")
    assert_stats_close(r1.mean.cpu().numpy()[rows], r1.rms.cpu().numpy()[rows], mean, rms)
