"""RFI mitigation on the device (dd_bandpass, dd_bandpass_fit, dd_rfi_clip) against the FP64
oracle (run on an MI355X with -m gpu). Flags are integer decisions taken in FP64 on both
sides; each case checks that no oracle mean lies within 1e-6 of its threshold, so the two
fits (which agree to 1e-9) cannot decide differently. The corrected output (fitted bandpass
subtracted, Ch. 3 Sec. "Bandpass Correction") is one FP32 subtraction of the FP32 fit on the
device: it differs from the FP64 oracle by at most the fit's rounding plus half an ulp of
the result, and a replaced sample is exactly 0 on both sides."""
import sys

import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import cuda

pytestmark = pytest.mark.gpu
GUARD = 1e-6


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


def _dirty(nchan, n, seed):
    rng = np.random.default_rng(seed)
    c = np.arange(nchan)
    x = (10.0 + 3.0 * np.sin(np.pi * c / nchan))[:, None] + rng.standard_normal((nchan, n))
    x = x.astype(np.float32)
    x[nchan // 7, n // 10: n // 10 + 3 * n // 40] += 5.0       # narrowband burst
    x[nchan // 3, : n // 50 + 1] = 0.0                          # lost data
    x[:, n // 2: n // 2 + 3] += 3.0                             # broadband spike
    return x


def _corr_tol(fit, want):
    """|float32(x - float32(fit)) - (x - fit)| <= ulp(fit)/2 + ulp(result)/2 (x is FP32)."""
    return 2.0 ** -24 * (np.abs(fit)[:, None] + np.abs(want)) * 1.01 + 1e-30


def _window_margin(x, fit, thr, window):
    n = x.shape[1]
    worst = np.inf
    for w in range(-(-n // window)):
        m = x[:, w * window:(w + 1) * window].astype(np.float64).mean(axis=1)
        worst = min(worst, float(np.min(np.abs(np.abs(m - fit) - thr))))
    return worst


@pytest.mark.parametrize("nchan,n,stride,window,order", [
    (64, 16384, 16384, 64, 4), (5, 1001, 1013, 7, 2), (1, 300, 300, 16, 0), (33, 4099, 4100, 256, 6)])
def test_rfi_parity(torch, dd, nchan, n, stride, window, order):
    _say(f"case: rfi {nchan}x{n} stride {stride} window {window} order {order}")
    full = np.zeros((nchan, stride), np.float32)
    full[:, :n] = _dirty(nchan, n, nchan * 31 + n)
    x = full[:, :n]
    cthr, sthr = 1.0, 1.0
    want, fit, rmse, fmean, cf, sf = orc.rfi_mitigate(x, order, cthr, window, sthr)
    assert _window_margin(x, fit, cthr, window) > GUARD
    after_chan, _ = orc.channel_clip(x, fit, cthr, window)
    assert float(np.min(np.abs(np.abs(after_chan.mean(axis=0) - fmean) - sthr))) > GUARD
    dev = torch.from_numpy(full).cuda()[:, :n]
    avg = dd.bandpass(dev).cpu().numpy()
    np.testing.assert_allclose(avg, orc.bandpass_average(x), rtol=0, atol=1e-12 * 16)
    avg2, wmeans = dd.bandpass(dev, window)
    np.testing.assert_allclose(avg2.cpu().numpy(), orc.bandpass_average(x), rtol=0, atol=1e-12 * 16)
    want_means = np.array([[x[c, w * window:(w + 1) * window].astype(np.float64).mean()
                            for w in range(-(-n // window))] for c in range(nchan)])
    np.testing.assert_allclose(wmeans.cpu().numpy(), want_means, rtol=0, atol=1e-12 * 16)
    gfit, grmse, gmean, flags = dd.rfi_mitigate(dev, order, cthr, window, sthr)
    got = dev.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(gfit, fit, rtol=0, atol=1e-9)
    np.testing.assert_array_equal(flags.cpu().numpy() != 0, cf)
    replaced = want == 0.0
    assert replaced.any() and cf.any() and sf.any()
    np.testing.assert_array_equal(got[replaced], 0.0)        # replaced, then corrected: exactly 0
    err = np.abs(got - want)
    assert np.all(err <= _corr_tol(fit, want)), float(np.max(err - _corr_tol(fit, want)))
    # the uncorrected form: replaced samples hold the FP32 fit, the rest keep their bits
    dev = torch.from_numpy(full).cuda()[:, :n]
    dd.rfi_mitigate(dev, order, cthr, window, sthr, subtract=False)
    raw = dev.cpu().numpy()
    want_raw = orc.rfi_mitigate(x, order, cthr, window, sthr, subtract=False)[0]
    same = want_raw == x.astype(np.float64)
    np.testing.assert_array_equal(raw[same], x[same])
    np.testing.assert_allclose(raw[~same], want_raw[~same], rtol=0, atol=1e-5)


def test_rfi_stages_skip(torch, dd):
    x = _dirty(16, 2048, 3)
    dev = torch.from_numpy(x.copy()).cuda()
    _, _, _, flags = dd.rfi_mitigate(dev, 2, 0.0, 64, 0.0, subtract=False)
    assert flags is None
    np.testing.assert_array_equal(dev.cpu().numpy(), x)
    # correction alone: one FP32 subtraction per sample, bit for bit
    dev = torch.from_numpy(x.copy()).cuda()
    fit = dd.rfi_mitigate(dev, 2, 0.0, 64, 0.0)[0]
    np.testing.assert_array_equal(dev.cpu().numpy(), x - fit.astype(np.float32)[:, None])


def test_rfi_full_size(torch, dd):
    """The full 1024 x 2^20 FP32 filterbank with injected RFI: bandpass, fit, every channel
    window flag and every spectrum decision against the oracle; sampled rows of the result."""
    _say("case: rfi full size, generating input")
    b = fbsynth.config2()
    x = b.data
    x[100, 200000:260000] += 2.0
    x[700, :5000] = -1.0
    x[:, 500000:500004] += 1.0
    window, order, cthr, sthr = 256, 6, 0.5, 0.2
    dev = torch.from_numpy(x).cuda()
    _say("case: rfi full size, running")
    gfit, grmse, gmean, flags = dd.rfi_mitigate(dev, order, cthr, window, sthr)
    torch.cuda.synchronize()
    _say("case: rfi full size, oracle")
    fit, rmse, fmean = orc.bandpass_fit(orc.bandpass_average(x), order)
    np.testing.assert_allclose(gfit, fit, rtol=0, atol=1e-9)
    nwin = x.shape[1] // window
    means = x.reshape(x.shape[0], nwin, window).astype(np.float64).mean(axis=2)
    dist = np.abs(means - fit[:, None])
    assert float(np.min(np.abs(dist - cthr))) > GUARD
    np.testing.assert_array_equal(flags.cpu().numpy() != 0, dist > cthr)
    assert flags[100].sum().item() >= 234 and flags[700, :19].all()
    got = dev.cpu().numpy()
    del dev
    # every channel's corrected mean is near 0 (noise of unit variance over 2^20 samples,
    # plus the injected RFI that was not replaced)
    assert np.max(np.abs(got.astype(np.float64).mean(axis=1))) < 0.05
    for c in (0, 100, 700, 1023):
        row, _ = orc.channel_clip(x[c:c + 1], fit[c:c + 1], cthr, window)
        col = [t for t in range(500000, 500004)]
        row[0, col] = fit[c]                           # the broadband spike is replaced
        want = orc.bandpass_correct(row, fit[c:c + 1])[0]
        replaced = want == 0.0
        np.testing.assert_array_equal(got[c][replaced], 0.0)
        err = np.abs(got[c].astype(np.float64) - want)
        assert np.all(err <= _corr_tol(fit[c:c + 1], want[None, :])[0])


def _codes_dirty(nchan, n, seed):
    rng = np.random.default_rng(seed)
    c = np.arange(nchan)
    x = (100.0 + 30.0 * np.sin(np.pi * c / nchan))[:, None] + 8.0 * rng.standard_normal((nchan, n))
    x[nchan // 7, n // 10: n // 10 + 3 * n // 40] += 60.0      # narrowband burst
    x[nchan // 3, : n // 50 + 1] = 0.0                          # lost data
    x[:, n // 2: n // 2 + 3] += 40.0                            # broadband spike
    return np.clip(np.floor(x + 0.5), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("nchan,n,stride,window,order", [
    (64, 16384, 16384, 64, 4), (5, 1001, 1013, 7, 2), (1, 300, 300, 16, 0), (33, 4099, 4112, 256, 6),
    (4096, 12207, 12207, 256, 6), (16, 5000, 5008, 1024, 3), (8, 2000, 2000, 32, 2), (24, 3000, 3008, 512, 3),
    (12, 2500, 2512, 128, 2), (16, 4096, 4096, 16, 2)])
def test_rfi_u8_parity(torch, dd, nchan, n, stride, window, order):
    """8-bit codes (dd_bandpass_u8, dd_rfi_clip_u8): averages and window means are exact sums
    divided once, equal to the oracle's bit for bit; every flag and every replaced code
    equals the oracle's (no decision and no fitted value within 1e-6 of flipping); rows
    unaligned (strides 1013, 12207) and ragged windows included; 16-byte aligned rows take
    windows of 16 x 2^k bytes (k = 0..6, with and without a ragged last window) through the
    lane-group path; the fifth case is a 1 s block of a 4096-channel serving beam."""
    _say(f"case: rfi u8 {nchan}x{n} stride {stride} window {window} order {order}")
    full = np.zeros((nchan, stride), np.uint8)
    full[:, :n] = _codes_dirty(nchan, n, nchan * 37 + n)
    x = full[:, :n]
    cthr, sthr = 20.0, 20.0
    want, fit, rmse, fmean, cf, sf = orc.rfi_mitigate_codes(x, order, cthr, window, sthr)
    assert _window_margin(x, fit, cthr, window) > GUARD
    after_chan = orc.rfi_mitigate_codes(x, order, cthr, window, 0.0)[0]
    assert float(np.min(np.abs(np.abs(after_chan.astype(np.float64).mean(axis=0) - fmean) - sthr))) > GUARD
    assert float(np.min(np.abs(fit - np.floor(fit) - 0.5))) > GUARD
    dev = torch.from_numpy(full).cuda()[:, :n]
    np.testing.assert_array_equal(dd.bandpass(dev).cpu().numpy(), orc.bandpass_average(x))
    avg2, wmeans = dd.bandpass(dev, window)
    np.testing.assert_array_equal(avg2.cpu().numpy(), orc.bandpass_average(x))
    want_means = np.array([[x[c, w * window:(w + 1) * window].astype(np.float64).mean()
                            for w in range(-(-n // window))] for c in range(nchan)])
    np.testing.assert_array_equal(wmeans.cpu().numpy(), want_means)
    with pytest.raises(ValueError):
        dd.rfi_mitigate(dev, order, cthr, window, sthr, subtract=True)
    gfit, grmse, gmean, flags = dd.rfi_mitigate(dev, order, cthr, window, sthr)
    np.testing.assert_allclose(gfit, fit, rtol=0, atol=1e-9)
    np.testing.assert_array_equal(flags.cpu().numpy() != 0, cf)
    assert cf.any() and sf.any()
    np.testing.assert_array_equal(dev.cpu().numpy(), want)
    assert np.array_equal(full[:, n:], np.zeros((nchan, stride - n), np.uint8))


def test_rfi_u8_stages_skip(torch, dd):
    """Thresholds <= 0 leave the codes as they are; the spectrum stage alone replaces the
    spike's spectra only."""
    x = _codes_dirty(16, 2048, 4)
    dev = torch.from_numpy(x.copy()).cuda()
    _, _, _, flags = dd.rfi_mitigate(dev, 2, 0.0, 64, 0.0)
    assert flags is None
    np.testing.assert_array_equal(dev.cpu().numpy(), x)
    want, fit, _, fmean, _, sf = orc.rfi_mitigate_codes(x, 2, 0.0, 64, 20.0)
    assert list(np.nonzero(sf)[0]) == [1024, 1025, 1026]
    dd.rfi_mitigate(dev, 2, 0.0, 64, 20.0)
    np.testing.assert_array_equal(dev.cpu().numpy(), want)
