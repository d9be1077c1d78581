"""Pins of the oracle's RFI mitigation (Sec. 3 "Bandpass Correction", "Channel
Thresholding", "Spectrum Thresholding").

Checked against what is fixed outside the oracle's code: an exact polynomial bandpass is
fitted with zero residual and corrects to zero; a literal pure-Python loop over windows,
spectra and the subtraction agrees on tiny inputs; corrected noise has each channel's mean
near zero; injected narrowband bursts, dropouts and broadband spikes become exactly 0 after
correction while every other sample loses only its channel's fitted value.
"""
import math

import numpy as np
import pytest

from oracle import dedisp_oracle as orc


def _bandpass(nchan):
    c = np.arange(nchan)
    return 10.0 + 3.0 * np.sin(np.pi * c / nchan) + 0.002 * c


@pytest.mark.parametrize("order,nchan", [(0, 1), (1, 2), (3, 17), (5, 64), (8, 1024)])
def test_polynomial_bandpass_is_fitted_exactly(order, nchan):
    x = np.zeros(nchan) if nchan == 1 else 2.0 * np.arange(nchan) / (nchan - 1) - 1.0
    coef = np.arange(1, order + 2) * 0.5
    poly = sum(cf * x ** i for i, cf in enumerate(coef))
    data = np.repeat(poly[:, None], 7, axis=1)
    avg = orc.bandpass_average(data)
    np.testing.assert_allclose(avg, poly, rtol=0, atol=1e-12)
    fit, rmse, fmean = orc.bandpass_fit(avg, order)
    np.testing.assert_allclose(fit, poly, rtol=0, atol=1e-9)
    assert rmse < 1e-9 and abs(fmean - poly.mean()) < 1e-9
    # a pure bandpass is all response: the corrected spectra are zero (to the fit's residual)
    out = orc.rfi_mitigate(data, order, 0.0, 1, 0.0)[0]
    assert np.max(np.abs(out)) < 1e-9


def _literal(data, fit, fit_mean, cthr, window, sthr):
    """Pure-Python loops: the stages written out sample by sample."""
    nchan, n = len(data), len(data[0])
    x = [list(map(float, row)) for row in data]
    nwin = (n + window - 1) // window
    flag = [[False] * nwin for _ in range(nchan)]
    for c in range(nchan):
        for w in range(nwin):
            idx = range(w * window, min(n, (w + 1) * window))
            m = sum(x[c][t] for t in idx) / len(idx)
            flag[c][w] = abs(m - fit[c]) > cthr
    y = [row[:] for row in x]
    for c in range(nchan):
        for w in range(nwin):
            if flag[c][w] or (w > 0 and flag[c][w - 1]) or (w + 1 < nwin and flag[c][w + 1]):
                for t in range(w * window, min(n, (w + 1) * window)):
                    y[c][t] = fit[c]
    for t in range(n):
        m = sum(y[c][t] for c in range(nchan)) / nchan
        if abs(m - fit_mean) > sthr:
            for c in range(nchan):
                y[c][t] = fit[c]
    for c in range(nchan):
        for t in range(n):
            y[c][t] = y[c][t] - fit[c]
    return np.array(y)


def test_against_literal_loops():
    rng = np.random.default_rng(11)
    nchan, n, window = 6, 53, 8
    data = _bandpass(nchan)[:, None] + rng.standard_normal((nchan, n))
    data[2, 17:21] += 9.0
    data[4, 40:53] = 0.0
    data[:, 30] += 6.0
    out, fit, rmse, fmean, cf, sf = orc.rfi_mitigate(data, 2, 1.5, window, 2.0)
    np.testing.assert_allclose(out, _literal(data, fit, fmean, 1.5, window, 2.0), rtol=0, atol=1e-12)
    assert cf[2, 2] and cf[4, 5] and cf[4, 6] and sf[30]


def test_corrected_noise_has_zero_channel_means():
    """Noise on a bandpass: after correction every channel's mean is within a few standard
    errors of 0 (the fit absorbs the response), and no stage flags clean data."""
    rng = np.random.default_rng(5)
    nchan, n, window = 64, 4096, 64
    data = _bandpass(nchan)[:, None] + rng.standard_normal((nchan, n))
    out, fit, rmse, fmean, cf, sf = orc.rfi_mitigate(data, 4, 1.0, window, 1.0)
    assert not cf.any() and not sf.any()
    assert np.max(np.abs(out.mean(axis=1))) < 5.0 / np.sqrt(n)
    # with no clipping the correction is the data minus the fit, sample by sample
    np.testing.assert_allclose(out, data - fit[:, None], rtol=0, atol=1e-12)
    # the uncorrected form (subtract=False) leaves clean data as it was
    raw = orc.rfi_mitigate(data, 4, 1.0, window, 1.0, subtract=False)[0]
    np.testing.assert_array_equal(raw, data)


def test_bursts_replaced_and_corrected_to_zero():
    rng = np.random.default_rng(5)
    nchan, n, window = 64, 4096, 64
    data = _bandpass(nchan)[:, None] + rng.standard_normal((nchan, n))
    dirty = data.copy()
    dirty[7, 640:830] += 5.0        # narrowband burst across windows 10..12
    dirty[20, 0:64] = 0.0           # lost data in window 0
    dirty[:, 2000:2003] += 3.0      # broadband spike
    out, fit, rmse, fmean, cf, sf = orc.rfi_mitigate(dirty, 4, 1.0, window, 1.0)
    assert set(np.nonzero(cf[7])[0]) == {10, 11, 12} and list(np.nonzero(cf[20])[0]) == [0]
    assert list(np.nonzero(sf)[0]) == [2000, 2001, 2002]
    np.testing.assert_array_equal(out[7, 9 * 64:14 * 64], 0.0)
    np.testing.assert_array_equal(out[20, 0:128], 0.0)
    np.testing.assert_array_equal(out[:, 2000:2003], 0.0)
    keep = np.ones_like(dirty, dtype=bool)
    keep[7, 9 * 64:14 * 64] = keep[20, 0:128] = False
    keep[:, 2000:2003] = False
    np.testing.assert_allclose(out[keep], (dirty - fit[:, None])[keep], rtol=0, atol=1e-12)
    # uncorrected: the replaced samples hold the fitted value, the rest is untouched
    raw = orc.rfi_mitigate(dirty, 4, 1.0, window, 1.0, subtract=False)[0]
    np.testing.assert_array_equal(raw[7, 9 * 64:14 * 64], np.full(5 * 64, fit[7]))
    np.testing.assert_array_equal(raw[keep], dirty[keep])


def _literal_codes(data, fit, fit_mean, cthr, window, sthr):
    """The 8-bit stage as pure-Python loops: integer window and spectrum sums, replaced
    samples take the nearest code of the fit (halves up, clamped to 0..255)."""
    nchan, n = len(data), len(data[0])
    code = [min(255, max(0, math.floor(f + 0.5))) for f in fit]
    y = [[int(v) for v in row] for row in data]
    nwin = (n + window - 1) // window
    flag = [[False] * nwin for _ in range(nchan)]
    for c in range(nchan):
        for w in range(nwin):
            idx = range(w * window, min(n, (w + 1) * window))
            flag[c][w] = abs(sum(y[c][t] for t in idx) / len(idx) - fit[c]) > cthr
    for c in range(nchan):
        for w in range(nwin):
            if flag[c][w] or (w > 0 and flag[c][w - 1]) or (w + 1 < nwin and flag[c][w + 1]):
                for t in range(w * window, min(n, (w + 1) * window)):
                    y[c][t] = code[c]
    for t in range(n):
        if abs(sum(y[c][t] for c in range(nchan)) / nchan - fit_mean) > sthr:
            for c in range(nchan):
                y[c][t] = code[c]
    return np.array(y, dtype=np.uint8)


def _codes(rng, nchan, n):
    x = _bandpass(nchan)[:, None] * 10.0 + 6.0 * rng.standard_normal((nchan, n))
    return np.clip(np.floor(x + 0.5), 0, 255).astype(np.uint8)


def test_codes_against_literal_loops_and_planted_rfi():
    """8-bit codes: a narrowband burst, a dropout and a broadband spike are replaced by the
    fitted codes, exactly as the literal loops do, and nothing else changes."""
    rng = np.random.default_rng(13)
    nchan, n, window = 8, 203, 16
    x = _codes(rng, nchan, n)
    x[3, 40:60] = 255
    x[5, 160:203] = 0
    x[:, 100] = 250
    out, fit, rmse, fmean, cf, sf = orc.rfi_mitigate_codes(x, 2, 20.0, window, 30.0)
    np.testing.assert_array_equal(out, _literal_codes(x, fit, fmean, 20.0, window, 30.0))
    assert cf[3, 2] and cf[3, 3] and cf[5, 11] and cf[5, 12] and sf[100]
    code = orc.fit_codes(fit)
    np.testing.assert_array_equal(out[3, 16:80], np.full(64, code[3], np.uint8))
    np.testing.assert_array_equal(out[:, 100], code)
    keep = np.ones(x.shape, dtype=bool)
    for c in range(nchan):
        for w in np.nonzero(cf[c])[0]:
            keep[c, max(0, w - 1) * window:(w + 2) * window] = False
    keep[:, sf] = False
    np.testing.assert_array_equal(out[keep], x[keep])


def test_fit_codes_round_halves_up_and_clamp():
    np.testing.assert_array_equal(orc.fit_codes([-3.0, -0.5, 0.49, 0.5, 1.5, 2.5, 254.5, 255.4, 300.0]),
                                  np.array([0, 0, 0, 1, 2, 3, 255, 255, 255], np.uint8))


def test_codes_stage_agrees_with_the_float_stage_on_integer_fits():
    """Where the fitted bandpass is integral (levels linear in the channel index, which a fit
    of order 1 or 2 reproduces, plus excursions that leave each channel mean as it was), the
    8-bit stage equals the float stage without correction: the same decisions and the same
    replaced values."""
    nchan, n, window = 5, 96, 8
    levels = np.array([40, 80, 120, 160, 200], np.float64)
    x = np.repeat(levels[:, None], n, axis=1)
    x[:, 10] += 4
    x[:, 11] -= 4
    x[2, 48:56] = levels[2] + 60
    x[2, 56:64] = levels[2] - 60  # a burst and a dropout: the channel mean stays integral
    u8 = x.astype(np.uint8)
    ran = 0
    for order in (1, 2):
        out8 = orc.rfi_mitigate_codes(u8, order, 30.0, window, 3.0)
        outf = orc.rfi_mitigate(x, order, 30.0, window, 3.0, subtract=False)
        if not np.allclose(outf[1], np.round(outf[1]), atol=1e-9):
            continue
        np.testing.assert_array_equal(out8[0], np.round(outf[0]).astype(np.uint8))
        np.testing.assert_array_equal(out8[4], outf[4])
        np.testing.assert_array_equal(out8[5], outf[5])
        assert out8[4].any() and out8[5].any()
        ran += 1
    assert ran >= 1


def test_correction_of_codes_is_a_constant_offset_of_the_series():
    """Eq. bruteEquation sums each channel once, so subtracting b[c] from every sample of
    channel c lowers every dedispersed sample by sum(b): the series' RMS and its n-sigma
    candidates (value and S/N) stay as they are, which is why the 8-bit stage leaves the
    correction to the caller."""
    rng = np.random.default_rng(3)
    freq = 428.0 - 0.3125 * np.arange(32)
    dm = np.arange(0, 20) * 0.5
    x = _codes(rng, 32, 3000).astype(np.float64)
    b = np.floor(orc.bandpass_fit(orc.bandpass_average(x), 3)[0])  # integral: exact in FP64
    tab = orc.delay_table(freq, dm, 51.2e-6)
    d0 = orc.dedisperse(x, tab)
    d1 = orc.dedisperse(x - b[:, None], tab)
    np.testing.assert_array_equal(d1, d0 - b.sum())
    m0, r0 = orc.series_stats(d0)
    m1, r1 = orc.series_stats(d1)
    np.testing.assert_allclose(m1, m0 - b.sum(), rtol=0, atol=1e-9)
    np.testing.assert_allclose(r1, r0, rtol=1e-12)
    c0, c1 = orc.candidates(d0, m0, r0, 3.0), orc.candidates(d1, m1, r1, 3.0)
    assert c0["t"].size > 0
    np.testing.assert_array_equal(c0["dm_index"], c1["dm_index"])
    np.testing.assert_array_equal(c0["t"], c1["t"])
    np.testing.assert_allclose(c1["snr"], c0["snr"], rtol=1e-9)
