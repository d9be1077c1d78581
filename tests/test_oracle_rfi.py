"""Pins of the oracle's RFI mitigation (Sec. 3 "Bandpass Correction", "Channel
Thresholding", "Spectrum Thresholding").

Checked against what is fixed outside the oracle's code: an exact polynomial bandpass is
fitted with zero residual and corrects to zero; a literal pure-Python loop over windows,
spectra and the subtraction agrees on tiny inputs; corrected noise has each channel's mean
near zero; injected narrowband bursts, dropouts and broadband spikes become exactly 0 after
correction while every other sample loses only its channel's fitted value.
"""
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
