"""Pins of the oracle's boxcar template matching (Sec. 6 "Transient Surveys"; Sec. 2
Eq. pulseSNREquation): a literal loop, the single-width case against the plain n-sigma
threshold, closed-form S/N of rectangular pulses at aligned and unaligned starts, and
the rules for rows without variance and for ties between widths."""
import math

import numpy as np

from oracle import dedisp_oracle as orc


def _literal(x, mean, rms, max_log2, k):
    """Every start, every width, written out as loops."""
    out = []
    nrows, n = x.shape
    for d in range(nrows):
        if rms[d] <= 0:
            continue
        for t in range(n):
            best, bw, bv = -math.inf, 0, 0.0
            for j in range(max_log2 + 1):
                w = 1 << j
                if t + w > n:
                    break
                b = 0.0
                for i in range(w):
                    b += float(x[d, t + i])
                snr = (b - w * float(mean[d])) / (float(rms[d]) * math.sqrt(w))
                if snr > best:
                    best, bw, bv = snr, w, b
            if best > k:
                out.append((d, t, bw, bv, best))
    return out


def test_matches_a_literal_loop():
    rng = np.random.default_rng(42)
    x = rng.standard_normal((3, 57))
    x[1, 20:28] += 1.2  # a pulse so that several widths detect
    mean, rms = x.mean(axis=1), x.std(axis=1)
    got = orc.boxcar_search(x, mean, rms, 4, 1.5)
    want = _literal(x, mean, rms, 4, 1.5)
    assert len(want) > 10
    assert list(got["row"]) == [w[0] for w in want]
    assert list(got["t"]) == [w[1] for w in want]
    assert list(got["width"]) == [w[2] for w in want]
    np.testing.assert_allclose(got["value"], [w[3] for w in want], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(got["snr"], [w[4] for w in want], rtol=1e-12, atol=1e-12)


def test_width_one_is_the_plain_threshold():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((4, 300))
    mean, rms = x.mean(axis=1), x.std(axis=1)
    got = orc.boxcar_search(x, mean, rms, 0, 2.0)
    want = orc.candidates(x, mean, rms, 2.0)
    np.testing.assert_array_equal(got["row"], want["dm_index"])
    np.testing.assert_array_equal(got["t"], want["t"])
    assert np.all(got["width"] == 1)
    np.testing.assert_array_equal(got["value"], want["value"])
    np.testing.assert_allclose(got["snr"], want["snr"], rtol=1e-15)


def test_unaligned_pulse_closed_form():
    """A rectangular pulse of amplitude a and width 8 starting at sample 13 (not a multiple
    of 8) on a zero series with mean 0 and rms 1: the width-8 boxcar that starts on it
    holds all its area, S/N = 8a / sqrt(8) = a sqrt(8), and is the only detection at
    k = 0.95 a sqrt(8). The non-overlapping (decimated) sums split the pulse 3 + 5 and
    reach only 5a / sqrt(8)."""
    a = 1.7
    x = np.zeros((1, 200))
    x[0, 13:21] = a
    mean, rms = np.zeros(1), np.ones(1)
    k = 0.95 * a * math.sqrt(8)
    got = orc.boxcar_search(x, mean, rms, 6, k)
    assert list(got["t"]) == [13] and list(got["width"]) == [8]
    assert math.isclose(got["snr"][0], a * math.sqrt(8), rel_tol=1e-14)
    assert math.isclose(got["value"][0], 8 * a, rel_tol=1e-14)
    # the neighbours: one sample of the pulse missed (width 8) or half the width empty (16)
    snr = orc.boxcar_snr(x, mean, rms, 6)
    assert math.isclose(snr[3][0, 12], 7 * a / math.sqrt(8), rel_tol=1e-14)
    assert math.isclose(snr[4][0, 5], 8 * a / 4.0, rel_tol=1e-14)
    levels = orc.boxcar_levels(x, 3)
    assert math.isclose(levels[3].max(), 5 * a / math.sqrt(8), rel_tol=1e-14)
    assert levels[3].max() < k


def test_pulse_of_width_five_and_aligned_widths():
    """Width 5 is not among the templates: the best is width 4 inside the pulse,
    S/N 4a / 2 = 2a, beside width 8 covering it, 5a / sqrt(8) = 1.77a."""
    a = 1.0
    x = np.zeros((1, 64))
    x[0, 30:35] = a
    got = orc.boxcar_search(x, np.zeros(1), np.ones(1), 6, 1.9 * a)
    assert list(got["t"]) == [30, 31] and list(got["width"]) == [4, 4]
    np.testing.assert_allclose(got["snr"], [2 * a, 2 * a], rtol=1e-14)


def test_rows_without_variance_and_short_rows():
    x = np.vstack([np.full(20, 3.0), np.arange(20.0)])
    got = orc.boxcar_search(x, x.mean(axis=1), x.std(axis=1), 6, 0.5)
    assert set(got["row"]) == {1}  # the constant row has rms 0: no detections
    # widths longer than the row are not defined; the last starts use the widths that fit
    assert got["t"].max() == 19 and got["width"][got["t"] == 19][0] == 1


def test_ties_take_the_narrower_width():
    """x[t] = 1, x[t+1] = sqrt(2) - 1 (built so widths 1 and 2 tie in exact arithmetic): the
    search takes width 1 unless width 2's S/N is strictly larger in FP64."""
    x = np.zeros((1, 16))
    x[0, 5] = 1.0
    x[0, 6] = math.sqrt(2.0) - 1.0
    snr = orc.boxcar_snr(x, np.zeros(1), np.ones(1), 1)
    got = orc.boxcar_search(x, np.zeros(1), np.ones(1), 1, 0.9)
    i = list(got["t"]).index(5)
    assert got["width"][i] == (2 if snr[1][0, 5] > snr[0][0, 5] else 1)


def test_margin_reports_threshold_and_width_gaps():
    """A pulse of 4 ones at t = 10..13 and k = 1.6: the one detection (t = 10, width 4,
    S/N 2) is 0.4 above k and 2 - 4/sqrt(8) = 0.586 above the next width; the closest
    non-detection is a width-4 boxcar holding 3 of the ones (S/N 1.5), 0.1 below k."""
    x = np.zeros((1, 40))
    x[0, 10:14] = 1.0
    k = 1.6
    got = orc.boxcar_search(x, np.zeros(1), np.ones(1), 3, k)
    assert list(got["t"]) == [10] and list(got["width"]) == [4]
    m = orc.boxcar_margin(x, np.zeros(1), np.ones(1), 3, k)
    assert math.isclose(m, 0.1, rel_tol=1e-12)
    assert orc.boxcar_margin(x, np.zeros(1), np.ones(1), 3, 1.95) < 0.05 + 1e-12
