"""Pins of the oracle's detrending and normalisation (Sec. 3.5 "Signal Post-processing").

Each check is fixed by the mathematics of a least-squares line, not by the oracle's own
formula: a pure line leaves nothing; the residual is orthogonal to 1 and t (the normal
equations); numpy.polyfit, an independent fit, gives the same residual; adding any line
changes nothing; a normalised residual has unit population RMS.
"""
import numpy as np
import pytest

from oracle import dedisp_oracle as orc


@pytest.mark.parametrize("n", [2, 3, 10, 1001])
def test_pure_line_vanishes(n):
    t = np.arange(n, dtype=np.float64)
    x = np.stack([3.5 + 0.25 * t, -7.0 + 1e-3 * t, np.full(n, 2.0)])
    y, rms = orc.detrend(x)
    assert np.max(np.abs(y)) < 1e-9 * (1 + np.max(np.abs(x)))
    assert np.max(rms) < 1e-9 * (1 + np.max(np.abs(x)))


@pytest.mark.parametrize("n", [2, 7, 512, 4097])
def test_normal_equations_and_polyfit(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((4, n)) * 5 + 100
    y, rms = orc.detrend(x)
    t = np.arange(n, dtype=np.float64)
    scale = np.abs(x).sum(axis=1) * n
    assert np.all(np.abs(y.sum(axis=1)) < 1e-9 * scale)
    assert np.all(np.abs((y * t).sum(axis=1)) < 1e-9 * scale * n)
    for r in range(x.shape[0]):
        b, a = np.polyfit(t, x[r], 1)
        np.testing.assert_allclose(y[r], x[r] - (a + b * t), rtol=0, atol=1e-8)
        np.testing.assert_allclose(rms[r], np.std(x[r] - (a + b * t)), rtol=1e-9, atol=1e-9 * np.abs(x[r]).max())


def test_adding_a_line_changes_nothing():
    rng = np.random.default_rng(3)
    n = 3000
    x = rng.standard_normal((3, n))
    t = np.arange(n)
    y0, r0 = orc.detrend(x)
    y1, r1 = orc.detrend(x + 12.0 - 0.003 * t)
    np.testing.assert_allclose(y1, y0, atol=1e-9)
    np.testing.assert_allclose(r1, r0, rtol=1e-9)


def test_normalised_has_unit_population_rms_and_edge_cases():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((5, 777)) * 3 + 1
    z, rms = orc.detrend(x, normalise=True)
    np.testing.assert_allclose(np.sqrt(np.mean(z * z, axis=1)), 1.0, rtol=1e-12)
    y, _ = orc.detrend(x)
    np.testing.assert_allclose(z * rms[:, None], y, atol=1e-12)
    # one sample: the line is the sample itself; zero residual, left as is when normalising
    z1, r1 = orc.detrend(np.array([[5.0], [-2.0]]), normalise=True)
    assert np.all(z1 == 0) and np.all(r1 == 0)


def test_boxcar_levels_closed_forms():
    """Boxcar levels: constant input, the pairwise recursion, conservation of sums and a
    matched top-hat pulse."""
    n, K = 1000, 6
    lv = orc.boxcar_levels(np.full((2, n), 3.0), K)
    for k in range(K + 1):
        assert lv[k].shape == (2, n >> k)
        np.testing.assert_allclose(lv[k], 3.0 * np.sqrt(2.0 ** k), rtol=1e-14)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((3, n))
    lv = orc.boxcar_levels(x, K)
    np.testing.assert_array_equal(lv[0], x)
    for k in range(1, K + 1):
        m = lv[k].shape[1]
        prev = lv[k - 1][:, : 2 * m]
        np.testing.assert_allclose(lv[k], (prev[:, 0::2] + prev[:, 1::2]) / np.sqrt(2.0), rtol=1e-12, atol=1e-12)
        cover = m << k
        np.testing.assert_allclose(lv[k].sum(axis=1) * np.sqrt(2.0 ** k), x[:, :cover].sum(axis=1), rtol=1e-10,
                                   atol=1e-9)
    for m in range(K + 1):
        w = 1 << m
        pulse = np.zeros((1, n))
        pulse[0, 5 * w: 6 * w] = 2.0
        lv = orc.boxcar_levels(pulse, K)
        assert np.isclose(lv[m].max(), 2.0 * np.sqrt(w)) and lv[m].argmax() == 5
