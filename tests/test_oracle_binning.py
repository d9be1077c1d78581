"""Pins of the oracle's time binning (Sec. 2 "Direct Dedispersion" and "Computing Larger DMs").

Each check comes from outside the oracle's own code: the diagonal DM printed in closed
form in Ch. 6 (dt f0^3 / (8300 df)) and its one-sample smear under the delay law; the
paper's count of binning stages, ceil(log2(DM_max / DM_diag)) + 1; closed forms of a
downfactored ramp; an impulse's binned position; factor 1 reducing to plain dedispersion.
"""
import math

import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc

BANDS = [(428.0, 64, 20.0, 51.2e-6), (428.0, 1024, 20.0, 51.2e-6), (180.0, 4096, 60.0, 81.92e-6)]


@pytest.mark.parametrize("f_top,nchan,bw,tsamp", BANDS)
def test_diagonal_dm_against_paper_closed_form(golden, f_top, nchan, bw, tsamp):
    df = bw / nchan
    freq = fbsynth.channel_freqs(f_top, df, nchan)
    f0 = float(freq.min())
    closed = tsamp * f0 ** 3 / (golden["diagonal_dm_constant"]["value"] * df)
    dd = orc.diagonal_dm(freq, tsamp)
    # the paper's form is the derivative at the lower edge: equal to first order in df / f0
    assert abs(dd - closed) / closed < 3.0 * df / f0, (dd, closed)
    # at DM_diag the bottom pair's continuous delays (delay law, seconds) differ by one sample
    x = orc.delay_seconds(np.sort(freq)[:2], [dd]) / tsamp
    assert abs(abs(float(x[0, 0] - x[1, 0])) - 1.0) < 1e-9
    # and no neighbouring pair differs by more
    xs = orc.delay_seconds(np.sort(freq), [dd])[:, 0] / tsamp
    assert np.max(np.abs(np.diff(xs))) < 1.0 + 1e-9


def test_diagonal_dm_order_and_single_channel():
    freq = fbsynth.channel_freqs(428.0, 0.3125, 64)
    perm = np.random.default_rng(0).permutation(64)
    assert orc.diagonal_dm(freq[perm], 51.2e-6) == orc.diagonal_dm(freq, 51.2e-6)
    assert math.isinf(orc.diagonal_dm([400.0], 1e-4))


@pytest.mark.parametrize("f_top,nchan,bw,tsamp", BANDS)
@pytest.mark.parametrize("mult", [0.5, 1.0, 1.7, 2.0, 3.1, 8.0, 40.0, 1000.0])
def test_number_of_binning_stages(f_top, nchan, bw, tsamp, mult):
    """Ch. 6 counts ceil(log2(DM_max / DM_diag)) + 1 stages for DMs up to DM_max."""
    freq = fbsynth.channel_freqs(f_top, bw / nchan, nchan)
    dd = orc.diagonal_dm(freq, tsamp)
    dm_max = dd * mult * (1 + 1e-9)
    dms = np.linspace(0.0, dm_max, 4001)
    segs = orc.binning_segments(freq, tsamp, dms, max_log2=30)
    expect = max(1, math.ceil(math.log2(dm_max / dd)) + 1)
    assert len(segs) == expect
    assert [k for k, _, _ in segs] == list(range(expect))
    # each stage covers (2^(k-1) DM_diag, 2^k DM_diag]
    for k, d0, d1 in segs:
        lo = 0.0 if k == 0 else dd * 2.0 ** (k - 1)
        assert np.all(dms[d0:d1] <= dd * 2.0 ** k) and (k == 0 or np.all(dms[d0:d1] > lo))


def test_binning_cap_and_boundaries():
    freq = fbsynth.channel_freqs(428.0, 0.3125, 64)
    dd = orc.diagonal_dm(freq, 51.2e-6)
    dms = [0.0, dd, np.nextafter(dd, np.inf), 2 * dd, np.nextafter(2 * dd, np.inf), 100 * dd]
    assert list(orc.binning_factors(freq, 51.2e-6, dms, 10)) == [0, 0, 1, 1, 2, 7]
    assert list(orc.binning_factors(freq, 51.2e-6, dms, 2)) == [0, 0, 1, 1, 2, 2]
    assert list(orc.binning_factors(freq, 51.2e-6, dms, 0)) == [0] * 6


def test_downfactor_closed_forms():
    n = 11
    ramp = np.stack([np.arange(n, dtype=np.float64), np.full(n, 3.0)])
    out = orc.downfactor(ramp)
    assert out.shape == (2, 5)                          # the odd last sample is dropped
    np.testing.assert_array_equal(out[0], 4 * np.arange(5) + 1)
    np.testing.assert_array_equal(out[1], np.full(5, 6.0))
    x = np.random.default_rng(1).integers(0, 256, (3, 64)).astype(np.uint8)
    assert np.array_equal(orc.downfactor(x).sum(axis=1), x.astype(np.int64).sum(axis=1))
    twice = orc.downfactor(orc.downfactor(x))
    np.testing.assert_array_equal(twice, x.reshape(3, 16, 4).astype(np.int64).sum(axis=2))


def test_factor_one_is_plain_dedispersion():
    b = fbsynth.config1(1)
    segs = orc.dedisperse_binned(b.data[:, :2048], b.freq_mhz, b.tsamp_s, b.dm[:40], max_log2=0)
    assert len(segs) == 1 and segs[0][:3] == (0, 0, 40)
    plain = orc.dedisperse(b.data[:, :2048], orc.delay_table(b.freq_mhz, b.dm[:40], b.tsamp_s))
    np.testing.assert_array_equal(segs[0][3], plain)


def test_impulse_lands_at_binned_index():
    """An impulse at (c0, t0) appears in a factor-2^k run at j = floor(t0 / 2^k) - delay_k,
    with delay_k the rounded delay law at sampling time 2^k t_samp (computed here from the
    delay law in seconds, not from the oracle's table)."""
    freq = fbsynth.channel_freqs(428.0, 0.3125, 64)
    tsamp = 51.2e-6
    dms = fbsynth.dm_trials(0.0, 0.1, 128)
    nsamp = 4096
    for c0, t0 in [(63, 3001), (40, 2222), (0, 1500), (17, 2047)]:
        a = np.zeros((64, nsamp))
        a[c0, t0] = 1.0
        for k, d0, d1, s in orc.dedisperse_binned(a, freq, tsamp, dms, max_log2=4):
            sec = orc.delay_seconds(freq, dms[d0:d1])
            for i in range(d1 - d0):
                x = sec[c0, i] / (tsamp * 2 ** k)
                j = (t0 >> k) - int(math.floor(x + 0.5))
                expect = np.zeros(s.shape[1])
                if 0 <= j < s.shape[1]:
                    expect[j] = 1.0
                np.testing.assert_array_equal(s[i], expect)


def test_binned_lengths_and_work():
    b = fbsynth.config1(1)
    segs = orc.dedisperse_binned(b.data, b.freq_mhz, b.tsamp_s, b.dm, max_log2=4)
    assert [k for k, _, _, _ in segs] == [0, 1, 2, 3, 4]
    assert segs[0][1] == 0 and segs[-1][2] == 128
    for k, d0, d1, s in segs:
        delays = orc.delay_table(b.freq_mhz, b.dm[d0:d1], b.tsamp_s * 2 ** k)
        assert s.shape == (d1 - d0, (b.data.shape[1] >> k) - int(delays.max()))
    plain = 128 * 64 * (b.data.shape[1] - 555)
    assert orc.binned_adds(segs, 64) < plain / 3
