"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: a literal
triple loop, exact rational arithmetic, a formula printed elsewhere in the
paper, closed forms, invariants and Gaussian statistics.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc


# ----------------------------------------------------------------------------- delays

def _exact_delay(f, f_ref, dm, tsamp, k=orc.K_DM):
    """Delta_t of Eq. deltaTEq in exact rational arithmetic from the double-valued inputs."""
    x = (Fraction(k) * Fraction(dm) * (1 / (Fraction(f) ** 2) - 1 / (Fraction(f_ref) ** 2))
         / Fraction(tsamp))
    fl = math.floor(x)
    return fl + (1 if x - fl >= Fraction(1, 2) else 0), x


@pytest.mark.parametrize("nchan,f_top,df,tsamp,step,ndm", [
    (64, 428.0, 0.3125, 51.2e-6, 0.1, 128),       # small FP32 workload
    (48, 428.0, 20.0 / 1024, 51.2e-6, 0.1, 40),   # 1024-ch band, subsampled below
    (32, 180.0, 60.0 / 4096, 81.92e-6, 0.05, 30),
])
def test_delay_table_equals_exact_rational_rounding(nchan, f_top, df, tsamp, step, ndm):
    freq = fbsynth.channel_freqs(f_top, df, nchan)
    if nchan == 48:  # spread over the full 1024-channel band
        freq = fbsynth.channel_freqs(f_top, df, 1024)[:: 1024 // 48][:48]
    dms = fbsynth.dm_trials(0.0, step, ndm)
    if ndm == 40:
        dms = fbsynth.dm_trials(0.0, step, 2048)[::51][:40]
    tab = orc.delay_table(freq, dms, tsamp)
    near_tie = 0
    for c in range(freq.size):
        for d in range(dms.size):
            want, x = _exact_delay(freq[c], freq.max(), dms[d], tsamp)
            frac = x - math.floor(x)
            if abs(frac - Fraction(1, 2)) < Fraction(1, 10 ** 9):
                near_tie += 1
                continue
            assert tab[c, d] == want, (c, d, float(x))
    assert near_tie == 0


def test_delay_worked_values():
    # Bottom channel of the 64-channel band at DM 12.7:
    # 4150 * 12.7 * (1/408.3125^2 - 1/428^2) / 51.2e-6 = 554.98... samples -> 555.
    freq = fbsynth.channel_freqs(428.0, 0.3125, 64)
    tab = orc.delay_table(freq, fbsynth.dm_trials(0.0, 0.1, 128), 51.2e-6)
    assert tab[63, 127] == 555
    assert orc.max_delay(tab) == 555
    assert orc.output_length(16384, tab) == 16384 - 555
    # Top channel is the reference: zero delay for every DM; zero DM gives zero delay.
    assert np.all(tab[0] == 0) and np.all(tab[:, 0] == 0)
    # Lower frequencies are delayed more; larger DMs are delayed more.
    assert np.all(np.diff(tab, axis=0) >= 0) and np.all(np.diff(tab, axis=1) >= 0)


def test_delay_law_constant_against_paper(golden):
    k = orc.K_DM
    assert abs(k - golden["dispersion_constant_exact_s_mhz2"]["value"]) / k < 1e-3
    assert abs(k - 1.0 / golden["dispersion_constant_approx_inverse"]["value"]) / k < 1e-3


def test_diagonal_dm_matches_delay_derivative(golden):
    """At the diagonal DM the smear across the bottom channel is one sample (Ch. 6)."""
    c8300 = golden["diagonal_dm_constant"]["value"]
    for f_top, nchan, bw, tsamp in [(428.0, 1024, 20.0, 51.2e-6), (180.0, 4096, 60.0, 81.92e-6),
                                    (428.0, 64, 20.0, 51.2e-6)]:
        df = bw / nchan
        freq = fbsynth.channel_freqs(f_top, df, nchan)
        f0 = freq[-1]
        dm_diag = tsamp * f0 ** 3 / (c8300 * df)
        # continuous delays (samples) of the two bottom channels from the oracle's law
        x = orc.delay_seconds(freq[-2:], [dm_diag]) / tsamp
        # the oracle's delays are relative to f_ref = max(freq[-2:]) here: x[-1] is the smear
        smear = float(x[-1, 0] - x[-2, 0])
        assert abs(smear - 1.0) < 3.0 * df / f0, (f_top, nchan, smear)


def test_delay_validation():
    f = [428.0, 427.0]
    with pytest.raises(ValueError):
        orc.delay_table(f, [-1.0], 1e-4)
    with pytest.raises(ValueError):
        orc.delay_table([428.0, 0.0], [1.0], 1e-4)
    with pytest.raises(ValueError):
        orc.delay_table(f, [1.0], 0.0)
    with pytest.raises(ValueError):
        orc.delay_table(f, [float("nan")], 1e-4)
    with pytest.raises(ValueError):
        orc.output_length(10, np.array([[0], [10]]))


# ------------------------------------------------------------------------ dedispersion

def _triple_loop(a, delays):
    nchan, nsamp = a.shape
    ndm = delays.shape[1]
    nout = nsamp - int(delays.max())
    out = [[0.0] * nout for _ in range(ndm)]
    for d in range(ndm):
        for t in range(nout):
            s = 0.0
            for c in range(nchan):
                s += float(a[c][t + int(delays[c][d])])
            out[d][t] = s
    return np.array(out)


@pytest.mark.parametrize("seed", range(12))
def test_dedisperse_equals_triple_loop(seed):
    rng = np.random.default_rng(seed)
    nchan = int(rng.integers(1, 9))
    ndm = int(rng.integers(1, 6))
    nsamp = int(rng.integers(8, 65))
    maxd = int(rng.integers(0, nsamp - 1))
    delays = rng.integers(0, maxd + 1, size=(nchan, ndm)).astype(np.int32)
    delays[0, 0] = 0
    delays[-1, -1] = maxd
    a = rng.standard_normal((nchan, nsamp))
    got = orc.dedisperse(a, delays)
    assert got.shape == (ndm, nsamp - maxd)
    np.testing.assert_array_equal(got, _triple_loop(a, delays))


def test_zero_dm_row_is_channel_sum():
    b = fbsynth.config1()
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    nout = orc.output_length(b.nsamp, tab)
    d0 = orc.dedisperse(b.data, tab, rows=[0])[0]
    np.testing.assert_allclose(d0, b.data[:, :nout].astype(np.float64).sum(axis=0), rtol=0, atol=1e-12)


def test_linearity_and_time_shift():
    rng = np.random.default_rng(5)
    freq = fbsynth.channel_freqs(428.0, 0.3125, 16)
    tab = orc.delay_table(freq, fbsynth.dm_trials(0.0, 0.5, 9), 51.2e-6)
    x = rng.integers(-50, 50, size=(16, 400)).astype(np.float64)
    y = rng.integers(-50, 50, size=(16, 400)).astype(np.float64)
    dx, dy = orc.dedisperse(x, tab), orc.dedisperse(y, tab)
    np.testing.assert_array_equal(orc.dedisperse(3 * x - 2 * y, tab), 3 * dx - 2 * dy)
    s = 37
    shifted = orc.dedisperse(x[:, s:], tab)
    np.testing.assert_array_equal(shifted, dx[:, s:])


def test_impulse_response_recovers_delay_column():
    freq = fbsynth.channel_freqs(428.0, 0.3125, 64)
    tab = orc.delay_table(freq, fbsynth.dm_trials(0.0, 0.1, 128), 51.2e-6)
    c0, t0 = 63, 700
    a = np.zeros((64, 2000))
    a[c0, t0] = 1.0
    out = orc.dedisperse(a, tab)
    for d in range(128):
        nz = np.flatnonzero(out[d])
        assert list(nz) == [t0 - tab[c0, d]]
        assert out[d, nz[0]] == 1.0


def test_on_grid_pulse_sums_exactly():
    """A pulse placed on the trial's own delay track adds A * nchan at every pulse sample."""
    freq = fbsynth.channel_freqs(428.0, 0.3125, 64)
    tab = orc.delay_table(freq, fbsynth.dm_trials(0.0, 0.1, 128), 51.2e-6)
    a = np.zeros((64, 2048), dtype=np.float32)
    dstar, t0, w = 50, 900, 8
    for c in range(64):
        a[c, t0 + tab[c, dstar]: t0 + tab[c, dstar] + w] += 0.5
    out = orc.dedisperse(a, tab)
    np.testing.assert_array_equal(out[dstar, t0:t0 + w], 32.0)
    assert out[dstar].sum() == 32.0 * w


def test_pulse_recovery_config1():
    b = fbsynth.config1()
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    out = orc.dedisperse(b.data, tab)
    p = b.pulses[0]
    t0 = int(p.t0)
    box = out[:, t0:t0 + p.width].sum(axis=1)
    assert abs(int(np.argmax(box)) - 50) <= 1


# ------------------------------------------------------------------ stats, candidates

def test_stats_closed_forms():
    s = np.array([[3.5] * 10, [1.0] * 5 + [5.0] * 5, [0.0, 2.0, 4.0, 6.0]  + [3.0] * 6])
    mean, rms = orc.series_stats(s)
    assert mean[0] == 3.5 and rms[0] == 0.0
    assert mean[1] == 3.0 and rms[1] == 2.0
    assert mean[2] == 3.0 and abs(rms[2] - math.sqrt(20.0 / 10.0)) < 1e-15


def test_noise_rms_is_sqrt_nchan():
    b = fbsynth.config1()
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    out = orc.dedisperse(b.data, tab, rows=[0, 64, 127])
    _, rms = orc.series_stats(out)
    assert np.all(np.abs(rms / 8.0 - 1.0) < 0.02)


def test_candidates_strict_and_ordered():
    s = np.array([[0.0, 10.0, 0.0, 10.0], [5.0, 0.0, 9.0, 1.0]])
    mean = np.array([1.0, 2.0])
    rms = np.array([1.0, 1.0])
    c = orc.candidates(s, mean, rms, k_sigma=5.0)
    # row 0: threshold 6 -> t=1,3 ; row 1: threshold 7 -> t=2 (5.0 is below)
    assert list(c["dm_index"]) == [0, 0, 1] and list(c["t"]) == [1, 3, 2]
    np.testing.assert_array_equal(c["snr"], [9.0, 9.0, 7.0])
    exact = orc.candidates(np.array([[6.0]]), np.array([1.0]), np.array([1.0]), 5.0)
    assert exact["t"].size == 0


def test_functional_test_snr_convention(golden):
    """Height 8/sqrt(1024) per channel gives a band-integrated S/N of 8 (Ch. 2 functional test)."""
    g = golden["functional_test_snr"]
    rng = np.random.default_rng(11)
    nchan = g["nchan"]
    freq = fbsynth.channel_freqs(428.0, 20.0 / nchan, nchan)
    dm = fbsynth.dm_trials(20.0, 1.0, 1)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    nsamp = 12000
    a = rng.standard_normal((nchan, nsamp))
    starts = np.arange(200, nsamp - int(tab.max()) - 200, 97)
    for t0 in starts:
        for c in range(nchan):
            a[c, t0 + tab[c, 0]] += g["height"]
    out = orc.dedisperse(a, tab)
    mean, rms = orc.series_stats(out)
    snr = (out[0, starts] - mean[0]) / math.sqrt(nchan)
    assert abs(snr.mean() - g["snr"]) < 4.0 / math.sqrt(starts.size)


def test_false_alarm_count_is_gaussian_tail():
    """Pure noise: counts above k sigma follow the Gaussian tail (Ch. 1, single-pulse S/N)."""
    rng = np.random.default_rng(3)
    nchan, nsamp = 16, 200_000
    freq = fbsynth.channel_freqs(428.0, 0.3125, nchan)
    tab = orc.delay_table(freq, fbsynth.dm_trials(0.0, 10.0, 3), 51.2e-6)
    a = rng.standard_normal((nchan, nsamp))
    out = orc.dedisperse(a, tab)
    mean, rms = orc.series_stats(out)
    k = 3.0
    c = orc.candidates(out, mean, rms, k)
    expected = out.size * 0.5 * math.erfc(k / math.sqrt(2.0))
    assert abs(c["t"].size - expected) < 6.0 * math.sqrt(expected)


def test_op_count_convention(golden):
    g = golden["realtime_op_rate"]
    # per second of data: samples_per_s outputs per DM series (4 s of data to stay integral)
    ops = g["beams"] * orc.algorithmic_adds(g["ndm"], g["nchan"], int(4 * g["samples_per_s"])) / 4
    assert round(ops / 1e9) == round(g["ops_per_s_approx"] / 1e9)


# ------------------------------------------------------------------------- streaming

def test_stream_expected_covers_one_shot():
    rng = np.random.default_rng(9)
    freq = fbsynth.channel_freqs(428.0, 0.3125, 8)
    tab = orc.delay_table(freq, fbsynth.dm_trials(0.0, 2.0, 5), 51.2e-6)
    m = orc.max_delay(tab)
    blocks = [rng.standard_normal((8, n)) for n in (m // 2, 40, 40, 7, 100)]
    res = orc.stream_expected(blocks, tab)
    full = orc.dedisperse(np.concatenate(blocks, axis=1), tab)
    assert res[0][1] == 0  # still filling after fewer than maxshift samples
    prev = 0
    for t0, t1, s in res:
        assert t0 == prev and t1 >= t0
        np.testing.assert_array_equal(s, full[:, t0:t1])
        prev = t1
    assert prev == full.shape[1]
