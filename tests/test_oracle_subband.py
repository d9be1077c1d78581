"""Pins of the oracle's subband dedispersion (Sec. "Subband Dedispersion").

Fixed outside the oracle's code: with one channel per subband and one trial per group it is
plain dedispersion; an impulse lands where the two rounded delays of the delay law (the
channel's within its subband at the nominal DM, the subband's at the trial DM) put it; its
positions differ from brute force by no more than the rounding of those delays plus the
nominal-DM offset.
"""
import math

import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc


def test_one_channel_subbands_single_trials_are_plain():
    b = fbsynth.config1()
    x = b.data[:, :4096]
    got = orc.subband_dedisperse(x, b.freq_mhz, b.tsamp_s, b.dm[:20], 1, 1)
    want = orc.dedisperse(x, orc.delay_table(b.freq_mhz, b.dm[:20], b.tsamp_s))
    for d0, d1, s in got:
        assert d1 == d0 + 1
        np.testing.assert_array_equal(s[0][:want.shape[1]], want[d0])


def _rnd(x):
    return int(math.floor(x + 0.5))


@pytest.mark.parametrize("nsub_ch,ngrp", [(8, 4), (16, 8), (64, 16), (5, 3)])
def test_impulse_position_from_the_delay_law(nsub_ch, ngrp):
    freq = fbsynth.channel_freqs(428.0, 0.3125, 64)
    tsamp = 51.2e-6
    dms = fbsynth.dm_trials(0.0, 0.1, 48)
    k = orc.K_DM
    for c0, t0 in [(63, 3000), (10, 2500), (37, 2900)]:
        a = np.zeros((64, 4096))
        a[c0, t0] = 1.0
        out = orc.subband_dedisperse(a, freq, tsamp, dms, nsub_ch, ngrp)
        s = c0 // nsub_ch
        f_s = max(freq[s * nsub_ch:(s + 1) * nsub_ch])
        for d0, d1, ser in out:
            nom = dms[d0 + (d1 - d0 - 1) // 2]
            inner = _rnd(k * nom * (1 / freq[c0] ** 2 - 1 / f_s ** 2) / tsamp)
            for i in range(d1 - d0):
                outer = _rnd(k * dms[d0 + i] * (1 / f_s ** 2 - 1 / freq[0] ** 2) / tsamp)
                j = t0 - inner - outer
                expect = np.zeros(ser.shape[1])
                if 0 <= j < ser.shape[1]:
                    expect[j] = 1.0
                np.testing.assert_array_equal(ser[i], expect)
                # against brute force: off by the two roundings plus the nominal-DM offset
                exact = k * dms[d0 + i] * (1 / freq[c0] ** 2 - 1 / freq[0] ** 2) / tsamp
                off = k * abs(dms[d0 + i] - nom) * (1 / freq[c0] ** 2 - 1 / f_s ** 2) / tsamp
                assert abs((t0 - j) - exact) <= 1.0 + off + 1e-9
