"""Seeded synthetic filterbanks in the style of the paper's simulations.

Conventions (Magro 2013):
* Noise is i.i.d. N(0, 1) per channel sample; a top-hat pulse of height
  SNR / sqrt(nchan) per channel integrates to per-sample S/N = SNR over the
  band (functional test of Sec. 2.2, height 8/sqrt(1024) for S/N 8).
* BEST-II-like bands: 408-428 MHz, 51.2 us sampling (Ch. 3 and 4); a
  low-frequency 120-180 MHz band at 81.92 us for the 4096-channel beams.
* Power stored as u8 (Sec. 3.7 persister): code = clip(rint(128 + 16 x), 0, 255).

The pulse is placed by a sky model, not by the dedispersion method: a boxcar of
W samples arriving at the top of the band at continuous time t0 reaches channel
c at t0 + k * DM * (f_c^-2 - f_top^-2) / tsamp (cold-plasma dispersion,
Sec. 1.2) and each sample receives the fraction of the boxcar that overlaps it.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Dispersion constant used by the sky model (s MHz^2 pc^-1 cm^3).
SKY_K_DM = 4.15e3
U8_OFFSET = 128.0
U8_SCALE = 16.0


@dataclasses.dataclass
class Pulse:
    dm: float        # true DM (may lie between trials)
    t0: float        # arrival time at the top of the band, in samples
    width: int       # boxcar width in samples
    amp: float       # height per channel sample, in input units


@dataclasses.dataclass
class Beam:
    name: str
    freq_mhz: np.ndarray        # [nchan] float64, descending
    tsamp_s: float
    dm: np.ndarray              # [ndm] float64
    data: np.ndarray            # [nchan][nsamp], float32 / float16 / uint8
    pulses: List[Pulse]
    k_sigma: float = 6.0

    @property
    def nchan(self) -> int:
        return int(self.data.shape[0])

    @property
    def nsamp(self) -> int:
        return int(self.data.shape[1])

    @property
    def ndm(self) -> int:
        return int(self.dm.shape[0])


def channel_freqs(f_top: float, df: float, nchan: int) -> np.ndarray:
    """Channel c at f_top - c * df (channel 0 is the top of the band)."""
    return f_top - np.arange(nchan, dtype=np.float64) * df


def dm_trials(dm0: float, step: float, n: int) -> np.ndarray:
    """DM(d) = dm0 + d * step, each trial computed directly (no running sum)."""
    return dm0 + np.arange(n, dtype=np.float64) * step


def sky_delay_s(freq_mhz, f_top: float, dm: float, k_dm: float = SKY_K_DM) -> np.ndarray:
    """Continuous arrival delay of a dispersed signal at each frequency, relative to f_top."""
    f = np.asarray(freq_mhz, dtype=np.float64)
    return k_dm * dm * (1.0 / (f * f) - 1.0 / (f_top * f_top))


def noise(rng: np.random.Generator, nchan: int, nsamp: int, dtype=np.float32) -> np.ndarray:
    """i.i.d. N(0, 1) samples, [nchan][nsamp]."""
    return rng.standard_normal((nchan, nsamp), dtype=np.float32).astype(dtype, copy=False)


def inject_boxcar(data: np.ndarray, freq_mhz, tsamp_s: float, p: Pulse) -> None:
    """Add a dispersed top-hat to data in place (sky model with fractional sample overlap)."""
    f = np.asarray(freq_mhz, dtype=np.float64)
    f_top = float(f.max())
    start = p.t0 + sky_delay_s(f, f_top, p.dm) / tsamp_s
    nsamp = data.shape[1]
    for c in range(f.size):
        a = start[c]
        b = a + p.width
        j0 = max(int(math.floor(a)), 0)
        j1 = min(int(math.ceil(b)), nsamp)
        if j1 <= j0:
            continue
        j = np.arange(j0, j1, dtype=np.float64)
        overlap = np.clip(np.minimum(j + 1.0, b) - np.maximum(j, a), 0.0, 1.0)
        data[c, j0:j1] += (p.amp * overlap).astype(data.dtype)


def to_u8(x: np.ndarray) -> np.ndarray:
    """Power stored as unsigned 8-bit codes: clip(rint(128 + 16 x), 0, 255), round half to even."""
    return np.clip(np.rint(U8_OFFSET + U8_SCALE * np.asarray(x, np.float32)), 0, 255).astype(np.uint8)


def to_f16(x: np.ndarray) -> np.ndarray:
    """Power stored as IEEE half precision (round to nearest even)."""
    return np.asarray(x, np.float32).astype(np.float16)


def config1(seed: int = 1) -> Beam:
    """Small FP32 case: 64 ch over 408-428 MHz, 51.2 us, 16384 samples, one pulse at DM 5."""
    rng = np.random.default_rng(seed)
    freq = channel_freqs(428.0, 0.3125, 64)
    tsamp = 51.2e-6
    data = noise(rng, 64, 16384)
    pulses = [Pulse(dm=5.0, t0=8192.0, width=8, amp=0.5)]
    for p in pulses:
        inject_boxcar(data, freq, tsamp, p)
    return Beam("config1: 64ch 16384 samples 128 DMs f32", freq, tsamp, dm_trials(0.0, 0.1, 128),
                data, pulses, k_sigma=6.0)


def config2(seed: int = 2, nsamp: int = 1 << 20, nchan: int = 1024, ndm: int = 2048,
            npulse: int = 20) -> Beam:
    """Full-size FP32 case: 1024 ch over 408-428 MHz, 2^20 samples, 2048 DMs, 20 pulses.

    Smaller nsamp/nchan/ndm give the same recipe at test sizes.
    """
    rng = np.random.default_rng(seed)
    freq = channel_freqs(428.0, 20.0 / nchan, nchan)
    tsamp = 51.2e-6
    dms = dm_trials(0.0, 0.1, ndm)
    pulse_rng = np.random.default_rng([seed, 7])
    data = noise(rng, nchan, nsamp)
    span = float(sky_delay_s(freq[-1:], 428.0, float(dms[-1]))[0] / tsamp) + 2.0
    pulses = []
    for _ in range(npulse):
        dm = float(pulse_rng.uniform(10.0, min(200.0, float(dms[-1]))))
        w = int(pulse_rng.integers(1, 65))
        snr = float(pulse_rng.uniform(6.0, 20.0))
        hi = max(int(nsamp - span - w), 1)
        t0 = float(pulse_rng.integers(0, hi))
        pulses.append(Pulse(dm=dm, t0=t0, width=w, amp=snr / math.sqrt(nchan)))
    for p in pulses:
        inject_boxcar(data, freq, tsamp, p)
    return Beam(f"config2: {nchan}ch {nsamp} samples {ndm} DMs f32", freq, tsamp, dms, data,
                pulses, k_sigma=6.0)


def config3(seed: int = 1):
    """Config 1's input stored as u8 and as f16 (returns the FP32 beam plus the two encodings)."""
    b = config1(seed)
    return b, to_u8(b.data), to_f16(b.data)


def make_beam(name: str, nchan: int, f_top: float, bw: float, tsamp: float, dm0: float,
              step: float, ndm: int, nsamp: int, rng: np.random.Generator,
              npulse: int, storage: str = "u8", snr_range=(6.0, 20.0)) -> Beam:
    """One beam of N(0, 1) noise plus dispersed pulses, stored as u8 (or f32/f16)."""
    freq = channel_freqs(f_top, bw / nchan, nchan)
    dms = dm_trials(dm0, step, ndm)
    x = noise(rng, nchan, nsamp)
    span = float(sky_delay_s(freq[-1:], f_top, float(dms[-1]))[0] / tsamp) + 2.0
    pulses = []
    for _ in range(npulse):
        dm = float(rng.uniform(float(dms[0]), float(dms[-1])))
        w = int(rng.integers(1, 65))
        snr = float(rng.uniform(*snr_range))
        hi = max(int(nsamp - span - w), 1)
        pulses.append(Pulse(dm=dm, t0=float(rng.integers(0, hi)), width=w,
                            amp=snr / math.sqrt(nchan)))
    for p in pulses:
        inject_boxcar(x, freq, tsamp, p)
    if storage == "u8":
        data = to_u8(x)
        for p in pulses:
            p.amp *= U8_SCALE
    elif storage == "f16":
        data = to_f16(x)
    else:
        data = x
    return Beam(name, freq, tsamp, dms, data, pulses)


def _band(nchan: int):
    if nchan == 4096:
        return 180.0, 60.0, 81.92e-6
    return 428.0, 20.0, 51.2e-6


def config4_specs(seed: int = 4, scale: float = 1.0):
    """Parameters of the 16 uneven u8 beams of the batched workload (no data drawn yet).

    nchan cycles over {256, 512, 1024, 4096}; ndm ~ U{500..4096}; DM step in
    {0.05, 0.1, 0.2}; nsamp in {2^16..2^19}; redrawn until the sky-model delay
    across the band at the largest DM is at most nsamp/2. ``scale`` < 1 shrinks
    ndm and nsamp for test-sized runs.
    """
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(16):
        nchan = (256, 512, 1024, 4096)[i % 4]
        f_top, bw, tsamp = _band(nchan)
        f_bot = f_top - bw * (nchan - 1) / nchan
        while True:
            ndm = int(rng.integers(500, 4097))
            step = float(rng.choice([0.05, 0.1, 0.2]))
            nsamp = int(1 << int(rng.integers(16, 20)))
            if scale != 1.0:
                ndm = max(8, int(ndm * scale))
                nsamp = max(1024, int(nsamp * scale))
            span = SKY_K_DM * step * (ndm - 1) * (f_bot ** -2 - f_top ** -2) / tsamp
            if span + 1.0 <= nsamp / 2:
                break
        specs.append(dict(name=f"beam{i:02d}", nchan=nchan, f_top=f_top, bw=bw, tsamp=tsamp,
                          dm0=0.0, step=step, ndm=ndm, nsamp=nsamp,
                          npulse=int(rng.integers(1, 5)), seed=[seed, i]))
    return specs


def config5_specs(seed: int = 5, n1024: int = 48, n4096: int = 16, dm_step_4096: float = 0.05):
    """Beams of the streaming workload: 1 s blocks, u8, 1024-ch and 4096-ch beams.

    Returns a list of dicts with the band, DM list parameters, block length
    floor(1 s / tsamp) and a per-beam arrival phase drawn from U[0, 1 s).
    """
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n1024 + n4096):
        nchan = 1024 if i < n1024 else 4096
        f_top, bw, tsamp = _band(nchan)
        ndm = 2048 if nchan == 1024 else 4096
        step = 0.1 if nchan == 1024 else dm_step_4096
        specs.append(dict(name=f"beam{i:02d}", nchan=nchan, f_top=f_top, bw=bw, tsamp=tsamp,
                          dm0=0.0, step=step, ndm=ndm, block=int(math.floor(1.0 / tsamp)),
                          phase_s=float(rng.uniform(0.0, 1.0)), seed=[seed, i]))
    return specs


def arrival_times(n_blocks: int, block_s: float, phase_s: float, rng: np.random.Generator,
                  jitter_mean_s: float = 0.1) -> np.ndarray:
    """arrival_k = k * T + phase + J_k, J_k ~ Exp(mean) truncated below T (Poisson jitter)."""
    j = rng.exponential(jitter_mean_s, size=n_blocks)
    j = np.minimum(j, np.nextafter(block_s, 0.0))
    return np.arange(n_blocks) * block_s + phase_s + j
