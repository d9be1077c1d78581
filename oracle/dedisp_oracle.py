"""Plain FP64 CPU oracle for brute-force incoherent dedispersion.

TEST INFRASTRUCTURE ONLY. This module exists to check the HIP library. Only the
test suite, the package's smoke check and the benchmark's CPU-baseline leg may
import it; the product path never calls it and shares no code with it.

What it computes, in the paper's notation (Magro 2013, Ch. 2 and 3):

* Dispersion delay law, Eq. dispRelationshipEquation (Sec. "Dispersion"):
  dt = k_DM * DM * (f_1^-2 - f_2^-2), f in MHz. The constant is the paper's
  approximate dispersion constant, 4.15e3 s MHz^2 pc^-1 cm^3 (the exact value
  quoted beside it is 4.148808e3; the approximation is the one the method uses).
* Discretised delay, Eq. deltaTEq (Sec. "Direct Dedispersion"):
  Delta_t(d, c) = round(DM(d) * k_DM * (f_c^-2 - f_ref^-2) / t_samp), f_ref the
  top of the band. "round" is read as round-half-away-from-zero in IEEE double.
* Direct dedispersion, Eq. bruteEquation: D[d, t] = sum_c A[c, t + Delta_t(d, c)],
  the sum taken in FP64 over every channel, for t in [0, nsamp - maxshift).
  maxshift = max Delta_t (Sec. 3.4 "Dedispersion", buffer sizing).
* Per-series mean and standard deviation (population, ddof 0), the
  normalisation of Sec. 3.5 "Signal Post-processing".
* n-sigma thresholding into (time, DM, intensity) detections, Sec. 3.6
  "Detection and Candidate Selection": every (d, t) with D > mean_d + k*rms_d.
* Detrending and normalisation, Sec. 3.5 "Signal Post-processing": subtract from each
  dedispersed series its least-squares line (linear regression over the sample index),
  then optionally divide by the residual's population standard deviation.
* Boxcar smoothing by successively adding adjacent samples (single-pulse detection,
  Sec. 2; boxcar templates downfactor the series, Sec. 6): level k holds the sums of
  2^k consecutive samples over sqrt(2^k), non-overlapping.
* Boxcar template matching (Sec. 6 "Transient Surveys": boxcars of varying width
  convolved with each dedispersed series, then thresholded; Sec. 2 Eq. pulseSNREquation:
  S/N grows as the square root of the samples a matched boxcar adds): for widths
  w = 2^j, the sum of w samples at every start offset, its S/N about the series mean in
  units of rms sqrt(w), and a detection wherever the best width's S/N exceeds k.
* Time binning (Sec. 2 "Direct Dedispersion", Sec. "Computing Larger DMs"): above the
  diagonal DM (where adjacent channels' delays differ by one sample) the input is
  downfactored by 2 by summing adjacent samples, again at twice the diagonal, and so on:
  a DM trial in (2^(k-1) DM_diag, 2^k DM_diag] is dedispersed at factor 2^k, i.e. on the
  input downfactored k times with sampling time 2^k t_samp.
* Subband dedispersion (Sec. "Subband Dedispersion"): nominal DMs, one per group of
  consecutive trials; each subband of channels is dedispersed at the nominal DMs with
  delays relative to the subband's top frequency; each trial then dedisperses the reduced
  filterbank of its group's subband series with the delays of the subbands' top
  frequencies. An approximation: the paper defers its error bound to another work, so
  beyond the pins below its error is "parity unpinned".
* RFI mitigation before dedispersion (Sec. 3 "Bandpass Correction", "Channel
  Thresholding", "Spectrum Thresholding"): the time-averaged bandpass, its least-squares
  polynomial fit over the channel index and the fit's RMSE; windows of W samples whose
  mean deviates from the channel's fitted value by more than a threshold are flagged, and
  each flagged window and its neighbours take the fitted value; then every spectrum whose
  mean over channels deviates from the fit's mean by more than a threshold takes the
  fitted bandpass; last the fitted bandpass is subtracted from every spectrum. For 8-bit
  codes the replacement is the nearest code of the fit and there is no subtraction.

Pins (tests/test_oracle_pins.py): a literal triple loop on tiny inputs; exact
rational delays (fractions.Fraction) away from ties; the paper's diagonal-DM
formula (Sec. 6.3, 8300 = 2 * 4150) as the derivative of the delay law; the
zero-DM row equal to the plain channel sum; linearity; impulse response;
time-shift equivariance; closed-form statistics; the E1 S/N convention (height
8/sqrt(1024) gives S/N 8); Gaussian-tail false-alarm counts; the paper's
op-count convention (138e9 ops/s). Detrending (tests/test_oracle_detrend.py): a pure
line vanishes; the residual satisfies the normal equations; numpy.polyfit's residual;
invariance under adding a line; unit population RMS after normalisation. No function
here is "parity unpinned". Boxcar levels (same file): a constant gives c sqrt(2^k); each
level is the pairwise sum of the one below over sqrt(2); sums are conserved; a top-hat
of width 2^m aligned to 2^m peaks at h sqrt(2^m) on level m.
Time binning (tests/test_oracle_binning.py): the diagonal DM against the paper's closed
form dt f0^3 / (8300 df) (Sec. 6) and against a one-sample smear of the bottom channel
pair; the number of binning stages against the paper's ceil(log2(DM_max / DM_diag)) + 1;
a ramp's downfactored closed form and conserved sums; an impulse lands at the binned
index floor(t0 / 2^k) - delay; factor 1 reduces to plain dedispersion.
Subband dedispersion (tests/test_oracle_subband.py): one-channel subbands with one trial per
group reduce to plain dedispersion exactly; an impulse lands at t0 minus the sum of its
in-subband delay at the nominal DM and its subband's delay at the trial DM, both from the
delay law in seconds; the residual against brute force stays within the rounding of those
two delays.
RFI mitigation (tests/test_oracle_rfi.py): a polynomial bandpass is fitted exactly with
zero RMSE; a literal pure-Python loop over windows and spectra on tiny inputs; clean data
under a high threshold is unchanged; a narrowband burst, a dropout and a broadband spike
are replaced by the fitted bandpass and nothing else changes. The 8-bit stage: literal
integer loops; nearest-code rounding; equality with the float stage where the fit is
integral; and the constant-offset identity (subtracting a per-channel constant lowers every
dedispersed sample by its sum, leaving RMS and candidates) that lets it skip the correction.
"""
from __future__ import annotations

import math

import numpy as np

# Approximate dispersion constant of Eq. dispRelationshipEquation, in
# s * MHz^2 * pc^-1 * cm^3 (the paper writes it as 1/2.41e-4 in ms units).
K_DM = 4.15e3


def reference_frequency(freq_mhz) -> float:
    """f_ref of Eq. deltaTEq: the top of the band, i.e. the largest channel frequency."""
    f = np.asarray(freq_mhz, dtype=np.float64)
    return float(f.max())


def delay_seconds(freq_mhz, dm, k_dm: float = K_DM):
    """Continuous delay of every channel relative to f_ref, Eq. dispRelationshipEquation.

    Returns a float64 array [nchan][ndm] in seconds; no rounding.
    """
    f = np.asarray(freq_mhz, dtype=np.float64)
    dms = np.asarray(dm, dtype=np.float64)
    f_ref = reference_frequency(f)
    inv_ref = 1.0 / (f_ref * f_ref)
    inv_c = 1.0 / (f * f)
    return (k_dm * dms[None, :]) * (inv_c - inv_ref)[:, None]


def delay_table(freq_mhz, dm, tsamp_s: float, k_dm: float = K_DM) -> np.ndarray:
    """Integer delays Delta_t(d, c) of Eq. deltaTEq, laid out [nchan][ndm] (DM fastest).

    Every entry is evaluated in IEEE double in the fixed order
    x = ((k_dm * DM) * (1/(f*f) - 1/(f_ref*f_ref))) / tsamp, then rounded half
    away from zero (x >= 0 here). The layout is the channel/DM order the paper
    stores its shift table in (Sec. 3.4).
    """
    f = np.asarray(freq_mhz, dtype=np.float64)
    dms = np.asarray(dm, dtype=np.float64)
    if f.ndim != 1 or dms.ndim != 1 or f.size < 1 or dms.size < 1:
        raise ValueError("need non-empty 1-D frequency and DM lists")
    if not np.all(np.isfinite(f)) or np.any(f <= 0):
        raise ValueError("frequencies must be finite and positive")
    if not np.all(np.isfinite(dms)) or np.any(dms < 0):
        raise ValueError("DMs must be finite and non-negative")
    if not (tsamp_s > 0 and math.isfinite(tsamp_s)):
        raise ValueError("tsamp must be finite and positive")
    f_ref = reference_frequency(f)
    inv_ref = 1.0 / (f_ref * f_ref)
    out = np.empty((f.size, dms.size), dtype=np.int64)
    for c in range(f.size):
        diff = 1.0 / (f[c] * f[c]) - inv_ref
        x = ((k_dm * dms) * diff) / tsamp_s
        fl = np.floor(x)
        out[c, :] = fl.astype(np.int64) + ((x - fl) >= 0.5)
    if out.max() > np.iinfo(np.int32).max:
        raise ValueError("delay exceeds int32")
    return out.astype(np.int32)


def max_delay(delays: np.ndarray) -> int:
    """maxshift of Sec. 3.4: the largest delay in the table."""
    return int(np.asarray(delays).max())


def output_length(nsamp: int, delays: np.ndarray) -> int:
    """Number of output samples per DM series: nsamp - maxshift (must be positive)."""
    nout = int(nsamp) - max_delay(delays)
    if nout <= 0:
        raise ValueError("nsamp must exceed the maximum delay")
    return nout


def dedisperse_row(data: np.ndarray, delay_col: np.ndarray, nout: int) -> np.ndarray:
    """One dedispersed series D[d, :] of Eq. bruteEquation, summed in FP64.

    data is [nchan][nsamp] in any real dtype (u8 codes are summed as raw codes);
    delay_col holds Delta_t(d, c) for every channel c of this DM trial.
    """
    acc = np.zeros(nout, dtype=np.float64)
    for c in range(data.shape[0]):
        s = int(delay_col[c])
        np.add(acc, data[c, s:s + nout], out=acc)
    return acc


def dedisperse(data: np.ndarray, delays: np.ndarray, rows=None) -> np.ndarray:
    """Every (or the selected) DM series of Eq. bruteEquation, as float64 [len(rows)][nout]."""
    data = np.asarray(data)
    delays = np.asarray(delays)
    if data.ndim != 2 or delays.ndim != 2 or delays.shape[0] != data.shape[0]:
        raise ValueError("data must be [nchan][nsamp] and delays [nchan][ndm]")
    nout = output_length(data.shape[1], delays)
    sel = range(delays.shape[1]) if rows is None else list(rows)
    out = np.empty((len(sel), nout), dtype=np.float64)
    for i, d in enumerate(sel):
        out[i] = dedisperse_row(data, delays[:, d], nout)
    return out


def series_stats(series: np.ndarray):
    """Per-series mean and population standard deviation (Sec. 3.5 normalisation)."""
    s = np.asarray(series, dtype=np.float64)
    mean = s.mean(axis=1)
    rms = np.sqrt(np.mean((s - mean[:, None]) ** 2, axis=1))
    return mean, rms


def detrend(series: np.ndarray, normalise: bool = False):
    """Detrending and normalisation of Sec. 3.5 "Signal Post-processing", in FP64.

    Each row x_t (t = 0 .. n-1) loses its least-squares line a + b*t: with
    tbar = (n-1)/2 and S_tt = sum (t - tbar)^2 = n(n^2-1)/12, b = sum (t - tbar) x_t / S_tt
    and a = mean(x) - b*tbar (a single sample keeps b = 0). With normalise, the residual
    is divided by its population standard deviation, unless that is 0. Returns (series,
    rms of the residual per row).
    """
    x = np.atleast_2d(np.asarray(series, dtype=np.float64))
    n = x.shape[1]
    t = np.arange(n, dtype=np.float64)
    tbar = (n - 1) / 2.0
    if n > 1:
        s_tt = n * (n * n - 1) / 12.0
        b = ((t - tbar)[None, :] * x).sum(axis=1) / s_tt
    else:
        b = np.zeros(x.shape[0])
    a = x.mean(axis=1) - b * tbar
    y = x - (a[:, None] + b[:, None] * t[None, :])
    rms = np.sqrt(np.mean(y * y, axis=1))
    if normalise:
        y = np.where(rms[:, None] > 0, y / np.where(rms > 0, rms, 1.0)[:, None], y)
    return y, rms


def boxcar_levels(series: np.ndarray, levels: int):
    """Smoothing by successively adding adjacent samples (Sec. 2 single-pulse detection;
    the boxcar templates that downfactor a series, Sec. 6): level k (k = 0 .. levels)
    holds s_k[j] = sum_{i < 2^k} x[j 2^k + i] / sqrt(2^k) for j < floor(n / 2^k), in FP64,
    so a normalised series keeps unit variance on every level. Returns a list of arrays
    [nrows][floor(n / 2^k)].
    """
    x = np.atleast_2d(np.asarray(series, dtype=np.float64))
    out = []
    for k in range(levels + 1):
        w = 1 << k
        m = x.shape[1] // w
        out.append(x[:, : m * w].reshape(x.shape[0], m, w).sum(axis=2) / math.sqrt(w))
    return out


def boxcar_snr(series: np.ndarray, mean: np.ndarray, rms: np.ndarray, max_log2: int):
    """S/N of every boxcar (Sec. 6 template matching, at every start offset): for width
    w = 2^j (j = 0 .. max_log2), B_w[d, t] = sum_{i < w} x[d, t + i] for t + w <= n, and
    S/N_w = (B_w - w mean_d) / (rms_d sqrt(w)), in FP64. Returns a list over j of arrays
    [nrows][n - w + 1] (rows with rms <= 0 hold -inf: no detection is defined there).
    """
    x = np.atleast_2d(np.asarray(series, dtype=np.float64))
    m = np.asarray(mean, np.float64)[:, None]
    r = np.asarray(rms, np.float64)[:, None]
    out = []
    for j in range(max_log2 + 1):
        w = 1 << j
        if x.shape[1] < w:
            out.append(np.full((x.shape[0], 0), -np.inf))
            continue
        b = np.lib.stride_tricks.sliding_window_view(x, w, axis=1).sum(axis=2)
        with np.errstate(divide="ignore", invalid="ignore"):
            snr = np.where(r > 0, (b - w * m) / (r * math.sqrt(w)), -np.inf)
        out.append(snr)
    return out


def boxcar_search(series: np.ndarray, mean: np.ndarray, rms: np.ndarray, max_log2: int, k_sigma: float):
    """Boxcar template matching and thresholding (Sec. 6; Sec. 3.6 n-sigma detections):
    at each start t of row d, the width with the largest S/N among those defined there
    (t + w <= n; the smallest such width on ties); a detection when that S/N exceeds
    k_sigma strictly. Ascending (d, t). Returns a dict of arrays: row, t, width, value
    (the boxcar sum B_w) and snr."""
    x = np.atleast_2d(np.asarray(series, dtype=np.float64))
    n = x.shape[1]
    snrs = boxcar_snr(x, mean, rms, max_log2)
    best = np.full(x.shape, -np.inf)
    bestj = np.zeros(x.shape, np.int64)
    for j, s in enumerate(snrs):
        better = s > best[:, : s.shape[1]]  # strictly larger: a wider width must beat a narrower one
        best[:, : s.shape[1]] = np.where(better, s, best[:, : s.shape[1]])
        bestj[:, : s.shape[1]] = np.where(better, j, bestj[:, : s.shape[1]])
    d, t = np.nonzero(best > k_sigma)
    width = (1 << bestj[d, t]).astype(np.int64)
    value = np.array([x[di, ti:ti + wi].sum() for di, ti, wi in zip(d, t, width)], dtype=np.float64)
    return {"row": d.astype(np.int64), "t": t.astype(np.int64), "width": width, "value": value,
            "snr": best[d, t] if d.size else np.zeros(0)}


def boxcar_margin(series: np.ndarray, mean: np.ndarray, rms: np.ndarray, max_log2: int, k_sigma: float):
    """How far the boxcar search's decisions are from flipping: the smallest, over every
    (d, t), of |best S/N - k|, and, where a detection is made, the gap between the best and
    the second-best width's S/N (the width a detection reports). A plain FP32 evaluation
    agrees with this oracle wherever the margin exceeds its rounding."""
    snrs = boxcar_snr(series, mean, rms, max_log2)
    x = np.atleast_2d(np.asarray(series))
    first = np.full(x.shape, -np.inf)
    second = np.full(x.shape, -np.inf)
    for s in snrs:
        f, sc = first[:, : s.shape[1]], second[:, : s.shape[1]]
        second[:, : s.shape[1]] = np.maximum(sc, np.minimum(f, s))
        first[:, : s.shape[1]] = np.maximum(f, s)
    ok = np.isfinite(first)
    if not np.any(ok):
        return float("inf")
    m = float(np.min(np.abs(first[ok] - k_sigma)))
    det = ok & (first > k_sigma) & np.isfinite(second)
    if np.any(det):
        m = min(m, float(np.min(first[det] - second[det])))
    return m


def candidates(series: np.ndarray, mean: np.ndarray, rms: np.ndarray, k_sigma: float,
               row_ids=None):
    """n-sigma detections of Sec. 3.6 in ascending (d, t) order.

    Returns a dict of arrays: dm_index, t, value, snr, where value > mean + k*rms
    strictly and snr = (value - mean) / rms.
    """
    s = np.asarray(series, dtype=np.float64)
    thr = np.asarray(mean, np.float64) + k_sigma * np.asarray(rms, np.float64)
    r, t = np.nonzero(s > thr[:, None])
    ids = np.arange(s.shape[0]) if row_ids is None else np.asarray(row_ids)
    value = s[r, t]
    snr = (value - mean[r]) / rms[r]
    return {"dm_index": ids[r].astype(np.int64), "t": t.astype(np.int64),
            "value": value, "snr": snr}


def threshold_margin(series: np.ndarray, mean: np.ndarray, rms: np.ndarray, k_sigma: float):
    """min over (d, t) of |D - (mean + k*rms)| / rms: how far every value sits from its threshold.

    Rows with rms = 0 (constant series) have no value above their threshold and are skipped."""
    s = np.asarray(series, dtype=np.float64)
    thr = mean + k_sigma * rms
    keep = np.asarray(rms) > 0
    if not np.any(keep):
        return float("inf")
    return float(np.min(np.abs(s[keep] - thr[keep, None]) / rms[keep, None]))


def stream_expected(blocks, delays: np.ndarray):
    """What a stream of consecutive blocks must return, from the one-shot definition.

    The stream's input is the concatenation of the blocks (Sec. 3.4: the last
    maxshift spectra of one buffer are carried into the next). After block j
    (j = 0, 1, ...) the outputs that become computable are the global output
    times [t0, t1) with t1 = (total samples received) - maxshift and t0 the
    previous t1 (or 0); an empty range means the stream is still filling.
    Returns a list of (t0, t1, series[ndm][t1-t0] float64) per block.
    """
    data = np.concatenate([np.asarray(b) for b in blocks], axis=1)
    m = max_delay(delays)
    full = dedisperse(data, delays)
    res = []
    total = 0
    prev = 0
    for b in blocks:
        total += np.asarray(b).shape[1]
        t1 = max(0, total - m)
        t0 = prev
        res.append((t0, t1, full[:, t0:t1]))
        prev = t1
    return res


def algorithmic_adds(ndm: int, nchan: int, nout: int) -> int:
    """The paper's op convention: one channel-sample add per DM trial (Sec. 3.9, GPU versus FPGA rates)."""
    return int(ndm) * int(nchan) * int(nout)


def diagonal_dm(freq_mhz, tsamp_s: float, k_dm: float = K_DM) -> float:
    """The diagonal DM (Sec. 2 "Direct Dedispersion"): the DM at which the dispersion
    curve crosses one time sample per channel step. With the channels in frequency order,
    the delay difference between neighbours a < b is k_DM DM (a^-2 - b^-2) / t_samp
    samples, largest for the bottom pair of a uniform band; DM_diag is one over the largest
    per-DM difference. A single channel has no diagonal (infinity). Sec. 6 prints the
    derivative form of the same limit, dt f0^3 / (8300 df)."""
    f = np.sort(np.asarray(freq_mhz, dtype=np.float64))
    if f.size < 2:
        return math.inf
    worst = 0.0
    for a, b in zip(f[:-1], f[1:]):
        per_dm = (k_dm * (1.0 / (a * a) - 1.0 / (b * b))) / tsamp_s
        worst = max(worst, per_dm)
    return math.inf if worst <= 0.0 else 1.0 / worst


def binning_factors(freq_mhz, tsamp_s: float, dm, max_log2: int, k_dm: float = K_DM) -> np.ndarray:
    """log2 of each DM trial's time-binning factor (Sec. 2 time binning): 0 up to the
    diagonal DM, k for DM in (2^(k-1) DM_diag, 2^k DM_diag], capped at max_log2."""
    dd = diagonal_dm(freq_mhz, tsamp_s, k_dm)
    out = np.zeros(len(dm), dtype=np.int32)
    for i, v in enumerate(np.asarray(dm, dtype=np.float64)):
        k = 0
        while k < max_log2 and v > dd * float(1 << k):
            k += 1
        out[i] = k
    return out


def binning_segments(freq_mhz, tsamp_s: float, dm, max_log2: int):
    """Runs of DM trials that share a binning factor, as (log2 factor, d0, d1) with the
    trials d0 .. d1-1 (DMs are non-decreasing, so each factor is one run)."""
    f = binning_factors(freq_mhz, tsamp_s, dm, max_log2)
    segs = []
    d0 = 0
    for d in range(1, len(f) + 1):
        if d == len(f) or f[d] != f[d0]:
            segs.append((int(f[d0]), d0, d))
            d0 = d
    return segs


def downfactor(data: np.ndarray) -> np.ndarray:
    """Downfactor a filterbank in time by 2, summing adjacent samples (Sec. "Computing
    Larger DMs", step iv): out[c][j] = A[c][2j] + A[c][2j+1] for j < floor(nsamp / 2), in
    FP64 (u8 codes are summed as raw codes)."""
    a = np.asarray(data, dtype=np.float64)
    m = a.shape[1] // 2
    return a[:, 0:2 * m:2] + a[:, 1:2 * m:2]


def dedisperse_binned(data: np.ndarray, freq_mhz, tsamp_s: float, dm, max_log2: int):
    """Brute-force dedispersion with time binning: each run of DM trials with factor 2^k
    is dedispersed (Eq. bruteEquation) on the input downfactored k times, with the delay
    table of sampling time 2^k t_samp. Returns a list of (k, d0, d1, series[d1-d0][nout_k])
    with nout_k = floor(nsamp / 2^k) - maxshift_k."""
    dm = np.asarray(dm, dtype=np.float64)
    level = np.asarray(data, dtype=np.float64)
    cur = 0
    res = []
    for k, d0, d1 in binning_segments(freq_mhz, tsamp_s, dm, max_log2):
        while cur < k:
            level = downfactor(level)
            cur += 1
        delays = delay_table(freq_mhz, dm[d0:d1], tsamp_s * float(1 << k))
        res.append((k, d0, d1, dedisperse(level, delays)))
    return res


def binned_adds(segments, nchan: int) -> int:
    """Algorithmic adds of a binned pass: sum over runs of ndm_k * nchan * nout_k (the
    downfactoring adds, nchan * nsamp in all, are not counted)."""
    return sum(int(d1 - d0) * int(nchan) * int(s.shape[1]) for _, d0, d1, s in segments)


def bandpass_average(data: np.ndarray) -> np.ndarray:
    """The averaged bandpass (Sec. "Bandpass Correction"): each channel's mean power over
    the buffer's samples, FP64."""
    return np.asarray(data, dtype=np.float64).mean(axis=1)


def bandpass_fit(avg, order: int):
    """Least-squares polynomial of the given order fitted to the averaged bandpass over the
    channel index, mapped to x = 2c/(nchan-1) - 1 (x = 0 for one channel). Returns the
    fitted bandpass [nchan], the RMSE between fit and average, and the fit's mean over
    channels. numpy's polynomial least squares is the fitting primitive."""
    a = np.asarray(avg, dtype=np.float64)
    n = a.size
    if order < 0 or order >= n:
        raise ValueError("need 0 <= order < nchan")
    x = np.zeros(n) if n == 1 else 2.0 * np.arange(n) / (n - 1) - 1.0
    coef = np.polynomial.polynomial.polyfit(x, a, order)
    fit = np.polynomial.polynomial.polyval(x, coef)
    rmse = float(np.sqrt(np.mean((a - fit) ** 2)))
    return fit, rmse, float(fit.mean())


def channel_clip(data: np.ndarray, fit, threshold: float, window: int):
    """Channel thresholding (Sec. "Channel Thresholding"): each channel is cut into
    non-overlapping windows of `window` samples (the last one may be shorter); a window is
    flagged when its mean differs from the channel's fitted value by more than `threshold`
    (too high: RFI; too low: lost data). Every flagged window and its two neighbours are
    replaced by the fitted value. Returns (data as FP64 with replacements, flags[nchan][nwin])."""
    x = np.array(data, dtype=np.float64)
    nchan, n = x.shape
    nwin = -(-n // window)
    flags = np.zeros((nchan, nwin), dtype=bool)
    for w in range(nwin):
        seg = x[:, w * window:(w + 1) * window]
        flags[:, w] = np.abs(seg.mean(axis=1) - np.asarray(fit)) > threshold
    spread = flags.copy()
    spread[:, 1:] |= flags[:, :-1]
    spread[:, :-1] |= flags[:, 1:]
    for c in range(nchan):
        for w in np.nonzero(spread[c])[0]:
            x[c, w * window:(w + 1) * window] = fit[c]
    return x, flags


def spectrum_clip(data: np.ndarray, fit, fit_mean: float, threshold: float):
    """Spectrum thresholding (Sec. "Spectrum Thresholding"): a spectrum (all channels at one
    sample) whose mean over channels differs from the fitted bandpass's mean by more than
    `threshold` is replaced by the fitted bandpass. Returns (data FP64, flags[nsamp])."""
    x = np.array(data, dtype=np.float64)
    m = x.mean(axis=0)
    flags = np.abs(m - fit_mean) > threshold
    x[:, flags] = np.asarray(fit, dtype=np.float64)[:, None]
    return x, flags


def bandpass_correct(data: np.ndarray, fit) -> np.ndarray:
    """Bandpass correction (Sec. "Bandpass Correction"): the fitted bandpass subtracted from
    every spectrum, equalising the response and moving each channel's mean to about 0."""
    return np.asarray(data, dtype=np.float64) - np.asarray(fit, dtype=np.float64)[:, None]


def rfi_mitigate(data: np.ndarray, order: int, chan_threshold: float, window: int, spec_threshold: float,
                 subtract: bool = True):
    """The RFI stage: fit the averaged bandpass; clip channel windows (when chan_threshold > 0)
    and then spectra (when spec_threshold > 0), replacing with the fitted bandpass; finally
    subtract the fitted bandpass from every spectrum (subtract=True), so replaced samples
    become exactly 0. The clipping compares the uncorrected data with the fit, as the
    paper's replacement by the fitted value presumes; the subtraction comes last."""
    fit, rmse, fit_mean = bandpass_fit(bandpass_average(data), order)
    x = np.asarray(data, dtype=np.float64)
    cflags = sflags = None
    if chan_threshold > 0:
        x, cflags = channel_clip(x, fit, chan_threshold, window)
    if spec_threshold > 0:
        x, sflags = spectrum_clip(x, fit, fit_mean, spec_threshold)
    if subtract:
        x = bandpass_correct(x, fit)
    return x, fit, rmse, fit_mean, cflags, sflags



def fit_codes(fit) -> np.ndarray:
    """The fitted bandpass as 8-bit codes: nearest integer, halves away from zero (the fit is
    a power level, so halves round up), clamped to 0..255."""
    f = np.asarray(fit, dtype=np.float64)
    return np.clip(np.floor(f + 0.5), 0.0, 255.0).astype(np.uint8)


def rfi_mitigate_codes(data: np.ndarray, order: int, chan_threshold: float, window: int, spec_threshold: float):
    """The RFI stage on 8-bit codes (reading: the paper's replacement by the fitted bandpass,
    with the replacement value the nearest code, since the samples stay 8-bit). The same fit,
    channel and spectrum decisions as rfi_mitigate on the codes as numbers, the replaced
    samples taking fit_codes(fit). No bandpass subtraction: an 8-bit sample cannot hold
    x - fit, and since Eq. bruteEquation sums each channel once, subtracting fit[c] from
    every sample of channel c lowers every dedispersed sample by sum(fit) and changes
    neither RMS nor candidates (pinned by a test). Returns (codes uint8, fit, rmse,
    fit_mean, channel flags, spectrum flags)."""
    codes = np.asarray(data)
    if codes.dtype != np.uint8:
        raise ValueError("8-bit codes expected")
    fit, rmse, fit_mean = bandpass_fit(bandpass_average(codes), order)
    rep = fit_codes(fit).astype(np.float64)
    x = codes.astype(np.float64)
    cflags = sflags = None
    if chan_threshold > 0:
        nchan, n = x.shape
        nwin = -(-n // window)
        cflags = np.zeros((nchan, nwin), dtype=bool)
        for w in range(nwin):
            cflags[:, w] = np.abs(x[:, w * window:(w + 1) * window].mean(axis=1) - fit) > chan_threshold
        spread = cflags.copy()
        spread[:, 1:] |= cflags[:, :-1]
        spread[:, :-1] |= cflags[:, 1:]
        for c in range(nchan):
            for w in np.nonzero(spread[c])[0]:
                x[c, w * window:(w + 1) * window] = rep[c]
    if spec_threshold > 0:
        sflags = np.abs(x.mean(axis=0) - fit_mean) > spec_threshold
        x[:, sflags] = rep[:, None]
    return x.astype(np.uint8), fit, rmse, fit_mean, cflags, sflags

def subband_dedisperse(data: np.ndarray, freq_mhz, tsamp_s: float, dm, chans_per_sub: int, dms_per_group: int):
    """Subband dedispersion (Sec. "Subband Dedispersion"). Subband s holds channels
    [s n_c, (s+1) n_c) (the last may be shorter) with reference f_s = its largest frequency.
    Trials are grouped in runs of n_dm consecutive trials; a group's nominal DM is the trial
    at its middle (index d0 + (len - 1) // 2).
    Step 1: S[g][s][t] = sum_{c in s} A[c][t + round(k DM_g (f_c^-2 - f_s^-2) / t_samp)]
    for t < nsamp - max over subbands and groups of the step-1 delays.
    Step 2: D[d][t] = sum_s S[g(d)][s][t + round(k DM_d (f_s^-2 - f_ref^-2) / t_samp)],
    f_ref the top of the band, for t < len(S) - the group's largest step-2 delay.
    Returns a list of (d0, d1, series[d1-d0][nout_g]) per group, in FP64."""
    f = np.asarray(freq_mhz, dtype=np.float64)
    dm = np.asarray(dm, dtype=np.float64)
    a = np.asarray(data, dtype=np.float64)
    nchan = f.size
    subs = [list(range(s, min(nchan, s + chans_per_sub))) for s in range(0, nchan, chans_per_sub)]
    groups = [(d0, min(dm.size, d0 + dms_per_group)) for d0 in range(0, dm.size, dms_per_group)]
    nominal = np.array([dm[d0 + (d1 - d0 - 1) // 2] for d0, d1 in groups])
    inner = [delay_table(f[idx], nominal, tsamp_s) for idx in subs]      # relative to f_s
    m1 = max(int(t.max()) for t in inner)
    len1 = a.shape[1] - m1
    if len1 <= 0:
        raise ValueError("nsamp must exceed the step-1 delays")
    f_sub = np.array([f[idx].max() for idx in subs])
    out = []
    for g, (d0, d1) in enumerate(groups):
        red = np.empty((len(subs), len1))
        for s, idx in enumerate(subs):
            acc = np.zeros(len1)
            for i, c in enumerate(idx):
                k = int(inner[s][i, g])
                acc += a[c, k:k + len1]
            red[s] = acc
        # step 2: the delay table of the subbands' top frequencies (max of them = f_ref)
        out.append((d0, d1, dedisperse(red, delay_table(f_sub, dm[d0:d1], tsamp_s))))
    return out
