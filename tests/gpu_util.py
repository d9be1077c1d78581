"""Shared helpers for the GPU parity tests (comparison rules, device fixture)."""
import numpy as np
import pytest

# FP32 outputs agree with the FP64 oracle within this many series RMS (per DM row).
RMS_TOL = 1e-5
# Candidates are compared only where no oracle value lies within this many RMS of its
# threshold; FP32 rounding of the series cannot move a value across it.
GUARD = 5e-5


def cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch


def assert_rows_close(got, want, rms, tol=RMS_TOL, what=""):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    scale = np.where(rms > 0, rms, 1.0)
    err = np.max(np.abs(got - want), axis=1) / scale
    worst = int(np.argmax(err))
    assert err[worst] <= tol, f"{what} row {worst}: max|err| = {err[worst]:.3e} rms (tol {tol})"


def assert_stats_close(mean_got, rms_got, mean_want, rms_want, tol=RMS_TOL):
    """Mean and RMS within tol series RMS, beyond the half ulp of their FP32 storage (the
    library returns both as FP32: a mean far above the RMS, as sums of many 8-bit codes
    give, is rounded by more than tol RMS on storage alone)."""
    mean_got = np.asarray(mean_got, np.float64)
    rms_got = np.asarray(rms_got, np.float64)
    scale = np.where(rms_want > 0, rms_want, 1.0)
    half_ulp = 2.0 ** -24
    assert np.max((np.abs(mean_got - mean_want) - half_ulp * np.abs(mean_want)) / scale) <= tol
    assert np.max((np.abs(rms_got - rms_want) - half_ulp * np.abs(rms_want)) / scale) <= tol


def compare_candidates(got, series, mean, rms, k, row_ids=None, t_offset=0):
    """got: structured array from the library. The oracle decides in FP64 from its own series;
    values within GUARD*rms of the threshold are ambiguous and must not occur."""
    from oracle import dedisp_oracle as orc
    margin = orc.threshold_margin(series, mean, rms, k)
    assert margin > GUARD, f"ill-conditioned seed: a value lies {margin:.2e} rms from its threshold"
    want = orc.candidates(series, mean, rms, k, row_ids=row_ids)
    assert got is not None
    assert got.size == want["t"].size, (got.size, want["t"].size)
    np.testing.assert_array_equal(got["dm_index"], want["dm_index"])
    np.testing.assert_array_equal(got["t"], want["t"] + t_offset)
    rr = np.asarray(rms)[np.searchsorted(np.asarray(row_ids) if row_ids is not None else
                                         np.arange(len(rms)), want["dm_index"])] if want["t"].size else []
    if want["t"].size:
        assert np.max(np.abs(got["value"] - want["value"]) / rr) <= RMS_TOL * 2
        assert np.max(np.abs(got["snr"] - want["snr"])) <= 1e-3
