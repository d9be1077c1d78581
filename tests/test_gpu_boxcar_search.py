"""dd_boxcar_search (boxcar template matching at every start, Ch. 6 "Transient Surveys")
against the oracle's boxcar_search.

Detections (row, t, width) must equal the oracle's exactly; the boxcar sums agree within
FP32 rounding of a pairwise sum, the S/N within 1e-4. The series are FP32 arrays given to
both sides, with the FP32 mean/rms the library takes; seeds are chosen so that no decision
(threshold or best width) lies within 1e-3 S/N of flipping (oracle boxcar_margin). Each case
prints its shape before it runs.
"""
import math

import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import cuda

pytestmark = pytest.mark.gpu

MARGIN = 1e-3


@pytest.fixture(scope="module")
def torch():
    return cuda()


@pytest.fixture(scope="module")
def dd():
    import paper_1401_8258_amd as dd
    dd.load_library()
    return dd


def _say(msg):
    print(msg, flush=True)


def _pulsed_rows(rng, nrows, n, npulse=3):
    x = rng.standard_normal((nrows, n)).astype(np.float32)
    for d in range(nrows):
        for _ in range(npulse):
            w = int(rng.choice([1, 3, 8, 13, 40, 64]))
            if w >= n:
                continue
            t0 = int(rng.integers(0, n - w))
            x[d, t0:t0 + w] += np.float32(rng.uniform(4.0, 9.0) / math.sqrt(w))
    return x


def _compare(got, want, rms_of_row):
    assert got.size == want["t"].size, (got.size, want["t"].size)
    np.testing.assert_array_equal(got["row"], want["row"])
    np.testing.assert_array_equal(got["t"], want["t"])
    np.testing.assert_array_equal(got["width"], want["width"])
    if got.size:
        scale = np.sqrt(want["width"]) * rms_of_row[want["row"]]
        assert np.max(np.abs(got["value"] - want["value"]) / scale) <= 1e-5
        assert np.max(np.abs(got["snr"] - want["snr"])) <= 1e-4


def _seeded(nrows, n, max_log2, k, first, stats=True):
    for seed in range(first, first + 60):
        rng = np.random.default_rng(seed)
        x = _pulsed_rows(rng, nrows, n)
        if stats:
            mean = x.astype(np.float64).mean(axis=1).astype(np.float32)
            rms = x.astype(np.float64).std(axis=1).astype(np.float32)
        else:
            mean = np.zeros(nrows, np.float32)
            rms = np.ones(nrows, np.float32)
        m = orc.boxcar_margin(x, mean.astype(np.float64), rms.astype(np.float64), max_log2, k)
        if m > MARGIN:
            return x, mean, rms
    raise AssertionError("no well-conditioned seed in 60")


@pytest.mark.parametrize("nrows,n,max_log2,k", [
    (16, 10000, 6, 4.0),    # several 4096-start segments and a ragged tail
    (3, 4096, 6, 3.5),      # exactly one segment
    (5, 4097, 3, 3.5),      # one start in the second segment; widths up to 8
    (2, 63, 6, 2.5),        # shorter than the widest boxcar
    (1, 1, 6, 0.0),         # one sample (rms 0: no detections)
])
def test_equals_oracle(torch, dd, nrows, n, max_log2, k):
    _say(f"case: boxcar search nrows={nrows} n={n} max_log2={max_log2} k={k}")
    x, mean, rms = _seeded(nrows, n, max_log2, k, first=nrows * 1000 + n)
    want = orc.boxcar_search(x, mean.astype(np.float64), rms.astype(np.float64), max_log2, k)
    got = dd.boxcar_search(torch.from_numpy(x).cuda(), torch.from_numpy(mean).cuda(), torch.from_numpy(rms).cuda(),
                           max_log2=max_log2, k_sigma=k)
    _compare(got, want, rms.astype(np.float64))
    if nrows * n > 1000:
        assert want["t"].size > 0


def test_normalised_rows_and_row_stride(torch, dd):
    """mean/rms omitted (normalised rows, mean 0 and rms 1) and rows padded in memory."""
    _say("case: boxcar search normalised, padded rows")
    x, mean, rms = _seeded(7, 5000, 6, 4.0, first=77, stats=False)
    want = orc.boxcar_search(x, mean.astype(np.float64), rms.astype(np.float64), 6, 4.0)
    full = torch.full((7, 5003), 99.0, device="cuda")
    full[:, :5000] = torch.from_numpy(x).cuda()
    got = dd.boxcar_search(full[:, :5000], max_log2=6, k_sigma=4.0)
    _compare(got, want, rms.astype(np.float64))


def test_width_one_is_the_plain_threshold(torch, dd):
    _say("case: boxcar search max_log2=0 against the plain threshold")
    x, mean, rms = _seeded(6, 9000, 0, 3.0, first=500)
    want = orc.candidates(x, mean.astype(np.float64), rms.astype(np.float64), 3.0)
    got = dd.boxcar_search(torch.from_numpy(x).cuda(), torch.from_numpy(mean).cuda(), torch.from_numpy(rms).cuda(),
                           max_log2=0, k_sigma=3.0)
    np.testing.assert_array_equal(got["row"], want["dm_index"])
    np.testing.assert_array_equal(got["t"], want["t"])
    assert np.all(got["width"] == 1)
    np.testing.assert_array_equal(got["value"], want["value"].astype(np.float32))


def test_constant_row_and_unaligned_pulse(torch, dd):
    """A constant row has no detections; an unaligned width-8 pulse on a zero row is found
    at its start with S/N a sqrt(8) (the oracle's closed-form pin)."""
    _say("case: boxcar search constant row, unaligned pulse")
    x = np.zeros((2, 300), np.float32)
    x[0] = 5.0
    x[1, 13:21] = 1.5
    mean = np.array([5.0, 0.0], np.float32)
    rms = np.array([0.0, 1.0], np.float32)
    k = 0.95 * 1.5 * math.sqrt(8)
    got = dd.boxcar_search(torch.from_numpy(x).cuda(), torch.from_numpy(mean).cuda(), torch.from_numpy(rms).cuda(),
                           max_log2=6, k_sigma=k)
    assert got.size == 1 and got["row"][0] == 1 and got["t"][0] == 13 and got["width"][0] == 8
    assert abs(got["snr"][0] - 1.5 * math.sqrt(8)) < 1e-5


def test_overflow_keeps_the_first(torch, dd):
    _say("case: boxcar search overflow")
    x, mean, rms = _seeded(4, 500, 6, 2.0, first=900)
    want = orc.boxcar_search(x, mean.astype(np.float64), rms.astype(np.float64), 6, 2.0)
    assert want["t"].size > 20
    with pytest.warns(dd.CandidateOverflow):
        got = dd.boxcar_search(torch.from_numpy(x).cuda(), torch.from_numpy(mean).cuda(),
                               torch.from_numpy(rms).cuda(), max_log2=6, k_sigma=2.0, cap=17)
    assert got.size == 17
    np.testing.assert_array_equal(got["t"], want["t"][:17])
    np.testing.assert_array_equal(got["width"], want["width"][:17])


def test_after_full_size_dedispersion(torch, dd):
    """Config 2 dedispersed on the device (FP32 series and statistics), then searched on the
    device; on the brightest pulses' trials and both ends the detections equal the oracle's
    search of its own FP64 series and statistics (rows whose decisions keep the margin)."""
    _say("case: boxcar search after config-2 dedispersion")
    b = fbsynth.config2()
    plan = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm)
    r = plan.dedisperse(torch.from_numpy(b.data).cuda())
    got = dd.boxcar_search(r.out, r.mean, r.rms, max_log2=6, k_sigma=6.5, cap=1 << 22)
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    bright = sorted(b.pulses, key=lambda p: -p.amp * math.sqrt(p.width))[:3]
    rows = sorted({0, b.ndm - 1} | {int(np.argmin(np.abs(b.dm - p.dm))) for p in bright})
    series = orc.dedisperse(b.data, tab, rows=rows)
    mean, rms = orc.series_stats(series)
    checked = 0
    for i, d in enumerate(rows):
        if orc.boxcar_margin(series[i:i + 1], mean[i:i + 1], rms[i:i + 1], 6, 6.5) <= MARGIN:
            continue
        want = orc.boxcar_search(series[i:i + 1], mean[i:i + 1], rms[i:i + 1], 6, 6.5)
        g = got[got["row"] == d]
        assert g.size == want["t"].size, (d, g.size, want["t"].size)
        np.testing.assert_array_equal(g["t"], want["t"])
        np.testing.assert_array_equal(g["width"], want["width"])
        if g.size:
            assert np.max(np.abs(g["snr"] - want["snr"])) <= 1e-3
        checked += 1
    assert checked >= 3
    # the brightest pulses are detected on their trials
    assert any(got[got["row"] == int(np.argmin(np.abs(b.dm - p.dm)))].size > 0 for p in bright)
