"""Edge shapes for every storage type against the oracle (FP32 is also covered by the
edge cases in test_gpu_parity.py; here all three run the same shapes).

8-bit input takes its own tile body (byte copies in LDS, a workspace copy of the input
tail for windows that would read past the end of the array); 16-bit input uses the
zero-extending 2-byte DMA with per-lane clamping at the end of the data. Each case
prints its shape before it runs.
"""
import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import GUARD, assert_rows_close, assert_stats_close, compare_candidates, cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return cuda()


@pytest.fixture(scope="module")
def dd():
    import paper_1401_8258_amd as dd
    dd.load_library()
    return dd


# nchan, channel width (MHz), ndm, DM step, nsamp, tuning, row padding (samples)
NARROW = [
    (1, 0.3125, 1, 0.1, 300, None, 0),            # one channel, one trial
    (64, 0.3125, 128, 0.1, 556, None, 0),         # nout = 1
    (64, 0.3125, 128, 0.1, 1000, (8, 2), 3),      # nout < one tile; odd row padding
    (37, 0.5, 33, 0.3, 2000, None, 0),            # odd channel count, partial group
    (96, 0.2, 70, 0.5, 5001, (8, 4, 1), 0),       # one channel per stage
    (200, 0.1, 40, 0.2, 4097, (8, 8, 5), 1),      # stage size not a divisor
    (16, 3.75, 64, 2.0, 40000, None, 0),          # wide band: large delay spread
]


def _data(nchan, nsamp, pad, dtype, seed):
    rng = np.random.default_rng(seed)
    x = fbsynth.noise(rng, nchan, nsamp)
    x = fbsynth.to_u8(x) if dtype == "u8" else fbsynth.to_f16(x) if dtype == "f16" else x
    if pad:
        full = np.zeros((nchan, nsamp + pad), dtype=x.dtype)
        full[:, :nsamp] = x
        return full
    return x


@pytest.mark.parametrize("dtype", ["u8", "f16", "f32"])
@pytest.mark.parametrize("nchan,df,ndm,step,nsamp,tuning,pad", NARROW)
def test_narrow_storage_edges(torch, dd, dtype, nchan, df, ndm, step, nsamp, tuning, pad):
    print(f"case: {dtype} nchan={nchan} ndm={ndm} step={step} nsamp={nsamp} tuning={tuning} pad={pad}",
          flush=True)
    freq = fbsynth.channel_freqs(428.0, df, nchan)
    dm = fbsynth.dm_trials(0.0, step, ndm)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    if nsamp <= int(tab.max()):
        pytest.skip("shape shorter than the delay spread")
    # the first seed whose oracle values all keep a clear margin from their thresholds
    for seed in range(nchan * 7 + ndm, nchan * 7 + ndm + 50):
        full = _data(nchan, nsamp, pad, dtype, seed=seed)
        data = np.ascontiguousarray(full[:, :nsamp])
        want = orc.dedisperse(data, tab)
        mean, rms = orc.series_stats(want)
        if orc.threshold_margin(want, mean, rms, 3.0) > 4 * GUARD:
            break
    plan = dd.Plan(freq, 51.2e-6, dm, dtype=dtype, tuning=tuning)
    xt = torch.from_numpy(np.ascontiguousarray(full)).cuda()[:, :nsamp]  # strided rows when padded
    res = plan.dedisperse(xt, k_sigma=3.0)
    torch.cuda.synchronize()
    got = res.out.cpu().numpy()
    if dtype == "u8":
        np.testing.assert_array_equal(got.astype(np.float64), want)
    else:
        assert_rows_close(got, want, rms, what=f"{dtype} edge")
    assert_stats_close(res.mean.cpu().numpy(), res.rms.cpu().numpy(), mean, rms)
    compare_candidates(res.candidates(), want, mean, rms, 3.0)


@pytest.mark.parametrize("dtype", ["u8", "f16"])
def test_narrow_stream_ragged_blocks(torch, dd, dtype):
    print(f"case: {dtype} stream with ragged blocks", flush=True)
    freq = fbsynth.channel_freqs(428.0, 20.0 / 128, 128)
    dm = fbsynth.dm_trials(0.0, 0.1, 96)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    sizes = [700, 700, 333, 700, 1, 700, 650, 700]
    x = _data(128, sum(sizes), 0, dtype, seed=33)
    plan = dd.Plan(freq, 51.2e-6, dm, dtype=dtype)
    st = dd.Stream(plan, 700)
    expected = orc.stream_expected(np.split(x, np.cumsum(sizes)[:-1], axis=1), tab)
    pos = 0
    for n, (t0, t1, want) in zip(sizes, expected):
        r = st.push(torch.from_numpy(np.ascontiguousarray(x[:, pos:pos + n])).cuda())
        pos += n
        if t1 <= t0:
            assert r is None
            continue
        assert r.t0 == t0 and r.out.shape[1] == t1 - t0
        got = r.out.cpu().numpy()
        if dtype == "u8":
            np.testing.assert_array_equal(got.astype(np.float64), want)
        else:
            _, rms = orc.series_stats(want) if want.shape[1] > 1 else (None, np.ones(want.shape[0]))
            assert_rows_close(got, want, np.maximum(rms, 1.0), what="f16 stream")
