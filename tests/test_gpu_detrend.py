"""Detrending and normalisation on the device (dd_detrend) against the FP64 oracle.

Sec. 3.5 "Signal Post-processing". Shapes span one sample, two samples, less than one
workgroup pass, ragged tails over several passes and long rows; rows are padded (row
stride > n) and the padding must stay untouched. The end-to-end case detrends the
dedispersed config-1 series. Each case prints its shape first.
"""
import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import cuda

pytestmark = pytest.mark.gpu

SHAPES = [(3, 1, 0), (5, 2, 3), (7, 255, 1), (4, 256, 0), (9, 1000, 24), (2, 70001, 7)]


@pytest.fixture(scope="module")
def torch():
    return cuda()


@pytest.mark.parametrize("normalise", [False, True])
@pytest.mark.parametrize("nrows,n,pad", SHAPES)
def test_detrend_matches_oracle(torch, nrows, n, pad, normalise):
    import paper_1401_8258_amd as dd
    print(f"case: detrend nrows={nrows} n={n} pad={pad} normalise={normalise}", flush=True)
    rng = np.random.default_rng(nrows * 1000 + n)
    t = np.arange(n)
    x = (rng.standard_normal((nrows, n)) * 3 + 50 + 0.01 * t[None, :] * rng.standard_normal((nrows, 1)))
    x = x.astype(np.float32)
    full = np.full((nrows, n + pad), -7.0, dtype=np.float32)
    full[:, :n] = x
    dev = torch.from_numpy(full).cuda()
    rms = dd.detrend(dev[:, :n], normalise=normalise)
    torch.cuda.synchronize()
    got = dev.cpu().numpy()
    want, want_rms = orc.detrend(x.astype(np.float64), normalise=normalise)
    scale = 1.0 if normalise else np.maximum(want_rms, 1e-30)[:, None]
    assert np.max(np.abs(got[:, :n] - want) / scale) <= 1e-6
    np.testing.assert_allclose(rms.cpu().numpy(), want_rms, rtol=1e-6, atol=1e-6)
    assert np.all(got[:, n:] == -7.0)  # padding untouched


def test_detrend_of_dedispersed_config1(torch):
    import paper_1401_8258_amd as dd
    print("case: detrend of the dedispersed config-1 series", flush=True)
    b = fbsynth.config1()
    plan = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm)
    res = plan.dedisperse(torch.from_numpy(b.data).cuda(), k_sigma=0.0, stats=False)
    rms = dd.detrend(res.out, normalise=True)
    torch.cuda.synchronize()
    want, want_rms = orc.detrend(orc.dedisperse(b.data, orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)),
                                 normalise=True)
    # the dedispersed input carries its own FP32 error (<= 1e-5 of its RMS); normalised
    # values are in units of that RMS
    assert np.max(np.abs(res.out.cpu().numpy() - want)) <= 2e-5
    np.testing.assert_allclose(rms.cpu().numpy(), want_rms, rtol=2e-5)
