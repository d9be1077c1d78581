"""Boxcar levels on the device (dd_boxcar) against the FP64 oracle, and the single-pulse
search on config 1: detrend, normalise, boxcar, then the injected pulse stands out at
its width and DM. Each case prints its shape first."""
import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import cuda

pytestmark = pytest.mark.gpu

SHAPES = [(3, 1, 0, 0), (2, 63, 6, 1), (4, 64, 6, 0), (3, 777, 3, 5), (5, 1000, 6, 0), (2, 100001, 6, 3)]


@pytest.fixture(scope="module")
def torch():
    return cuda()


@pytest.mark.parametrize("nrows,n,levels,pad", SHAPES)
def test_boxcar_matches_oracle(torch, nrows, n, levels, pad):
    import paper_1401_8258_amd as dd
    print(f"case: boxcar nrows={nrows} n={n} levels={levels} pad={pad}", flush=True)
    rng = np.random.default_rng(n + levels)
    full = np.zeros((nrows, n + pad), dtype=np.float32)
    full[:, :n] = rng.standard_normal((nrows, n)).astype(np.float32)
    got = dd.boxcar(torch.from_numpy(full).cuda()[:, :n], levels=levels)
    torch.cuda.synchronize()
    want = orc.boxcar_levels(full[:, :n].astype(np.float64), levels)
    assert len(got) == levels + 1
    for k in range(levels + 1):
        g = got[k].cpu().numpy()
        assert g.shape == want[k].shape
        # FP32 pairwise sums of at most 64 unit-variance samples
        assert np.max(np.abs(g - want[k]), initial=0.0) <= 2e-6 * np.sqrt(2.0 ** k) + 1e-6


def test_single_pulse_search_config1(torch):
    import paper_1401_8258_amd as dd
    print("case: config 1 single-pulse search (detrend, normalise, boxcar)", flush=True)
    b = fbsynth.config1()
    plan = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm)
    res = plan.dedisperse(torch.from_numpy(b.data).cuda(), stats=False)
    dd.detrend(res.out, normalise=True)
    lv = dd.boxcar(res.out, levels=6)
    torch.cuda.synchronize()
    want = orc.boxcar_levels(orc.detrend(orc.dedisperse(b.data, orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)),
                                         normalise=True)[0], 6)
    for k in range(7):
        assert np.max(np.abs(lv[k].cpu().numpy() - want[k])) <= 1e-4
    # the pulse (8 samples wide, DM 5.0 = trial 50) peaks on the width-8 level near its DM
    l3 = lv[3].cpu().numpy()
    d, j = np.unravel_index(np.argmax(l3), l3.shape)
    assert abs(d - 50) <= 1 and l3[d, j] > 7.0, (d, j, l3[d, j])
