"""Subband dedispersion on the device (two steps of ordinary plans through the C ABI)
against the FP64 oracle's two-step definition (run on an MI355X with -m gpu)."""
import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import assert_rows_close, assert_stats_close, compare_candidates, cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return cuda()


@pytest.fixture(scope="module")
def dd():
    import paper_1401_8258_amd as dd
    dd.load_library()
    return dd


@pytest.mark.parametrize("nsub_ch,ngrp", [(8, 8), (16, 16), (5, 3), (64, 48), (1, 1)])
def test_subband_config1(torch, dd, nsub_ch, ngrp):
    """Every group's series, statistics and 6-sigma candidates (ragged last subband and group
    included); one-channel subbands with single-trial groups are plain dedispersion."""
    print(f"case: subband config1 {nsub_ch} ch/subband, {ngrp} trials/group", flush=True)
    b = fbsynth.config1()
    sp = dd.SubbandPlan(b.freq_mhz, b.tsamp_s, b.dm, chans_per_sub=nsub_ch, dms_per_group=ngrp)
    res = sp.dedisperse(torch.from_numpy(b.data).cuda(), k_sigma=6.0)
    torch.cuda.synchronize()
    want = orc.subband_dedisperse(b.data, b.freq_mhz, b.tsamp_s, b.dm, nsub_ch, ngrp)
    assert [g for g, _ in res] == [(d0, d1) for d0, d1, _ in want]
    for (_, r), (d0, d1, s) in zip(res, want):
        mean, rms = orc.series_stats(s)
        assert_rows_close(r.out.cpu().numpy(), s, rms, what=f"group {d0}")
        assert_stats_close(r.mean.cpu().numpy(), r.rms.cpu().numpy(), mean, rms)
        compare_candidates(r.candidates(), s, mean, rms, 6.0)
    if nsub_ch == 1 and ngrp == 1:
        plain = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm).dedisperse(torch.from_numpy(b.data).cuda()).out.cpu().numpy()
        for (d0, _), r in res:
            got = r.out.cpu().numpy()[0, :plain.shape[1]]
            assert np.max(np.abs(got - plain[d0])) <= 1e-5 * np.sqrt(64)


def test_subband_batched_equals_per_plan(torch, dd):
    """Each step in one persistent launch equals one launch per plan, bit for bit."""
    b = fbsynth.config1()
    x = torch.from_numpy(b.data).cuda()
    sp = dd.SubbandPlan(b.freq_mhz, b.tsamp_s, b.dm, chans_per_sub=8, dms_per_group=8)
    a = sp.dedisperse(x, k_sigma=4.0)
    c = sp.dedisperse(x, k_sigma=4.0, batched=True)
    torch.cuda.synchronize()
    for (g1, r1), (g2, r2) in zip(a, c):
        assert g1 == g2
        assert torch.equal(r1.out, r2.out) and torch.equal(r1.mean, r2.mean) and torch.equal(r1.rms, r2.rms)
        np.testing.assert_array_equal(r1.candidates(), r2.candidates())
