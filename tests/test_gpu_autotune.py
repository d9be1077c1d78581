"""The autotuner on the device: whatever tiling it picks computes the same series (the channel
summation order is fixed), so the tuned plan's output equals the default plan's bit for bit
and the FP64 oracle within 1e-5 rms (u8: exactly)."""
import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import assert_rows_close, assert_stats_close, cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return cuda()


@pytest.fixture(scope="module")
def at():
    import paper_1401_8258_amd as dd
    dd.load_library()
    from paper_1401_8258_amd import autotune
    return autotune


def test_tuned_plan_equals_default_and_oracle(torch, at):
    print("case: autotune config 1 shape, FP32, both forms", flush=True)
    import paper_1401_8258_amd as dd
    b = fbsynth.config1()
    x = torch.from_numpy(b.data).cuda()
    res = at.tune(b.freq_mhz, b.tsamp_s, b.dm, "f32", b.nsamp, waves=(8, 4, 2, 1), stages=(0, 2, 4),
                  forms=("lds", "regwin"), reps=1, x=x)
    assert sum("ms" in t for t in res["trials"]) >= 2
    tuned = at.make_plan(b.freq_mhz, b.tsamp_s, b.dm, "f32", res)
    default = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm)
    r1 = tuned.dedisperse(x)
    r2 = default.dedisperse(x)
    torch.cuda.synchronize()
    assert torch.equal(r1.out, r2.out), f"tuned {res['form']} {res['tuning']} differs from the default plan"
    tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
    want = orc.dedisperse(b.data, tab)
    mean, rms = orc.series_stats(want)
    assert_rows_close(r1.out.cpu().numpy(), want, rms, what="tuned")
    assert_stats_close(r1.mean.cpu().numpy(), r1.rms.cpu().numpy(), mean, rms)


def test_tune_batch_u8_beams_exact(torch, at):
    print("case: tune_batch over three small u8 beams", flush=True)
    specs = fbsynth.config4_specs(seed=4, scale=1 / 64)[:3]
    beams, xs, data = [], [], []
    for sp in specs:
        rng = np.random.default_rng(sp["seed"])
        bm = fbsynth.make_beam(sp["name"], sp["nchan"], sp["f_top"], sp["bw"], sp["tsamp"], sp["dm0"], sp["step"],
                               sp["ndm"], sp["nsamp"], rng, sp["npulse"], storage="u8")
        beams.append((bm.freq_mhz, bm.tsamp_s, bm.dm, "u8", bm.nsamp))
        xs.append(torch.from_numpy(bm.data).cuda())
        data.append(bm)
    res = at.tune_batch(beams, waves=(8, 4, 2), stages=(0,), reps=1, inputs=xs)
    assert res["waves"] in (8, 4, 2) and len(res["tunings"]) == 3
    # the chosen plans (each beam's own best) in one batched call equal their single calls
    plans = [at.make_plan(bm.freq_mhz, bm.tsamp_s, bm.dm, "u8", c) for bm, c in zip(data, res["choices"])]
    import paper_1401_8258_amd as dd
    batched = dd.batch_dedisperse(list(zip(plans, xs)), k_sigma=6.0)
    for p, x, r in zip(plans, xs, batched):
        s = p.dedisperse(x, k_sigma=6.0)
        np.testing.assert_array_equal(s.out.cpu().numpy(), r.out.cpu().numpy())
        np.testing.assert_array_equal(s.candidates(), r.candidates())
    for bm, choice, x in zip(data, res["choices"], xs):
        plan = at.make_plan(bm.freq_mhz, bm.tsamp_s, bm.dm, "u8", choice)
        assert plan.form == choice["form"]
        got = plan.dedisperse(x).out.cpu().numpy()
        rows = [0, bm.ndm // 2, bm.ndm - 1]
        want = orc.dedisperse(bm.data, orc.delay_table(bm.freq_mhz, bm.dm, bm.tsamp_s), rows=rows)
        np.testing.assert_array_equal(got[rows].astype(np.float64), want)
