"""Batched persistent launch against one-at-a-time calls (bit for bit) and the oracle."""
import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from tests.gpu_util import GUARD, assert_rows_close, compare_candidates, cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return cuda()


@pytest.fixture(scope="module")
def dd():
    import paper_1401_8258_amd as dd
    dd.load_library()
    return dd


def _beams(scale, dtype="u8", seed=4):
    specs = fbsynth.config4_specs(seed=seed, scale=scale)
    out = []
    for sp in specs:
        rng = np.random.default_rng(sp["seed"])
        b = fbsynth.make_beam(sp["name"], sp["nchan"], sp["f_top"], sp["bw"], sp["tsamp"], sp["dm0"], sp["step"],
                              sp["ndm"], sp["nsamp"], rng, sp["npulse"], storage=dtype)
        out.append(b)
    return out


def test_batch_equals_single_calls_uneven_u8(torch, dd):
    print("case: batch of uneven u8 beams", flush=True)
    beams = _beams(scale=1 / 64)[:8]
    tuning = (8, 2)
    plans = [dd.Plan(b.freq_mhz, b.tsamp_s, b.dm, dtype="u8", tuning=tuning) for b in beams]
    xs = [torch.from_numpy(b.data).cuda() for b in beams]
    singles = [p.dedisperse(x, k_sigma=6.0) for p, x in zip(plans, xs)]
    batched = dd.batch_dedisperse(list(zip(plans, xs)), k_sigma=6.0)
    torch.cuda.synchronize()
    for b, p, s1, s2 in zip(beams, plans, singles, batched):
        o1, o2 = s1.out.cpu().numpy(), s2.out.cpu().numpy()
        np.testing.assert_array_equal(o1, o2)
        np.testing.assert_array_equal(s1.mean.cpu().numpy(), s2.mean.cpu().numpy())
        np.testing.assert_array_equal(s1.rms.cpu().numpy(), s2.rms.cpu().numpy())
        c1, c2 = s1.candidates(), s2.candidates()
        np.testing.assert_array_equal(c1, c2)
        # and against the oracle: u8 codes sum exactly
        tab = orc.delay_table(b.freq_mhz, b.dm, b.tsamp_s)
        rows = [0, b.ndm // 2, b.ndm - 1]
        want = orc.dedisperse(b.data, tab, rows=rows)
        np.testing.assert_array_equal(o2[rows].astype(np.float64), want)


def test_batch_f32_mixed_shapes(torch, dd):
    print("case: batch of f32 beams", flush=True)
    jobs, refs = [], []
    for i, (nchan, ndm, nsamp, step) in enumerate([(64, 100, 6000, 0.1), (128, 40, 9000, 0.3), (32, 300, 4000, 0.05)]):
        freq = fbsynth.channel_freqs(428.0, 20.0 / nchan, nchan)
        dm = fbsynth.dm_trials(0.0, step, ndm)
        tab = orc.delay_table(freq, dm, 51.2e-6)
        # a seed whose oracle values keep a margin from their thresholds (candidates compared)
        for seed in range(100 * i, 100 * i + 50):
            x = np.random.default_rng(seed).standard_normal((nchan, nsamp)).astype(np.float32)
            want = orc.dedisperse(x, tab)
            mean, rms = orc.series_stats(want)
            if orc.threshold_margin(want, mean, rms, 4.0) > 4 * GUARD:
                break
        else:
            raise AssertionError("no well-conditioned seed in 50")
        p = dd.Plan(freq, 51.2e-6, dm, tuning=(8, 4))
        jobs.append((p, torch.from_numpy(x).cuda()))
        refs.append((want, mean, rms))
    res = dd.batch_dedisperse(jobs, k_sigma=4.0)
    torch.cuda.synchronize()
    for (p, x), r, (want, mean, rms) in zip(jobs, res, refs):
        s = p.dedisperse(x, k_sigma=4.0)
        np.testing.assert_array_equal(s.out.cpu().numpy(), r.out.cpu().numpy())
        assert_rows_close(r.out.cpu().numpy(), want, rms, what="batch f32")
        compare_candidates(r.candidates(), want, mean, rms, 4.0)


def test_batched_stream_windows_equal_push(torch, dd):
    print("case: batched stream windows", flush=True)
    rng = np.random.default_rng(8)
    freq = fbsynth.channel_freqs(428.0, 20.0 / 64, 64)
    dm = fbsynth.dm_trials(0.0, 0.2, 64)
    block = 600
    nblk = 6
    data = [rng.integers(0, 256, size=(64, block * nblk)).astype(np.uint8) for _ in range(3)]
    plan = dd.Plan(freq, 51.2e-6, dm, dtype="u8", tuning=(8, 4))
    pushed = [dd.Stream(plan, block) for _ in range(3)]
    batched = [dd.Stream(plan, block) for _ in range(3)]
    for k in range(nblk):
        blocks = [torch.from_numpy(np.ascontiguousarray(d[:, k * block:(k + 1) * block])).cuda() for d in data]
        want = [s.push(b, k_sigma=3.0) for s, b in zip(pushed, blocks)]
        wins = [s.append(b) for s, b in zip(batched, blocks)]
        assert all((w is None) == (r is None) for w, r in zip(wins, want))
        if wins[0] is None:
            continue
        got = dd.batch_dedisperse(list(zip(batched, wins)), k_sigma=3.0)
        torch.cuda.synchronize()
        for g, r in zip(got, want):
            assert g.t0 == r.t0
            np.testing.assert_array_equal(g.out.cpu().numpy(), r.out.cpu().numpy())
            np.testing.assert_array_equal(g.candidates(), r.candidates())


def test_batch_mixed_dma_forms_and_f16(torch, dd):
    """FP32 items whose plans differ in DMA form (16-byte DMAs for narrow windows, 4-byte
    DMAs for windows too wide for the 16 descriptors) share one launch through the kernel
    that picks the form per item; FP16 items batch through their own kernel."""
    rng = np.random.default_rng(21)
    shapes = [(64, 0.3125, 128, 0.1, 6000), (16, 3.75, 64, 2.0, 40000)]  # narrow, wide band
    for dtype in ("f32", "f16"):
        print(f"case: batch of {dtype} items, narrow and wide-band windows", flush=True)
        jobs, refs = [], []
        for nchan, df, ndm, step, nsamp in shapes:
            freq = fbsynth.channel_freqs(428.0, df, nchan)
            dm = fbsynth.dm_trials(0.0, step, ndm)
            x = fbsynth.noise(rng, nchan, nsamp)
            x = fbsynth.to_f16(x) if dtype == "f16" else x
            p = dd.Plan(freq, 51.2e-6, dm, dtype=dtype, tuning=(8, 1, 0, -1))
            jobs.append((p, torch.from_numpy(np.ascontiguousarray(x)).cuda()))
            refs.append((freq, dm, x))
        if dtype == "f32":
            launch = [p.query(x.shape[1])["launch_buf"] for p, x in jobs]
            assert launch[0] // 64 <= 16 < launch[1] // 64, launch  # one item of each DMA form
        res = dd.batch_dedisperse(jobs, k_sigma=4.0)
        torch.cuda.synchronize()
        for (p, x), r, (freq, dm, xh) in zip(jobs, res, refs):
            s = p.dedisperse(x, k_sigma=4.0)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(s.out.cpu().numpy(), r.out.cpu().numpy())
            want = orc.dedisperse(xh, orc.delay_table(freq, dm, 51.2e-6))
            _, rms = orc.series_stats(want)
            assert_rows_close(r.out.cpu().numpy(), want, rms, what=f"batch {dtype}")


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_batch_same_plan_twice(torch, dd, dtype):
    """One plan, two inputs of the same length in one batch: each item gets a workspace of its
    own, so statistics, candidates and (u8) the input-tail copy equal the single calls."""
    print(f"case: batch with one {dtype} plan twice", flush=True)
    freq = fbsynth.channel_freqs(428.0, 20.0 / 64, 64)
    dm = fbsynth.dm_trials(0.0, 0.1, 96)
    rng = np.random.default_rng(77)
    xs = []
    for _ in range(2):
        x = fbsynth.noise(rng, 64, 5000)
        xs.append(torch.from_numpy(fbsynth.to_u8(x) if dtype == "u8" else x).cuda())
    plan = dd.Plan(freq, 51.2e-6, dm, dtype=dtype, tuning=(8, 4))
    singles = [plan.dedisperse(x, k_sigma=3.0) for x in xs]
    torch.cuda.synchronize()
    single_out = [(s.out.cpu().numpy(), s.mean.cpu().numpy(), s.rms.cpu().numpy(), s.candidates()) for s in singles]
    batched = dd.batch_dedisperse([(plan, xs[0]), (plan, xs[1])], k_sigma=3.0)
    torch.cuda.synchronize()
    for (o, m, r, c), b in zip(single_out, batched):
        np.testing.assert_array_equal(b.out.cpu().numpy(), o)
        np.testing.assert_array_equal(b.mean.cpu().numpy(), m)
        np.testing.assert_array_equal(b.rms.cpu().numpy(), r)
        np.testing.assert_array_equal(b.candidates(), c)


def test_batch_rejects_shared_workspace(torch, dd):
    """The C ABI refuses two items whose workspaces overlap."""
    import ctypes as C
    from paper_1401_8258_amd import _lib
    freq = fbsynth.channel_freqs(428.0, 20.0 / 64, 64)
    dm = fbsynth.dm_trials(0.0, 0.1, 96)
    plan = dd.Plan(freq, 51.2e-6, dm, tuning=(8, 4))
    x = torch.zeros((64, 3000), device="cuda")
    ws = plan.workspace(3000)
    out = torch.empty((96, 3000), device="cuda")
    items = (_lib.BatchItem * 2)()
    for it in items:
        it.plan = plan.handle.value
        it.d_in = x.data_ptr()
        it.nsamp = 3000
        it.in_row_stride = 3000
        it.d_out = out.data_ptr()
        it.out_row_stride = 3000
        it.d_plan_workspace = ws.data_ptr()
    bws = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    lib = _lib.load()
    rc = lib.dd_batch_dedisperse(items, 2, C.c_void_p(bws.data_ptr()), bws.numel(),
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == _lib.DD_ERR_INVALID_ARG
    assert "share workspace" in lib.dd_last_error().decode()


def test_batch_mixes_every_kernel_shape(torch, dd):
    """One batched call over items on every kernel shape: FP32 with 8 and with 4 trials per
    computing wavefront beside producers, FP32 without producers, FP16, 8-bit in the LDS form
    and 8-bit in the direct-read form at two tile shapes and wavefront counts. Each shape
    gets its own launch; every item equals its single call bit for bit (outputs, statistics,
    candidates) and the oracle."""
    print("case: batch mixing every kernel shape", flush=True)
    nchan, ndm, nsamp = 64, 128, 6000
    freq = fbsynth.channel_freqs(428.0, 20.0 / nchan, nchan)
    dm = fbsynth.dm_trials(0.0, 0.1, ndm)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    rng = np.random.default_rng(31)
    x32 = fbsynth.noise(rng, nchan, nsamp)
    inputs = {"f32": x32, "f16": fbsynth.to_f16(x32), "u8": fbsynth.to_u8(x32)}
    cases = [("f32", (8, 6, 0, 2), "lds"), ("f32", (4, 14, 0, 2), "lds"), ("f32", (8, 4, 0, -1), "lds"),
             ("f16", (8, 2), "lds"), ("u8", (8, 4), "lds"), ("u8", (2, 4, 16), "direct"),
             ("u8", (1, 8, 32), "direct")]
    jobs = []
    for dtype, tun, form in cases:
        p = dd.Plan(freq, 51.2e-6, dm, dtype=dtype, tuning=tun, form=form)
        assert p.form == form, (dtype, tun, p.form)
        jobs.append((p, torch.from_numpy(np.ascontiguousarray(inputs[dtype])).cuda()))
    assert jobs[0][0].tiles[:2] == (8, 6) and jobs[1][0].tiles[:2] == (4, 14)
    assert jobs[0][0].producer_waves == 2 and jobs[2][0].producer_waves == 0
    res = dd.batch_dedisperse(jobs, k_sigma=4.0)
    torch.cuda.synchronize()
    rows = [0, 57, ndm - 1]
    for (dtype, tun, form), (p, x), r in zip(cases, jobs, res):
        s = p.dedisperse(x, k_sigma=4.0)
        torch.cuda.synchronize()
        got = r.out.cpu().numpy()
        np.testing.assert_array_equal(s.out.cpu().numpy(), got)
        np.testing.assert_array_equal(s.mean.cpu().numpy(), r.mean.cpu().numpy())
        np.testing.assert_array_equal(s.rms.cpu().numpy(), r.rms.cpu().numpy())
        np.testing.assert_array_equal(s.candidates(), r.candidates())
        want = orc.dedisperse(inputs[dtype].astype(np.float64), tab, rows=rows)
        if dtype == "u8":
            np.testing.assert_array_equal(got[rows].astype(np.float64), want)
        else:
            full = orc.dedisperse(inputs[dtype].astype(np.float64), tab)
            _, rms = orc.series_stats(full)
            assert_rows_close(got, full, rms, what=f"batch {dtype} {tun}")


@pytest.mark.parametrize("tuning", [(4, 14, 0, 2), (8, 4, 0, -1)])
def test_batch_short_window_many_groups(torch, dd, tuning):
    """An item with two time tiles and many DM groups (its units spread over the XCDs by DM
    group) beside one with many tiles (spread by tile), in one launch: both equal their
    single calls bit for bit, and the oracle."""
    print(f"case: batch, short window over many DM groups, tuning {tuning}", flush=True)
    nchan, ndm = 64, 700
    freq = fbsynth.channel_freqs(428.0, 20.0 / nchan, nchan)
    dm = fbsynth.dm_trials(0.0, 0.05, ndm)
    tab = orc.delay_table(freq, dm, 51.2e-6)
    plan = dd.Plan(freq, 51.2e-6, dm, tuning=tuning)
    rng = np.random.default_rng(41)
    xs = [fbsynth.noise(rng, nchan, plan.maxdelay + n) for n in (700, 40000)]
    jobs = [(plan, torch.from_numpy(x).cuda()) for x in xs]
    res = dd.batch_dedisperse(jobs, k_sigma=4.0)
    torch.cuda.synchronize()
    for (p, x), r, xh in zip(jobs, res, xs):
        s = p.dedisperse(x, k_sigma=4.0)
        torch.cuda.synchronize()
        got = r.out.cpu().numpy()
        np.testing.assert_array_equal(s.out.cpu().numpy(), got)
        np.testing.assert_array_equal(s.mean.cpu().numpy(), r.mean.cpu().numpy())
        np.testing.assert_array_equal(s.rms.cpu().numpy(), r.rms.cpu().numpy())
        np.testing.assert_array_equal(s.candidates(), r.candidates())
        rows = list(range(0, ndm, 97)) + [ndm - 1]
        want = orc.dedisperse(xh, tab, rows=rows)
        rms = np.sqrt(np.mean((want - want.mean(axis=1, keepdims=True)) ** 2, axis=1))
        assert_rows_close(got[rows], want, rms, what=f"batch short window {tuning}")
