"""Serving on the device: continuous batching of streaming beams through the library.

Each block result that the server produces in a mixed batch must equal, bit for bit,
the result of pushing the same blocks through the beam's own stream alone; one beam is
also checked against the oracle (u8 codes sum exactly).
"""
import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc
from paper_1401_8258_amd import serve
from tests.gpu_util import cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return cuda()


def _specs():
    # (name, nchan, channel width MHz, ndm, DM step, block): uneven beams, u8 storage
    shapes = [("a", 64, 0.3125, 96, 0.1, 2048), ("b", 128, 0.15625, 64, 0.2, 1500),
              ("c", 32, 0.625, 40, 0.3, 3000)]
    out = []
    for name, nchan, df, ndm, step, block in shapes:
        out.append(serve.BeamSpec(name, fbsynth.channel_freqs(428.0, df, nchan), 51.2e-6,
                                  fbsynth.dm_trials(0.0, step, ndm), "u8", block, k_sigma=6.0))
    return out


def _blocks(spec, nblocks, seed):
    rng = np.random.default_rng(seed)
    x = fbsynth.to_u8(fbsynth.noise(rng, len(spec.freq_mhz), spec.block * nblocks))
    return [np.ascontiguousarray(x[:, k * spec.block:(k + 1) * spec.block]) for k in range(nblocks)]


def test_server_results_equal_alone_and_oracle(torch):
    import paper_1401_8258_amd as dd
    dd.load_library()
    specs = _specs()
    nblocks = 4
    host = [_blocks(sp, nblocks, 100 + i) for i, sp in enumerate(specs)]
    dev = [[torch.from_numpy(b).cuda() for b in bs] for bs in host]

    # alone: each beam through its own stream, block by block
    alone = {}
    for i, sp in enumerate(specs):
        plan = dd.Plan(sp.freq_mhz, sp.tsamp_s, sp.dm, dtype="u8")
        st = dd.Stream(plan, sp.block)
        for k, x in enumerate(dev[i]):
            r = st.push(x, k_sigma=sp.k_sigma)
            if r is not None:
                alone[(i, k)] = (r.t0, r.out.cpu().numpy(), r.mean.cpu().numpy(), r.rms.cpu().numpy(),
                                 r.candidates())
    torch.cuda.synchronize()

    # mixed: the server batches whatever has arrived across beams
    print("case: server over 3 uneven u8 beams, 4 blocks each", flush=True)
    ex = serve.LibraryExecutor(k_sigma=6.0, keep=True)
    srv = serve.Server(specs, ex, hbm_budget=1 << 40, max_inflight=2)
    for i in range(len(specs)):
        assert srv.request(i) == "admitted"
    sched = serve.poisson_schedule(specs, nblocks, seed=7, jitter_mean_s=0.01, phases=[0.0, 0.001, 0.002],
                                   make_data=lambda i, k: dev[i][k], time_scale=0.02)
    stats = srv.run(sched)
    torch.cuda.synchronize()
    assert stats.blocks == len(specs) * nblocks
    assert max(stats.batch_sizes) > 1, "no two beams were ever batched"
    assert set(ex.kept) == set(alone)
    for key, (t0, out, mean, rms, cand) in alone.items():
        got = ex.kept[key]
        assert got["t0"] == t0
        np.testing.assert_array_equal(got["out"].cpu().numpy(), out)
        np.testing.assert_array_equal(got["mean"].cpu().numpy(), mean)
        np.testing.assert_array_equal(got["rms"].cpu().numpy(), rms)
        np.testing.assert_array_equal(got["cand"], cand)
    # the counts the server reports (read from pinned copies taken before each launch's event)
    reported = {(br.beam, br.seq): br.ncand for br in srv.results if not br.filling}
    assert reported == {key: int(v[4].size) for key, v in alone.items()}

    # beam 0 against the oracle on the concatenated blocks
    sp = specs[0]
    tab = orc.delay_table(sp.freq_mhz, sp.dm, sp.tsamp_s)
    exp = orc.stream_expected(host[0], tab)
    for k, (t0, t1, want) in enumerate(exp):
        if t1 <= t0:
            assert (0, k) not in ex.kept
            continue
        got = ex.kept[(0, k)]
        assert got["t0"] == t0
        np.testing.assert_array_equal(got["out"].cpu().numpy().astype(np.float64), want)


def test_footprint_and_admission(torch):
    import paper_1401_8258_amd as dd
    dd.load_library()
    specs = _specs()
    ex = serve.LibraryExecutor(k_sigma=6.0)
    fps = [ex.footprint(sp) for sp in specs]
    assert all(f > 0 for f in fps)
    # budget for the first two beams only: the third queues, a fourth request is rejected
    srv = serve.Server(specs + [specs[0]], ex, hbm_budget=fps[0] + fps[1], max_queue=1)
    assert srv.request(0) == "admitted"
    assert srv.request(1) == "admitted"
    assert srv.request(2) == "queued"
    assert srv.request(3) == "rejected"
    srv.release(0)
    assert 2 in srv.active or fps[2] > fps[0]


def test_queued_beam_admitted_mid_run_equals_alone(torch):
    import paper_1401_8258_amd as dd
    dd.load_library()
    specs = _specs()
    nblocks = 3
    host = [_blocks(sp, nblocks, 200 + i) for i, sp in enumerate(specs)]
    dev = [[torch.from_numpy(b).cuda() for b in bs] for bs in host]
    alone = {}
    for i, sp in enumerate(specs):
        st = dd.Stream(dd.Plan(sp.freq_mhz, sp.tsamp_s, sp.dm, dtype="u8"), sp.block)
        for k, x in enumerate(dev[i]):
            r = st.push(x, k_sigma=sp.k_sigma)
            if r is not None:
                alone[(i, k)] = r.out.cpu().numpy()
    torch.cuda.synchronize()
    print("case: beam 2 queued by the HBM budget, admitted when beam 0 finishes", flush=True)
    ex = serve.LibraryExecutor(k_sigma=6.0, keep=True)
    fps = [ex.footprint(sp) for sp in specs]
    srv = serve.Server(specs, ex, hbm_budget=fps[0] + fps[1] + min(fps[2] - 1, fps[0] - 1), max_inflight=2)
    assert [srv.request(i) for i in range(3)] == ["admitted", "admitted", "queued"]
    # beam 0 gets one block, so it finishes first and frees its memory for beam 2
    sched = [b for b in serve.poisson_schedule(specs, nblocks, seed=9, jitter_mean_s=0.01,
                                               phases=[0.0, 0.001, 0.002],
                                               make_data=lambda i, k: dev[i][k], time_scale=0.02)
             if not (b.beam == 0 and b.seq > 0)]
    st = srv.run(sched, release_done=True)
    torch.cuda.synchronize()
    assert st.admitted_in_run == 1 and not srv.active
    want = {key: v for key, v in alone.items() if not (key[0] == 0 and key[1] > 0)}
    assert set(ex.kept) == set(want)
    for key, out in want.items():
        np.testing.assert_array_equal(ex.kept[key]["out"].cpu().numpy(), out)


def test_server_with_a_binned_beam_equals_alone(torch):
    """A beam with time binning (BinnedStream: one ring per run at its binned sampling time)
    served beside two plain beams: per block, its runs' outputs, statistics and merged
    candidates equal those of its own BinnedStream pushed alone, and its footprint is its
    binned ring and workspace plus two output sets."""
    import paper_1401_8258_amd as dd
    dd.load_library()
    specs = _specs()[:2] + [serve.BeamSpec("binned", fbsynth.channel_freqs(428.0, 0.3125, 64), 51.2e-6,
                                           fbsynth.dm_trials(0.0, 0.1, 128), "u8", 1024, k_sigma=6.0,
                                           max_log2=4)]
    nblocks = 4
    host = [_blocks(sp, nblocks, 300 + i) for i, sp in enumerate(specs)]
    dev = [[torch.from_numpy(b).cuda() for b in bs] for bs in host]
    sp = specs[2]
    bp = dd.BinnedPlan(sp.freq_mhz, sp.tsamp_s, sp.dm, dtype="u8", max_log2=4)
    assert len(bp.segments) == 5
    st = dd.BinnedStream(bp, sp.block)
    alone = {}
    for k, x in enumerate(dev[2]):
        r = st.push(x, k_sigma=6.0)
        if r is not None:
            alone[k] = ([(t0, None if x is None else (x.out.cpu().numpy(), x.mean.cpu().numpy(),
                                                      x.rms.cpu().numpy())) for _, t0, x in r.segments],
                        r.candidates())
    torch.cuda.synchronize()
    assert alone
    print("case: server with a binned beam beside two plain u8 beams", flush=True)
    ex = serve.LibraryExecutor(k_sigma=6.0, keep=True)
    ring, ws = bp.stream_sizes(sp.block)
    outs = 128 * sp.block * 4 + 2 * 128 * 4 + ex.cand_cap * 24 + 8
    assert ex.footprint(sp) == ring + ws + 2 * outs
    srv = serve.Server(specs, ex, hbm_budget=1 << 40, max_inflight=2)
    assert [srv.request(i) for i in range(3)] == ["admitted"] * 3
    sched = serve.poisson_schedule(specs, nblocks, seed=11, jitter_mean_s=0.01, phases=[0.0, 0.001, 0.002],
                                   make_data=lambda i, k: dev[i][k], time_scale=0.02)
    stats = srv.run(sched)
    torch.cuda.synchronize()
    assert stats.blocks == 3 * nblocks
    got = {k: v for (i, k), v in ex.kept.items() if i == 2}
    assert set(got) == set(alone)
    for k, (runs, cand) in alone.items():
        g = got[k]
        assert [t0 for t0, _, _, _ in g["runs"]] == [t0 for t0, _ in runs]
        for (t0, o, m, r), (_, want) in zip(g["runs"], runs):
            assert (o is None) == (want is None)
            if want is not None:
                np.testing.assert_array_equal(o.cpu().numpy(), want[0])
                np.testing.assert_array_equal(m.cpu().numpy(), want[1])
                np.testing.assert_array_equal(r.cpu().numpy(), want[2])
        np.testing.assert_array_equal(g["cand"], cand)
