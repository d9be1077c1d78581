"""Benchmark: brute-force dedispersion of the full-size FP32 workload on one MI355X.

Workload: 1024 channels over 408-428 MHz, 51.2 us sampling, 2^20 samples of N(0,1)
noise with 20 dispersed boxcars, 2048 DM trials 0-204.7 step 0.1; output FP32
plus per-DM mean/RMS and candidates above 6 sigma. Inputs are resident in HBM
before timing starts. One step = one dd_dedisperse call (dedispersion kernel,
statistics and candidate kernels).

Prints one JSON line: the whole-step throughput in DM-trial*samples/s, the
dedispersion kernel's own duration against the published FP32 vector peak (and the
add issue rate), the FP64 oracle timed on a bounded sample of the same workload on
the host (one core and all cores), the 16-beam u8 batch (config 4: batched against
one at a time) and the 64-beam u8 serving run (config 5).
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 2.4 GHz. The published FP32 vector peak of 157.3 TFLOP/s counts a
# fused multiply-add as two flops on 128 lanes/clk/CU (256 x 2.4e9 x 128 x 2). A plain add
# is one flop per lane, so the add issue rate is half of it, 256 x 2.4e9 x 128 = 78.6e12
# adds/s (v_add_f32 issues at ~118 lanes/clk/CU measured). The roofline reports achieved
# adds/s against the published peak; the add-rate fraction is printed beside it.
PEAK_FP32_TFLOPS = 157.3
PEAK_ADD_TFLOPS = 256 * 2.4e9 * 128 / 1e12
# The kernel's own ceiling: every add consumes one 4-byte LDS word, and ds_read_b128
# delivers ~221 B/clk/CU, so at most 256 x 2.4e9 x 221 / 4 = 33.9e12 adds/s.
LDS_CEILING_TADDS = 256 * 2.4e9 * 221 / 4 / 1e12
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dedisp_tile_full_fp32_1024ch_2048dm_traffic.json")
_CSRC = os.path.join(ROOT, "paper_1401_8258_amd", "csrc")
# what the LDS-form kernel's counters depend on: its device code (and the launch geometry,
# compared separately)
KERNEL_SOURCES = [os.path.join(_CSRC, f) for f in ("dedisp.hip", "dd_device.h")]
GEOMETRY_KEYS = ("dms_per_wave", "waves", "producer_waves", "launch_buf", "launch_stage", "launch_ring",
                 "launch_lds")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-rows", type=int, default=12, help="DM rows in the oracle sample")
    ap.add_argument("--tuning", type=str, default=None, help="dms_per_wave,waves[,chan_stage] tile override")
    ap.add_argument("--traffic", type=str, default=TRAFFIC_FILE,
                    help="JSON with measured HBM fetch/write bytes per launch of the dedispersion kernel "
                         "(used only while the kernel source is the one it was measured on)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain device copy of the input (known bytes) to calibrate HBM counters")
    ap.add_argument("--mode", choices=("plain", "batch", "serve", "subband", "u8beam", "binstream"), default="plain",
                    help="plain: the full-size FP32 workload (default); batch: 16 uneven u8 beams in one "
                         "batched call; serve: 64 streaming u8 beams with continuous batching; "
                         "subband: only the subband passes over the full-size FP32 workload; u8beam: the "
                         "largest 4096-channel u8 beam of the batch in its default (direct-read) plan "
                         "(both for profiling); binstream: a 4096-channel serving beam streamed plain and "
                         "with time binning")
    ap.add_argument("--serve-blocks", type=int, default=60,
                    help="1 s blocks per beam after the ring fill in the serving run (plain mode appends a "
                         "serving summary when > 0)")
    ap.add_argument("--batch-reps", type=int, default=3,
                    help="timed repetitions of the config-4 batch (plain mode appends it when > 0)")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="processes of the all-core oracle leg (at most the host's cores)")
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0, help="serving admission budget")
    return ap.parse_args()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ORC = {}


def _oracle_rows(rows):
    """One worker's share of the all-core leg (the beam and delay table come by fork)."""
    from oracle import dedisp_oracle as orc
    out = orc.dedisperse(_ORC["data"], _ORC["tab"], rows=rows)
    orc.series_stats(out)
    return out.shape[0] * out.shape[1]


def cpu_baseline(beam, rows, workers):
    """The FP64 oracle on the host: evenly spaced DM rows on one core, then on `workers`
    processes (fork, the input shared copy-on-write) with `rows` rows each."""
    import multiprocessing as mp

    from oracle import dedisp_oracle as orc
    tab = orc.delay_table(beam.freq_mhz, beam.dm, beam.tsamp_s)
    sel = [int(r) for r in np.linspace(0, beam.ndm - 1, rows)]
    t = time.perf_counter()
    out = orc.dedisperse(beam.data, tab, rows=sel)
    orc.series_stats(out)
    dt = time.perf_counter() - t
    nout = out.shape[1]
    one = {"value": len(sel) * nout / dt, "unit": "DM-trial*samples/s", "cores": 1, "kind": "oracle",
           "sample": f"{len(sel)} of {beam.ndm} DM rows (evenly spaced) x {nout} output samples x "
                     f"{beam.nchan} channels, FP64 NumPy, single thread; {dt:.1f} s"}
    ncpu = os.cpu_count() or 1
    nw = max(1, min(workers, ncpu))
    res = dict(one)
    res["single_core"] = dict(one)
    res["cpu_model"] = _cpu_model()
    res["host_cpus"] = ncpu
    if nw > 1:
        _ORC["data"], _ORC["tab"] = beam.data, tab
        allrows = [int(r) for r in np.linspace(0, beam.ndm - 1, nw * rows)]
        shares = [allrows[i::nw] for i in range(nw)]
        ctx = mp.get_context("fork")
        t = time.perf_counter()
        with ctx.Pool(nw) as pool:
            done = sum(pool.map(_oracle_rows, shares))
        dt_all = time.perf_counter() - t
        res.update({"value": done / dt_all, "cores": nw,
                    "sample": f"{nw * rows} of {beam.ndm} DM rows (evenly spaced) x {nout} output samples x "
                              f"{beam.nchan} channels, FP64 NumPy, {nw} processes x 1 thread; {dt_all:.1f} s"})
    return res


def serve_run(nblocks, budget_bytes, seed=5):
    """Config-5 serving: 48 x 1024-ch and 16 x 4096-ch u8 beams, 1 s blocks, Poisson arrival
    jitter, rings prefilled past their fill, then real-time arrivals for nblocks blocks."""
    import torch

    import fbsynth
    from paper_1401_8258_amd import serve

    specs5 = fbsynth.config5_specs(seed=seed)
    specs = [serve.BeamSpec(sp["name"], fbsynth.channel_freqs(sp["f_top"], sp["bw"] / sp["nchan"], sp["nchan"]),
                            sp["tsamp"], fbsynth.dm_trials(sp["dm0"], sp["step"], sp["ndm"]), "u8", sp["block"],
                            k_sigma=6.0) for sp in specs5]
    ex = serve.LibraryExecutor(k_sigma=6.0, cand_cap=1 << 14)
    srv = serve.Server(specs, ex, hbm_budget=budget_bytes, max_inflight=2)
    admitted = [i for i in range(len(specs)) if srv.request(i) == "admitted"]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    pool = {}
    for sp in specs:
        key = (len(sp.freq_mhz), sp.block)
        if key not in pool:  # N(128, 16) codes, three distinct blocks per shape
            pool[key] = [torch.clamp(torch.round(128.0 + 16.0 * torch.randn(key, generator=g, device="cuda")),
                                     0, 255).to(torch.uint8) for _ in range(3)]
    nfill = {}
    for i in admitted:
        sp = specs[i]
        nf = ex.plan(sp).maxdelay // sp.block  # blocks after which the ring still holds <= maxdelay samples
        key = (len(sp.freq_mhz), sp.block)
        ex.prefill(i, [pool[key][k % 3] for k in range(nf)])
        nfill[i] = nf
    torch.cuda.synchronize()
    sched = serve.poisson_schedule(specs, nblocks, seed=seed, jitter_mean_s=0.1,
                                   phases=[sp["phase_s"] for sp in specs5],
                                   make_data=lambda i, k: pool[(len(specs[i].freq_mhz), specs[i].block)][
                                       (nfill.get(i, 0) + k) % 3])
    sched = [b for b in sched if b.beam in srv.active]
    st = srv.run(sched)
    out = st.summary()
    out["batch_vs_single"] = _serve_batch_vs_single(ex, specs, admitted, pool, nfill, nblocks)
    out.update({"beams": len(specs), "blocks_per_beam": nblocks,
                "workload": "48 x 1024-ch (408-428 MHz, 51.2 us, 2048 DMs) + 16 x 4096-ch (120-180 MHz, "
                            "81.92 us, 4096 DMs step 0.05) u8 beams, 1 s blocks, Poisson arrival jitter "
                            "(mean 0.1 s), rings prefilled", "hbm_budget_gb": budget_bytes / 1e9})
    return out


def _serve_batch_vs_single(ex, specs, beams, pool, nfill, nblocks, rounds=3):
    """After the serving run: every admitted beam's next 1 s block, all of them in one
    batched call (ring appends, then one dedispersion launch and one launch per statistics /
    candidate step), against the same blocks pushed one beam at a time; device time per
    round of blocks, alternating the two ways."""
    import torch

    from paper_1401_8258_amd import api
    streams = {i: ex._beams[i]["stream"] for i in beams}
    outs = {i: api.alloc_outputs(streams[i].plan.ndm, specs[i].block, ex.device, ex.k_sigma, ex.cand_cap)
            for i in beams}
    seqk = {i: nfill.get(i, 0) + nblocks for i in beams}

    def block(i):
        sp = specs[i]
        b = pool[(len(sp.freq_mhz), sp.block)][seqk[i] % 3]
        seqk[i] += 1
        return b

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms_b, ms_s = [], []
    for _ in range(rounds):
        torch.cuda.synchronize()
        e0.record(ex.stream)
        jobs, o = [], []
        for i in beams:
            w = streams[i].append(block(i), stream=ex.stream)
            jobs.append((streams[i], w))
            o.append(outs[i])
        api.batch_dedisperse(jobs, k_sigma=ex.k_sigma, cand_cap=ex.cand_cap, stream=ex.stream, outputs=o)
        e1.record(ex.stream)
        torch.cuda.synchronize()
        ms_b.append(e0.elapsed_time(e1))
        e0.record(ex.stream)
        for i in beams:
            w = streams[i].append(block(i), stream=ex.stream)
            api.batch_dedisperse([(streams[i], w)], k_sigma=ex.k_sigma, cand_cap=ex.cand_cap, stream=ex.stream,
                                 outputs=[outs[i]])
        e1.record(ex.stream)
        torch.cuda.synchronize()
        ms_s.append(e0.elapsed_time(e1))
    return {"beams": len(beams), "rounds": rounds, "batched_ms": round(float(np.median(ms_b)), 3),
            "one_at_a_time_ms": round(float(np.median(ms_s)), 3),
            "batched_speedup": round(float(np.median(ms_s)) / float(np.median(ms_b)), 3)}


def batch_run(reps):
    """Config-4 batch: 16 uneven u8 beams (N(128,16) codes drawn on the device) with
    direct-read tiles from the autotuner (each beam's own best) in one batched call (one
    launch per distinct tile shape and wavefront count, then one launch per
    statistics/candidate step for all beams), against each beam alone on the same tiles."""
    import torch

    import fbsynth
    import paper_1401_8258_amd as dd
    from paper_1401_8258_amd import autotune

    specs = fbsynth.config4_specs()
    beams, xs = [], []
    for i, sp in enumerate(specs):
        freq = fbsynth.channel_freqs(sp["f_top"], sp["bw"] / sp["nchan"], sp["nchan"])
        dms = fbsynth.dm_trials(sp["dm0"], sp["step"], sp["ndm"])
        beams.append((freq, sp["tsamp"], dms, "u8", sp["nsamp"]))
        xs.append(autotune.synthetic_input(sp["nchan"], sp["nsamp"], "u8", seed=i))
    t_tune = time.perf_counter()
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    tb = autotune.tune_batch(beams, waves=(8, 4, 2, 1), stages=(0,), reps=1, inputs=xs, log=log,
                             forms=("direct",))
    t_tune = time.perf_counter() - t_tune
    # each beam's own best tiles over all wavefront counts, batched and one at a time
    plans = [autotune.make_plan(f, ts, dm, "u8", c) for (f, ts, dm, _, _), c in zip(beams, tb["choices"])]
    outs = [dd.api.alloc_outputs(p.ndm, x.shape[1] - p.maxdelay, x.device, 6.0, 1 << 16) for p, x in zip(plans, xs)]
    jobs = list(zip(plans, xs))
    for p, x in jobs:  # workspaces allocated before timing
        p.workspace(x.shape[1], x.device)

    def batched():
        dd.batch_dedisperse(jobs, k_sigma=6.0, cand_cap=1 << 16, outputs=outs)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_batch = timed(batched)
    # each beam alone with its own best tiles, timed one by one
    per_beam = []
    for p, x, o in zip(plans, xs, outs):
        ms = timed(lambda: dd.batch_dedisperse([(p, x)], k_sigma=6.0, cand_cap=1 << 16, outputs=[o]))
        nout = x.shape[1] - p.maxdelay
        per_beam.append({"nchan": p.nchan, "ndm": p.ndm, "nout": nout, "form": p.form, "tiles": list(p.tiles[:2]),
                         "ms": round(ms, 3), "adds_per_s": p.ndm * p.nchan * nout / (ms * 1e-3)})
    ms_single = sum(b["ms"] for b in per_beam)
    trials_samples = sum(p.ndm * (x.shape[1] - p.maxdelay) for p, x in jobs)
    adds = sum(p.ndm * p.nchan * (x.shape[1] - p.maxdelay) for p, x in jobs)
    return {"metric": "DM-trial*samples/s", "value": trials_samples / (ms_batch * 1e-3),
            "unit": "DM-trial*samples/s", "n_gpus": 1, "steps": reps, "ms_per_step": round(ms_batch, 3),
            "higher_is_better": True, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "16 uneven u8 beams (nchan 256/512/1024/4096, 500-4096 DMs, nsamp 2^16-2^19), "
                                   "batched, stats + 6-sigma candidates",
                       "tunings": tb["choices"],
                       "kernel_launches": len({(c["form"], tuple(c["tuning"])) for c in tb["choices"]}),
                       "tune_s": round(t_tune, 1)},
            "adds_per_s": adds / (ms_batch * 1e-3),
            "one_at_a_time_ms": round(ms_single, 3),
            "batched_speedup": round(ms_single / ms_batch, 3),
            "per_beam_alone": per_beam}


def binned_stream_run(nblocks):
    """One 4096-channel serving beam (120-180 MHz, 81.92 us, 4096 u8 DMs step 0.05, maxdelay
    ~400k samples) streamed in blocks of 12208 samples (1.0001 s, a multiple of 16): a plain
    stream against a time-binned one (factors up to 16, one ring per run at its binned
    sampling time). Both are filled first; then the device time of nblocks pushes (ring
    appends, dedispersion, statistics and 6-sigma candidates) by HIP events, and the ring
    bytes each keeps."""
    import torch

    import fbsynth
    import paper_1401_8258_amd as dd
    from paper_1401_8258_amd import api

    sp = fbsynth.config5_specs()[48]
    assert sp["nchan"] == 4096
    freq = fbsynth.channel_freqs(sp["f_top"], sp["bw"] / sp["nchan"], sp["nchan"])
    dms = fbsynth.dm_trials(sp["dm0"], sp["step"], sp["ndm"])
    block = 12208
    g = torch.Generator(device="cuda")
    g.manual_seed(9)
    pool = [torch.clamp(torch.round(128.0 + 16.0 * torch.randn((sp["nchan"], block), generator=g, device="cuda")),
                        0, 255).to(torch.uint8) for _ in range(3)]
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {"workload": f"u8 beam: 4096 ch 120-180 MHz, tsamp 81.92 us, {sp['ndm']} DMs step {sp['step']}, "
                       f"blocks of {block} samples, stats + 6-sigma candidates", "blocks_timed": nblocks}
    plan = dd.Plan(freq, sp["tsamp"], dms, dtype="u8")
    st = dd.Stream(plan, block)
    nf = plan.maxdelay // block
    for k in range(nf):
        st.append(pool[k % 3])
    out = api.alloc_outputs(plan.ndm, block, "cuda", 6.0, 1 << 16)
    torch.cuda.synchronize()
    e0.record(stream)
    for k in range(nblocks):
        w = st.append(pool[(nf + k) % 3])
        dd.batch_dedisperse([(st, w)], k_sigma=6.0, cand_cap=1 << 16, outputs=[out])
    e1.record(stream)
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1) / nblocks
    res["plain"] = {"ring_bytes": int(st.ring.numel()), "maxdelay": plan.maxdelay, "form": plan.form,
                    "ms_per_block": round(ms_plain, 3), "adds_per_block": plan.ndm * plan.nchan * block}
    del st
    torch.cuda.empty_cache()
    bp = dd.BinnedPlan(freq, sp["tsamp"], dms, dtype="u8", max_log2=4)
    bs = dd.BinnedStream(bp, block)
    outs = api.alloc_outputs(bp.dm.size, block, "cuda", 6.0, 1 << 16)
    nfb = -(-bp.fill_nsamp // block)
    for k in range(nfb):
        bs.push(pool[k % 3], stats=False)
    torch.cuda.synchronize()
    ms_by = {}
    for batched in (False, True) if bp.batchable else (False,):  # the runs one launch each, then batched
        e0.record(stream)
        for k in range(nblocks):
            r = bs.push(pool[(nfb + k) % 3], k_sigma=6.0, outputs=outs, batched=batched)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_by[batched] = e0.elapsed_time(e1) / nblocks
        assert r is not None and all(x is not None for _, _, x in r.segments)
    ms_b = min(ms_by.values())
    adds_b = sum((sg.d1 - sg.d0) * bp.freq.size * (block >> sg.log2) for sg in bp.segments)
    res["binned"] = {"ring_bytes": bs.ring_bytes, "max_log2": 4, "dm_diag": round(bp.dm_diag, 4),
                     "runs": [{"factor": 1 << sg.log2, "ndm": sg.d1 - sg.d0, "maxdelay": sg.plan.maxdelay,
                               "form": sg.plan.form} for sg in bp.segments],
                     "ms_per_block": round(ms_b, 3), "ms_per_block_unbatched": round(ms_by[False], 3),
                     "ms_per_block_batched": round(ms_by[True], 3) if True in ms_by else None,
                     "adds_per_block": adds_b}
    res["ring_bytes_ratio"] = round(res["plain"]["ring_bytes"] / bs.ring_bytes, 2)
    res["speedup_per_block"] = round(ms_plain / ms_b, 3)
    res["block_s"] = block * sp["tsamp"]
    del bs
    torch.cuda.empty_cache()
    return res


def u8beam_run(steps, warmup):
    """The 4096-channel 120-180 MHz u8 beam of config 4 with the most work, default plan
    (direct-read form): kernel-only launches (no statistics), then whole steps."""
    import torch

    import fbsynth
    import paper_1401_8258_amd as dd
    from paper_1401_8258_amd import autotune

    specs = [sp for sp in fbsynth.config4_specs() if sp["nchan"] == 4096]
    sp = max(specs, key=lambda s: s["ndm"] * s["nsamp"])
    freq = fbsynth.channel_freqs(sp["f_top"], sp["bw"] / sp["nchan"], sp["nchan"])
    dms = fbsynth.dm_trials(sp["dm0"], sp["step"], sp["ndm"])
    x = autotune.synthetic_input(sp["nchan"], sp["nsamp"], "u8", seed=3)
    plan = dd.Plan(freq, sp["tsamp"], dms, dtype="u8")
    nout = sp["nsamp"] - plan.maxdelay
    out = torch.empty((plan.ndm, nout), dtype=torch.float32, device="cuda")
    ws = plan.workspace(sp["nsamp"])
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for stats in (False, True):
        for _ in range(warmup):
            plan.dedisperse(x, stats=stats, k_sigma=6.0 if stats else 0.0, out=out, workspace=ws)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            plan.dedisperse(x, stats=stats, k_sigma=6.0 if stats else 0.0, out=out, workspace=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        res["step_ms" if stats else "prep_and_kernel_ms"] = round(e0.elapsed_time(e1) / steps, 3)
    adds = plan.ndm * plan.nchan * nout
    return {"workload": f"u8 beam: {plan.nchan} ch 120-180 MHz, tsamp 81.92 us, nsamp {sp['nsamp']}, "
                        f"{plan.ndm} DMs step {sp['step']}, maxdelay {plan.maxdelay}",
            "form": plan.form, "tiles": list(plan.tiles[:2]), "nout": nout, "adds": adds,
            "adds_per_s_prep_and_kernel": adds / (res["prep_and_kernel_ms"] * 1e-3), **res}


def subband_run(dd, beam, steps, warmup):
    """Times the subband passes alone (32-channel subbands; 16 and 48 trials per nominal DM)
    over the full-size FP32 workload, with statistics and 6-sigma candidates."""
    import torch
    x = torch.from_numpy(beam.data).cuda()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    res = {"workload": "subband dedispersion, full size: FP32 1024 ch 408-428 MHz, tsamp 51.2 us, "
                       "nsamp 2^20, 2048 DMs 0-204.7 step 0.1, 32-channel subbands", "passes": []}
    for group in (16, 48):
        sp = dd.SubbandPlan(beam.freq_mhz, beam.tsamp_s, beam.dm, chans_per_sub=32, dms_per_group=group)
        for _ in range(max(warmup, 1)):
            sp.dedisperse(x, k_sigma=6.0, cand_cap=1 << 20)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            sp.dedisperse(x, k_sigma=6.0, cand_cap=1 << 20)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res["passes"].append({"dms_per_group": group, "ms": round(ms, 3), "steps": steps,
                              "launches": sp.launches})
        print(f"bench: subband groups of {group}: {ms:.3f} ms", file=sys.stderr, flush=True)
        del sp
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this path has no "
              "multi-GPU mode: beams are independent and would be spread across GPUs by the caller.",
              file=sys.stderr)
        sys.exit(2)
    global np
    import numpy as np
    import torch

    import fbsynth
    import paper_1401_8258_amd as dd
    from paper_1401_8258_amd import _lib

    dd.load_library()
    if args.mode == "batch":
        print(json.dumps(batch_run(args.steps)), flush=True)
        return
    if args.mode == "u8beam":
        print(json.dumps(u8beam_run(args.steps, args.warmup)), flush=True)
        return
    if args.mode == "binstream":
        print(json.dumps(binned_stream_run(max(args.steps, 1))), flush=True)
        return
    if args.mode == "serve":
        res = serve_run(max(args.serve_blocks, 1), int(args.hbm_budget_gb * 1e9))
        print(json.dumps({"metric": "blocks/s", "value": res["blocks_per_s"], "unit": "blocks/s", "n_gpus": 1,
                          "higher_is_better": True, "dtype": "u8", "data": "synthetic", "serving": res}),
              flush=True)
        return
    print("bench: generating workload", file=sys.stderr, flush=True)
    beam = fbsynth.config2()
    if args.mode == "subband":
        print(json.dumps(subband_run(dd, beam, args.steps, args.warmup)), flush=True)
        return
    tuning = tuple(int(v) for v in args.tuning.split(",")) if args.tuning else None
    plan = dd.Plan(beam.freq_mhz, beam.tsamp_s, beam.dm, tuning=tuning)
    x = torch.from_numpy(beam.data).cuda()
    nsamp = beam.nsamp
    nout = nsamp - plan.maxdelay
    out = torch.empty((beam.ndm, nout), dtype=torch.float32, device="cuda")
    ws = plan.workspace(nsamp)
    stream = torch.cuda.current_stream()
    st = C.c_void_p(stream.cuda_stream)
    lib = _lib.load()
    mean = torch.empty(beam.ndm, dtype=torch.float32, device="cuda")
    rms = torch.empty_like(mean)
    cap = 1 << 20
    cand = torch.empty(cap * 24, dtype=torch.uint8, device="cuda")
    ncand = torch.zeros(1, dtype=torch.int64, device="cuda")
    k = 6.0

    def vp(t):
        return C.c_void_p(t.data_ptr())

    def step(full=True):
        rc = lib.dd_dedisperse(plan.handle, vp(x), nsamp, nsamp, vp(out), nout,
                               vp(mean) if full else None, vp(rms) if full else None, k if full else 0.0,
                               vp(cand) if full else None, cap if full else 0, vp(ncand) if full else None,
                               vp(ws), ws.numel(), st)
        _lib.check(rc)

    print("bench: warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step(True)
    torch.cuda.synchronize()

    # whole steps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step(True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    n_found = int(ncand.item())

    # the dedispersion kernel alone (no statistics/candidates): the roofline's launch duration
    print("bench: kernel-only timing", file=sys.stderr, flush=True)
    e0.record(stream)
    for _ in range(args.steps):
        step(False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_kernel = e0.elapsed_time(e1) / args.steps

    adds = beam.ndm * beam.nchan * nout
    achieved = adds / (ms_kernel * 1e-3) / 1e12
    info = plan.query(nsamp)
    geometry = {k: int(info[k]) for k in GEOMETRY_KEYS}
    traffic, traffic_note = None, "no counter record"
    if args.traffic and os.path.exists(args.traffic):
        from paper_1401_8258_amd.profiling import source_digest
        with open(args.traffic) as f:
            rec = json.load(f)
        if rec.get("kernel_source_sha256") == source_digest(KERNEL_SOURCES) and rec.get("geometry") == geometry:
            traffic = rec["hbm_bytes_per_launch"]
            traffic_note = (f"FETCH_SIZE x {rec['fetch_scale']} + WRITE_SIZE x {rec['write_scale']} "
                            f"(copy-kernel calibration), {os.path.relpath(args.traffic, ROOT)}")
        else:
            traffic_note = "kernel changed since the counters were taken"
    algo_bytes = beam.nchan * nsamp * 4 + beam.ndm * nout * 4
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
            "traffic_note": traffic_note, "algorithmic_bytes": algo_bytes,
            "kernel": "dedisp_tile", "kernel_ms": round(ms_kernel, 3), "geometry": geometry,
            "achieved_note": "one FP32 add per (DM trial, channel, output sample) = one flop",
            "peak_note": "published FP32 vector peak: 256 CU x 2.4 GHz x 128 lanes x 2 (FMA)",
            "add_issue_rate": round(PEAK_ADD_TFLOPS, 2),
            "frac_of_add_issue_rate": round(achieved / PEAK_ADD_TFLOPS, 4),
            "add_issue_rate_note": "256 CU x 2.4 GHz x 128 lanes x 1 (an add is one flop per lane)",
            "frac_of_lds_ceiling": round(achieved / LDS_CEILING_TADDS, 4),
            "algorithmic_hbm_gbs": round(algo_bytes / (ms_kernel * 1e-3) / 1e9, 1)}

    # detrending and normalisation of the dedispersed series (Sec. 3.5, downstream of the
    # step and not part of it): an HBM-bound kernel reading the output twice and writing
    # it once; algorithmic bytes are one read and one write
    print("bench: detrend timing", file=sys.stderr, flush=True)
    _lib.check(lib.dd_detrend(vp(out), beam.ndm, nout, nout, 1, vp(rms), st))
    e0.record(stream)
    for _ in range(3):
        _lib.check(lib.dd_detrend(vp(out), beam.ndm, nout, nout, 1, vp(rms), st))
    e1.record(stream)
    torch.cuda.synchronize()
    ms_dt = e0.elapsed_time(e1) / 3
    dt_bytes = 2 * beam.ndm * nout * 4
    detrend = {"kernel": "detrend_rows", "ms": round(ms_dt, 3), "bound": "hbm", "unit": "GB/s",
               "achieved": round(dt_bytes / (ms_dt * 1e-3) / 1e9, 1), "peak": 8000.0,
               "frac": round(dt_bytes / (ms_dt * 1e-3) / 1e9 / 8000.0, 4), "algorithmic_bytes": dt_bytes,
               "bytes_moved": 3 * beam.ndm * nout * 4}

    # boxcar levels 0..6 of the normalised series (widths 1..64): one read of the series,
    # one write of all levels (level 0 included)
    print("bench: boxcar timing", file=sys.stderr, flush=True)
    offs = [0]
    for kk in range(7):
        offs.append(offs[-1] + (nout >> kk))
    bx = torch.empty((beam.ndm, offs[-1]), dtype=torch.float32, device=out.device)
    _lib.check(lib.dd_boxcar(vp(out), beam.ndm, nout, nout, 6, vp(bx), offs[-1], st))
    e0.record(stream)
    for _ in range(3):
        _lib.check(lib.dd_boxcar(vp(out), beam.ndm, nout, nout, 6, vp(bx), offs[-1], st))
    e1.record(stream)
    torch.cuda.synchronize()
    ms_bx = e0.elapsed_time(e1) / 3
    bx_bytes = beam.ndm * nout * 4 + beam.ndm * offs[-1] * 4
    boxcar = {"kernel": "boxcar_rows", "levels": 6, "ms": round(ms_bx, 3), "bound": "hbm", "unit": "GB/s",
              "achieved": round(bx_bytes / (ms_bx * 1e-3) / 1e9, 1), "peak": 8000.0,
              "frac": round(bx_bytes / (ms_bx * 1e-3) / 1e9 / 8000.0, 4), "algorithmic_bytes": bx_bytes}
    del bx

    # boxcar template matching at every start (widths 1..64) with 6.5-sigma detections and
    # their widths: a counting pass over the series and a writing pass over the segments
    # with detections
    print("bench: boxcar search timing", file=sys.stderr, flush=True)
    # the series as dedispersed (the detrend above normalised `out` in place): fresh output
    step(True)
    nws = C.c_int64()
    _lib.check(lib.dd_boxcar_search_workspace(beam.ndm, nout, C.byref(nws)))
    sws = torch.empty(int(nws.value), dtype=torch.uint8, device=out.device)
    pcap = 1 << 22
    pulses = torch.empty(pcap * 24, dtype=torch.uint8, device=out.device)
    npulse = torch.zeros(1, dtype=torch.int64, device=out.device)

    def search():
        _lib.check(lib.dd_boxcar_search(vp(out), beam.ndm, nout, nout, vp(mean), vp(rms), 6, 6.5, vp(pulses), pcap,
                                        vp(npulse), vp(sws), sws.numel(), st))
    search()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(3):
        search()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_bs = e0.elapsed_time(e1) / 3
    # algorithmic bytes: one read of the series and the detections written (the counting
    # pass reads every segment, the writing pass again only the segments with detections)
    bs_bytes = beam.ndm * nout * 4 + int(npulse.item()) * 24
    boxcar_search = {"kernels": "boxcar_count + count scan (3 launches) + boxcar_write", "max_width": 64, "k_sigma": 6.5,
                     "ms": round(ms_bs, 3), "bound": "hbm", "unit": "GB/s",
                     "achieved": round(bs_bytes / (ms_bs * 1e-3) / 1e9, 1), "peak": 8000.0,
                     "frac": round(bs_bytes / (ms_bs * 1e-3) / 1e9 / 8000.0, 4),
                     "algorithmic_bytes": bs_bytes, "detections": int(npulse.item())}
    del pulses, sws

    # time binning above the diagonal DM (factor 2^k for DM in (2^(k-1), 2^k] DM_diag, k <= 4):
    # the downfactored inputs and one plan per run of trials, stats and 6-sigma candidates
    print("bench: time-binning timing", file=sys.stderr, flush=True)
    bp = dd.BinnedPlan(beam.freq_mhz, beam.tsamp_s, beam.dm, max_log2=4)
    bp.workspace(nsamp)
    bp.dedisperse(x, k_sigma=k, cand_cap=cap)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(3):
        bp.dedisperse(x, k_sigma=k, cand_cap=cap)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_tb = e0.elapsed_time(e1) / 3
    dfo = torch.empty((beam.nchan, nsamp // 2), dtype=torch.float32, device=x.device)
    e0.record(stream)
    for _ in range(3):
        _lib.check(lib.dd_downfactor(vp(x), 0, beam.nchan, nsamp, nsamp, vp(dfo), nsamp // 2, st))
    e1.record(stream)
    torch.cuda.synchronize()
    ms_df = e0.elapsed_time(e1) / 3
    del dfo
    df_bytes = beam.nchan * nsamp * 4 + beam.nchan * (nsamp // 2) * 4
    tb_nout = bp.nout(nsamp)
    time_binning = {
        "max_log2": 4, "dm_diag": round(bp.dm_diag, 4), "ms": round(ms_tb, 3),
        "runs": [{"factor": 1 << sg.log2, "ndm": sg.d1 - sg.d0, "nout": n} for sg, n in zip(bp.segments, tb_nout)],
        "adds": bp.adds(nsamp), "adds_vs_plain": round(bp.adds(nsamp) / adds, 4),
        "speedup_vs_plain_step": round(ms_step / ms_tb, 3),
        "dm_trial_samples_per_s_full_res": beam.ndm * nout / (ms_tb * 1e-3),
        "downfactor": {"kernel": "downfactor_rows", "ms": round(ms_df, 3), "bound": "hbm", "unit": "GB/s",
                       "achieved": round(df_bytes / (ms_df * 1e-3) / 1e9, 1), "peak": 8000.0,
                       "frac": round(df_bytes / (ms_df * 1e-3) / 1e9 / 8000.0, 4), "algorithmic_bytes": df_bytes}}
    del bp

    # RFI mitigation before dedispersion (Ch. 3), the whole stage on a fresh copy of the
    # input each time: the averaged bandpass (one read), its polynomial fit on the host (the
    # 1024 averages cross PCIe), then one pass for the 256-sample channel windows and the
    # bandpass correction (a read and a write of every sample) and one for the spectra (a read)
    print("bench: RFI timing", file=sys.stderr, flush=True)
    xr = torch.empty_like(x)
    avg = torch.empty(beam.nchan, dtype=torch.float64, device=x.device)
    win = 256
    flg = torch.empty((beam.nchan, -(-nsamp // win)), dtype=torch.int32, device=x.device)
    wmeans = torch.empty((beam.nchan, -(-nsamp // win)), dtype=torch.float64, device=x.device)
    e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms_bp = ms_clip = ms_stage = 0.0
    nrep = 3
    for rep in range(nrep + 1):  # the first run warms up
        xr.copy_(x)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        e0.record(stream)
        _lib.check(lib.dd_bandpass(vp(xr), beam.nchan, nsamp, nsamp, win, vp(avg), vp(wmeans), st))
        e1.record(stream)
        fit, rmse_bp, fmean = dd.bandpass_fit(avg.cpu().numpy(), 6)
        d_fit = torch.from_numpy(fit).cuda()
        e2.record(stream)
        _lib.check(lib.dd_rfi_clip(vp(xr), beam.nchan, nsamp, nsamp, vp(d_fit), 0.5, win, vp(wmeans), vp(flg),
                                   fmean, 0.2, 1, st))
        e3.record(stream)
        torch.cuda.synchronize()
        if rep:
            ms_stage += (time.perf_counter() - w0) * 1e3 / nrep
            ms_bp += e0.elapsed_time(e1) / nrep
            ms_clip += e2.elapsed_time(e3) / nrep
    in_bytes = beam.nchan * nsamp * 4
    rfi = {"kernels": "bandpass_windows (channel and window means); chan_flag + chan_correct (replacement and "
                      "bandpass correction) + spec_clip",
           "window": win, "order": 6, "chan_threshold": 0.5, "spec_threshold": 0.2, "subtract_bandpass": True,
           "stage_ms": round(ms_stage, 3),
           "bandpass_ms": round(ms_bp, 3), "bandpass_gbs": round(in_bytes / (ms_bp * 1e-3) / 1e9, 1),
           "clip_ms": round(ms_clip, 3),
           "clip_gbs_two_reads_one_write": round(3 * in_bytes / (ms_clip * 1e-3) / 1e9, 1), "peak_gbs": 8000.0,
           "stage_reads_of_input": 3,
           "windows_flagged": int(flg.sum().item())}
    del xr, flg, wmeans

    # subband dedispersion (an approximation: 32-channel subbands, 16 trials per nominal DM)
    print("bench: subband timing", file=sys.stderr, flush=True)
    sp = dd.SubbandPlan(beam.freq_mhz, beam.tsamp_s, beam.dm, chans_per_sub=32, dms_per_group=16)
    sp.dedisperse(x, k_sigma=k, cand_cap=cap)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(3):
        sp.dedisperse(x, k_sigma=k, cand_cap=cap)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_sb = e0.elapsed_time(e1) / 3
    sp.dedisperse(x, k_sigma=k, cand_cap=cap, batched=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(3):
        sp.dedisperse(x, k_sigma=k, cand_cap=cap, batched=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_sb_b = e0.elapsed_time(e1) / 3
    # one workgroup's worth of trials (48) per nominal DM: fewer, larger launches, more smear
    sp48 = dd.SubbandPlan(beam.freq_mhz, beam.tsamp_s, beam.dm, chans_per_sub=32, dms_per_group=48)
    sp48.dedisperse(x, k_sigma=k, cand_cap=cap)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(3):
        sp48.dedisperse(x, k_sigma=k, cand_cap=cap)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_sb48 = e0.elapsed_time(e1) / 3
    groups48 = {"dms_per_group": 48, "ms": round(ms_sb48, 3), "adds_vs_plain": round(sp48.adds(nsamp) / adds, 4),
                "speedup_vs_plain_step": round(ms_step / ms_sb48, 3), "launches": sp48.launches}
    del sp48
    subband = {"chans_per_sub": 32, "dms_per_group": 16, "ms": round(ms_sb, 3), "adds": sp.adds(nsamp),
               "adds_vs_plain": round(sp.adds(nsamp) / adds, 4), "speedup_vs_plain_step": round(ms_step / ms_sb, 3),
               "launches": sp.launches,
               "ms_batched": round(ms_sb_b, 3), "speedup_batched_vs_plain_step": round(ms_step / ms_sb_b, 3),
               "groups_of_48": groups48}
    del sp

    # the same workload stored as 8-bit codes (clip(rint(128 + 16 x), 0, 255), made on the
    # device), in the 8-bit default plan (direct-read form, exact integer sums): the kernel
    # with its copy preparation alone, then whole steps with statistics and candidates
    print("bench: 8-bit storage of the same workload", file=sys.stderr, flush=True)
    x8 = torch.clamp(torch.round(128.0 + 16.0 * x), 0, 255).to(torch.uint8)
    plan8 = dd.Plan(beam.freq_mhz, beam.tsamp_s, beam.dm, dtype="u8")
    ws8 = plan8.workspace(nsamp)
    u8res = {}
    for full in (False, True):
        plan8.dedisperse(x8, stats=full, k_sigma=k if full else 0.0, cand_cap=cap, out=out, workspace=ws8)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(3):
            plan8.dedisperse(x8, stats=full, k_sigma=k if full else 0.0, cand_cap=cap, out=out, workspace=ws8)
        e1.record(stream)
        torch.cuda.synchronize()
        u8res["step_ms" if full else "prep_and_kernel_ms"] = round(e0.elapsed_time(e1) / 3, 3)
    u8 = {"form": plan8.form, "tiles": list(plan8.tiles[:2]), **u8res,
          "adds_per_s_prep_and_kernel": adds / (u8res["prep_and_kernel_ms"] * 1e-3),
          "dm_trial_samples_per_s": beam.ndm * nout / (u8res["step_ms"] * 1e-3)}
    # RFI mitigation of the 8-bit codes in place (window 256, order 6): the bandpass and
    # window means (one read), the host fit, then channel and spectrum clipping (a read for
    # the spectra; windows are written only where replaced)
    x8r = torch.empty_like(x8)
    win8 = 256
    avg8 = torch.empty(beam.nchan, dtype=torch.float64, device=x.device)
    wm8 = torch.empty((beam.nchan, -(-nsamp // win8)), dtype=torch.float64, device=x.device)
    fl8 = torch.empty((beam.nchan, -(-nsamp // win8)), dtype=torch.int32, device=x.device)
    ms_bp8 = ms_cl8 = 0.0
    for rep in range(4):  # the first run warms up
        x8r.copy_(x8)
        torch.cuda.synchronize()
        e0.record(stream)
        _lib.check(lib.dd_bandpass_u8(vp(x8r), beam.nchan, nsamp, nsamp, win8, vp(avg8), vp(wm8), st))
        e1.record(stream)
        fit8, _, fmean8 = dd.bandpass_fit(avg8.cpu().numpy(), 6)
        d_fit8 = torch.from_numpy(fit8).cuda()
        e2 = torch.cuda.Event(enable_timing=True)
        e3 = torch.cuda.Event(enable_timing=True)
        e2.record(stream)
        _lib.check(lib.dd_rfi_clip_u8(vp(x8r), beam.nchan, nsamp, nsamp, vp(d_fit8), 8.0, win8, vp(wm8), vp(fl8),
                                      fmean8, 3.2, st))
        e3.record(stream)
        torch.cuda.synchronize()
        if rep:
            ms_bp8 += e0.elapsed_time(e1) / 3
            ms_cl8 += e2.elapsed_time(e3) / 3
    u8["rfi"] = {"kernels": "bandpass_windows_u8; chan_flag + chan_apply_u8 + spec_clip_u8", "window": win8,
                 "order": 6, "chan_threshold": 8.0, "spec_threshold": 3.2,
                 "bandpass_ms": round(ms_bp8, 3),
                 "bandpass_gbs": round(beam.nchan * nsamp / (ms_bp8 * 1e-3) / 1e9, 1),
                 "clip_ms": round(ms_cl8, 3),
                 "clip_gbs_one_read": round(beam.nchan * nsamp / (ms_cl8 * 1e-3) / 1e9, 1),
                 "windows_flagged": int(fl8.sum().item())}
    del x8, x8r, ws8, plan8

    res = {
        "metric": "DM-trial*samples/s",
        "value": beam.ndm * nout / (ms_step * 1e-3),
        "unit": "DM-trial*samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plain brute-force dedispersion, full size: FP32 1024 ch 408-428 MHz, "
                               "tsamp 51.2 us, nsamp 2^20, 2048 DMs 0-204.7 step 0.1, stats + 6-sigma candidates",
                   "nchan": beam.nchan, "nsamp": nsamp, "ndm": beam.ndm, "nout": nout,
                   "tiles": list(plan.tiles), "producer_waves": plan.producer_waves, "candidates_found": n_found},
        "real_time_factor": round(nout * beam.tsamp_s / (ms_step * 1e-3), 2),
        "roofline": roof,
        "u8_storage": u8,
        "detrend": detrend,
        "boxcar": boxcar,
        "boxcar_search": boxcar_search,
        "time_binning": time_binning,
        "rfi": rfi,
        "subband": subband,
    }
    if args.copy_probe:
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        res["copy_probe_bytes"] = int(x.numel() * x.element_size())
        del y
    del x
    del out
    if args.batch_reps > 0:
        print("bench: config-4 batch (autotune, batched, one at a time)", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        res["batch"] = batch_run(args.batch_reps)
        torch.cuda.empty_cache()
    if args.serve_blocks > 0:
        print("bench: binned stream of a 4096-channel serving beam", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        res["binned_stream"] = binned_stream_run(8)
        print(f"bench: serving run ({args.serve_blocks} blocks per beam)", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        res["serving"] = serve_run(args.serve_blocks, int(args.hbm_budget_gb * 1e9))
    if not args.no_cpu:
        print("bench: oracle CPU baseline", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(beam, args.cpu_rows, args.cpu_workers)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
