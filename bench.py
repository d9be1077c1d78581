"""Benchmark: brute-force dedispersion of the full-size FP32 workload on one MI355X.

Workload: 1024 channels over 408-428 MHz, 51.2 us sampling, 2^20 samples of N(0,1)
noise with 20 dispersed boxcars, 2048 DM trials 0-204.7 step 0.1; output FP32
plus per-DM mean/RMS and candidates above 6 sigma. Inputs are resident in HBM
before timing starts. One step = one dd_dedisperse call (dedispersion kernel,
statistics and candidate kernels).

Prints one JSON line: the whole-step throughput in DM-trial*samples/s, the
dedispersion kernel's own duration against the FP32 add roofline, and the FP64
oracle timed on a bounded sample of the same workload on the host.
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

# MI355X: 256 CUs x 2.4 GHz. The FP32 vector peak of 157.3 TFLOP/s counts a fused
# multiply-add as two flops on 128 lanes/clk/CU; an add is one flop per lane, so the
# add roofline is 256 x 2.4e9 x 128 = 78.6e12 adds/s (v_add_f32 issues at that rate).
PEAK_ADD_TFLOPS = 256 * 2.4e9 * 128 / 1e12
# The kernel's own ceiling: every add consumes one 4-byte LDS word, and ds_read_b128
# delivers ~221 B/clk/CU, so at most 256 x 2.4e9 x 221 / 4 = 33.9e12 adds/s.
LDS_CEILING_TADDS = 256 * 2.4e9 * 221 / 4 / 1e12
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dedisp_tile_full_fp32_1024ch_2048dm_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1401_8258_amd", "csrc", "dedisp.hip")


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
    return ap.parse_args()


def cpu_baseline(beam, rows):
    from oracle import dedisp_oracle as orc
    tab = orc.delay_table(beam.freq_mhz, beam.dm, beam.tsamp_s)
    sel = [int(r) for r in np.linspace(0, beam.ndm - 1, rows)]
    t = time.perf_counter()
    out = orc.dedisperse(beam.data, tab, rows=sel)
    orc.series_stats(out)
    dt = time.perf_counter() - t
    nout = out.shape[1]
    return {"value": len(sel) * nout / dt, "unit": "DM-trial*samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(sel)} of {beam.ndm} DM rows (evenly spaced) x {nout} output samples x "
                      f"{beam.nchan} channels, FP64 NumPy, single thread; {dt:.1f} s"}


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
    print("bench: generating workload", file=sys.stderr, flush=True)
    beam = fbsynth.config2()
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
    traffic, traffic_note = None, "no counter record"
    if args.traffic and os.path.exists(args.traffic):
        from paper_1401_8258_amd.profiling import source_digest
        with open(args.traffic) as f:
            rec = json.load(f)
        if rec.get("kernel_source_sha256") == source_digest(KERNEL_SOURCE):
            traffic = rec["hbm_bytes_per_launch"]
            traffic_note = (f"FETCH_SIZE x {rec['fetch_scale']} + WRITE_SIZE x {rec['write_scale']} "
                            f"(copy-kernel calibration), {os.path.relpath(args.traffic, ROOT)}")
        else:
            traffic_note = "kernel changed since the counters were taken"
    algo_bytes = beam.nchan * nsamp * 4 + beam.ndm * nout * 4
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_ADD_TFLOPS, 2),
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_ADD_TFLOPS, 4), "traffic": traffic,
            "traffic_note": traffic_note, "algorithmic_bytes": algo_bytes,
            "kernel": "dedisp_tile", "kernel_ms": round(ms_kernel, 3),
            "frac_of_lds_ceiling": round(achieved / LDS_CEILING_TADDS, 4),
            "algorithmic_hbm_gbs": round(algo_bytes / (ms_kernel * 1e-3) / 1e9, 1)}

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
                   "tiles": list(plan.tiles), "candidates_found": n_found},
        "real_time_factor": round(nout * beam.tsamp_s / (ms_step * 1e-3), 2),
        "roofline": roof,
    }
    if args.copy_probe:
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        res["copy_probe_bytes"] = int(x.numel() * x.element_size())
        del y
    del x
    if not args.no_cpu:
        print("bench: oracle CPU baseline", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(beam, args.cpu_rows)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
