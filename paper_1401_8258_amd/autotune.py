"""Autotuner for the dedispersion tiles (kernel form, wavefronts per DM group, channels per
LDS stage, DM trials per wavefront).

The thesis tuned its kernel by sweeping accumulators per thread and threads per
block on the target GPU (Ch. 2, Sec. Performance and Benchmarks). Here the
tunables are the kernel form ("lds": every add reads LDS, lanes own 2 x 4 samples,
DM groups of 8 x waves trials; "regwin", FP32: lanes own 8 consecutive samples held
in a register window, DM groups of 64 trials; "direct", 8-bit: lanes own 16 or
32 samples read through the caches, DM groups of g x waves trials with g in 1, 2, 4),
the number of wavefronts sharing one LDS ring or workgroup and the channels staged
per ring slot. ``tune``
times every candidate on seeded random input of the beam's shape and keeps the
fastest; ``tune_batch`` tunes a set of beams at every wavefront count and returns each
beam's own best (a batched call runs every beam on its own tiles, one launch per kernel
shape), or on request each beam's best under the one count that minimises their summed
time (fewer launches). The timer is a parameter (``time_plan`` on the
device by default). Results are cached by (nchan, ndm, dtype, nsamp, DM list hash).
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from .api import Plan, torch_dtype

WAVES = (14, 8, 4, 2, 1)  # 14: 4 trials per wavefront beside 2 producers (FP32 LDS form only)
STAGES = (0, 2, 4)
FORMS = ("lds", "direct")
# (DM trials per wavefront, samples per lane) of the direct-read form
DIRECT_SHAPES = ((1, 16), (2, 16), (4, 16), (1, 32), (2, 32))


def _key(freq, tsamp, dm, dtype, nsamp) -> str:
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(freq, np.float64).tobytes())
    h.update(np.ascontiguousarray(dm, np.float64).tobytes())
    h.update(np.float64(tsamp).tobytes())
    return f"{len(freq)}x{len(dm)}:{dtype}:{nsamp}:{h.hexdigest()[:16]}"


class TuneCache:
    def __init__(self, path: Optional[str] = None):
        self.path = path
        self.data: Dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def get(self, key):
        return self.data.get(key)

    def put(self, key, val):
        self.data[key] = val
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def synthetic_input(nchan: int, nsamp: int, dtype, seed: int = 0, device="cuda") -> torch.Tensor:
    """Seeded random input of the beam's shape for timing (noise only)."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    x = torch.randn((nchan, nsamp), generator=g, device=device)
    dt = torch_dtype(dtype)
    if dt == torch.uint8:
        return torch.clamp(torch.round(128.0 + 16.0 * x), 0, 255).to(torch.uint8)
    return x.to(dt)


def time_plan(plan: Plan, x: torch.Tensor, reps: int = 3) -> float:
    """Milliseconds per dedispersion (kernel only, no statistics) on the current stream."""
    nout = x.shape[1] - plan.maxdelay
    out = torch.empty((plan.ndm, nout), dtype=torch.float32, device=x.device)
    ws = plan.workspace(x.shape[1], x.device)
    plan.dedisperse(x, stats=False, out=out, workspace=ws)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        plan.dedisperse(x, stats=False, out=out, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def make_plan(freq, tsamp, dm, dtype, choice: dict) -> Plan:
    """The plan a tuning result (or one of its trials) describes."""
    return Plan(freq, tsamp, dm, dtype=dtype, tuning=choice.get("tuning"), form=choice.get("form", "lds"))


def tune(freq, tsamp, dm, dtype, nsamp, waves: Sequence[int] = WAVES, stages: Sequence[int] = STAGES,
         reps: int = 3, cache: Optional[TuneCache] = None, x: Optional[torch.Tensor] = None,
         forms: Sequence[str] = FORMS, timer: Callable[[Plan, torch.Tensor, int], float] = time_plan) -> dict:
    """The fastest of the candidate tilings for one beam shape: {"form", "tuning", "ms",
    "trials"} ("tuning" is (dms_per_wave, waves, chan_stage) for the LDS form, (dms_per_wave,
    waves, samples_per_lane) for the direct-read form, None for the register-window form,
    whose groups are fixed at 8 x 8 trials)."""
    key = _key(freq, tsamp, dm, str(dtype), nsamp) + f":{tuple(waves)}:{tuple(stages)}:{tuple(forms)}"
    if cache is not None and cache.get(key):
        return cache.get(key)
    if x is None:
        x = synthetic_input(len(freq), nsamp, dtype)
    cands = []
    u8 = torch_dtype(dtype) == torch.uint8
    for form in forms:
        if form == "regwin":
            cands.append({"form": "regwin", "tuning": None})
        elif form == "direct":
            if u8:  # the direct-read form takes 8-bit input only
                cands += [{"form": "direct", "tuning": [g, w, spl]} for w in waves if w <= 8
                          for g, spl in DIRECT_SHAPES]
        else:
            # up to 8 wavefronts: 8 trials each; more (FP32 only): the 4-trial producer form
            cands += [{"form": "lds", "tuning": [8 if w <= 8 else 4, w, cc]} for w in waves for cc in stages
                      if w <= 8 or torch_dtype(dtype) == torch.float32]
    trials = []
    for cand in cands:
        try:
            plan = make_plan(freq, tsamp, dm, dtype, cand)
            ms = timer(plan, x, reps)
        except Exception as e:  # a tiling that does not fit this beam
            trials.append(dict(cand, error=str(e)))
            continue
        trials.append(dict(cand, ms=ms))
    ok = [t for t in trials if "ms" in t]
    if not ok:
        raise RuntimeError("no tiling fits this beam")
    best = min(ok, key=lambda t: t["ms"])
    res = {"form": best["form"], "tuning": best["tuning"], "ms": best["ms"], "trials": trials}
    if cache is not None:
        cache.put(key, res)
    return res


def tune_batch(beams: List[Tuple], waves: Sequence[int] = WAVES, stages: Sequence[int] = STAGES, reps: int = 2,
               cache: Optional[TuneCache] = None, inputs: Optional[List[torch.Tensor]] = None,
               log=None, timer: Callable[[Plan, torch.Tensor, int], float] = time_plan,
               forms: Sequence[str] = FORMS, common_waves: bool = False) -> dict:
    """Tiles for a batch of beams.

    beams: (freq, tsamp, dm, dtype, nsamp) per beam. Every beam is tuned at each wavefront
    count. Returns {"waves": w, "choices": [...], "tunings": [...], "own_best": [...],
    "total_ms": t, "by_waves": {w: t}}: ``own_best`` is each beam's fastest choice over all
    counts ({"form", "tuning", "ms"}); ``w`` the count that minimises the summed time over
    the counts every beam fits (None if there is none), ``total_ms`` that sum. ``choices``
    (what make_plan takes) is ``own_best``, or with ``common_waves`` each beam's best under
    ``w`` (a batched call then needs one launch per tile shape instead of one per distinct
    tiling).
    """
    per_w: Dict[int, List[Optional[dict]]] = {}
    for w in waves:
        per_w[w] = []
        for i, (freq, tsamp, dm, dtype, nsamp) in enumerate(beams):
            x = inputs[i] if inputs is not None else None
            try:
                r = tune(freq, tsamp, dm, dtype, nsamp, waves=(w,), stages=stages, reps=reps, cache=cache, x=x,
                         timer=timer, forms=forms)
            except RuntimeError:
                r = None  # no tiling with w wavefronts fits this beam
            per_w[w].append(r)
            if log is not None and r is not None:
                log(f"tune: waves {w} beam {i}: {r['form']} {r['tuning']} {r['ms']:.2f} ms")
    totals = {w: sum(r["ms"] for r in rs) for w, rs in per_w.items() if all(r is not None for r in rs)}
    wbest = min(totals, key=totals.get) if totals else None
    own = []
    for i in range(len(beams)):
        fits = [rs[i] for rs in per_w.values() if rs[i] is not None]
        if not fits:
            raise RuntimeError(f"no tiling fits beam {i}")
        r = min(fits, key=lambda t: t["ms"])
        own.append({"form": r["form"], "tuning": r["tuning"], "ms": r["ms"]})
    if common_waves:
        if wbest is None:
            raise RuntimeError("no common wavefront count fits every beam")
        choices = [{"form": r["form"], "tuning": r["tuning"]} for r in per_w[wbest]]
    else:
        choices = [{"form": r["form"], "tuning": r["tuning"]} for r in own]
    return {"waves": wbest, "choices": choices, "tunings": [c["tuning"] for c in choices], "own_best": own,
            "total_ms": totals.get(wbest), "by_waves": totals}
