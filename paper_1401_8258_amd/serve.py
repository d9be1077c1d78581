"""Streaming server: many beams' blocks, device-resident overlap rings, continuous batching.

The thesis's pipeline (Ch. 3, Sec. Pipeline Overview) runs one processing thread
per beam and carries the last maxshift spectra of every buffer into the next
(Ch. 3, Sec. Dedispersion). Here one scheduler feeds the GPU instead:

* admission: a beam is admitted when its device footprint (ring with the
  overlap, workspace, output block) fits in the HBM budget; beams that do not
  fit wait in a bounded queue (admitted as admitted beams finish) or are
  rejected when the queue is full;
* continuous batching: at every scheduling point all blocks that have arrived
  for admitted beams (in per-beam sequence order) form one launch; blocks that
  arrive while a launch is on the GPU join the next one, and up to
  ``max_inflight`` launches overlap on the device;
* accounting: per block latency = completion - arrival against the real-time
  deadline (one block duration), blocks/s, real-time factor, p50/p99.

The executor does the device work. ``LibraryExecutor`` appends each block to its
beam's ring (dd_stream_append) and dedisperses the whole batch in one batched
launch (dd_batch_dedisperse); tests drive the scheduler with a fake executor.
"""
from __future__ import annotations

import collections
import dataclasses
import heapq
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class BeamSpec:
    name: str
    freq_mhz: np.ndarray
    tsamp_s: float
    dm: np.ndarray
    dtype: str              # "u8", "f16" or "f32"
    block: int              # samples per block
    k_sigma: float = 6.0
    max_log2: int = 0       # > 0: time binning above the diagonal DM up to factor 2^max_log2
                            # (block must then be a multiple of 2^K, K the largest run factor)

    @property
    def block_s(self) -> float:
        return self.block * self.tsamp_s


@dataclasses.dataclass(order=True)
class Block:
    arrival: float
    beam: int = dataclasses.field(compare=False)
    seq: int = dataclasses.field(compare=False)
    data: object = dataclasses.field(compare=False, default=None)


@dataclasses.dataclass
class BlockResult:
    beam: int
    seq: int
    arrival: float
    done: float
    t0: int
    nout: int
    ncand: int
    filling: bool

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Executor:
    """Device side of the server (interface)."""

    def footprint(self, spec: BeamSpec) -> int:          # bytes a beam keeps on the device
        raise NotImplementedError

    def open(self, beam: int, spec: BeamSpec) -> None:    # allocate the beam's ring/workspace
        raise NotImplementedError

    def close(self, beam: int) -> None:
        raise NotImplementedError

    def submit(self, blocks: List[Block]):                # enqueue one batched launch; returns a handle
        raise NotImplementedError

    def done(self, handle) -> bool:                       # non-blocking completion check
        raise NotImplementedError

    def results(self, handle) -> List[dict]:              # per block: t0, nout, ncand, filling (after done)
        raise NotImplementedError

    def gpu_seconds(self, handle) -> float:               # device time of a finished launch (0 if unknown)
        return 0.0


@dataclasses.dataclass
class ServeStats:
    admitted: int = 0
    queued: int = 0
    rejected: int = 0
    launches: int = 0
    blocks: int = 0
    fill_blocks: int = 0
    deadline_misses: int = 0
    admitted_in_run: int = 0   # beams admitted while the run was going (freed slots and memory)
    wall_s: float = 0.0
    data_s: float = 0.0
    gpu_busy_s: float = 0.0    # device time of every launch (ring appends, dedispersion, tails)
    stream_s: float = 0.0      # seconds of stream time served: the data of the busiest beam
    latencies: List[float] = dataclasses.field(default_factory=list)
    batch_sizes: List[int] = dataclasses.field(default_factory=list)

    def summary(self) -> dict:
        lat = np.asarray(self.latencies) if self.latencies else np.zeros(1)
        return {
            "admitted_beams": self.admitted, "queued_beams": self.queued, "rejected_beams": self.rejected,
            "launches": self.launches, "blocks": self.blocks, "fill_blocks": self.fill_blocks,
            "blocks_per_s": self.blocks / self.wall_s if self.wall_s > 0 else 0.0,
            "real_time_factor": self.data_s / self.wall_s if self.wall_s > 0 else 0.0,
            "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_max_s": float(lat.max()), "deadline_misses": self.deadline_misses,
            "admitted_in_run": self.admitted_in_run,
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "data_s": self.data_s, "stream_s": self.stream_s, "gpu_busy_s": self.gpu_busy_s,
            # device seconds per second of stream time (all beams together): below 1 the GPU
            # keeps up with every beam in real time, and 1 - this is the real-time margin
            "gpu_busy_s_per_stream_s": self.gpu_busy_s / self.stream_s if self.stream_s > 0 else 0.0,
        }


class Server:
    """Admission by HBM budget plus continuous batching over a simulated arrival schedule.

    ``clock`` returns seconds (wall clock by default); ``sleep`` waits. Arrival times
    are in the same clock, relative to ``start``.
    """

    def __init__(self, specs: Sequence[BeamSpec], executor: Executor, hbm_budget: int,
                 max_queue: int = 1 << 30, max_inflight: int = 2, max_batch: int = 1 << 30,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep):
        self.specs = list(specs)
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_queue = max_queue
        self.max_inflight = max_inflight
        self.max_batch = max_batch
        self.clock = clock
        self.sleep = sleep
        self.used = 0
        self.active: Dict[int, int] = {}         # beam -> footprint
        self.waiting: collections.deque = collections.deque()
        self.rejected: List[int] = []
        self.stats = ServeStats()
        self.results: List[BlockResult] = []

    # ---------------------------------------------------------------- admission
    def request(self, beam: int) -> str:
        """Ask to admit a beam: 'admitted', 'queued' or 'rejected'."""
        need = self.ex.footprint(self.specs[beam])
        if need > self.budget:
            self.rejected.append(beam)
            self.stats.rejected += 1
            return "rejected"
        if self.used + need <= self.budget and not self.waiting:
            self._admit(beam, need)
            return "admitted"
        if len(self.waiting) >= self.max_queue:
            self.rejected.append(beam)
            self.stats.rejected += 1
            return "rejected"
        self.waiting.append(beam)
        self.stats.queued += 1
        return "queued"

    def _admit(self, beam: int, need: int) -> None:
        self.ex.open(beam, self.specs[beam])
        self.active[beam] = need
        self.used += need
        self.stats.admitted += 1

    def release(self, beam: int) -> None:
        """A beam finished: free its memory and admit waiting beams in order while they fit."""
        need = self.active.pop(beam)
        self.ex.close(beam)
        self.used -= need
        while self.waiting:
            b = self.waiting[0]
            nb = self.ex.footprint(self.specs[b])
            if self.used + nb > self.budget:
                break
            self.waiting.popleft()
            self._admit(b, nb)

    # ---------------------------------------------------------------- serving loop
    def run(self, schedule: List[Block], fill: Optional[Callable[[int], bool]] = None,
            release_done: bool = False) -> ServeStats:
        """Serve every block of ``schedule`` (arrival times relative to the start).

        Blocks of beams that are not admitted wait until their beam is. ``fill(beam)``
        tells whether a block result belongs to the ring fill (excluded from latency).
        With ``release_done`` a beam is released as soon as its last scheduled block
        has completed, which admits waiting beams while the others keep streaming;
        their queued blocks count their wait in their latency.
        """
        pending = list(schedule)
        heapq.heapify(pending)
        left: Dict[int, int] = collections.Counter(b.beam for b in schedule)
        ready: Dict[int, collections.deque] = collections.defaultdict(collections.deque)
        next_seq: Dict[int, int] = collections.defaultdict(int)
        inflight: collections.deque = collections.deque()
        start = self.clock()
        data_s = 0.0
        beam_s: Dict[int, float] = collections.defaultdict(float)
        while pending or any(ready.values()) or inflight:
            now = self.clock() - start
            while pending and pending[0].arrival <= now:
                b = heapq.heappop(pending)
                ready[b.beam].append(b)
            # retire finished launches (in order)
            while inflight and self.ex.done(inflight[0][0]):
                h, blocks = inflight.popleft()
                t_done = self.clock() - start
                self.stats.gpu_busy_s += self.ex.gpu_seconds(h)
                for blk, r in zip(blocks, self.ex.results(h)):
                    br = BlockResult(blk.beam, blk.seq, blk.arrival, t_done, r["t0"], r["nout"], r["ncand"],
                                     r["filling"])
                    self.results.append(br)
                    self.stats.blocks += 1
                    data_s += self.specs[blk.beam].block_s
                    beam_s[blk.beam] += self.specs[blk.beam].block_s
                    if br.filling or (fill is not None and fill(blk.beam)):
                        self.stats.fill_blocks += 1
                        continue
                    self.stats.latencies.append(br.latency)
                    if br.latency > self.specs[blk.beam].block_s:
                        self.stats.deadline_misses += 1
                for blk in blocks:
                    left[blk.beam] -= 1
                    if release_done and left[blk.beam] == 0 and blk.beam in self.active:
                        before = len(self.active)
                        self.release(blk.beam)
                        self.stats.admitted_in_run += len(self.active) - before + 1
            # form the next launch from every ready block of an admitted beam
            if len(inflight) < self.max_inflight:
                batch: List[Block] = []
                for beam in sorted(ready):
                    if beam not in self.active:
                        continue
                    q = ready[beam]
                    # one block per beam per launch: a ring holds one pending window
                    if q and q[0].seq == next_seq[beam] and len(batch) < self.max_batch:
                        batch.append(q.popleft())
                        next_seq[beam] += 1
                if batch:
                    h = self.ex.submit(batch)
                    inflight.append((h, batch))
                    self.stats.launches += 1
                    self.stats.batch_sizes.append(len(batch))
                    continue
            # nothing to launch: wait for the next arrival or completion
            if inflight:
                self.sleep(2e-4)
            elif pending:
                wait = pending[0].arrival - (self.clock() - start)
                if wait > 0:
                    self.sleep(min(wait, 0.05))
            elif any(ready.values()):
                # ready blocks whose beams are not admitted and nothing in flight: cannot progress
                if not any(b in self.active for b in ready if ready[b]):
                    break
        self.stats.wall_s = self.clock() - start
        self.stats.data_s = data_s
        self.stats.stream_s = max(beam_s.values()) if beam_s else 0.0
        return self.stats


class LibraryExecutor(Executor):
    """Device side on libdedisp: one Stream (device ring with the maxdelay overlap) per
    admitted beam, and per submitted set of blocks one batched call over all of them (one
    persistent launch per kernel shape, each beam on its own tiles).
    A beam with time binning (``max_log2 > 0``) has a BinnedStream instead, one ring per run
    at its binned sampling time, and is pushed on its own after the batched calls.

    Each beam owns two output sets (dedispersed block, mean, rms, candidates), used by
    alternate blocks, so a block's results stay intact while the next block of the same
    beam is already queued behind it. ``keep`` stores copies of every result (for tests).
    """

    def __init__(self, k_sigma: float = 6.0, cand_cap: int = 1 << 14, device="cuda", stream=None,
                 tunings: Optional[Dict[str, object]] = None, keep: bool = False):
        import torch

        from . import api
        self._torch = torch
        self._api = api
        self.k_sigma = float(k_sigma)
        self.cand_cap = int(cand_cap)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.tunings = dict(tunings or {})
        self.keep = keep
        self.kept: Dict[tuple, dict] = {}
        self._plans: Dict[str, object] = {}
        self._beams: Dict[int, dict] = {}

    def plan(self, spec: BeamSpec):
        p = self._plans.get(spec.name)
        if p is None:
            # a tuning is an LDS-form tile tuple or an autotuner choice {"form", "tuning"}
            t = self.tunings.get(spec.name)
            form = "auto"
            if isinstance(t, dict):
                form, t = t.get("form", "auto"), t.get("tuning")
            if spec.max_log2 > 0:
                p = self._api.BinnedPlan(spec.freq_mhz, spec.tsamp_s, spec.dm, dtype=spec.dtype,
                                         max_log2=spec.max_log2, tuning=t, form=form)
            else:
                p = self._api.Plan(spec.freq_mhz, spec.tsamp_s, spec.dm, dtype=spec.dtype, tuning=t, form=form)
            self._plans[spec.name] = p
        return p

    def footprint(self, spec: BeamSpec) -> int:
        p = self.plan(spec)
        ndm = len(spec.dm)
        outs = ndm * spec.block * 4 + 2 * ndm * 4 + self.cand_cap * 24 + 8
        if spec.max_log2 > 0:
            ring, ws = p.stream_sizes(spec.block)
            return int(ring + ws + 2 * outs)
        q = p.query(spec.block, allow_short=True)
        return int(q["ring_bytes"] + q["stream_workspace_bytes"] + 2 * outs)

    def open(self, beam: int, spec: BeamSpec) -> None:
        p = self.plan(spec)
        ndm = len(spec.dm)
        if spec.max_log2 > 0:
            st = self._api.BinnedStream(p, spec.block, device=self.device, stream=self.stream)
        else:
            st = self._api.Stream(p, spec.block, device=self.device, stream=self.stream)
        outs = [self._api.alloc_outputs(ndm, spec.block, self.device, self.k_sigma, self.cand_cap)
                for _ in range(2)]
        self._beams[beam] = {"stream": st, "outs": outs, "n": 0, "spec": spec,
                             "binned": spec.max_log2 > 0}

    def close(self, beam: int) -> None:
        self._beams.pop(beam, None)

    def prefill(self, beam: int, blocks) -> int:
        """Append blocks without dedispersing (fast-forward a ring past its fill); returns how
        many blocks were still filling. Must precede the beam's first submitted block."""
        b = self._beams[beam]
        filling = 0
        for x in blocks:
            if b["binned"]:
                # no append without dedispersion here: runs past their own fill dedisperse
                # (without statistics), the others only fill
                w = b["stream"].push(x, stats=False, stream=self.stream)
            else:
                w = b["stream"].append(x, stream=self.stream)
            if w is None:
                filling += 1
            elif not b["binned"]:
                raise ValueError("prefill went past the ring fill; use fewer blocks")
        return filling

    def submit(self, blocks: List[Block]):
        # the stream runs launches in order, so the time between these two events is this
        # launch's own device time even when it was queued behind the previous one
        ev0 = self._torch.cuda.Event(enable_timing=True)
        ev0.record(self.stream)
        pend = []
        for blk in blocks:
            b = self._beams[blk.beam]
            pend.append(None if b["binned"] else b["stream"].append(blk.data, stream=self.stream))
        # plans of any tiles share one batched call (one launch per kernel shape)
        idx = [i for i, w in enumerate(pend) if w is not None]
        res: List[object] = [None] * len(blocks)
        if idx:
            jobs, outs = [], []
            for i in idx:
                b = self._beams[blocks[i].beam]
                jobs.append((b["stream"], pend[i]))
                outs.append(b["outs"][b["n"] & 1])
            rs = self._api.batch_dedisperse(jobs, k_sigma=self.k_sigma, cand_cap=self.cand_cap, stream=self.stream,
                                            outputs=outs)
            for i, r in zip(idx, rs):
                res[i] = r
        for i, blk in enumerate(blocks):
            b = self._beams[blk.beam]
            if b["binned"]:
                res[i] = b["stream"].push(blk.data, k_sigma=self.k_sigma, cand_cap=self.cand_cap,
                                          outputs=b["outs"][b["n"] & 1], stream=self.stream,
                                          batched=False)  # one launch per run: measured faster
                if res[i] is not None:
                    b["n"] += 1
        for blk, w in zip(blocks, pend):
            if w is not None:
                self._beams[blk.beam]["n"] += 1
        # candidate counts to pinned host memory on the serving stream, before the completion
        # event: once the event has completed they are there, and retiring this launch does
        # not wait for the next launch in flight on the stream
        counts = []
        with self._torch.cuda.stream(self.stream):
            for r in res:
                m = r.merged if isinstance(r, self._api.BinnedStreamResult) else r
                if m is None or m._ncand is None:
                    counts.append(None)
                    continue
                h = self._torch.empty(1, dtype=self._torch.int64, pin_memory=True)
                h.copy_(m._ncand, non_blocking=True)
                counts.append(h)
        ev = self._torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        return ev, list(blocks), res, ev0, counts

    def done(self, handle) -> bool:
        return handle[0].query()

    def gpu_seconds(self, handle) -> float:
        return handle[3].elapsed_time(handle[0]) * 1e-3

    def results(self, handle) -> List[dict]:
        _, blocks, res, _, counts = handle
        out = []
        for blk, r, h in zip(blocks, res, counts):
            if r is None:
                out.append({"t0": 0, "nout": 0, "ncand": 0, "filling": True})
                continue
            n = int(h[0]) if h is not None else 0  # copied before the launch's event
            if isinstance(r, self._api.BinnedStreamResult):
                # a binned beam: t0 of its factor-1 run, outputs summed over the runs
                m = r.merged
                nout = sum(int(x.out.shape[1]) for _, _, x in r.segments if x is not None)
                out.append({"t0": int(r.segments[0][1]), "nout": nout, "ncand": n, "filling": False})
                if self.keep:
                    self.kept[(blk.beam, blk.seq)] = {
                        "runs": [(t0, None if x is None else x.out.clone(), None if x is None else x.mean.clone(),
                                  None if x is None else x.rms.clone()) for _, t0, x in r.segments],
                        "cand": m.candidates()}
                continue
            out.append({"t0": int(r.t0), "nout": int(r.out.shape[1]), "ncand": n, "filling": False})
            if self.keep:
                self.kept[(blk.beam, blk.seq)] = {
                    "t0": int(r.t0), "out": r.out.clone(), "mean": r.mean.clone(), "rms": r.rms.clone(),
                    "cand": r.candidates()}
        return out


def poisson_schedule(specs: Sequence[BeamSpec], n_blocks: int, seed: int = 5, jitter_mean_s: float = 0.1,
                     phases=None, make_data: Optional[Callable[[int, int], object]] = None,
                     time_scale: float = 1.0) -> List[Block]:
    """arrival_k = (k * T + phase + J_k) * time_scale with J_k ~ Exp(mean) truncated below T."""
    rng = np.random.default_rng(seed)
    out = []
    for i, sp in enumerate(specs):
        T = sp.block_s
        ph = float(phases[i]) if phases is not None else float(rng.uniform(0.0, T))
        j = np.minimum(rng.exponential(jitter_mean_s, size=n_blocks), np.nextafter(T, 0.0))
        for k in range(n_blocks):
            data = make_data(i, k) if make_data else None
            out.append(Block((k * T + ph + float(j[k])) * time_scale, i, k, data))
    return out
