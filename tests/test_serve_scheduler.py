"""Serving scheduler logic on the CPU with a fake executor and a virtual clock.

The fake executor is a test double (fixed launch cost, canned results); it is not
a product code path. Device results of the real executor are covered on the GPU.
"""
import numpy as np

from paper_1401_8258_amd.serve import BeamSpec, Block, Executor, Server, poisson_schedule


class VClock:
    def __init__(self):
        self.t = 0.0

    def clock(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor(Executor):
    def __init__(self, vc, per_block=0.01, fixed=0.02, foot=100, fill_blocks=0):
        self.vc, self.per_block, self.fixed, self.foot, self.fill_blocks = vc, per_block, fixed, foot, fill_blocks
        self.opened, self.closed, self.launches = [], [], []
        self.count = {}

    def footprint(self, spec):
        return self.foot if not isinstance(self.foot, dict) else self.foot[spec.name]

    def open(self, beam, spec):
        self.opened.append(beam)

    def close(self, beam):
        self.closed.append(beam)

    def submit(self, blocks):
        t_end = self.vc.t + self.fixed + self.per_block * len(blocks)
        res = []
        for b in blocks:
            n = self.count.get(b.beam, 0)
            self.count[b.beam] = n + 1
            res.append({"t0": 0, "nout": 10, "ncand": 0, "filling": n < self.fill_blocks})
        self.launches.append([(b.beam, b.seq) for b in blocks])
        return (t_end, res)

    def done(self, h):
        return self.vc.t >= h[0]

    def results(self, h):
        return h[1]


def _specs(n, block_s=1.0):
    f = np.array([428.0, 427.0])
    return [BeamSpec(f"b{i}", f, block_s / 1000, np.array([0.0]), "u8", 1000) for i in range(n)]


def test_admission_queue_and_release():
    vc = VClock()
    ex = FakeExecutor(vc, foot=40)
    srv = Server(_specs(4), ex, hbm_budget=100, max_queue=1, clock=vc.clock, sleep=vc.sleep)
    assert [srv.request(i) for i in range(4)] == ["admitted", "admitted", "queued", "rejected"]
    assert srv.used == 80 and list(srv.waiting) == [2]
    srv.release(0)
    assert 2 in srv.active and srv.used == 80 and not srv.waiting
    big = FakeExecutor(vc, foot={"b0": 500})
    srv2 = Server(_specs(1), big, hbm_budget=100, clock=vc.clock, sleep=vc.sleep)
    assert srv2.request(0) == "rejected"


def test_continuous_batching_and_order():
    vc = VClock()
    ex = FakeExecutor(vc, per_block=0.02, fixed=0.15)
    specs = _specs(6)
    srv = Server(specs, ex, hbm_budget=10_000, max_inflight=2, clock=vc.clock, sleep=vc.sleep)
    for i in range(6):
        assert srv.request(i) == "admitted"
    sched = poisson_schedule(specs, n_blocks=8, seed=1, jitter_mean_s=0.05, phases=[0.01 * i for i in range(6)])
    st = srv.run(sched)
    assert st.blocks == 48
    # each beam's blocks complete in sequence order, each exactly once
    for i in range(6):
        seqs = [r.seq for r in srv.results if r.beam == i]
        assert seqs == list(range(8))
    # launches carry blocks of several beams; no beam appears twice in one launch
    assert max(len(l) for l in ex.launches) > 1
    for l in ex.launches:
        beams = [b for b, _ in l]
        assert len(beams) == len(set(beams))
    # blocks that arrived while a launch ran went into a later launch, not a new queue
    assert st.launches < st.blocks


def test_inflight_limit_and_latency_accounting():
    vc = VClock()
    ex = FakeExecutor(vc, per_block=0.0, fixed=0.4)
    specs = _specs(2, block_s=1.0)
    srv = Server(specs, ex, hbm_budget=10_000, max_inflight=1, clock=vc.clock, sleep=vc.sleep)
    srv.request(0), srv.request(1)
    sched = [Block(0.0, 0, 0), Block(0.0, 1, 0), Block(1.0, 0, 1), Block(1.0, 1, 1)]
    st = srv.run(sched)
    assert st.blocks == 4 and st.deadline_misses == 0
    assert all(abs(l - 0.4) < 0.01 for l in st.latencies)
    slow = FakeExecutor(vc, per_block=0.0, fixed=1.5)
    srv2 = Server(specs, slow, hbm_budget=10_000, max_inflight=1, clock=vc.clock, sleep=vc.sleep)
    srv2.request(0), srv2.request(1)
    st2 = srv2.run([Block(0.0, 0, 0), Block(1.0, 0, 1), Block(2.0, 0, 2)])
    assert st2.deadline_misses >= 2


def test_fill_blocks_excluded_from_latency():
    vc = VClock()
    ex = FakeExecutor(vc, fixed=0.1, fill_blocks=3)
    specs = _specs(1)
    srv = Server(specs, ex, hbm_budget=10_000, clock=vc.clock, sleep=vc.sleep)
    srv.request(0)
    st = srv.run([Block(float(k), 0, k) for k in range(5)])
    assert st.fill_blocks == 3 and len(st.latencies) == 2
    s = st.summary()
    assert s["blocks"] == 5 and s["latency_p99_s"] > 0


def test_blocks_wait_for_admission():
    vc = VClock()
    ex = FakeExecutor(vc, foot=60, fixed=0.1)
    specs = _specs(2)
    srv = Server(specs, ex, hbm_budget=100, clock=vc.clock, sleep=vc.sleep)
    assert srv.request(0) == "admitted" and srv.request(1) == "queued"
    st = srv.run([Block(0.0, 0, 0), Block(0.0, 1, 0)])
    # beam 1 never got memory: its block is still unserved, beam 0's was served
    assert [r.beam for r in srv.results] == [0]


def test_waiting_beam_admitted_when_memory_frees_during_run():
    vc = VClock()
    specs = _specs(3)
    ex = FakeExecutor(vc, foot=100)
    srv = Server(specs, ex, hbm_budget=200, clock=vc.clock, sleep=vc.sleep)
    assert [srv.request(i) for i in range(3)] == ["admitted", "admitted", "queued"]
    # beam 0 streams 2 blocks, beam 1 six, beam 2 (queued) four from the start
    sched = ([Block(k * 1.0, 0, k) for k in range(2)] + [Block(k * 1.0, 1, k) for k in range(6)]
             + [Block(k * 1.0, 2, k) for k in range(4)])
    st = srv.run(sched, release_done=True)
    assert st.blocks == 12 and st.admitted == 3 and st.admitted_in_run == 1
    assert ex.opened == [0, 1, 2] and sorted(ex.closed) == [0, 1, 2]
    # beam 2 could only start after beam 0's last block completed (~t = 1 s)
    first2 = min(r.done for r in srv.results if r.beam == 2)
    last0 = max(r.done for r in srv.results if r.beam == 0)
    assert first2 >= last0
    # its blocks keep their order and all complete
    seqs = [r.seq for r in srv.results if r.beam == 2]
    assert seqs == sorted(seqs) == [0, 1, 2, 3]
    assert srv.used == 0 and not srv.active
