"""The autotuner's search logic with a fake timer (no GPU): plans are created by the
library's host code, the timer is a table of made-up milliseconds."""
import numpy as np
import pytest

import fbsynth

lib_mod = pytest.importorskip("paper_1401_8258_amd._lib")


@pytest.fixture(scope="module")
def at():
    try:
        lib_mod.load()
    except lib_mod.LibraryMissing as e:
        pytest.skip(str(e))
    from paper_1401_8258_amd import autotune
    return autotune


def _beam(nchan, ndm, step=0.1):
    return (fbsynth.channel_freqs(428.0, 20.0 / nchan, nchan), 51.2e-6, fbsynth.dm_trials(0.0, step, ndm), "f32", 20000)


class FakeClock:
    """ms = base[nchan] * wave_cost[waves] * stage_cost[chan_stage]; counts its calls."""

    def __init__(self, wave_cost, stage_cost, regwin_ms=None):
        self.wave_cost, self.stage_cost, self.regwin_ms = wave_cost, stage_cost, regwin_ms
        self.calls = 0

    def __call__(self, plan, x, reps):
        self.calls += 1
        if plan.form == "regwin":
            return self.regwin_ms
        g, w, cc = plan.tiles
        return plan.nchan / 64.0 * self.wave_cost[w] * self.stage_cost[cc]


def test_tune_picks_fastest_and_caches(at, tmp_path):
    clock = FakeClock({8: 3.0, 4: 1.0, 2: 2.0, 1: 5.0}, {0: 1.0, 2: 0.5, 4: 2.0})
    cache = at.TuneCache(str(tmp_path / "tune.json"))
    r = at.tune(*_beam(64, 96), waves=(8, 4, 2, 1), stages=(0, 2, 4), cache=cache, x=object(), timer=clock)
    assert r["form"] == "lds" and r["tuning"] == [8, 4, 2] and r["ms"] == pytest.approx(0.5)
    assert clock.calls == 12 and len(r["trials"]) == 12
    # a second call is served from the cache file, without timing
    again = at.tune(*_beam(64, 96), waves=(8, 4, 2, 1), stages=(0, 2, 4), cache=at.TuneCache(cache.path),
                    x=object(), timer=clock)
    assert again["tuning"] == [8, 4, 2] and clock.calls == 12


def test_tune_compares_kernel_forms(at):
    clock = FakeClock({8: 1.0, 4: 1.0}, {0: 1.0}, regwin_ms=0.25)
    r = at.tune(*_beam(64, 128), waves=(8, 4), stages=(0,), forms=("lds", "regwin"), x=object(), timer=clock)
    assert r["form"] == "regwin" and r["tuning"] is None
    assert at.make_plan(*_beam(64, 128)[:4], r).form == "regwin"
    clock = FakeClock({8: 1.0, 4: 1.0}, {0: 1.0}, regwin_ms=5.0)
    r = at.tune(*_beam(64, 128), waves=(8, 4), stages=(0,), forms=("lds", "regwin"), x=object(), timer=clock)
    assert r["form"] == "lds"


def test_tune_records_tilings_that_do_not_fit(at):
    # a wide band at a coarse DM step: groups of 64 trials spread beyond the LDS ring, and
    # eight consecutive trials beyond the register window
    beam = (fbsynth.channel_freqs(428.0, 3.75, 16), 51.2e-6, fbsynth.dm_trials(0.0, 2.0, 512), "f32", 200000)
    clock = FakeClock({8: 1.0, 1: 2.0}, {0: 1.0}, regwin_ms=0.1)
    r = at.tune(*beam, waves=(8, 1), stages=(0,), forms=("lds", "regwin"), x=object(), timer=clock)
    errs = [t for t in r["trials"] if "error" in t]
    assert any(t["form"] == "regwin" for t in errs)
    assert r["form"] == "lds" and "ms" in next(t for t in r["trials"] if t.get("tuning") == r["tuning"])


def test_tune_batch_own_best_or_one_wave_count(at):
    # per wave count: beam A prefers 8 waves, beam B 2; summed, 4 waves is best
    class Clock(FakeClock):
        def __call__(self, plan, x, reps):
            self.calls += 1
            g, w, cc = plan.tiles
            table = {64: {8: 1.0, 4: 1.5, 2: 3.0}, 128: {8: 5.0, 4: 2.0, 2: 1.8}}
            return table[plan.nchan][w] * (0.9 if cc == 2 else 1.0)
    clock = Clock({}, {})
    res = at.tune_batch([_beam(64, 96), _beam(128, 64)], waves=(8, 4, 2), stages=(0, 2), inputs=[object(), object()],
                        timer=clock, common_waves=True)
    assert res["waves"] == 4
    assert res["tunings"] == [[8, 4, 2], [8, 4, 2]]
    assert res["choices"] == [{"form": "lds", "tuning": [8, 4, 2]}] * 2
    # each beam's own best over all counts
    assert [o["tuning"] for o in res["own_best"]] == [[8, 8, 2], [8, 2, 2]]
    free = at.tune_batch([_beam(64, 96), _beam(128, 64)], waves=(8, 4, 2), stages=(0, 2),
                         inputs=[object(), object()], timer=clock)
    assert free["choices"] == [{"form": "lds", "tuning": [8, 8, 2]}, {"form": "lds", "tuning": [8, 2, 2]}]
    assert free["waves"] == 4 and free["total_ms"] == pytest.approx(3.15)
    assert res["by_waves"] == pytest.approx({8: 5.4, 4: 3.15, 2: 4.32})


def test_tune_batch_beam_that_misses_a_wave_count(at):
    """A beam that fits no tiling at one wavefront count keeps its own best over the others;
    that count drops out of the common-count sums."""
    class Clock(FakeClock):
        def __call__(self, plan, x, reps):
            self.calls += 1
            g, w, cc = plan.tiles
            if plan.nchan == 128 and w == 8:
                raise RuntimeError("does not fit")
            return {8: 1.0, 4: 2.0, 2: 3.0}[w] * (2.0 if plan.nchan == 128 else 1.0)
    res = at.tune_batch([_beam(64, 96), _beam(128, 64)], waves=(8, 4, 2), stages=(0,), inputs=[object(), object()],
                        timer=Clock({}, {}))
    assert [c["tuning"] for c in res["choices"]] == [[8, 8, 0], [8, 4, 0]]
    assert set(res["by_waves"]) == {4, 2} and res["waves"] == 4


def test_tune_offers_the_direct_form_for_8bit_beams(at):
    """8-bit beams: direct-read candidates (g trials per wavefront, waves) beside the LDS
    ones; other dtypes get none."""
    class Clock(FakeClock):
        def __call__(self, plan, x, reps):
            self.calls += 1
            g, w, cc = plan.tiles
            if plan.form == "direct":  # tiles = (g, w, samples_per_lane)
                return {1: 1.0, 2: 0.4, 4: 0.7}[g] * (1.0 if w == 4 else 1.5) * (0.9 if cc == 32 else 1.0)
            return 2.0
    clock = Clock({}, {})
    freq, tsamp, dm, _, nsamp = _beam(64, 96)
    r = at.tune(freq, tsamp, dm, "u8", nsamp, waves=(8, 4), stages=(0,), x=object(), timer=clock)
    assert r["form"] == "direct" and r["tuning"] == [2, 4, 32] and r["ms"] == pytest.approx(0.36)
    forms = [t["form"] for t in r["trials"]]
    assert forms.count("direct") == 10 and forms.count("lds") == 2
    assert at.make_plan(freq, tsamp, dm, "u8", r).form == "direct"
    r = at.tune(freq, tsamp, dm, "f32", nsamp, waves=(8, 4), stages=(0,), x=object(), timer=clock)
    assert all(t["form"] == "lds" for t in r["trials"])
