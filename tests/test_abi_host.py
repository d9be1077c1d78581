"""The C ABI without a GPU: every declared symbol is exported, host-only calls validate and
the FP64 delay table matches the oracle bit for bit (Eq. deltaTEq)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import fbsynth
from oracle import dedisp_oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
lib_mod = pytest.importorskip("paper_1401_8258_amd._lib")


@pytest.fixture(scope="module")
def lib():
    try:
        return lib_mod.load()
    except lib_mod.LibraryMissing as e:  # the build step has not run in this checkout
        pytest.skip(str(e))


def _header_functions():
    with open(os.path.join(ROOT, "include", "dedisp.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dd_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = _header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
        assert n in lib_mod.SIGNATURES, n
    assert lib.dd_version().decode() == "1.5"


def _create(lib, freq, dm, tsamp, dtype=0, tuning=None):
    h = C.c_void_p()
    f = np.ascontiguousarray(freq, np.float64)
    d = np.ascontiguousarray(dm, np.float64)
    dbl = C.POINTER(C.c_double)
    tun = C.byref(lib_mod.Tuning(*tuning)) if tuning else None
    rc = lib.dd_plan_create(C.byref(h), f.ctypes.data_as(dbl), f.size, tsamp, d.ctypes.data_as(dbl), d.size,
                            dtype, tun)
    return rc, h


def _delays(lib, h, nchan, ndm):
    out = np.empty((nchan, ndm), np.int32)
    assert lib.dd_plan_delays(h, out.ctypes.data_as(C.POINTER(C.c_int32))) == 0
    return out


@pytest.mark.parametrize("name,nchan,f_top,bw,tsamp,step,ndm", [
    ("64ch small", 64, 428.0, 20.0, 51.2e-6, 0.1, 128),
    ("1024ch full", 1024, 428.0, 20.0, 51.2e-6, 0.1, 2048),
    ("4096ch low band", 4096, 180.0, 60.0, 81.92e-6, 0.05, 4096),
    ("256ch wide step", 256, 428.0, 20.0, 51.2e-6, 0.2, 4096),
])
def test_delay_table_bit_exact(lib, name, nchan, f_top, bw, tsamp, step, ndm):
    freq = fbsynth.channel_freqs(f_top, bw / nchan, nchan)
    dm = fbsynth.dm_trials(0.0, step, ndm)
    rc, h = _create(lib, freq, dm, tsamp)
    assert rc == 0
    try:
        got = _delays(lib, h, nchan, ndm)
        want = orc.delay_table(freq, dm, tsamp)
        np.testing.assert_array_equal(got, want)
        # guard: no entry sits within 1e-9 of a rounding tie, so FP64 evaluation order cannot flip one
        x = orc.delay_seconds(freq, dm) / tsamp
        frac = x - np.floor(x)
        assert np.min(np.abs(frac - 0.5)) > 1e-9
        info = lib_mod.PlanInfo()
        assert lib.dd_plan_query(h, 1 << 20, C.byref(info)) in (0, -2)
        assert info.maxdelay == want.max()
    finally:
        lib.dd_plan_destroy(h)


def test_known_maxdelays(lib):
    for freq, dm, tsamp, want in [
        (fbsynth.channel_freqs(428.0, 0.3125, 64), fbsynth.dm_trials(0, 0.1, 128), 51.2e-6, 555),
        (fbsynth.channel_freqs(428.0, 20 / 1024, 1024), fbsynth.dm_trials(0, 0.1, 2048), 51.2e-6, 9088),
    ]:
        rc, h = _create(lib, freq, dm, tsamp)
        assert rc == 0
        info = lib_mod.PlanInfo()
        assert lib.dd_plan_query(h, 16384 if want == 555 else 1 << 20, C.byref(info)) == 0
        assert info.maxdelay == want
        assert info.nout == (16384 if want == 555 else 1 << 20) - want
        assert info.adds == info.ndm * info.nchan * info.nout
        lib.dd_plan_destroy(h)


def test_plan_validation_codes(lib):
    f = [428.0, 427.0, 426.0]
    bad = [
        ([428.0, -1.0], [1.0], 1e-4, 0),
        ([428.0, float("inf")], [1.0], 1e-4, 0),
        (f, [-0.1], 1e-4, 0),
        (f, [float("nan")], 1e-4, 0),
        (f, [2.0, 1.0], 1e-4, 0),        # decreasing DMs
        (f, [1.0], 0.0, 0),
        (f, [1.0], -1.0, 0),
        (f, [1.0], 1e-4, 7),             # unknown dtype
        (f, [1e12], 1e-9, 0),            # delay beyond int32
    ]
    for freq, dm, tsamp, dt in bad:
        rc, h = _create(lib, freq, dm, tsamp, dt)
        assert rc == lib_mod.DD_ERR_INVALID_ARG, (freq, dm, tsamp, dt)
        assert not h.value
        assert len(lib.dd_last_error()) > 0
    rc, h = _create(lib, f, [1.0], 1e-4, 0, tuning=(3, 4, 8, 0))
    assert rc == lib_mod.DD_ERR_UNSUPPORTED
    rc, h = _create(lib, f, [1.0], 1e-4, 0, tuning=(8, 4, 16, 0))
    assert rc == lib_mod.DD_ERR_UNSUPPORTED
    rc, h = _create(lib, f, [1.0], 1e-4, 0, tuning=(8, 4, 8, 33))
    assert rc == lib_mod.DD_ERR_UNSUPPORTED
    rc, h = _create(lib, [], [1.0], 1e-4)
    assert rc == lib_mod.DD_ERR_INVALID_ARG
    lib.dd_plan_destroy(None)  # null-safe
    lib.dd_stream_destroy(None)
    # detrending rejects bad shapes before any launch
    assert lib.dd_detrend(None, 1, 1, 1, 0, None, None) == lib_mod.DD_ERR_INVALID_ARG
    for nrows, n, stride in [(0, 5, 5), (1, 0, 5), (2, 6, 5)]:
        assert lib.dd_detrend(C.c_void_p(256), nrows, n, stride, 1, None, None) == lib_mod.DD_ERR_INVALID_ARG
    # boxcar levels: bad shapes, levels out of range, an output row too short
    p256 = C.c_void_p(256)
    for args in [(None, 1, 8, 8, 2, p256, 100), (p256, 1, 8, 8, 7, p256, 100), (p256, 1, 8, 8, -1, p256, 100),
                 (p256, 1, 8, 8, 2, p256, 13), (p256, 0, 8, 8, 2, p256, 100), (p256, 1, 8, 7, 2, p256, 100)]:
        assert lib.dd_boxcar(*args, None) == lib_mod.DD_ERR_INVALID_ARG, args


def test_query_too_short_and_sizes(lib):
    freq = fbsynth.channel_freqs(428.0, 0.3125, 64)
    rc, h = _create(lib, freq, fbsynth.dm_trials(0, 0.1, 128), 51.2e-6)
    assert rc == 0
    info = lib_mod.PlanInfo()
    assert lib.dd_plan_query(h, 555, C.byref(info)) == lib_mod.DD_ERR_TOO_SHORT
    assert info.maxdelay == 555 and info.nout == 0
    assert b"maxdelay" in lib.dd_last_error()
    assert lib.dd_plan_query(h, 556, C.byref(info)) == 0 and info.nout == 1
    assert info.workspace_bytes >= 64 * 128 * 4
    assert info.ring_bytes >= 64 * (556 + 555) * 4
    # device entry points reject bad arguments before touching the GPU
    assert lib.dd_dedisperse(h, None, 1000, 1000, None, 1000, None, None, 0.0, None, 0, None, None, 0,
                             None) == lib_mod.DD_ERR_INVALID_ARG
    lib.dd_plan_destroy(h)


def test_explicit_channel_order(lib):
    """Frequencies in any order: f_ref is the largest, each channel keeps its own delay."""
    freq = fbsynth.channel_freqs(428.0, 0.3125, 64)
    perm = np.random.default_rng(0).permutation(64)
    dm = fbsynth.dm_trials(0, 0.1, 40)
    rc, h = _create(lib, freq[perm], dm, 51.2e-6)
    assert rc == 0
    got = _delays(lib, h, 64, 40)
    np.testing.assert_array_equal(got, orc.delay_table(freq, dm, 51.2e-6)[perm])
    lib.dd_plan_destroy(h)


def _launch_ok(lib, freq, dm, tsamp, dtype=0, tuning=None, nsamp=1 << 20):
    rc, h = _create(lib, freq, dm, tsamp, dtype, tuning)
    assert rc == 0, lib.dd_last_error()
    info = lib_mod.PlanInfo()
    lib.dd_plan_query(h, nsamp, C.byref(info))
    lib.dd_plan_destroy(h)
    return info


def test_every_workload_has_a_launch_geometry(lib):
    """Each plan the tests and the benchmark build must have a ring that fits in LDS."""
    cases = []
    b1 = fbsynth.config1()
    cases.append((b1.freq_mhz, b1.dm, b1.tsamp_s, 0, None))
    f2 = fbsynth.channel_freqs(428.0, 20 / 1024, 1024)
    cases.append((f2, fbsynth.dm_trials(0, 0.1, 2048), 51.2e-6, 0, None))
    for scale, tun in [(1.0, None), (1 / 64, (8, 2, 8, 0)), (1 / 16, (8, 1, 8, 0))]:
        for sp in fbsynth.config4_specs(scale=scale):
            f = fbsynth.channel_freqs(sp["f_top"], sp["bw"] / sp["nchan"], sp["nchan"])
            cases.append((f, fbsynth.dm_trials(sp["dm0"], sp["step"], sp["ndm"]), sp["tsamp"], 2, tun))
    for sp in fbsynth.config5_specs()[::8]:
        f = fbsynth.channel_freqs(sp["f_top"], sp["bw"] / sp["nchan"], sp["nchan"])
        cases.append((f, fbsynth.dm_trials(sp["dm0"], sp["step"], sp["ndm"]), sp["tsamp"], 2, None))
    for freq, dm, tsamp, dt, tun in cases:
        info = _launch_ok(lib, freq, dm, tsamp, dt, tun)
        if dt == 2 and tun is None:
            # 8-bit input takes the direct-read form by default: no LDS, 1024-sample tiles
            assert info.kernel_form == lib_mod.DD_FORM_DIRECT
            assert info.launch_lds == 0 and info.launch_buf == 2048 and info.samples_per_lane == 16
            assert (info.dms_per_wave, info.waves) == (2, 4)
            # the same beam in the LDS form must also fit
            info = _launch_ok(lib, freq, dm, tsamp, dt, (0, 0, 0, 0, 0, lib_mod.DD_FORM_LDS))
            assert info.kernel_form == lib_mod.DD_FORM_LDS
        assert info.launch_ring >= 2 and 0 < info.launch_lds <= 160 * 1024, (len(freq), len(dm), tun)
        assert info.launch_buf % 64 == 0 and info.launch_copies == 4


def test_producer_wavefront_plans(lib):
    """Producer wavefronts (FP32 only; the default there): tuning checks and the ring bounds
    they need. The automatic FP32 plan is the 4-trial form, 14 computing wavefronts beside 2
    producers.

    Each producer issues whole stage channels: L/64 16-byte DMAs for the four copies and
    one for the trial offsets, so (cs / producers) * (L/64 + 1) per stage, and with nb - 1
    stages ahead no more than the 63 a wavefront can have outstanding.
    """
    freq = fbsynth.channel_freqs(428.0, 20 / 1024, 1024)
    dm = fbsynth.dm_trials(0, 0.1, 2048)
    auto = _launch_ok(lib, freq, dm, 51.2e-6)
    assert (auto.dms_per_wave, auto.waves, auto.producer_waves, auto.launch_stage, auto.launch_ring) == \
        (4, 14, 2, 6, 2)
    eight = _launch_ok(lib, freq, dm, 51.2e-6, 0, (8, 0, 8, 0, 0))
    assert (eight.dms_per_wave, eight.waves, eight.producer_waves, eight.launch_stage) == (8, 6, 2, 6)
    plain = _launch_ok(lib, freq, dm, 51.2e-6, 0, (8, 0, 8, 0, -1))
    assert plain.producer_waves == 0 and plain.waves == 8  # every wavefront issues its share
    assert _launch_ok(lib, freq, dm, 51.2e-6, 0, (8, 8, 8, 0, 0)).producer_waves == 0  # no room beside 8
    for dt in (1, 2):
        assert _launch_ok(lib, freq, dm, 51.2e-6, dt).producer_waves == 0
    for pw in (1, 2, 3, 4):
        info = _launch_ok(lib, freq, dm, 51.2e-6, 0, (8, 0, 8, 0, pw))
        assert info.producer_waves == pw and info.waves + pw <= 8
        assert info.launch_stage % pw == 0 and info.launch_buf % 64 == 0 and info.launch_buf // 64 <= 16
        ndw = info.launch_stage // pw * (info.launch_buf // 64 + 1)
        assert (info.launch_ring - 1) * ndw <= 63 and info.launch_ring >= 2
        assert info.launch_lds == info.launch_ring * info.launch_stage * (4 * info.launch_buf + 64) * 4
        assert info.launch_lds <= 160 * 1024
    # explicit shapes
    info = _launch_ok(lib, freq, dm, 51.2e-6, 0, (8, 6, 8, 6, 2))
    assert (info.waves, info.producer_waves, info.launch_stage, info.launch_ring) == (6, 2, 6, 2)
    for bad in [(8, 7, 8, 0, 2), (8, 8, 8, 0, 1), (8, 5, 8, 0, 4), (8, 0, 8, 0, 5)]:
        rc, _ = _create(lib, freq, dm, 51.2e-6, 0, bad)
        assert rc == lib_mod.DD_ERR_UNSUPPORTED, bad
    for dt in (1, 2):  # FP16 and u8 input take no producer
        rc, _ = _create(lib, freq, dm, 51.2e-6, dt, (8, 0, 8, 0, 1))
        assert rc == lib_mod.DD_ERR_UNSUPPORTED and b"FP32" in lib.dd_last_error()
    # one channel, two producers: the stage repeats the channel for the second producer
    info = _launch_ok(lib, [400.0], [0.0, 1.0], 51.2e-6, 0, (8, 0, 8, 0, 2))
    assert info.producer_waves == 2 and info.launch_stage == 2
    # windows wider than 1024 words cannot go through the 16 per-lane descriptors: an
    # explicit request fails, the automatic choice falls back to every wavefront issuing
    wide_f, wide_dm = fbsynth.channel_freqs(428.0, 3.75, 16), fbsynth.dm_trials(0, 2.0, 64)
    rc, _ = _create(lib, wide_f, wide_dm, 51.2e-6, 0, (8, 0, 8, 0, 1))
    assert rc == lib_mod.DD_ERR_UNSUPPORTED
    assert _launch_ok(lib, wide_f, wide_dm, 51.2e-6).producer_waves == 0


def _binning(lib, freq, tsamp, dms, max_log2):
    freq = np.ascontiguousarray(freq, dtype=np.float64)
    dms = np.ascontiguousarray(dms, dtype=np.float64)
    out = np.full(dms.size, -7, dtype=np.int32)
    diag = C.c_double()
    dbl = C.POINTER(C.c_double)
    rc = lib.dd_time_binning(freq.ctypes.data_as(dbl), int(freq.size), float(tsamp), dms.ctypes.data_as(dbl),
                             int(dms.size), int(max_log2), C.byref(diag), out.ctypes.data_as(C.POINTER(C.c_int32)))
    return rc, diag.value, out



def test_four_trial_producer_plans(lib):
    """4 DM trials per computing wavefront: FP32 producer form only, at most 14 computing
    wavefronts and 16 in all (1024 threads); other dtypes, no producer, or too many
    wavefronts are refused."""
    freq = fbsynth.channel_freqs(428.0, 20.0 / 1024, 1024)
    dms = fbsynth.dm_trials(0.0, 0.1, 2048)
    info = lib_mod.PlanInfo()
    for tun, waves in [((4, 14, 8, 0, 2, 0), 14), ((4, 0, 8, 0, 2, 0), 14), ((4, 7, 8, 3, 1, 0), 7)]:
        rc, h = _create(lib, freq, dms, 51.2e-6, 0, tun)
        assert rc == 0, lib.dd_last_error()
        lib.dd_plan_query(h, 1 << 20, C.byref(info))
        assert (info.dms_per_wave, info.waves) == (4, waves)
        assert info.producer_waves == tun[4] and info.kernel_form == lib_mod.DD_FORM_LDS
        assert 4 * waves <= 64  # one DMA of 64 lanes carries a group's trial offsets
        lib.dd_plan_destroy(h)
    for dtype, tun in [(0, (4, 15, 8, 0, 1, 0)), (0, (4, 14, 8, 0, 3, 0)), (0, (4, 8, 8, 0, -1, 0)),
                       (1, (4, 8, 8, 0, 0, 0)), (2, (4, 8, 8, 0, 0, lib_mod.DD_FORM_LDS)),
                       (0, (6, 8, 8, 0, 2, 0))]:
        rc, h = _create(lib, freq, dms, 51.2e-6, dtype, tun)
        assert rc == lib_mod.DD_ERR_UNSUPPORTED, (dtype, tun)
        assert not h.value

@pytest.mark.parametrize("f_top,nchan,bw,tsamp,step,ndm,max_log2", [
    (428.0, 64, 20.0, 51.2e-6, 0.1, 128, 4),
    (428.0, 1024, 20.0, 51.2e-6, 0.1, 2048, 4),
    (428.0, 1024, 20.0, 51.2e-6, 0.1, 2048, 2),
    (180.0, 4096, 60.0, 81.92e-6, 0.05, 4096, 16),
    (428.0, 256, 20.0, 51.2e-6, 0.2, 700, 0),
])
def test_time_binning_matches_oracle(lib, f_top, nchan, bw, tsamp, step, ndm, max_log2):
    """The planner's diagonal DM and factors equal the oracle's (same FP64 decision)."""
    freq = fbsynth.channel_freqs(f_top, bw / nchan, nchan)
    dms = fbsynth.dm_trials(0.0, step, ndm)
    rc, diag, k = _binning(lib, freq[::-1].copy(), tsamp, dms, max_log2)  # any channel order
    assert rc == 0
    assert diag == orc.diagonal_dm(freq, tsamp)
    np.testing.assert_array_equal(k, orc.binning_factors(freq, tsamp, dms, max_log2))
    # boundary trials at exactly 2^k DM_diag and one ulp above
    edge = np.array(sorted({0.0} | {v for j in range(4) for v in (diag * 2 ** j, np.nextafter(diag * 2 ** j, np.inf))}))
    rc, _, k2 = _binning(lib, freq, tsamp, edge, 10)
    assert rc == 0
    np.testing.assert_array_equal(k2, orc.binning_factors(freq, tsamp, edge, 10))


def test_time_binning_and_downfactor_arguments(lib):
    freq = fbsynth.channel_freqs(428.0, 0.3125, 64)
    assert _binning(lib, [400.0], 1e-4, [0.0, 5.0], 3)[:2] == (0, float("inf"))
    for f, ts, dms, ml in [(freq, 0.0, [1.0], 2), (freq, 1e-4, [2.0, 1.0], 2), (freq, 1e-4, [-1.0], 2),
                           (freq, 1e-4, [1.0], 17), (freq, 1e-4, [1.0], -1), ([400.0, float("nan")], 1e-4, [1.0], 2),
                           ([400.0, 0.0], 1e-4, [1.0], 2)]:
        assert _binning(lib, f, ts, dms, ml)[0] == lib_mod.DD_ERR_INVALID_ARG, (ts, dms, ml)
    p256 = C.c_void_p(256)
    for args in [(None, 0, 4, 8, 8, p256, 4), (p256, 0, 4, 8, 8, None, 4), (p256, 3, 4, 8, 8, p256, 4),
                 (p256, 0, 0, 8, 8, p256, 4), (p256, 0, 4, 1, 8, p256, 4), (p256, 0, 4, 8, 7, p256, 4),
                 (p256, 0, 4, 9, 9, p256, 3)]:
        assert lib.dd_downfactor(*args, None) == lib_mod.DD_ERR_INVALID_ARG, args
    assert lib.dd_downfactor(p256, 0, 70000, 8, 8, p256, 4, None) == lib_mod.DD_ERR_UNSUPPORTED



def _binned(lib, freq, tsamp, dms, dtype, max_log2):
    h = C.c_void_p()
    f = np.ascontiguousarray(freq, np.float64)
    d = np.ascontiguousarray(dms, np.float64)
    dbl = C.POINTER(C.c_double)
    rc = lib.dd_binned_create(C.byref(h), f.ctypes.data_as(dbl), f.size, tsamp, d.ctypes.data_as(dbl), d.size,
                              dtype, max_log2, None)
    assert rc == 0
    n = C.c_int32()
    assert lib.dd_binned_query(h, 0, C.byref(n), None, 0, None, None) == lib_mod.DD_ERR_INVALID_ARG
    runs = (lib_mod.BinnedRun * n.value)()
    lib.dd_binned_query(h, 0, None, runs, n.value, None, None)
    return h, list(runs)


def test_binned_runs_and_stream_sizes(lib):
    """Binned runs follow the oracle's factors; a binned stream's ring is every run's stream
    ring (each at block >> log2 samples, 256-byte aligned) and its blocks must be multiples
    of the largest factor."""
    freq = fbsynth.channel_freqs(428.0, 20.0 / 1024, 1024)
    dms = fbsynth.dm_trials(0.0, 0.1, 2048)
    h, runs = _binned(lib, freq, 51.2e-6, dms, 0, 4)
    try:
        k = orc.binning_factors(freq, 51.2e-6, dms, 4)
        assert [(r.log2, r.d0, r.d1) for r in runs] == [
            (int(k[d0]), d0, d1) for d0, d1 in zip([0] + [i for i in range(1, k.size) if k[i] != k[i - 1]],
                                                   [i for i in range(1, k.size) if k[i] != k[i - 1]] + [k.size])]
        kmax = max(r.log2 for r in runs)
        assert kmax == 4
        block = 19536  # a multiple of 16
        rb, wb = C.c_int64(), C.c_int64()
        assert lib.dd_binned_stream_query(h, block, C.byref(rb), C.byref(wb)) == 0
        want = 0
        for r in runs:
            rc, p = _create(lib, freq, dms[r.d0:r.d1], 51.2e-6 * (1 << r.log2))
            assert rc == 0
            info = lib_mod.PlanInfo()
            lib.dd_plan_query(p, block >> r.log2, C.byref(info))
            want += -(-info.ring_bytes // 256) * 256
            lib.dd_plan_destroy(p)
        assert rb.value == want
        assert wb.value > 0
        for bad in (0, -16, 8, 19537, 19528):
            assert lib.dd_binned_stream_query(h, bad, C.byref(rb), C.byref(wb)) == lib_mod.DD_ERR_INVALID_ARG, bad
            assert rb.value == 0 and wb.value == 0
        assert lib.dd_binned_stream_query(None, block, None, None) == lib_mod.DD_ERR_INVALID_ARG
        out = C.c_void_p(1)
        assert lib.dd_binned_stream_create(h, block, None, 1 << 40, None, C.byref(out)) == lib_mod.DD_ERR_INVALID_ARG
        assert out.value is None
        assert lib.dd_binned_stream_create(h, block, C.c_void_p(256), rb.value - 1, None,
                                           C.byref(out)) == lib_mod.DD_ERR_WORKSPACE
        assert lib.dd_binned_stream_create(h, 8, C.c_void_p(256), 1 << 40, None,
                                           C.byref(out)) == lib_mod.DD_ERR_INVALID_ARG
        t0 = (C.c_int64 * len(runs))(*([7] * len(runs)))
        assert lib.dd_binned_stream_push(None, None, 16, 16, 0, None, 16, None, None, 0.0, None, 0, None, 0, None, 0,
                                         None, t0, None) == lib_mod.DD_ERR_INVALID_ARG
        assert lib.dd_binned_stream_set_gap_fill(None, 1) == lib_mod.DD_ERR_INVALID_ARG
        lib.dd_binned_stream_destroy(None)
    finally:
        lib.dd_binned_destroy(h)

@pytest.mark.parametrize("nchan,order", [(1, 0), (2, 1), (64, 4), (1024, 8), (4096, 12)])
def test_bandpass_fit_matches_oracle(lib, nchan, order):
    """The host fit (Gram-Schmidt projection) equals the oracle's numpy least squares."""
    rng = np.random.default_rng(nchan + order)
    c = np.arange(nchan)
    avg = 10.0 + 3.0 * np.sin(np.pi * c / max(nchan, 1)) + 0.05 * rng.standard_normal(nchan)
    avg[nchan // 3] += 4.0
    fit = np.empty(nchan)
    rmse, fmean = C.c_double(), C.c_double()
    dbl = C.POINTER(C.c_double)
    assert lib.dd_bandpass_fit(avg.ctypes.data_as(dbl), nchan, order, fit.ctypes.data_as(dbl), C.byref(rmse),
                               C.byref(fmean)) == 0
    want, wr, wm = orc.bandpass_fit(avg, order)
    np.testing.assert_allclose(fit, want, rtol=0, atol=1e-9)
    assert abs(rmse.value - wr) < 1e-9 and abs(fmean.value - wm) < 1e-9


def test_rfi_arguments(lib):
    dbl = C.POINTER(C.c_double)
    a = np.ones(8)
    f = np.empty(8)
    for n, order in [(0, 0), (8, 8), (8, -1), (20, 17)]:
        assert lib.dd_bandpass_fit(a.ctypes.data_as(dbl), n, order, f.ctypes.data_as(dbl), None, None) == \
            lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_bandpass_fit(None, 8, 1, f.ctypes.data_as(dbl), None, None) == lib_mod.DD_ERR_INVALID_ARG
    p = C.c_void_p(256)
    assert lib.dd_bandpass(None, 4, 8, 8, 0, p, None, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_bandpass(p, 4, 8, 7, 0, p, None, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_bandpass(p, 4, 8, 8, 4, p, None, None) == lib_mod.DD_ERR_INVALID_ARG   # window without means
    assert lib.dd_bandpass(p, 4, 8, 8, 0, p, p, None) == lib_mod.DD_ERR_INVALID_ARG      # means without window
    assert lib.dd_rfi_clip(p, 4, 8, 8, None, 1.0, 4, p, p, 0.0, 1.0, 1, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_rfi_clip(p, 4, 8, 8, p, 1.0, 0, p, p, 0.0, 1.0, 1, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_rfi_clip(p, 4, 8, 8, p, 1.0, 4, p, None, 0.0, 1.0, 1, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_rfi_clip(p, 4, 8, 8, p, 1.0, 4, None, p, 0.0, 1.0, 1, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_rfi_clip(p, 70000, 8, 8, p, 1.0, 4, p, p, 0.0, 1.0, 1, None) == lib_mod.DD_ERR_UNSUPPORTED
    # the 8-bit forms validate the same way (no correction argument)
    assert lib.dd_bandpass_u8(None, 4, 8, 8, 0, p, None, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_bandpass_u8(p, 4, 8, 7, 0, p, None, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_bandpass_u8(p, 4, 8, 8, 4, p, None, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_bandpass_u8(p, 0, 8, 8, 0, p, None, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_rfi_clip_u8(p, 4, 8, 8, None, 1.0, 4, p, p, 0.0, 1.0, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_rfi_clip_u8(p, 4, 8, 8, p, 1.0, 0, p, p, 0.0, 1.0, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_rfi_clip_u8(p, 4, 8, 8, p, 1.0, 4, p, None, 0.0, 1.0, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_rfi_clip_u8(p, 4, 0, 8, p, 0.0, 4, p, p, 0.0, 1.0, None) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_rfi_clip_u8(p, 70000, 8, 8, p, 1.0, 4, p, p, 0.0, 1.0, None) == lib_mod.DD_ERR_UNSUPPORTED


def test_boxcar_search_arguments(lib):
    """Workspace sizes and every refused argument of dd_boxcar_search (checked before any launch)."""
    ws = C.c_int64()
    assert lib.dd_boxcar_search_workspace(3, 10000, C.byref(ws)) == 0
    # counts int32 and offsets int64 per (row, 4096-start segment), each region 256-aligned
    assert ws.value == 256 + 256
    assert lib.dd_boxcar_search_workspace(2048, 1 << 20, C.byref(ws)) == 0 and ws.value == 2048 * 256 * 12
    assert lib.dd_boxcar_search_workspace(0, 10, C.byref(ws)) == lib_mod.DD_ERR_INVALID_ARG
    assert lib.dd_boxcar_search_workspace(1, 10, None) == lib_mod.DD_ERR_INVALID_ARG
    p = C.c_void_p(256)
    ok = dict(series=p, nrows=4, n=100, stride=100, mean=p, rms=p, ml=6, k=5.0, out=p, cap=8, cnt=p, ws=p,
              wsb=1 << 20)

    def call(**kw):
        a = dict(ok, **kw)
        return lib.dd_boxcar_search(a["series"], a["nrows"], a["n"], a["stride"], a["mean"], a["rms"], a["ml"],
                                    a["k"], a["out"], a["cap"], a["cnt"], a["ws"], a["wsb"], None)

    bad = lib_mod.DD_ERR_INVALID_ARG
    for kw in [dict(series=None), dict(cnt=None), dict(ws=None), dict(nrows=0), dict(n=0), dict(stride=99),
               dict(mean=None), dict(rms=None), dict(ml=7), dict(ml=-1), dict(k=float("nan")), dict(k=float("inf")),
               dict(cap=-1), dict(out=None)]:
        assert call(**kw) == bad, kw
    assert call(wsb=100) == lib_mod.DD_ERR_WORKSPACE
    assert call(nrows=70000) == lib_mod.DD_ERR_UNSUPPORTED


def _info(lib, h, nsamp=1 << 20):
    info = lib_mod.PlanInfo()
    assert lib.dd_plan_query(h, nsamp, C.byref(info)) in (0, -2)
    return info


def test_register_window_form_plan(lib):
    """DD_FORM_REGWIN: 64-trial groups, one staged copy, windows sized by the delay spread of
    eight consecutive trials; refused for other dtypes and for spreads past 40 samples."""
    freq = fbsynth.channel_freqs(428.0, 20.0 / 1024, 1024)
    dm = fbsynth.dm_trials(0.0, 0.1, 2048)
    rc, h = _create(lib, freq, dm, 51.2e-6, tuning=(0, 0, 0, 0, 0, lib_mod.DD_FORM_REGWIN))
    assert rc == 0
    try:
        info = _info(lib, h)
        assert info.kernel_form == lib_mod.DD_FORM_REGWIN and info.launch_copies == 1
        assert (info.dms_per_wave, info.waves, info.samples_per_lane) == (8, 8, 8)
        # eight consecutive trials spread at most 7 * 4.44 samples in the bottom channel; with up
        # to 7 samples of alignment and the lane's 8 outputs a window needs 12 chunks of 4
        tab = orc.delay_table(freq, dm, 51.2e-6)
        spread8 = max(int((tab[:, d + 7] - tab[:, d]).max()) for d in range(0, 2048, 8))
        assert spread8 == 32
        assert info.window_chunks == 12
        assert info.launch_lds <= 160 * 1024 and info.launch_ring >= 2
        np.testing.assert_array_equal(_delays(lib, h, 1024, 2048), tab)
    finally:
        lib.dd_plan_destroy(h)
    # the LDS form is chosen by default and on request
    rc, h = _create(lib, freq, dm, 51.2e-6, tuning=(0, 0, 0, 0, 0, lib_mod.DD_FORM_LDS))
    assert rc == 0
    assert _info(lib, h).kernel_form == lib_mod.DD_FORM_LDS and _info(lib, h).launch_copies == 4
    lib.dd_plan_destroy(h)
    # twice the DM step: 8 trials spread 62 samples in the bottom channel
    rc, h = _create(lib, freq, 2 * dm, 51.2e-6, tuning=(0, 0, 0, 0, 0, lib_mod.DD_FORM_REGWIN))
    assert rc == lib_mod.DD_ERR_UNSUPPORTED and not h.value
    assert "register window" in lib.dd_last_error().decode()
    rc, h = _create(lib, freq, dm, 51.2e-6, dtype=lib_mod.DD_U8, tuning=(0, 0, 0, 0, 0, lib_mod.DD_FORM_REGWIN))
    assert rc == lib_mod.DD_ERR_UNSUPPORTED
    rc, h = _create(lib, freq, dm, 51.2e-6, tuning=(0, 0, 0, 0, 0, 7))
    assert rc == lib_mod.DD_ERR_UNSUPPORTED
