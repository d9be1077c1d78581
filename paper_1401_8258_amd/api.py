"""Python face of libdedisp.so: plans, one-shot dedispersion and streams on torch device memory.

Every computation runs in the library's HIP kernels; this module only allocates
device buffers with torch, passes pointers and the current HIP stream, and
unpacks results. There is no fallback: without the built library every call
raises LibraryMissing.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import warnings
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import check

CAND_DTYPE = np.dtype([("dm_index", "<i4"), ("reserved", "<i4"), ("t", "<i8"), ("value", "<f4"),
                       ("snr", "<f4")])
PULSE_DTYPE = np.dtype([("row", "<i4"), ("width", "<i4"), ("t", "<i8"), ("value", "<f4"), ("snr", "<f4")])
_TORCH_DT = {torch.float32: _lib.DD_F32, torch.float16: _lib.DD_F16, torch.uint8: _lib.DD_U8}
_NAME_DT = {"f32": torch.float32, "f16": torch.float16, "u8": torch.uint8}
# kernel forms (dd_tuning.kernel_form): "lds" stages four shifted copies per channel and reads
# one LDS word per add; "regwin" (FP32) stages one copy and adds from register windows;
# "direct" (8-bit) reads each trial's window through the caches with no LDS staging
_FORMS = {"auto": _lib.DD_FORM_AUTO, "lds": _lib.DD_FORM_LDS, "regwin": _lib.DD_FORM_REGWIN,
          "direct": _lib.DD_FORM_DIRECT}
_FORM_NAMES = {v: k for k, v in _FORMS.items()}


def _tuning(tuning, form: str):
    """The dd_tuning a (tuning tuple, form name) pair describes, by reference, or None."""
    kf = _FORMS[form]
    if tuning is not None and kf == _lib.DD_FORM_DIRECT:  # (dms_per_wave, waves[, samples_per_lane])
        g, w = int(tuning[0]), int(tuning[1])
        spl = int(tuning[2]) if len(tuning) > 2 else 0
        return C.byref(_lib.Tuning(g, w, spl, 0, 0, kf))
    if tuning is not None:  # (dms_per_wave, waves[, chan_stage[, producer_waves]])
        g, w = int(tuning[0]), int(tuning[1])
        cc = int(tuning[2]) if len(tuning) > 2 else 0
        pw = int(tuning[3]) if len(tuning) > 3 else 0
        return C.byref(_lib.Tuning(g, w, 0, cc, pw, kf))
    if kf != _lib.DD_FORM_AUTO:
        return C.byref(_lib.Tuning(0, 0, 0, 0, 0, kf))
    return None


def _vp(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def torch_dtype(dtype) -> torch.dtype:
    return _NAME_DT[dtype] if isinstance(dtype, str) else dtype


class CandidateOverflow(UserWarning):
    """More candidates qualified than the buffer held (DD_WARN_CAND_OVERFLOW)."""


@dataclasses.dataclass
class Result:
    out: torch.Tensor                 # [ndm][nout] float32 (a view when out_row_stride > nout)
    mean: Optional[torch.Tensor]      # [ndm] float32
    rms: Optional[torch.Tensor]
    t0: int = 0                       # global output time of column 0 (streams)
    _cand: Optional[torch.Tensor] = None
    _ncand: Optional[torch.Tensor] = None
    cand_cap: int = 0
    _keep: object = None

    def _check(self, stream=None):
        n = C.c_int64()
        rc = check(_lib.load().dd_candidates_check(_vp(self._ncand), int(self.cand_cap), _stream(stream), C.byref(n)),
                   (_lib.DD_OK, _lib.DD_WARN_CAND_OVERFLOW))
        return int(n.value), rc == _lib.DD_WARN_CAND_OVERFLOW

    def candidates(self, stream=None) -> Optional[np.ndarray]:
        """Detections as a structured numpy array (synchronises the stream). When more
        qualified than cand_cap, the first cand_cap in (d, t) order are returned and a
        CandidateOverflow warning names the true count (dd_candidates_check)."""
        if self._ncand is None:
            return None
        n, over = self._check(stream)
        if over:
            warnings.warn(f"{n} candidates qualified; the first {self.cand_cap} were kept", CandidateOverflow)
        keep = min(n, self.cand_cap)
        raw = self._cand[: keep * CAND_DTYPE.itemsize].cpu().numpy()
        return raw.view(CAND_DTYPE)

    def ncand(self, stream=None) -> Optional[int]:
        """The true number of candidates (may exceed cand_cap)."""
        return None if self._ncand is None else self._check(stream)[0]


class Plan:
    """A dedispersion plan: channel frequencies (MHz), sampling time (s), DM trials, input dtype."""

    def __init__(self, freq_mhz, tsamp_s: float, dm, dtype=torch.float32, tuning=None, form: str = "auto"):
        lib = _lib.load()
        self._lib = lib
        self.freq = np.ascontiguousarray(freq_mhz, dtype=np.float64)
        self.dm = np.ascontiguousarray(dm, dtype=np.float64)
        self.tsamp = float(tsamp_s)
        self.dtype = torch_dtype(dtype)
        if self.dtype not in _TORCH_DT:
            raise ValueError(f"unsupported input dtype {dtype}")
        h = C.c_void_p()
        tun = _tuning(tuning, form)
        dbl = C.POINTER(C.c_double)
        check(lib.dd_plan_create(C.byref(h), self.freq.ctypes.data_as(dbl), int(self.freq.size), self.tsamp,
                                 self.dm.ctypes.data_as(dbl), int(self.dm.size), _TORCH_DT[self.dtype], tun))
        self._h = h
        self._ws = {}
        info = self.query(1, allow_short=True)
        self.maxdelay = int(info["maxdelay"])
        self.form = _FORM_NAMES[int(info["kernel_form"])]
        # (dms_per_wave, waves, chan_stage); the direct-read form has no stages and reports
        # its samples per lane third
        third = info["samples_per_lane"] if self.form == "direct" else info["chan_stage"]
        self.tiles = (int(info["dms_per_wave"]), int(info["waves"]), int(third))
        self.producer_waves = int(info["producer_waves"])
        self.max_span = int(info["max_span"])

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    @property
    def nchan(self) -> int:
        return int(self.freq.size)

    @property
    def ndm(self) -> int:
        return int(self.dm.size)

    def query(self, nsamp: int, allow_short: bool = False) -> dict:
        inf = _lib.PlanInfo()
        allow = (_lib.DD_OK, _lib.DD_ERR_TOO_SHORT) if allow_short else (_lib.DD_OK,)
        check(self._lib.dd_plan_query(self._h, int(nsamp), C.byref(inf)), allow)
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    def delays(self) -> np.ndarray:
        out = np.empty((self.nchan, self.ndm), dtype=np.int32)
        check(self._lib.dd_plan_delays(self._h, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def workspace(self, nsamp: int, device=None, stream=None) -> torch.Tensor:
        """A device workspace for nsamp-sample inputs with this plan's delay table uploaded (cached)."""
        device = torch.device(device if device is not None else "cuda")
        nbytes = int(self.query(nsamp, allow_short=True)["workspace_bytes"])
        key = (device.index if device.index is not None else torch.cuda.current_device(), nbytes)
        ws = self._ws.get(key)
        if ws is None:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
            check(self._lib.dd_plan_upload(self._h, _vp(ws), nbytes, _stream(stream)))
            self._ws[key] = ws
        return ws

    def dedisperse(self, x: torch.Tensor, k_sigma: float = 0.0, cand_cap: int = 1 << 16, stats: bool = True,
                   out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                   stream=None) -> Result:
        """D[d][t] = sum_c x[c][t + delay(d, c)] for t < nsamp - maxdelay (Eq. bruteEquation)."""
        if x.dim() != 2 or x.shape[0] != self.nchan or x.dtype != self.dtype or not x.is_cuda:
            raise ValueError(f"x must be a CUDA [nchan={self.nchan}][nsamp] {self.dtype} tensor")
        if x.stride(1) != 1:
            raise ValueError("x rows must be contiguous in time")
        nsamp = int(x.shape[1])
        nout = nsamp - self.maxdelay
        if out is None:
            out = torch.empty((self.ndm, max(nout, 1)), dtype=torch.float32, device=x.device)
        ws = workspace if workspace is not None else self.workspace(nsamp, x.device, stream)
        mean = rms = cand = ncand = None
        if stats:
            mean = torch.empty(self.ndm, dtype=torch.float32, device=x.device)
            rms = torch.empty(self.ndm, dtype=torch.float32, device=x.device)
            if k_sigma > 0:
                cand = torch.empty(max(cand_cap, 1) * CAND_DTYPE.itemsize, dtype=torch.uint8, device=x.device)
                ncand = torch.zeros(1, dtype=torch.int64, device=x.device)
        check(self._lib.dd_dedisperse(self._h, _vp(x), nsamp, int(x.stride(0)), _vp(out), int(out.stride(0)),
                                      _vp(mean), _vp(rms), float(k_sigma), _vp(cand), int(cand_cap if cand is not None else 0),
                                      _vp(ncand), _vp(ws), int(ws.numel()), _stream(stream)))
        return Result(out[:, :nout], mean, rms, 0, cand, ncand, cand_cap)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.dd_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stream:
    """A beam's stream: device ring of maxdelay + block samples per channel (Ch. 3, buffer overlap)."""

    def __init__(self, plan: Plan, block_nsamp: int, device=None, stream=None, gap_fill: bool = False):
        self.plan = plan
        self._lib = plan._lib
        self.block = int(block_nsamp)
        device = torch.device(device if device is not None else "cuda")
        self.device = device
        info = plan.query(self.block, allow_short=True)
        self.ring = torch.empty(int(info["ring_bytes"]), dtype=torch.uint8, device=device)
        self.ws = torch.empty(int(info["stream_workspace_bytes"]), dtype=torch.uint8, device=device)
        h = C.c_void_p()
        check(self._lib.dd_stream_create(plan.handle, self.block, _vp(self.ring), int(self.ring.numel()),
                                         _stream(stream), C.byref(h)))
        self._h = h
        self.seq = 0
        if gap_fill:
            check(self._lib.dd_stream_set_gap_fill(h, 1))

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def push(self, block: torch.Tensor, k_sigma: float = 0.0, cand_cap: int = 1 << 14, stats: bool = True,
             out: Optional[torch.Tensor] = None, stream=None, seq: Optional[int] = None) -> Optional[Result]:
        """Append a block; returns the newly computable outputs, or None while the ring fills.
        seq defaults to the next in order; a larger one (with gap_fill) zero-fills the blocks
        in between."""
        if seq is not None:
            self.seq = int(seq)
        p = self.plan
        if block.dim() != 2 or block.shape[0] != p.nchan or block.dtype != p.dtype or block.stride(1) != 1:
            raise ValueError("block must be [nchan][n] of the plan dtype, time contiguous")
        dev = block.device
        if out is None:
            out = torch.empty((p.ndm, self.block), dtype=torch.float32, device=dev)
        mean = rms = cand = ncand = None
        if stats:
            mean = torch.empty(p.ndm, dtype=torch.float32, device=dev)
            rms = torch.empty(p.ndm, dtype=torch.float32, device=dev)
            if k_sigma > 0:
                cand = torch.empty(max(cand_cap, 1) * CAND_DTYPE.itemsize, dtype=torch.uint8, device=dev)
                ncand = torch.zeros(1, dtype=torch.int64, device=dev)
        t0 = C.c_int64()
        n = C.c_int64()
        rc = check(self._lib.dd_stream_push(self._h, _vp(block), int(block.shape[1]), int(block.stride(0)),
                                            self.seq, _vp(out), int(out.stride(0)), _vp(mean), _vp(rms),
                                            float(k_sigma), _vp(cand), int(cand_cap if cand is not None else 0),
                                            _vp(ncand), _vp(self.ws), int(self.ws.numel()), _stream(stream),
                                            C.byref(t0), C.byref(n)), (_lib.DD_OK, _lib.DD_FILLING))
        self.seq += 1
        if rc == _lib.DD_FILLING:
            return None
        return Result(out[:, : n.value], mean, rms, t0.value, cand, ncand, cand_cap)

    def append(self, block: torch.Tensor, stream=None):
        """Copy a block into the ring without dedispersing (the first half of a batched push).

        Returns (t0, nout) of the window now pending, or None while the ring fills.
        """
        p = self.plan
        if block.dim() != 2 or block.shape[0] != p.nchan or block.dtype != p.dtype or block.stride(1) != 1:
            raise ValueError("block must be [nchan][n] of the plan dtype, time contiguous")
        t0 = C.c_int64()
        n = C.c_int64()
        rc = check(self._lib.dd_stream_append(self._h, _vp(block), int(block.shape[1]), int(block.stride(0)),
                                              self.seq, _stream(stream), C.byref(t0), C.byref(n)),
                   (_lib.DD_OK, _lib.DD_FILLING))
        self.seq += 1
        if rc == _lib.DD_FILLING:
            return None
        return int(t0.value), int(n.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.dd_stream_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _outputs(ndm: int, ncols: int, device, k_sigma: float, cand_cap: int, stats: bool):
    out = torch.empty((ndm, max(ncols, 1)), dtype=torch.float32, device=device)
    mean = rms = cand = ncand = None
    if stats:
        mean = torch.empty(ndm, dtype=torch.float32, device=device)
        rms = torch.empty(ndm, dtype=torch.float32, device=device)
        if k_sigma > 0:
            cand = torch.empty(max(cand_cap, 1) * CAND_DTYPE.itemsize, dtype=torch.uint8, device=device)
            ncand = torch.zeros(1, dtype=torch.int64, device=device)
    return out, mean, rms, cand, ncand


def alloc_outputs(ndm: int, ncols: int, device, k_sigma: float = 0.0, cand_cap: int = 1 << 16,
                  stats: bool = True):
    """Output buffers (out, mean, rms, cand, ncand) for one job, for reuse across calls."""
    return _outputs(ndm, ncols, device, k_sigma, cand_cap, stats)


def batch_dedisperse(jobs, k_sigma: float = 0.0, cand_cap: int = 1 << 16, stats: bool = True, stream=None,
                     outputs=None):
    """Dedisperse several inputs in one batched call (dd_batch_dedisperse): one persistent
    launch per kernel shape.

    jobs: a list of (Plan, tensor) pairs and/or (Stream, (t0, nout)) pairs, the latter
    after Stream.append returned a pending window. Plans of any tiles and forms mix, except
    the register-window form; the jobs on one kernel and workgroup shape share a persistent
    launch, each on its own tiles. Statistics and candidates of all jobs run in one launch
    per step. ``outputs`` optionally gives, per job, buffers from
    alloc_outputs (with ``stats`` and ``k_sigma`` matching) to write into instead of new
    ones. Returns one Result per job, equal bit for bit to the one-at-a-time calls.
    """
    lib = _lib.load()
    items = (_lib.BatchItem * len(jobs))()
    keep = []
    results = []
    used_ws = set()
    for i, (obj, arg) in enumerate(jobs):
        it = items[i]
        given = outputs[i] if outputs is not None else None
        if isinstance(obj, Stream):
            t0, n = arg
            plan = obj.plan
            dev = obj.device
            out, mean, rms, cand, ncand = given or _outputs(plan.ndm, obj.block, dev, k_sigma, cand_cap, stats)
            it.plan = plan.handle.value
            it.stream_item = obj.handle.value
            it.d_plan_workspace = obj.ws.data_ptr()
            cols = n
        else:
            plan, x = obj, arg
            if x.dim() != 2 or x.shape[0] != plan.nchan or x.dtype != plan.dtype or x.stride(1) != 1:
                raise ValueError("each input must be [nchan][nsamp] of its plan dtype, time contiguous")
            nsamp = int(x.shape[1])
            cols = nsamp - plan.maxdelay
            t0 = 0
            out, mean, rms, cand, ncand = given or _outputs(plan.ndm, cols, x.device, k_sigma, cand_cap, stats)
            ws = plan.workspace(nsamp, x.device, stream)
            if ws.data_ptr() in used_ws:  # the same plan twice at one length: a workspace of its own
                ws = torch.empty(ws.numel(), dtype=torch.uint8, device=x.device)
                check(lib.dd_plan_upload(plan.handle, _vp(ws), ws.numel(), _stream(stream)))
            used_ws.add(ws.data_ptr())
            it.plan = plan.handle.value
            it.d_in = x.data_ptr()
            it.nsamp = nsamp
            it.in_row_stride = int(x.stride(0))
            it.d_plan_workspace = ws.data_ptr()
            keep.append(ws)
        if out.shape[0] != plan.ndm or out.shape[1] < cols:
            raise ValueError(f"job {i}: output buffer smaller than [ndm][{cols}]")
        it.d_out = out.data_ptr()
        it.out_row_stride = int(out.stride(0))
        it.d_mean = mean.data_ptr() if mean is not None else None
        it.d_rms = rms.data_ptr() if rms is not None else None
        it.k_sigma = float(k_sigma)
        it.d_cand = cand.data_ptr() if cand is not None else None
        it.cand_cap = int(cand_cap) if cand is not None else 0
        it.d_ncand = ncand.data_ptr() if ncand is not None else None
        results.append(Result(out[:, :cols], mean, rms, t0, cand, ncand, cand_cap))
    need = C.c_int64()
    check(lib.dd_batch_query(items, len(jobs), C.byref(need)))
    dev = results[0].out.device
    bws = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
    check(lib.dd_batch_dedisperse(items, len(jobs), _vp(bws), int(bws.numel()), _stream(stream)))
    keep.append(bws)
    for r in results:
        r._keep = keep  # device buffers stay alive until the results are dropped
    return results


def detrend(series: torch.Tensor, normalise: bool = True, stream=None) -> torch.Tensor:
    """Subtract each row's least-squares line in place (dd_detrend, Sec. 3.5 "Signal
    Post-processing"); with normalise, divide by the residual's population standard
    deviation. series: [nrows][n] float32 on the device, rows may be strided. Returns the
    residuals' standard deviations, [nrows] float32 on the device."""
    if series.dim() != 2 or series.dtype != torch.float32 or not series.is_cuda or series.stride(1) != 1:
        raise ValueError("series must be a [nrows][n] float32 device tensor, time contiguous")
    lib = _lib.load()
    rms = torch.empty(series.shape[0], dtype=torch.float32, device=series.device)
    check(lib.dd_detrend(_vp(series), int(series.shape[0]), int(series.shape[1]), int(series.stride(0)),
                         1 if normalise else 0, _vp(rms), _stream(stream)))
    return rms


def boxcar_search(series: torch.Tensor, mean: Optional[torch.Tensor] = None, rms: Optional[torch.Tensor] = None,
                  max_log2: int = 6, k_sigma: float = 6.0, cap: int = 1 << 16, stream=None) -> np.ndarray:
    """Boxcar template matching with thresholding (dd_boxcar_search): at every start of each
    row, the boxcar of width 2^j (j <= max_log2) with the best S/N about the row's mean in
    units of rms sqrt(width); detections above k_sigma as a structured array (PULSE_DTYPE:
    row, width, t, value, snr) in (row, t) order. mean and rms default to 0 and 1
    (normalised rows). Synchronises the stream; warns CandidateOverflow when more than cap
    qualified (the first cap are returned)."""
    if series.dim() != 2 or series.dtype != torch.float32 or not series.is_cuda or series.stride(1) != 1:
        raise ValueError("series must be a [nrows][n] float32 device tensor, time contiguous")
    if (mean is None) != (rms is None):
        raise ValueError("give both mean and rms, or neither")
    lib = _lib.load()
    nrows, n = int(series.shape[0]), int(series.shape[1])
    need = C.c_int64()
    check(lib.dd_boxcar_search_workspace(nrows, n, C.byref(need)))
    dev = series.device
    ws = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=dev)
    out = torch.empty(max(int(cap), 1) * PULSE_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    m = mean.to(torch.float32).contiguous() if mean is not None else None
    r = rms.to(torch.float32).contiguous() if rms is not None else None
    check(lib.dd_boxcar_search(_vp(series), nrows, n, int(series.stride(0)), _vp(m), _vp(r), int(max_log2),
                               float(k_sigma), _vp(out), int(cap), _vp(cnt), _vp(ws), int(ws.numel()),
                               _stream(stream)))
    total = C.c_int64()
    rc = check(lib.dd_candidates_check(_vp(cnt), int(cap), _stream(stream), C.byref(total)),
               (_lib.DD_OK, _lib.DD_WARN_CAND_OVERFLOW))
    if rc == _lib.DD_WARN_CAND_OVERFLOW:
        warnings.warn(f"{total.value} boxcar detections qualified; the first {cap} were kept", CandidateOverflow)
    keep = min(int(total.value), int(cap))
    return out[: keep * PULSE_DTYPE.itemsize].cpu().numpy().view(PULSE_DTYPE)


def boxcar_offsets(n: int, levels: int):
    """Start of each level inside a dd_boxcar output row, and the row length."""
    offs = [0]
    for k in range(levels + 1):
        offs.append(offs[-1] + (n >> k))
    return offs


def boxcar(series: torch.Tensor, levels: int = 6, stream=None):
    """Boxcar levels 0..levels of each row (dd_boxcar): level k holds the sums of 2^k
    adjacent samples over sqrt(2^k). Returns a list of [nrows][n >> k] views of one
    device buffer."""
    if series.dim() != 2 or series.dtype != torch.float32 or not series.is_cuda or series.stride(1) != 1:
        raise ValueError("series must be a [nrows][n] float32 device tensor, time contiguous")
    nrows, n = int(series.shape[0]), int(series.shape[1])
    offs = boxcar_offsets(n, levels)
    out = torch.empty((nrows, offs[-1]), dtype=torch.float32, device=series.device)
    check(_lib.load().dd_boxcar(_vp(series), nrows, n, int(series.stride(0)), int(levels), _vp(out), offs[-1],
                                _stream(stream)))
    return [out[:, offs[k]:offs[k + 1]] for k in range(levels + 1)]


def downfactor(x: torch.Tensor, stream=None) -> torch.Tensor:
    """Sum adjacent sample pairs of every channel (dd_downfactor; the downfactor step of
    time binning): [nchan][nsamp] float32/float16/uint8 device tensor, time contiguous ->
    [nchan][nsamp // 2] float32."""
    if x.dim() != 2 or x.dtype not in _TORCH_DT or not x.is_cuda or x.stride(1) != 1:
        raise ValueError("x must be a [nchan][nsamp] float32/float16/uint8 device tensor, time contiguous")
    nchan, nsamp = int(x.shape[0]), int(x.shape[1])
    out = torch.empty((nchan, nsamp // 2), dtype=torch.float32, device=x.device)
    check(_lib.load().dd_downfactor(_vp(x), _TORCH_DT[x.dtype], nchan, nsamp, int(x.stride(0)), _vp(out),
                                    int(out.stride(0)), _stream(stream)))
    return out


def time_binning(freq_mhz, tsamp_s: float, dm, max_log2: int):
    """(diagonal DM, log2 binning factor per DM trial) from dd_time_binning."""
    f = np.ascontiguousarray(freq_mhz, dtype=np.float64)
    d = np.ascontiguousarray(dm, dtype=np.float64)
    k = np.empty(d.size, dtype=np.int32)
    diag = C.c_double()
    dbl = C.POINTER(C.c_double)
    check(_lib.load().dd_time_binning(f.ctypes.data_as(dbl), int(f.size), float(tsamp_s), d.ctypes.data_as(dbl),
                                      int(d.size), int(max_log2), C.byref(diag), k.ctypes.data_as(C.POINTER(C.c_int32))))
    return float(diag.value), k


@dataclasses.dataclass
class BinnedSegment:
    log2: int          # this run is dedispersed at 2^log2 times the sampling time
    d0: int            # first DM trial of the run
    d1: int            # one past its last trial
    plan: "Plan"       # host-side plan of the run (delay table, maximum delay), for inspection


class _PartResult(Result):
    """Rows [d0, d1) of a composite call: views of its output and statistics; candidates are
    the composite's merged list restricted to these trials, with dm_index local and t in
    this part's own samples (t >> log2)."""

    def __init__(self, parent, out, mean, rms, d0: int, d1: int, log2: int = 0):
        super().__init__(out, mean, rms, 0, None, parent._ncand, parent.cand_cap)
        self._parent, self._d0, self._d1, self._log2 = parent, d0, d1, log2

    def candidates(self, stream=None) -> Optional[np.ndarray]:
        c = self._parent.candidates(stream)
        if c is None:
            return None
        c = c[(c["dm_index"] >= self._d0) & (c["dm_index"] < self._d1)].copy()
        c["dm_index"] -= self._d0
        c["t"] >>= self._log2
        return c

    def ncand(self, stream=None) -> Optional[int]:
        c = self.candidates(stream)
        return None if c is None else int(c.size)


@dataclasses.dataclass
class BinnedResult:
    segments: list     # [(BinnedSegment, Result)]: rows d0..d1-1 at nsamp >> log2 resolution
    merged: Result     # the whole [ndm][nout_max] output and the merged candidate list

    def candidates(self) -> Optional[np.ndarray]:
        """All runs' detections in one list from the library: dm_index global and t in input
        samples (binned index << log2)."""
        return self.merged.candidates()


class _Composite:
    """Marshalling shared by the time-binned and subband plans (C objects with a per-nsamp
    workspace and one call over all their parts)."""

    def _workspace(self, nsamp: int, device, stream, query_bytes, upload):
        device = torch.device(device if device is not None else "cuda")
        nbytes = int(query_bytes(nsamp))
        key = (device.index if device.index is not None else torch.cuda.current_device(), nsamp)
        ws = self._ws.get(key)
        if ws is None:
            ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
            check(upload(self._h, int(nsamp), _vp(ws), nbytes, _stream(stream)))
            self._ws[key] = ws
        return ws


class BinnedPlan(_Composite):
    """Brute-force dedispersion with time binning above the diagonal DM (Ch. 2 Sec. "Direct
    Dedispersion"; Sec. "Computing Larger DMs"), a dd_binned object: DM trials in
    (2^(k-1), 2^k] x DM_diag are dedispersed on the input downfactored k times (k <=
    max_log2), with delays at sampling time 2^k tsamp, all in one library call."""

    def __init__(self, freq_mhz, tsamp_s: float, dm, dtype=torch.float32, max_log2: int = 4, tuning=None,
                 form: str = "auto"):
        lib = _lib.load()
        self._lib = lib
        self.freq = np.ascontiguousarray(freq_mhz, dtype=np.float64)
        self.dm = np.ascontiguousarray(dm, dtype=np.float64)
        self.tsamp = float(tsamp_s)
        self.dtype = torch_dtype(dtype)
        self.max_log2 = int(max_log2)
        dbl = C.POINTER(C.c_double)
        h = C.c_void_p()
        check(lib.dd_binned_create(C.byref(h), self.freq.ctypes.data_as(dbl), int(self.freq.size), self.tsamp,
                                   self.dm.ctypes.data_as(dbl), int(self.dm.size), _TORCH_DT[self.dtype],
                                   self.max_log2, _tuning(tuning, form)))
        self._h = h
        self._ws = {}
        n = C.c_int32()
        diag = C.c_double()
        check(lib.dd_binned_query(h, 0, C.byref(n), None, 0, None, C.byref(diag)), (_lib.DD_ERR_INVALID_ARG,))
        runs = (_lib.BinnedRun * n.value)()
        check(lib.dd_binned_query(h, 0, None, runs, n.value, None, None), (_lib.DD_ERR_INVALID_ARG,))
        self.dm_diag = float(diag.value)
        self.log2 = np.zeros(self.dm.size, dtype=np.int32)
        self.segments = []
        for r in runs:
            k, d0, d1 = int(r.log2), int(r.d0), int(r.d1)
            self.log2[d0:d1] = k
            # the run's plan on the host, with the form and tiles the library chose for it, for
            # its delay table, maximum delay and launch shape
            kf = int(r.kernel_form)
            if kf == _lib.DD_FORM_DIRECT:
                t, f = (int(r.dms_per_wave), int(r.waves)), "direct"
            elif kf == _lib.DD_FORM_REGWIN:
                t, f = None, "regwin"
            else:
                t, f = (int(r.dms_per_wave), int(r.waves), 0,
                        int(r.producer_waves) if r.producer_waves > 0 else -1), "lds"
            host = Plan(self.freq, self.tsamp * float(1 << k), self.dm[d0:d1], self.dtype if k == 0 else torch.float32,
                        t, f)
            self.segments.append(BinnedSegment(k, d0, d1, host))

    def nout(self, nsamp: int):
        """Output samples per run for an nsamp-sample input: (nsamp >> k) - maxdelay_k."""
        return [(int(nsamp) >> s.log2) - s.plan.maxdelay for s in self.segments]

    def adds(self, nsamp: int) -> int:
        return sum((s.d1 - s.d0) * s.plan.nchan * n for s, n in zip(self.segments, self.nout(nsamp)))

    @property
    def batchable(self) -> bool:
        """Whether the runs can share one batched call: none is in the register-window form."""
        return all(s.plan.form != "regwin" for s in self.segments)

    @property
    def fill_nsamp(self) -> int:
        """Input samples a stream needs before every run emits: max over runs of
        (maxdelay + 1) << log2."""
        return max((s.plan.maxdelay + 1) << s.log2 for s in self.segments)

    def stream_sizes(self, block_nsamp: int):
        """(ring bytes, workspace bytes) of a BinnedStream of block_nsamp-sample blocks."""
        rb, wb = C.c_int64(), C.c_int64()
        check(self._lib.dd_binned_stream_query(self._h, int(block_nsamp), C.byref(rb), C.byref(wb)))
        return int(rb.value), int(wb.value)

    def workspace(self, nsamp: int, device=None, stream=None) -> torch.Tensor:
        """A device workspace for nsamp-sample inputs with every run's delay table (cached)."""
        def query(ns):
            b = C.c_int64()
            check(self._lib.dd_binned_query(self._h, int(ns), None, None, 0, C.byref(b), None))
            return b.value
        return self._workspace(nsamp, device, stream, query, self._lib.dd_binned_upload)

    def dedisperse(self, x: torch.Tensor, k_sigma: float = 0.0, cand_cap: int = 1 << 16, stats: bool = True,
                   stream=None, batched: bool = False) -> BinnedResult:
        """Every run of trials on its downfactored input (dd_binned_dedisperse). With batched,
        the runs go through one dd_batch_dedisperse call, equal bit for bit."""
        if x.dim() != 2 or x.shape[0] != self.freq.size or x.dtype != self.dtype or x.stride(1) != 1:
            raise ValueError(f"x must be a [nchan={self.freq.size}][nsamp] {self.dtype} tensor, time contiguous")
        nsamp = int(x.shape[1])
        nouts = self.nout(nsamp)
        ncols = max(nouts)
        out, mean, rms, cand, ncand = _outputs(self.dm.size, ncols, x.device, k_sigma, cand_cap, stats)
        ws = self.workspace(nsamp, x.device, stream)
        check(self._lib.dd_binned_dedisperse(self._h, _vp(x), nsamp, int(x.stride(0)), _vp(out), int(out.stride(0)),
                                             _vp(mean), _vp(rms), float(k_sigma), _vp(cand),
                                             int(cand_cap if cand is not None else 0), _vp(ncand), 1 if batched else 0,
                                             _vp(ws), int(ws.numel()), _stream(stream)))
        merged = Result(out, mean, rms, 0, cand, ncand, cand_cap)
        merged._keep = ws
        parts = []
        for seg, n in zip(self.segments, nouts):
            r = _PartResult(merged, out[seg.d0:seg.d1, :n], mean[seg.d0:seg.d1] if mean is not None else None,
                            rms[seg.d0:seg.d1] if rms is not None else None, seg.d0, seg.d1, seg.log2)
            parts.append((seg, r))
        return BinnedResult(parts, merged)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.dd_binned_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass



@dataclasses.dataclass
class BinnedStreamResult:
    segments: list     # [(BinnedSegment, t0, Result or None)]: None while that run fills; t0 and the
                       # candidates' t in the run's own samples (input samples >> log2)
    merged: Result     # the [ndm][block] output and the merged candidate list (t in input samples)

    def candidates(self) -> Optional[np.ndarray]:
        return self.merged.candidates()


class BinnedStream:
    """A beam's stream over a time-binned plan (dd_binned_stream): each run keeps a ring of
    the input downfactored 2^log2 times, so the long delays of the high DMs are held at
    their binned sampling time. Blocks must be multiples of 2^K samples (K the largest
    log2)."""

    def __init__(self, plan: BinnedPlan, block_nsamp: int, device=None, stream=None, gap_fill: bool = False):
        self.plan = plan
        self._lib = plan._lib
        self.block = int(block_nsamp)
        device = torch.device(device if device is not None else "cuda")
        self.device = device
        self.ring_bytes, ws_bytes = plan.stream_sizes(self.block)
        self.batchable = plan.batchable
        self.ring = torch.empty(max(self.ring_bytes, 1), dtype=torch.uint8, device=device)
        self.ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=device)
        h = C.c_void_p()
        check(self._lib.dd_binned_stream_create(plan._h, self.block, _vp(self.ring), int(self.ring.numel()),
                                                _stream(stream), C.byref(h)))
        self._h = h
        self.seq = 0
        if gap_fill:
            check(self._lib.dd_binned_stream_set_gap_fill(h, 1))

    def push(self, block: torch.Tensor, k_sigma: float = 0.0, cand_cap: int = 1 << 14, stats: bool = True,
             out: Optional[torch.Tensor] = None, stream=None, seq: Optional[int] = None,
             batched: bool = False, outputs=None) -> Optional[BinnedStreamResult]:
        """Append a block; returns each run's newly computable outputs, or None while every
        run fills. seq defaults to the next in order. ``outputs`` optionally gives buffers
        from alloc_outputs(ndm, block, ...) to write into (``out`` then is ignored)."""
        if seq is not None:
            self.seq = int(seq)
        bp = self.plan
        if block.dim() != 2 or block.shape[0] != bp.freq.size or block.dtype != bp.dtype or block.stride(1) != 1:
            raise ValueError("block must be [nchan][n] of the plan dtype, time contiguous")
        dev = block.device
        ndm = bp.dm.size
        if outputs is not None:
            out, mean, rms, cand, ncand = outputs
            if ncand is not None:
                cand_cap = cand.numel() // CAND_DTYPE.itemsize
        else:
            if out is None:
                out = torch.empty((ndm, self.block), dtype=torch.float32, device=dev)
            _, mean, rms, cand, ncand = _outputs(ndm, 1, dev, k_sigma, cand_cap, stats)
        nr = len(bp.segments)
        t0 = (C.c_int64 * nr)()
        n = (C.c_int64 * nr)()
        rc = check(self._lib.dd_binned_stream_push(
            self._h, _vp(block), int(block.shape[1]), int(block.stride(0)), self.seq, _vp(out), int(out.stride(0)),
            _vp(mean), _vp(rms), float(k_sigma), _vp(cand), int(cand_cap if cand is not None else 0), _vp(ncand),
            1 if batched else 0, _vp(self.ws), int(self.ws.numel()), _stream(stream), t0, n),
            (_lib.DD_OK, _lib.DD_FILLING))
        self.seq += 1
        if rc == _lib.DD_FILLING:
            return None
        merged = Result(out, mean, rms, 0, cand, ncand, cand_cap)
        parts = []
        for i, seg in enumerate(bp.segments):
            if n[i] == 0:
                parts.append((seg, 0, None))
                continue
            r = _PartResult(merged, out[seg.d0:seg.d1, :n[i]], mean[seg.d0:seg.d1] if mean is not None else None,
                            rms[seg.d0:seg.d1] if rms is not None else None, seg.d0, seg.d1, seg.log2)
            r.t0 = int(t0[i])
            parts.append((seg, int(t0[i]), r))
        return BinnedStreamResult(parts, merged)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.dd_binned_stream_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

def bandpass(x: torch.Tensor, window: int = 0, stream=None):
    """The averaged bandpass (dd_bandpass, dd_bandpass_u8 for 8-bit codes): each channel's
    mean, [nchan] float64 on the device. With window >= 1 also the means of every window of
    that many samples, [nchan][nwin] float64 (returned as a second tensor): the channel
    stage's statistic, from the same read."""
    if x.dim() != 2 or x.dtype not in (torch.float32, torch.uint8) or not x.is_cuda or x.stride(1) != 1:
        raise ValueError("x must be a [nchan][nsamp] float32 or uint8 device tensor, time contiguous")
    avg = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
    means = None
    if window:
        means = torch.empty((x.shape[0], -(-int(x.shape[1]) // int(window))), dtype=torch.float64, device=x.device)
    lib = _lib.load()
    fn = lib.dd_bandpass_u8 if x.dtype == torch.uint8 else lib.dd_bandpass
    check(fn(_vp(x), int(x.shape[0]), int(x.shape[1]), int(x.stride(0)), int(window), _vp(avg), _vp(means),
             _stream(stream)))
    return (avg, means) if window else avg


def bandpass_fit(avg, order: int):
    """Host least-squares polynomial fit of an averaged bandpass (dd_bandpass_fit):
    (fitted values as a float64 numpy array, RMSE, mean of the fit)."""
    a = np.ascontiguousarray(avg, dtype=np.float64)
    fit = np.empty_like(a)
    rmse, fmean = C.c_double(), C.c_double()
    dbl = C.POINTER(C.c_double)
    check(_lib.load().dd_bandpass_fit(a.ctypes.data_as(dbl), int(a.size), int(order), fit.ctypes.data_as(dbl),
                                      C.byref(rmse), C.byref(fmean)))
    return fit, float(rmse.value), float(fmean.value)


def rfi_mitigate(x: torch.Tensor, order: int, chan_threshold: float, window: int, spec_threshold: float,
                 subtract: Optional[bool] = None, stream=None):
    """RFI mitigation in place on a [nchan][nsamp] float32 or uint8 device filterbank (Ch. 3):
    the averaged bandpass on the device, its polynomial fit on the host (the nchan averages
    cross PCIe, as in the paper), then channel and spectrum thresholding and the bandpass
    correction (dd_rfi_clip, dd_rfi_clip_u8). Thresholds are absolute deviations from the
    fit; <= 0 skips a stage. With subtract (the default for float32) the fitted bandpass is
    subtracted from every spectrum. 8-bit codes take the nearest code of the fit where
    replaced and cannot be corrected in place (subtract must be false): the correction is
    then the constant -sum(fit) on every dedispersed sample. Returns (fit, rmse, fit_mean,
    channel flags [nchan][nwin] int32 device tensor or None)."""
    u8 = x.dtype == torch.uint8
    if subtract is None:
        subtract = not u8
    if u8 and subtract:
        raise ValueError("8-bit codes cannot hold the corrected values; subtract sum(fit) from the dedispersed "
                         "series instead")
    chan = chan_threshold > 0
    if chan:
        avg_d, means = bandpass(x, int(window), stream)
    else:
        avg_d, means = bandpass(x, 0, stream), None
    fit, rmse, fmean = bandpass_fit(avg_d.cpu().numpy(), order)
    d_fit = torch.from_numpy(fit).to(x.device)
    flags = None
    if chan:
        flags = torch.empty(means.shape, dtype=torch.int32, device=x.device)
    lib = _lib.load()
    if u8:
        check(lib.dd_rfi_clip_u8(_vp(x), int(x.shape[0]), int(x.shape[1]), int(x.stride(0)), _vp(d_fit),
                                 float(chan_threshold), int(window), _vp(means), _vp(flags), float(fmean),
                                 float(spec_threshold), _stream(stream)))
    else:
        check(lib.dd_rfi_clip(_vp(x), int(x.shape[0]), int(x.shape[1]), int(x.stride(0)), _vp(d_fit),
                              float(chan_threshold), int(window), _vp(means), _vp(flags), float(fmean),
                              float(spec_threshold), int(bool(subtract)), _stream(stream)))
    return fit, rmse, fmean, flags


class SubbandPlan(_Composite):
    """Subband dedispersion (Sec. "Subband Dedispersion"), an approximation of Eq.
    bruteEquation at a fraction of the adds, a dd_subband object. Trials are grouped in runs
    of dms_per_group; each group's nominal DM is its middle trial. Step 1 dedisperses each
    subband of chans_per_sub channels at the nominal DMs into a reduced filterbank; step 2
    dedisperses each group's trials over its subband series. FP32 input; one library call."""

    def __init__(self, freq_mhz, tsamp_s: float, dm, chans_per_sub: int = 32, dms_per_group: int = 16):
        lib = _lib.load()
        self._lib = lib
        self.freq = np.ascontiguousarray(freq_mhz, dtype=np.float64)
        self.dm = np.ascontiguousarray(dm, dtype=np.float64)
        self.tsamp = float(tsamp_s)
        nchan, ndm = self.freq.size, self.dm.size
        dbl = C.POINTER(C.c_double)
        h = C.c_void_p()
        check(lib.dd_subband_create(C.byref(h), self.freq.ctypes.data_as(dbl), nchan, self.tsamp,
                                    self.dm.ctypes.data_as(dbl), ndm, int(chans_per_sub), int(dms_per_group)))
        self._h = h
        self._ws = {}
        self.subs = [(c0, min(nchan, c0 + chans_per_sub)) for c0 in range(0, nchan, chans_per_sub)]
        self.groups = [(d0, min(ndm, d0 + dms_per_group)) for d0 in range(0, ndm, dms_per_group)]

    @property
    def launches(self) -> int:
        """Dedispersion launches of an unbatched call: one per subband and one per group."""
        return len(self.subs) + len(self.groups)

    def _query(self, nsamp: int):
        ws = C.c_int64()
        adds = C.c_int64()
        nout = np.zeros(self.dm.size, dtype=np.int64)
        check(self._lib.dd_subband_query(self._h, int(nsamp), C.byref(ws), nout.ctypes.data_as(C.POINTER(C.c_int64)),
                                         C.byref(adds), None, None))
        return ws.value, nout, adds.value

    def adds(self, nsamp: int) -> int:
        """Step-1 and step-2 channel-sample adds for an nsamp-sample input."""
        return self._query(nsamp)[2]

    def workspace(self, nsamp: int, device=None, stream=None) -> torch.Tensor:
        return self._workspace(nsamp, device, stream, lambda ns: self._query(ns)[0], self._lib.dd_subband_upload)

    def dedisperse(self, x: torch.Tensor, k_sigma: float = 0.0, cand_cap: int = 1 << 16, stats: bool = True,
                   stream=None, batched: bool = False):
        """Returns [((d0, d1), Result)] per group of trials (dd_subband_dedisperse). With
        batched, each step goes through one dd_batch_dedisperse call, equal bit for bit."""
        if x.dim() != 2 or x.dtype != torch.float32 or x.shape[0] != self.freq.size or x.stride(1) != 1:
            raise ValueError("x must be a [nchan][nsamp] float32 device tensor, time contiguous")
        nsamp = int(x.shape[1])
        _, nout, _ = self._query(nsamp)
        out, mean, rms, cand, ncand = _outputs(self.dm.size, int(nout.max()), x.device, k_sigma, cand_cap, stats)
        ws = self.workspace(nsamp, x.device, stream)
        check(self._lib.dd_subband_dedisperse(self._h, _vp(x), nsamp, int(x.stride(0)), _vp(out), int(out.stride(0)),
                                              _vp(mean), _vp(rms), float(k_sigma), _vp(cand),
                                              int(cand_cap if cand is not None else 0), _vp(ncand), 1 if batched else 0,
                                              _vp(ws), int(ws.numel()), _stream(stream)))
        merged = Result(out, mean, rms, 0, cand, ncand, cand_cap)
        merged._keep = ws
        res = []
        for d0, d1 in self.groups:
            n = int(nout[d0])
            res.append(((d0, d1), _PartResult(merged, out[d0:d1, :n], mean[d0:d1] if mean is not None else None,
                                              rms[d0:d1] if rms is not None else None, d0, d1)))
        return res

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.dd_subband_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
