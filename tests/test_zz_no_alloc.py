"""dd_dedisperse_noalloc (static scratch, no allocation) against dd_dedisperse (caller
workspace) through the C ABI: two calls in a row, the second on a smaller input, each equal
bit for bit in series, statistics, candidate count and candidates; and the size limit."""
import ctypes as C

import numpy as np
import pytest

import fbsynth
from tests.gpu_util import cuda

pytestmark = pytest.mark.gpu


def _vp(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _outputs(torch, ndm, nout, cap):
    return (torch.empty((ndm, nout), device="cuda"), torch.empty(ndm, device="cuda"), torch.empty(ndm, device="cuda"),
            torch.empty(cap * 24, dtype=torch.uint8, device="cuda"), torch.zeros(1, dtype=torch.int64, device="cuda"))


@pytest.mark.parametrize("dtype", ["f32", "u8"])
def test_noalloc_equals_workspace_call(dtype):
    torch = cuda()
    import paper_1401_8258_amd as dd
    from paper_1401_8258_amd import _lib
    lib = _lib.load()
    b = fbsynth.config1()
    x_full = fbsynth.to_u8(b.data) if dtype == "u8" else b.data
    plan = dd.Plan(b.freq_mhz, b.tsamp_s, b.dm, dtype=dtype)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    table = plan.workspace(x_full.shape[1])  # dd_plan_upload'ed: the table is its first region
    cap, k = 4096, 3.0
    for nsamp in (x_full.shape[1], 8000):  # the second call is smaller
        print(f"case: noalloc {dtype} nsamp={nsamp}", flush=True)
        x = torch.from_numpy(np.ascontiguousarray(x_full[:, :nsamp])).cuda()
        nout = nsamp - plan.maxdelay
        a = _outputs(torch, plan.ndm, nout, cap)
        bb = _outputs(torch, plan.ndm, nout, cap)
        ws = plan.workspace(nsamp)
        rc = lib.dd_dedisperse(plan.handle, _vp(x), nsamp, nsamp, _vp(a[0]), nout, _vp(a[1]), _vp(a[2]), k, _vp(a[3]),
                               cap, _vp(a[4]), _vp(ws), ws.numel(), st)
        assert rc == 0, lib.dd_last_error()
        rc = lib.dd_dedisperse_noalloc(plan.handle, _vp(x), nsamp, nsamp, _vp(bb[0]), nout, _vp(bb[1]), _vp(bb[2]), k,
                                       _vp(bb[3]), cap, _vp(bb[4]), _vp(table), st)
        assert rc == 0, lib.dd_last_error()
        torch.cuda.synchronize()
        assert torch.equal(a[0], bb[0])
        assert torch.equal(a[1], bb[1]) and torch.equal(a[2], bb[2])
        n = int(a[4].item())
        assert n == int(bb[4].item()) and 0 < n <= cap
        assert torch.equal(a[3][: n * 24], bb[3][: n * 24])


def test_noalloc_refuses_oversize_shapes():
    cuda()
    import paper_1401_8258_amd as dd
    from paper_1401_8258_amd import _lib
    lib = _lib.load()
    freq = fbsynth.channel_freqs(428.0, 20.0 / 64, 64)
    plan = dd.Plan(freq, 51.2e-6, fbsynth.dm_trials(0.0, 0.1, 4096))
    p = C.c_void_p(256)  # never dereferenced: the size check comes first
    nsamp = 1 << 22      # 4096 trials x 8192 tiles x 16 bytes of partials: 512 MiB
    rc = lib.dd_dedisperse_noalloc(plan.handle, p, nsamp, nsamp, p, nsamp, p, p, 0.0, None, 0, None, p, None)
    assert rc == _lib.DD_ERR_UNSUPPORTED
    assert "scratch" in lib.dd_last_error().decode()
