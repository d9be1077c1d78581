"""Static checks of the gfx950 device code (CPU only; needs hipcc and llvm-mc/objdump).

The device code is assembled from the committed sources and checked before any of
it runs on a GPU: no packed FP32 VALU forms, no scratch or spills, and an inner
loop of the dedispersion kernel made of vector adds and LDS reads only.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1401_8258_amd", "csrc")
ROCM = "/opt/rocm"
HIPCC = os.path.join(ROCM, "bin", "hipcc")
MC = os.path.join(ROCM, "llvm", "bin", "llvm-mc")
OBJDUMP = os.path.join(ROCM, "llvm", "bin", "llvm-objdump")

pytestmark = pytest.mark.skipif(not all(os.path.exists(p) for p in (HIPCC, MC, OBJDUMP)),
                                reason="ROCm toolchain not found")


@pytest.fixture(scope="module")
def device_code(tmp_path_factory):
    import sys
    sys.path.insert(0, os.path.join(ROOT, "paper_1401_8258_amd"))
    from paper_1401_8258_amd import build
    d = tmp_path_factory.mktemp("codegen")
    flags = [f for f in build.FLAGS if f not in ("-shared", "-fPIC")]
    asm_all, dis_all = "", ""
    for name in ("dedisp", "direct", "regwin", "detrend", "boxcar", "downfactor", "rfi"):  # every device source
        asm = d / f"{name}.s"
        subprocess.run([HIPCC] + flags + ["--cuda-device-only", "-S", "-o", str(asm),
                                          os.path.join(CSRC, f"{name}.hip")], check=True, capture_output=True)
        obj = d / f"{name}.o"
        subprocess.run([MC, "-triple=amdgcn-amd-amdhsa", "-mcpu=gfx950", "-filetype=obj", "-o", str(obj),
                        str(asm)], check=True, capture_output=True)
        asm_all += asm.read_text()
        dis_all += subprocess.run([OBJDUMP, "-d", "--mcpu=gfx950", str(obj)], check=True, capture_output=True,
                                  text=True).stdout
    return asm_all, dis_all


def test_no_packed_fp32_and_no_scratch(device_code):
    asm, dis = device_code
    assert not re.search(r"\bv_pk_(add|mul|fma)_f32\b", dis)
    for m in re.finditer(r"\.private_segment_fixed_size:\s+(\d+)", asm):
        assert int(m.group(1)) == 0
    for m in re.finditer(r"\.vgpr_spill_count:\s+(\d+)", asm):
        assert int(m.group(1)) == 0


# FP32 kernels by DMA form: 16-byte DMAs from every wavefront, and producer wavefronts (8 and 4
# trials per computing wavefront)
FP32_KERNELS = ["_ZN12_GLOBAL__N_111dedisp_tileIfLi1EEEvNS_7KParamsE",
                "_ZN12_GLOBAL__N_111dedisp_tileIfLi2EEEvNS_7KParamsE",
                "_ZN12_GLOBAL__N_111dedisp_tileIfLi4EEEvNS_7KParamsE"]


@pytest.mark.parametrize("sym", FP32_KERNELS)
def test_inner_loop_has_no_scalar_work_per_trial(device_code, sym):
    """Per channel each wavefront does 8 trials x (1 address add + 2 ds_read_b128 + 8 adds)."""
    asm, _ = device_code
    assert sym + ":" in asm
    body = asm.split(sym + ":", 1)[1].split("s_endpgm", 1)[0]
    n_b128 = len(re.findall(r"ds_read_b128", body))
    n_add = len(re.findall(r"v_add_f32_e32", body))
    assert n_b128 >= 16 and n_add >= 64
