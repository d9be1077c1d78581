"""Static checks of the gfx950 device code (CPU only; needs hipcc and llvm-mc/objdump).

The dedispersion kernel jumps into tables of equal-sized cases (window_add): a
wrong case size or table offset would send a wavefront to an arbitrary address.
These tests assemble the device code built from the committed sources and check
every table instruction by instruction before any of it runs on a GPU.
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
    asm = d / "dedisp.s"
    flags = [f for f in build.FLAGS if f not in ("-shared", "-fPIC")]
    subprocess.run([HIPCC] + flags + ["--cuda-device-only", "-S", "-o", str(asm),
                                      os.path.join(CSRC, "dedisp.hip")], check=True, capture_output=True)
    obj = d / "dedisp.o"
    subprocess.run([MC, "-triple=amdgcn-amd-amdhsa", "-mcpu=gfx950", "-filetype=obj", "-o", str(obj), str(asm)],
                   check=True, capture_output=True)
    dis = subprocess.run([OBJDUMP, "-d", "--mcpu=gfx950", str(obj)], check=True, capture_output=True,
                         text=True).stdout
    return asm.read_text(), dis


def _kmax():
    src = open(os.path.join(CSRC, "gen_jumptable.py")).read()
    s = int(re.search(r"^S = (\d+)", src, re.M).group(1))
    k = int(re.search(r"^KMAX = (\d+)", src, re.M).group(1))
    return s, k


INSN = re.compile(r"^\s+(\S+)\s*(.*?)\s*//\s*([0-9A-F]+):", re.M)


def _instructions(dis):
    """[(address, mnemonic, operands)] in listing order, plus {label: (index, address)}.

    Template instantiations sit in separate sections whose addresses overlap, so labels
    are resolved to positions in the listing, and addresses are only compared locally."""
    out, labels = [], {}
    for line in dis.splitlines():
        m = re.match(r"^([0-9a-f]+) <([^>]+)>:", line)
        if m:
            labels[m.group(2)] = (len(out), int(m.group(1), 16))
            continue
        m = INSN.match(line)
        if m:
            out.append((int(m.group(3), 16), m.group(1), m.group(2)))
    return out, labels


def test_jump_tables_are_well_formed(device_code):
    _, dis = device_code
    S, KMAX = _kmax()
    insns, labels = _instructions(dis)
    tabs = sorted(n for n in labels if n.startswith("L_tab"))
    assert len(tabs) >= 8, "no window_add tables found"
    for name in tabs:
        uid = name[len("L_tab"):]
        i_tab, tab = labels[name]
        i_pc, pc = labels["L_pc" + uid]
        i_end, end = labels["L_end" + uid]
        assert insns[i_tab][0] == tab and insns[i_pc][0] == pc
        # addresses are unique inside one table
        by_addr = {insns[j][0]: j for j in range(i_tab, i_end)}
        # preamble: s_min_u32 k, s_mul_i32 case size, s_getpc, add (L_tab - L_pc), add/addc, s_setpc
        pre = insns[i_pc - 3:i_pc + 4]
        assert pre[0][1] == "s_min_u32" and pre[0][2].endswith(f", {KMAX}"), pre[0]
        assert pre[1][1] == "s_mul_i32" and pre[1][2].endswith(f", {4 * S + 4}"), pre[1]
        assert pre[2][1] == "s_getpc_b64"
        assert pre[3][1] == "s_add_u32" and pre[3][2].split(",")[-1].strip() == str(tab - pc), (pre[3], tab - pc)
        assert pre[6][1] == "s_setpc_b64" and i_pc + 4 == i_tab
        assert end == tab + (KMAX + 1) * (4 * S + 4)
        pos_reg = {}
        dst = None
        for k in range(KMAX + 1):
            i0 = by_addr[tab + k * (4 * S + 4)]
            rows = insns[i0:i0 + S + 1]
            assert [r[1] for r in rows[:S]] == ["v_add_f32_e32"] * S, rows
            assert rows[S][1] == "s_branch" and rows[S][0] == tab + k * (4 * S + 4) + 4 * S
            assert rows[S][2] == "L_end" + uid, rows[S]
            d_here = []
            for s, (_, _, ops) in enumerate(rows[:S]):
                d, src, d2 = [o.strip() for o in ops.split(",")]
                assert d == d2
                d_here.append(d)
                assert pos_reg.setdefault(k + s, src) == src, (name, k, s)
            if dst is None:
                dst = d_here
            assert d_here == dst
        assert len(set(pos_reg.values())) == S + KMAX, "window registers are not distinct"
        assert len(set(dst)) == S


def test_window_load_tables_are_well_formed(device_code):
    _, dis = device_code
    S, KMAX = _kmax()
    nchunk = (S + KMAX) // 4
    insns, labels = _instructions(dis)
    lds = sorted(n for n in labels if n.startswith("L_ld"))
    assert len(lds) >= 1, "no window_load tables found"
    for name in lds:
        uid = name[len("L_ld"):]
        i_ld, ld = labels[name]
        i_lp, lp = labels["L_lp" + uid]
        pre = insns[i_lp - 5:i_lp + 4]
        assert [p[1] for p in pre] == ["s_max_i32", "s_min_i32", "s_sub_u32", "s_lshl_b32", "s_getpc_b64",
                                       "s_add_u32", "s_add_u32", "s_addc_u32", "s_setpc_b64"], pre
        assert pre[1][2].endswith(f", {nchunk}") and pre[2][2].split(",")[1].strip() == str(nchunk)
        assert pre[3][2].endswith(", 3")  # entries are 8 bytes
        assert pre[5][2].split(",")[-1].strip() == str(ld - lp)
        assert i_lp + 4 == i_ld
        rows = insns[i_ld:i_ld + nchunk + 1]
        bases = set()
        dsts = []
        for e, (a, mnem, ops) in enumerate(rows[:nchunk]):
            j = nchunk - 1 - e
            assert mnem == "ds_read_b128" and a == ld + 8 * e, (a, mnem)
            parts = [o.strip() for o in ops.split(",")]
            dst, base = parts[0], parts[1].split()[0]
            off = 0
            m = re.search(r"offset:(\d+)", ops)
            if m:
                off = int(m.group(1))
            assert off == 16 * (j // 2), (j, ops)
            bases.add((j % 2, base))
            dsts.append(dst)
        assert len({b for _, b in bases}) == 2 and len(bases) == 2
        assert len(set(dsts)) == nchunk
        assert rows[nchunk][1] == "s_waitcnt" and "lgkmcnt(0)" in rows[nchunk][2]


def test_no_packed_fp32_and_no_scratch(device_code):
    asm, dis = device_code
    assert not re.search(r"\bv_pk_(add|mul|fma)_f32\b", dis)
    for m in re.finditer(r"\.private_segment_fixed_size:\s+(\d+)", asm):
        assert int(m.group(1)) == 0
    for m in re.finditer(r"\.vgpr_spill_count:\s+(\d+)", asm):
        assert int(m.group(1)) == 0
