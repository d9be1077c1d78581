"""Turn rocprofv3 counter CSVs into the HBM traffic record that bench.py reports.

Usage (after two counter runs of the same command, one with ``--pmc FETCH_SIZE`` and
one with ``--pmc WRITE_SIZE``, each also running one plain device copy of known size):

    python -m paper_1401_8258_amd.profiling traffic \
        --fetch <dir>/bench_counter_collection.csv --write <dir>/bench_counter_collection.csv \
        --kernel dedisp_tile --copy-bytes N --source <comma-separated kernel sources> \
        --out profiles/<kernel>_<workload>_traffic.json

FETCH_SIZE and WRITE_SIZE are KiB per dispatch summed over the L2 channels. Each is
scaled by bytes / counter of the copy kernel (``__amd_rocclr_copyBuffer``) of the same
run, which moves ``copy-bytes`` in each direction. With ``--largest-grid`` only the
kernel's dispatches with the largest grid count (the full-size launch, when the same
command also runs the kernel on smaller inputs). The record stores the SHA-256 of the
kernel source and the launch geometry of the profiled plan, so a reader can tell when the
kernel has changed since the counters were taken (``source_digest``: the device code of the
listed files, comments and layout aside).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import re
import statistics
import sys


# Host code of a .hip file starts after this line; the digest of a kernel covers only the
# device code above it (and every other file it names in full), so edits to host-side
# launch plumbing do not void a counter record.
HOST_MARKER = b"// ------------------------------------------------------------------ host side"


def _code_only(text: bytes) -> bytes:
    """The code of a C++ source without its comments, blank lines and indentation, so that a
    counter record only goes stale when the code changes (the device sources carry no
    comment markers inside string literals)."""
    t = re.sub(rb"/\*.*?\*/", b"", text, flags=re.S)
    t = re.sub(rb"//[^\n]*", b"", t)
    return b"\n".join(line.strip() for line in t.splitlines() if line.strip())


def source_digest(paths) -> str:
    """SHA-256 over the code of the device part of each file (all of it when it has no host
    marker), comments and layout aside."""
    if isinstance(paths, str):
        paths = paths.split(",")
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            text = f.read()
        cut = text.find(HOST_MARKER)
        h.update(_code_only(text if cut < 0 else text[:cut]))
    return h.hexdigest()


def _rows(path: str, counter: str):
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                yield r["Kernel_Name"], float(r["Counter_Value"]), int(r.get("Grid_Size") or 0)


def _kernel_and_copy(path: str, counter: str, kernel: str, largest_grid: bool = False):
    ks, cs = [], []
    for name, v, grid in _rows(path, counter):
        if kernel in name:
            ks.append((grid, v))
        elif "copyBuffer" in name:
            cs.append(v)
    if ks and largest_grid:
        top = max(g for g, _ in ks)
        ks = [(g, v) for g, v in ks if g == top]
    ks = [v for _, v in ks]
    if not ks:
        raise SystemExit(f"{path}: no {counter} rows for a kernel named like {kernel!r}")
    if not cs:
        raise SystemExit(f"{path}: no copy-kernel rows to calibrate {counter}")
    return ks, max(cs)  # the big copy (the probe); small copies are argument uploads


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, source: str,
            largest_grid: bool = False, geometry: dict = None) -> dict:
    fk, fc = _kernel_and_copy(fetch_csv, "FETCH_SIZE", kernel, largest_grid)
    wk, wc = _kernel_and_copy(write_csv, "WRITE_SIZE", kernel, largest_grid)
    f_scale = copy_bytes / (fc * 1024.0)
    w_scale = copy_bytes / (wc * 1024.0)
    fetch = statistics.mean(fk) * 1024.0 * f_scale
    write = statistics.mean(wk) * 1024.0 * w_scale
    return {
        "kernel": kernel,
        "hbm_bytes_per_launch": round(fetch + write),
        "fetch_bytes": round(fetch), "write_bytes": round(write),
        "fetch_kib_raw": statistics.mean(fk), "write_kib_raw": statistics.mean(wk),
        "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
        "copy_bytes": copy_bytes, "launches": len(fk),
        "kernel_source_sha256": source_digest(source),
        # the launch geometry the counters were taken with (the plan's tiles and LDS ring)
        "geometry": geometry,
    }


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1401_8258_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--source", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--largest-grid", action="store_true", help="only the dispatches with the largest grid")
    t.add_argument("--geometry", default=None,
                   help="JSON object: the launch geometry of the profiled plan (bench.py prints it)")
    a = ap.parse_args(argv)
    geo = json.loads(a.geometry) if a.geometry else None
    rec = traffic(a.fetch, a.write, a.kernel, a.copy_bytes, a.source, a.largest_grid, geo)
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    json.dump(rec, sys.stdout, indent=1)
    print()


if __name__ == "__main__":
    main()
