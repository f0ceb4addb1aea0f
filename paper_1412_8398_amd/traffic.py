"""HBM traffic per launch of each pass from two rocprofv3 counter runs.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d prof/pf -o pf -- \\
        python3 bench.py --size L --steps 3 --warmup 1 --no-cpu-baseline --no-tti --no-fp64 --copy-calibration
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d prof/pw -o pw -- (same)
    python -m paper_1412_8398_amd.traffic --size L --fetch prof/pf/pf_counter_collection.csv \\
        --write prof/pw/pw_counter_collection.csv --out profiles/traffic_ASR_fp32_L.json

The counters are read in KiB per dispatch.  The 1 GiB device copy that
``bench.py --copy-calibration`` runs first (a plain read-and-write kernel of
known size) calibrates them: its FETCH_SIZE and WRITE_SIZE readings against
the 1 GiB it reads and writes give the two scale factors.  Each pass's record
holds the mean scaled bytes per dispatch, the algorithmic bytes of bench.py's
model and a SHA-256 over the kernel's source files, so that bench.py can drop
the measured figure once the kernel has changed.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")

# the sources each pass's kernel is built from
_FFT = ["fe_passes.h", "fe_fft.h", "fe_device.h"]
_STENCIL = ["fe_pointwise.hip", "fe_stencil.h", "fe_device.h", "fe_kernels.h"]
PASSES = {
    "pointwise": (r"^void fe::k_div<\d+, \d+, float, float, float, 2>", _STENCIL),
    "zfwd": (r"^void fe::k_zr2c<float, {L}>", ["fe_pass_z.hip"] + _FFT),
    "yfwd": (r"^void fe::k_ypass<float, {L}, false>", ["fe_pass_y.hip"] + _FFT),
    "xgreen": (r"^void fe::k_xgreen3<float, {L}, 2>", ["fe_pass_x3.hip", "fe_green.h"] + _FFT),
    "yinv": (r"^void fe::k_ypass<float, {L}, true>", ["fe_pass_y.hip"] + _FFT),
    "zinv": (r"^void fe::k_zc2r<float, {L}>", ["fe_pass_z.hip"] + _FFT),
    "update": (r"^void fe::k_update_div<\d+, \d+, float, 2, true, false, true>", _STENCIL),
}
COPY_BYTES = 1 << 30


def sources_sha256(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _rows(path, counter):
    out = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                out.append((r["Kernel_Name"], int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    return sorted(out, key=lambda t: t[1])


def _calibration(rows):
    """The first copy dispatch of the run: bench.py's 1 GiB calibration copy."""
    for name, _, value in rows:
        if "copyBuffer" in name:
            return value
    raise ValueError("no calibration copy in the counter file (run bench.py with --copy-calibration)")


def build(size, fetch_csv, write_csv, commands):
    sys.path.insert(0, ROOT)
    from bench import pass_bytes

    fr, wr = _rows(fetch_csv, "FETCH_SIZE"), _rows(write_csv, "WRITE_SIZE")
    f_cal, w_cal = _calibration(fr), _calibration(wr)
    fscale, wscale = COPY_BYTES / 1024.0 / f_cal, COPY_BYTES / 1024.0 / w_cal
    algo = pass_bytes(size)
    kernels = {}
    for name, (pattern, files) in PASSES.items():
        rx = re.compile(pattern.replace("{L}", str(size)))
        fv = [v for k, _, v in fr if rx.search(k)]
        wv = [v for k, _, v in wr if rx.search(k)]
        if not fv or not wv:
            continue
        kname = next(re.sub(r"\(.*", "", k) for k, _, _ in fr if rx.search(k))
        fk, wk = sum(fv) / len(fv), sum(wv) / len(wv)
        kernels[name] = {
            "kernel": kname,
            "dispatches": len(fv),
            "fetch_kib": fk,
            "write_kib": wk,
            "bytes": (fk * fscale + wk * wscale) * 1024.0,
            "algorithmic_bytes": algo[name],
            "sources": files,
            "sources_sha256": sources_sha256(files),
        }
    return {
        "workload": f"{size}^3 sphere-Boolean, AS + rotated operator, float32 (bench.py recipe)",
        "commands": commands,
        "calibration": {"copy_bytes": COPY_BYTES, "fetch_kib_read": f_cal, "write_kib_read": w_cal,
                        "fetch_scale": fscale, "write_scale": wscale},
        "kernels": kernels,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", action="append", default=[], help="the profiling commands, for the record")
    a = ap.parse_args(argv)
    rec = build(a.size, a.fetch, a.write, a.command)
    with open(a.out, "w") as fh:
        json.dump(rec, fh, indent=1)
    for k, v in rec["kernels"].items():
        print(f"{k:10s} {v['kernel'][:56]:56s} {v['bytes'] / 1e9:8.3f} GB  x{v['bytes'] / v['algorithmic_bytes']:.3f}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
