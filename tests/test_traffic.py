"""Host logic of the measurement records: the algorithmic byte model of the
passes (bench.pass_bytes) and the traffic records built from rocprofv3
counter files (paper_1412_8398_amd.traffic), on synthetic counter files."""
import csv
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from bench import pass_bytes, spectrum_bytes  # noqa: E402
from paper_1412_8398_amd import traffic  # noqa: E402


def test_pass_bytes_per_voxel():
    L = 512
    N = L ** 3
    b = pass_bytes(L)
    # fused update: read U (12), eps^k (24), phase (1); write eps^(k+1) (24), D (12)
    assert b["update"] == 73 * N
    # stand-alone divergence: read eps (24), phase (1); write D (12)
    assert b["pointwise"] == 37 * N
    # each transform pass reads and writes about 12 B/voxel of spectra or real planes
    for k in ("zfwd", "yfwd", "xgreen", "yinv", "zinv"):
        assert 24 * N <= b[k] <= 24 * N * (1 + 4 / L)
    it = sum(v for k, v in b.items() if k != "pointwise") / N
    assert 193 <= it <= 194


def test_spectrum_bytes_follow_the_z_blocking():
    # half spectra: nz/2 + 1 planes rounded up to blocks of 8 (4, 2, 1 where 8 does not divide nz)
    assert spectrum_bytes(512) == 3 * 264 * 512 * 512 * 8
    assert spectrum_bytes(1024) == 3 * 520 * 1024 * 1024 * 8
    assert spectrum_bytes(36) == 3 * 20 * 36 * 36 * 8  # 36: blocks of 4, 19 planes -> 20


def _write(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, k, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v})


ZR2C = "void fe::k_zr2c<float, 64>(float const*, fe::cpx<float>*, fe::Dims, fe::cpx<float> const*, fe::Batch)"
UPD = "void fe::k_update_div<32, 8, float, 2, true, false, true>(float const*, ...)"
COPY = "__amd_rocclr_copyBuffer"


def test_traffic_record_from_counter_files(tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    # the first copy is the 1 GiB calibration: FETCH_SIZE reads half the bytes, WRITE_SIZE all
    _write(f, "FETCH_SIZE", [(1, COPY, 524288.0), (2, ZR2C, 100.0), (3, UPD, 300.0), (4, ZR2C, 120.0),
                             (5, COPY, 7.0)])
    _write(w, "WRITE_SIZE", [(1, COPY, 1048576.0), (2, ZR2C, 50.0), (3, UPD, 200.0), (4, ZR2C, 70.0),
                             (5, COPY, 9.0)])
    rec = traffic.build(64, str(f), str(w), ["cmd"])
    cal = rec["calibration"]
    assert cal["fetch_scale"] == pytest.approx(2.0) and cal["write_scale"] == pytest.approx(1.0)
    z = rec["kernels"]["zfwd"]
    assert z["dispatches"] == 2 and z["kernel"] == "void fe::k_zr2c<float, 64>"
    assert z["fetch_kib"] == pytest.approx(110.0) and z["write_kib"] == pytest.approx(60.0)
    assert z["bytes"] == pytest.approx((110.0 * 2.0 + 60.0) * 1024.0)
    assert z["algorithmic_bytes"] == pass_bytes(64)["zfwd"]
    assert re.fullmatch(r"[0-9a-f]{64}", z["sources_sha256"])
    assert z["sources_sha256"] == traffic.sources_sha256(z["sources"])
    u = rec["kernels"]["update"]
    assert u["bytes"] == pytest.approx((300.0 * 2.0 + 200.0) * 1024.0)
    # passes without dispatches in the files get no record
    assert "yfwd" not in rec["kernels"] and rec["commands"] == ["cmd"]


def test_traffic_record_needs_the_calibration_copy(tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(f, "FETCH_SIZE", [(1, ZR2C, 100.0)])
    _write(w, "WRITE_SIZE", [(1, ZR2C, 50.0)])
    with pytest.raises(ValueError):
        traffic.build(64, str(f), str(w), [])
