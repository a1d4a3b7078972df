"""Host logic of bench.py (CPU): the gate on committed counter figures and the one-GPU guard."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _digest(rel):
    return hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest()


def _traffic_file(tmp_path, digests):
    kernels = {
        "void jac::blk_inner_v_kernel<double, true>": {"fetch_bytes": 1.0, "write_bytes": 2.0, "bytes": 3.0,
                                                       "dispatches": 3},
        "void jac::blk_inner_kernel<double, false>": {"fetch_bytes": 4.0, "write_bytes": 3.0, "bytes": 7.0,
                                                      "dispatches": 1},
        "void jac::sytrd_reg_kernel<double, 256, 8, 8, double>": {"fetch_bytes": 5.0, "write_bytes": 6.0,
                                                                  "bytes": 11.0, "dispatches": 2},
    }
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps({"sources": digests, "kernels": kernels}))
    return str(p)


def test_traffic_is_gated_by_the_source_of_its_own_kernels(tmp_path, monkeypatch):
    blk, tri = "paper_2211_03339_amd/csrc/blocked.hip", "paper_2211_03339_amd/csrc/tridiag.hip"
    good = {blk: _digest(blk), tri: _digest(tri)}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path, good))
    # dispatch-weighted mean over the class's kernels: (3 * 3 + 7 * 1) / 4
    assert bench.measured_traffic("inner64") == 4.0
    assert bench.measured_traffic("tridiag_reduce") == 11.0
    assert bench.measured_traffic("elem64") is None          # no source recorded for it
    assert bench.measured_traffic("no_such_class") is None
    # a changed tridiagonal source voids only the tridiagonal figures
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path, {blk: good[blk], tri: "0" * 64}))
    assert bench.measured_traffic("inner64") == 4.0
    assert bench.measured_traffic("tridiag_reduce") is None
    # and a changed block-sweep source voids the inner-solve figure
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path, {blk: "0" * 64, tri: good[tri]}))
    assert bench.measured_traffic("inner64") is None
    assert bench.measured_traffic("tridiag_reduce") == 11.0


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
