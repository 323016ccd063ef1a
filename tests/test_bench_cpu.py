"""Host logic of bench.py: the choice of the counter record for the Krylov
kernel a run launched, the stale-record rule, and the one-GPU contract."""
import json
import os
import subprocess
import sys

import bench as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rec(kernel, threads, ratio):
    return {"kernel": kernel, "shape": {"krylov_threads": threads, "krylov_precond": 8},
            "hbm_bytes_per_iteration": 1.0e6 * ratio, "ratio": ratio}


def test_krylov_traffic_record_matches_form_and_width():
    tr = {"krylov_bicgstab": [_rec("k_bicgstab_ov<256>", 256, 0.5), _rec("k_bicgstab_ov<512>", 512, 0.6)]}
    overlapped = 1 | 4 | 8          # resident, block-Jacobi, overlapped
    barrier = 1 | 4
    assert B.krylov_traffic_record(tr, overlapped, {"krylov_threads": 512})["ratio"] == 0.6
    assert B.krylov_traffic_record(tr, overlapped, {"krylov_threads": 256})["ratio"] == 0.5
    # another width, or the barrier form: no record (the counters belong to one kernel)
    assert B.krylov_traffic_record(tr, overlapped, {"krylov_threads": 1024}) is None
    assert B.krylov_traffic_record(tr, barrier, {"krylov_threads": 256}) is None
    # a single record (earlier layout) is still read
    one = {"krylov_bicgstab": _rec("k_bicgstab_reg<256, 8>", 256, 0.2)}
    assert B.krylov_traffic_record(one, barrier, {"krylov_threads": 256})["ratio"] == 0.2
    assert B.krylov_traffic_record({}, barrier, {"krylov_threads": 256}) is None


def test_traffic_record_is_dropped_when_the_kernels_changed(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.json").write_text(json.dumps({"source_sha": "0000000000000000", "krylov_bicgstab": []}))
    monkeypatch.setattr(B, "ROOT", str(tmp_path))
    monkeypatch.setattr(B, "kernel_source_sha", lambda: "1111111111111111")
    assert B.load_traffic() is None
    monkeypatch.setattr(B, "kernel_source_sha", lambda: "0000000000000000")
    assert B.load_traffic() is not None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus 2" in r.stderr and r.stdout == ""
