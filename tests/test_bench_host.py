"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the rule that a
stored HBM-traffic record counts only while the kernel sources it names are
unchanged, the stage-C kernel names the records and profiles are keyed by,
and whether the committed traffic records match the current sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_counts_only_for_unchanged_sources(tmp_path, monkeypatch):
    import hashlib
    src = tmp_path / "k.hpp"
    src.write_text("kernel v1\n")
    rec = {"kernel": "K<1>", "bytes_per_launch": 123.0, "sources": ["k.hpp"],
           "source_sha256": hashlib.sha256(b"kernel v1\n").hexdigest()}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps({"w": [rec]}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(str(path), "w", "K<1>") == 123.0
    assert bench.measured_traffic(str(path), "w", "K<2>") is None
    assert bench.measured_traffic(str(path), "other", "K<1>") is None
    src.write_text("kernel v2\n")
    assert bench.measured_traffic(str(path), "w", "K<1>") is None


def test_stage_c_kernel_names():
    assert bench.stage_c_kernel("fp64", 2, 7) == \
        "tile_gemm_persistent<4,2,5,16,Batched<StageC<double>>>"
    assert bench.stage_c_kernel("fp32", 3, 7).startswith("tile_dma_persistent<")
    assert bench.stage_c_kernel("bf16x3", 0, 0).startswith("tile_bf16x3_kernel<")
    assert bench.stage_c_kernel("bf16x3", 3, 7) == "tile_bf3_dma_persistent<4,2,4,5,3,0,Batched<StageCBf>>"


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_committed_traffic_records_match_the_sources(prec):
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    rec = next(r for r in d["strip300"] if r["prec"] == prec)
    got = bench.measured_traffic(os.path.join(ROOT, "profiles", "traffic.json"), "strip300",
                                 rec["kernel"])
    if got is None:
        pytest.skip("kernel sources changed since the counters were taken: bench.py reports "
                    "traffic null until FETCH_SIZE / WRITE_SIZE are taken again")
    assert got == rec["bytes_per_launch"]

