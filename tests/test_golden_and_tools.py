"""Regression fixture of the oracle, and host-side behaviour of the bench and
profiling tools."""
import json
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_matches_frozen_fixture():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_golden
    ref = json.load(open(os.path.join(HERE, "golden", "oracle_sphere_tiny.json")))
    now = make_golden.sphere_tiny()
    assert now["row_ptr"] == ref["row_ptr"] and now["col"] == ref["col"]
    assert np.allclose(now["y_first_rows"], ref["y_first_rows"], rtol=1e-12, atol=1e-14)
    assert abs(now["loss"] - ref["loss"]) <= 1e-12 * abs(ref["loss"])
    assert np.allclose(now["grad_norm_per_tensor"], ref["grad_norm_per_tensor"], rtol=1e-10)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_profiling_summaries(tmp_path):
    from paper_2411_17164_amd import profiling
    d = tmp_path / "prof"
    d.mkdir()
    (d / "x_kernel_stats.csv").write_text(
        '"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n'
        '"void xmgn::k_edge_bwd<bf16>(xmgn::BatchView)",15,30000000,2000000,60.0,1,1,0\n'
        '"copy_kernel",1,1000,1000,1.0,1,1,0\n')
    rows = profiling.stats(str(d))
    assert rows[0][0].startswith("void xmgn::k_edge_bwd") and rows[0][1] == 15 and rows[0][3] == 2000.0
    f = tmp_path / "f"
    w = tmp_path / "w"
    f.mkdir()
    w.mkdir()
    hdr = '"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n'
    (f / "a_counter_collection.csv").write_text(
        hdr + '1,"copy_kernel","FETCH_SIZE",2048\n2,"k_edge_bwd","FETCH_SIZE",4000\n3,"k_edge_bwd","FETCH_SIZE",6000\n')
    (w / "a_counter_collection.csv").write_text(
        hdr + '1,"copy_kernel","WRITE_SIZE",1024\n2,"k_edge_bwd","WRITE_SIZE",1000\n3,"k_edge_bwd","WRITE_SIZE",3000\n')
    out = tmp_path / "t.json"
    profiling.main(["traffic", "--fetch", str(f), "--write", str(w), "--kernel", "k_edge_bwd", "--calib", "copy",
                    "--calib-bytes", str(2048 * 1024), "--workload", "x", "--source-hash", "h", "--out", str(out)])
    rec = json.load(open(out))
    # fetch scale 1.0, write scale 2.0
    assert rec["bytes_per_launch"] == 5000 * 1024 + 2000 * 1024 * 2.0
