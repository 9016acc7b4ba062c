"""Host logic of the measurement path (no GPU): the counter summary that
bench.py reports as roofline traffic, and the guard that reports it only for
the profiled kernel sources and launch plan.
"""
import csv
import importlib.util
import json
import os

import pytest

from paper_2002_08110_amd import profiling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

K64 = ["void hd::stage_k3_kernel<double, 1, 1>(hd::StageParams<double>)",
       "void hd::stage_k3_kernel<double, 1, 0>(hd::StageParams<double>)",
       "void hd::stage_k3_kernel<double, 1, 2>(hd::StageParams<double>)"]
PLAN64 = {"lds": 1, "cells_per_wg": 1, "wg_size": 256, "xcd_remap": 0, "reg_dims": 2, "kernel": 1,
          "options": 1, "split_dims": 0, "loop_dims": 0}


def _csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(("Kernel_Name", "Counter_Name", "Counter_Value"), r)))


def _fake_run(tmp):
    """Counter csv files as rocprofv3 writes them: per dispatch, per kernel."""
    # copy of 4096 MiB: FETCH reads half the bytes (scale 2), WRITE all (scale 1)
    _csv(os.path.join(tmp, "cfetch", "cfetch_counter_collection.csv"),
         [("hd::stream_copy_kernel", "FETCH_SIZE", 2097152.0)])
    _csv(os.path.join(tmp, "cwrite", "cwrite_counter_collection.csv"),
         [("hd::stream_copy_kernel", "WRITE_SIZE", 4194304.0)])
    fetch = [(K64[0], "FETCH_SIZE", 100.0), (K64[0], "FETCH_SIZE", 300.0),  # mean 200
             (K64[1], "FETCH_SIZE", 400.0)] + [(K64[2], "FETCH_SIZE", 50.0)]
    write = [(K64[0], "WRITE_SIZE", 10.0), (K64[0], "WRITE_SIZE", 10.0),
             (K64[1], "WRITE_SIZE", 20.0), (K64[2], "WRITE_SIZE", 30.0)]
    _csv(os.path.join(tmp, "fetch", "fetch_counter_collection.csv"), fetch)
    _csv(os.path.join(tmp, "write", "write_counter_collection.csv"), write)
    with open(os.path.join(tmp, "fetch.log"), "w") as f:
        f.write("W20261203 some profiler line\n")
        f.write("# ran 10 stage launches (fp64, plan %r)\n" % PLAN64)
        f.write("# ran 10 stage launches (fp32, plan %r)\n" % dict(PLAN64, xcd_remap=1, options=3))


def test_counter_summary_scales_and_records_plans(tmp_path):
    tmp = str(tmp_path)
    _fake_run(tmp)
    out_json, out_md = os.path.join(tmp, "t.json"), os.path.join(tmp, "t.md")
    profiling.counters(tmp, 4096, out_json, out_md)
    d = json.load(open(out_json))
    assert d["fetch_scale"] == pytest.approx(2.0)
    assert d["write_scale"] == pytest.approx(1.0)
    assert d["plans"]["fp64"] == PLAN64
    assert d["plans"]["fp32"]["xcd_remap"] == 1
    k = d["kernels"][K64[0]]
    assert k["launches"] == 2
    # (mean FETCH 200 KiB * 2 + mean WRITE 10 KiB * 1) * 1024 bytes
    assert k["bytes_per_launch"] == pytest.approx((200.0 * 2 + 10.0) * 1024)
    assert d["kernel_source_digest"] == profiling.kernel_source_digest()
    assert "stage_k3_kernel<double, 1, 0>" in open(out_md).read()


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_for_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_traffic_is_launch_weighted_and_guarded(tmp_path):
    bench = _bench_module()
    prof = tmp_path / "profiles"
    prof.mkdir()
    data = {"kernel_source_digest": profiling.kernel_source_digest(), "plans": {"fp64": PLAN64},
            "kernels": {K64[0]: {"launches": 2, "bytes_per_launch": 10.0},
                        K64[1]: {"launches": 6, "bytes_per_launch": 20.0},
                        K64[2]: {"launches": 2, "bytes_per_launch": 30.0}}}
    (prof / "stage_6d_8x6_k3_traffic.json").write_text(json.dumps(data))
    bench.ROOT = str(tmp_path)
    got = bench.profiled_kernel("fp64", {}, dict(PLAN64, lds=0, reg_dims=1))  # ignored fields differ
    assert got["launches"] == 10 and got["variants"] == 3
    assert got["bytes_per_launch"] == pytest.approx((2 * 10 + 6 * 20 + 2 * 30) / 10)
    # another cell order, another plan or kernel sources: no traffic reported
    assert bench.profiled_kernel("fp64", {}, dict(PLAN64, xcd_remap=1)) is None
    assert bench.profiled_kernel("fp64", {"kernel": 1}, PLAN64) is None
    assert bench.profiled_kernel("fp32", {}, PLAN64) is None
    data["kernel_source_digest"] = "0" * 16
    (prof / "stage_6d_8x6_k3_traffic.json").write_text(json.dumps(data))
    assert bench.profiled_kernel("fp64", {}, PLAN64) is None
