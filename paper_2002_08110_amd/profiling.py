"""Summaries of rocprofv3 output for the committed profiles.

The byte counters FETCH_SIZE and WRITE_SIZE are taken in separate runs (one
counter group per run). Each is scaled by what the same counter reports for
the library's plain streaming copy (hd_stream_copy) of a known size, which
reads and writes exactly that many bytes. The result is the bytes the fused
stage kernel moves between L2 and memory per launch, written to a small JSON
file that bench.py reports as roofline "traffic" while the kernel source is
unchanged (checked with a digest of the kernel headers).

Usage:
  python -m paper_2002_08110_amd.profiling counters DIR COPY_MIB OUT_JSON OUT_MD
  python -m paper_2002_08110_amd.profiling trace STATS_CSV COMMAND OUT_MD
"""
from __future__ import annotations

import ast
import collections
import csv
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/stage_kernel.h", "csrc/stage_k3.h")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _counter_means(path):
    agg = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}, {k: len(v) for k, v in agg.items()}


def _pick(means, needle):
    out = {}
    for (k, c), v in means.items():
        if needle in k:
            out[k] = v
    return out


def _plans(run_dir):
    """The launch plan per precision that the counted run printed."""
    plans = {}
    log = os.path.join(run_dir, "fetch.log")
    if os.path.exists(log):
        for line in open(log):
            m = re.match(r"# ran \d+ stage launches \((fp\d\d), plan (\{.*\})\)", line)
            if m:
                plans[m.group(1)] = ast.literal_eval(m.group(2))
    return plans


def counters(run_dir, copy_mib, out_json, out_md):
    """run_dir holds fetch/, write/, cfetch/, cwrite/ rocprofv3 csv outputs."""
    def csvp(name):
        return os.path.join(run_dir, name, name + "_counter_collection.csv")

    fetch, nf = _counter_means(csvp("fetch"))
    write, nw = _counter_means(csvp("write"))
    cfetch, _ = _counter_means(csvp("cfetch"))
    cwrite, _ = _counter_means(csvp("cwrite"))
    copy_kib = copy_mib * 1024.0
    cf = list(_pick(cfetch, "stream_copy").values())[0]
    cw = list(_pick(cwrite, "stream_copy").values())[0]
    f_scale = copy_kib / cf
    w_scale = copy_kib / cw
    res = {"kernel_source_digest": kernel_source_digest(), "copy_mib": copy_mib,
           "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": f_scale, "write_scale": w_scale, "plans": _plans(run_dir),
           "kernels": {}}
    valu = {}
    if os.path.exists(csvp("valu")):
        valu, _ = _counter_means(csvp("valu"))
    for (k, c), v in fetch.items():
        if "stage" not in k:
            continue
        wv = write.get((k, "WRITE_SIZE"))
        res["kernels"][k] = {
            "launches": nf[(k, c)], "fetch_kib": v, "write_kib": wv,
            "bytes_per_launch": (v * f_scale + wv * w_scale) * 1024.0,
        }
        if (k, "VALUBusy") in valu:
            res["kernels"][k]["valu_busy_pct"] = valu[(k, "VALUBusy")]
            res["kernels"][k]["flops_fp64_per_launch"] = valu.get((k, "SQ_INSTS_VALU_FLOPS_FP64"))
            res["kernels"][k]["flops_fp32_per_launch"] = valu.get((k, "SQ_INSTS_VALU_FLOPS_FP32"))
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    lines = ["# Byte counters of the fused stage kernels", "",
             "Counters per dispatch (KiB, mean over the dispatches of two RK steps of",
             "the 6D 8^6 k=3 workload), scaled by the library's plain copy of %d MiB:" % copy_mib,
             "", "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes/launch (scaled) |",
             "|---|---|---|---|---|"]
    for k, d in res["kernels"].items():
        lines.append("| `%s` | %d | %.4g | %.4g | %.4g GB |" % (k, d["launches"], d["fetch_kib"],
                                                                d["write_kib"],
                                                                d["bytes_per_launch"] / 1e9))
    if any("valu_busy_pct" in d for d in res["kernels"].values()):
        lines += ["", "VALU activity (derived counter VALUBusy = active VALU cycles / CUs / GPU",
                  "busy cycles; VALU FLOP counters per launch):", "",
                  "| kernel | VALUBusy % | FP64 FLOP/launch | FP32 FLOP/launch |", "|---|---|---|---|"]
        for k, d in res["kernels"].items():
            if "valu_busy_pct" in d:
                lines.append("| `%s` | %.1f | %.4g | %.4g |" % (
                    k, d["valu_busy_pct"], d["flops_fp64_per_launch"] or 0,
                    d["flops_fp32_per_launch"] or 0))
    lines += ["", "Commands (one counter per run, from the repository root after",
              "`cd /tmp && export TMPDIR=/tmp`):", "", "```"]
    for name, cnt, mode in (("fetch", "FETCH_SIZE", "--mode stages --steps 2"),
                            ("write", "WRITE_SIZE", "--mode stages --steps 2"),
                            ("valu", "VALUBusy SQ_INSTS_VALU_FLOPS_FP64 SQ_INSTS_VALU_FLOPS_FP32",
                             "--mode stages --steps 2"),
                            ("cfetch", "FETCH_SIZE", "--mode copy --copy-mib %d" % copy_mib),
                            ("cwrite", "WRITE_SIZE", "--mode copy --copy-mib %d" % copy_mib)):
        lines.append("rocprofv3 --pmc %s --output-format csv -d %s/%s -o %s -- "
                     "python3 bench.py %s" % (cnt, run_dir.rstrip("/"), name, name, mode))
    lines += ["python -m paper_2002_08110_amd.profiling counters %s %d "
              "profiles/<name>_traffic.json profiles/<name>_counters.md"
              % (run_dir.rstrip("/"), copy_mib), "```"]
    lines += ["", "Copy calibration: FETCH_SIZE %.4g KiB and WRITE_SIZE %.4g KiB for %d MiB "
              "read + %d MiB written: scales %.3f (fetch) and %.3f (write)."
              % (cf, cw, copy_mib, copy_mib, f_scale, w_scale),
              "", "Kernel source digest: `%s`." % res["kernel_source_digest"]]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return res


def trace(stats_csv, command, out_md):
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["# Kernel trace summary", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | average ms | min ms | max ms | share % |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append("| `%s` | %s | %.4f | %.4f | %.4f | %.2f |" % (
            r["Name"][:90], r["Calls"], float(r["AverageNs"]) / 1e6, float(r["MinNs"]) / 1e6,
            float(r["MaxNs"]) / 1e6, float(r["Percentage"])))
    # The stage launches of one precision run up to three kernel variants
    # (first stage, general, late increment): their launch-weighted mean is
    # the average stage launch.
    mean = []
    for prec, needle in (("FP64", "stage_k3_kernel<double"), ("FP32 mode", "stage_k3_kernel<float")):
        rs = [r for r in rows if needle in r["Name"]]
        if rs:
            calls = sum(int(r["Calls"]) for r in rs)
            avg = sum(int(r["Calls"]) * float(r["AverageNs"]) for r in rs) / calls / 1e6
            mean.append("| %s | %d | %d | %.4f |" % (prec, len(rs), calls, avg))
    if mean:
        lines += ["", "Mean stage launch of the 6D degree-3 kernel, weighted by calls:", "",
                  "| mode | variants | calls | average ms |", "|---|---|---|---|"] + mean
    vp = hashlib.sha256(open(os.path.join(HERE, "csrc/hd_vp.hip"), "rb").read()).hexdigest()[:16]
    lines += ["", "Kernel source digest: `%s` (stage kernels), `%s` (Vlasov-Poisson field)."
              % (kernel_source_digest(), vp)]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "counters":
        counters(sys.argv[2], int(sys.argv[3]), sys.argv[4], sys.argv[5])
    elif sys.argv[1] == "trace":
        trace(sys.argv[2], sys.argv[3], sys.argv[4])
    else:
        raise SystemExit(__doc__)
