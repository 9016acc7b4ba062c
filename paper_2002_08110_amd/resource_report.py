"""Register, scratch and LDS use of every compiled stage-kernel variant, from
hipcc's resource-usage remarks (-Rpass-analysis=kernel-resource-usage), for
each kernel's own launch form (stage_kernel, stage_k3_kernel) next to its
work-list form (stage_list_kernel, stage_k3_list_kernel).

The batched step runs a variant's work-list form only where, at the launch
shape in use, it keeps the own form's workgroups per CU and scratch (checked
at run time with hipFuncGetAttributes and the occupancy query); this report
shows the compile-time picture for all variants at once.

Usage: python -m paper_2002_08110_amd.resource_report OUT_MD
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

from paper_2002_08110_amd.build import CSRC, FLAGS, HIPCC

UNITS = ["stage_d%d_%s" % (d, p) for d in range(2, 7) for p in ("f32", "f64")] + ["stage_k3"]


def remarks(unit: str) -> str:
    src = os.path.join(CSRC, unit + ".hip")
    cmd = [HIPCC] + [f for f in FLAGS if f != "-fPIC"] + [
        "--cuda-device-only", "-c", src, "-o", os.devnull,
        "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-2000:])
    return r.stderr


def parse(text: str) -> dict:
    rows, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            rows[cur] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z][^:]*): (\S+)", line)
        if m and cur:
            rows[cur][m.group(1).strip()] = m.group(2)
    return rows


def demangle(names):
    r = subprocess.run(["c++filt"], input="\n".join(names), capture_output=True, text=True)
    return r.stdout.split("\n")


def table(rows: dict):
    names = list(rows)
    pairs = {}
    for n, d in zip(names, demangle(names)):
        m = re.match(r"void hd::(stage_list_kernel|stage_kernel|stage_k3_list_kernel|stage_k3_kernel)"
                     r"<(.*)>\(", d)
        if not m:
            continue
        form = "list" if "list" in m.group(1) else "own"
        fam = "stage_k3_kernel" if "k3" in m.group(1) else "stage_kernel"
        pairs.setdefault((fam, m.group(2)), {})[form] = rows[n]
    return pairs


def fmt(r):
    return "%s / %s / %s / %s" % (r.get("VGPRs"), r.get("AGPRs"), r.get("ScratchSize [bytes/lane]"),
                                  r.get("Occupancy [waves/SIMD]"))


def main(out_md: str):
    with cf.ThreadPoolExecutor(max_workers=min(len(UNITS), os.cpu_count() or 4)) as ex:
        texts = list(ex.map(remarks, UNITS))
    rows = {}
    for t in texts:
        rows.update(parse(t))
    pairs = table(rows)
    worse = []
    lines = ["| kernel | template arguments (D, N, DX, RD, P, LDS, SD, OPT, LD; k3: P, OPT, ROLE) | "
             "own form VGPR / AGPR / scratch B / waves | work-list form |", "|---|---|---|---|"]
    count = 0
    for (fam, args), v in sorted(pairs.items()):
        own, lst = v.get("own"), v.get("list")
        if not own or not lst:
            continue
        count += 1
        keeps = (int(lst["Occupancy [waves/SIMD]"]) >= int(own["Occupancy [waves/SIMD]"]) and
                 int(lst["ScratchSize [bytes/lane]"]) <= int(own["ScratchSize [bytes/lane]"]))
        if not keeps:
            worse.append(args)
            lines.append("| %s | %s | %s | %s |" % (fam, args, fmt(own), fmt(lst)))
    static_lds = sorted({r.get("LDS Size [bytes/block]") for r in rows.values()})
    head = ["# Resource use of the stage kernels (hipcc -Rpass-analysis=kernel-resource-usage)", "",
            "Command: `python -m paper_2002_08110_amd.resource_report %s` (compiles each stage "
            "translation unit for gfx950 with the library's flags)." % out_md, "",
            "%d variants; the work-list form keeps the own form's waves per SIMD and scratch for %d "
            "of them, and the table lists the others (a batched step launches those solves on "
            "their own). Static LDS of every kernel (bytes): %s; all LDS is dynamic (at most 160 "
            "KiB per workgroup, set per launch)." % (count, count - len(worse),
                                                    ", ".join(static_lds)), "",
            "Waves per SIMD is the compiler's occupancy bound from registers alone (LDS can lower "
            "it further at run time).", ""]
    with open(out_md, "w") as f:
        f.write("\n".join(head + lines) + "\n")
    print("%d variants, %d keep resources in the work-list form" % (count, count - len(worse)))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "profiles/kernel_resources.md")
