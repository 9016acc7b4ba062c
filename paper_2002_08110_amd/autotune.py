"""Autotuner of the fused stage kernel's launch plan per (d, k, precision).

For a representative mesh it times every valid plan - generic kernel with
one or two register dimensions, LDS or global line reads, cells per
workgroup, XCD-aware tile order; the 6D degree-3 kernel with its streaming
options; the dimension-split passes at degrees 4 and 5 (d = 5, 6) - over
full RK steps' worth of stage launches, and records the
fastest in a JSON cache keyed by (GPU architecture, d, k, precision). A
Solver picks its plan from the cache with `apply_tuned_plan`.

  python -m paper_2002_08110_amd.autotune --out PATH [--dims 3,4,5,6] [--degrees 2,3,4,5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

from . import workloads as W

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_plans.json")


def arch_name():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def key(arch, d, k, precision):
    return "%s|d%d|k%d|%s" % (arch, d, k, precision)


def candidate_plans(d, k, dim_v, precision):
    n = k + 1
    psize = 4 if precision == "fp32" else 8
    nd = n ** d
    plans = []
    if d == 6 and k == 3:
        for opt in ((0, 1, 2, 3) if precision == "fp32" else (0, 1)):
            for xcd in (0, 1):
                plans.append(dict(kernel=1, options=opt, xcd_remap=xcd, split_dims=0))
    for rd in (1, 2):
        if rd > dim_v:
            continue
        for sd in (1, 2):
            # slabs of cells too large to stage whole (degree >= 4, d >= 5)
            if n < 5 or d < 5 or rd + sd > dim_v or n ** (d - rd - sd) > 1024:
                continue
            Ts = n ** (d - rd - sd)
            ub = n ** (d - sd) * psize
            if ub > 160 * 1024:
                continue
            cpws = [1] if Ts > 256 else sorted({1, max(1, 256 // Ts)})
            for cpw in cpws:
                if cpw * ub <= 160 * 1024:
                    for xcd in (0, 1):
                        plans.append(dict(kernel=0, options=0, lds=1, cells_per_wg=cpw, reg_dims=rd,
                                          split_dims=sd, xcd_remap=xcd, wg_size=256))
        for sd in (0, 1, 2):
            # looped pencils: a thread covers the k+1 pencils of one fast dim
            nf = d - rd - sd
            if (n < 5 or d < 5 or rd + sd > dim_v or nf - 1 < d - dim_v
                    or n ** (nf - 1) > 1024 or n ** (d - sd) * psize > 160 * 1024):
                continue
            for xcd in (0, 1):
                plans.append(dict(kernel=0, options=0, lds=1, cells_per_wg=1, reg_dims=rd,
                                  split_dims=sd, loop_dims=1, xcd_remap=xcd, wg_size=256))
        T = n ** (d - rd)
        for xcd in (0, 1):
            plans.append(dict(kernel=0, options=0, lds=0, wg_size=256, reg_dims=rd, xcd_remap=xcd,
                              cells_per_wg=1, split_dims=0))
            if T <= 1024 and nd * psize <= 160 * 1024:
                cpws = [1] if T > 256 else sorted({1, max(1, 256 // T)})
                for cpw in cpws:
                    if cpw * nd * psize <= 160 * 1024 and (T > 256 or cpw * T <= 256):
                        plans.append(dict(kernel=0, options=0, lds=1, cells_per_wg=cpw,
                                          reg_dims=rd, xcd_remap=xcd, wg_size=256, split_dims=0))
    generic = [p for p in plans if p["kernel"] == 0]
    for p in generic:  # the streaming option of the generic kernel
        plans.append(dict(p, options=1))
    if dim_v in (2, 3) and d - dim_v == 3 and k in (4, 5):
        # the dimension-split passes (x terms, then v terms and the update)
        for xcd in (0, 1):
            for opt in (0, 1):
                plans.append(dict(kernel=2, options=opt, xcd_remap=xcd, split_dims=0))
    full = dict(lds=0, cells_per_wg=1, wg_size=256, xcd_remap=0, reg_dims=1, kernel=0, options=0,
                split_dims=0, loop_dims=0)
    return [dict(full, **p) for p in plans]


def same_launch(a, b):
    """True if two plans launch the same kernel the same way (fields that
    the chosen kernel ignores do not count)."""
    if a.get("kernel", 0) != b.get("kernel", 0):
        return False
    keys = ["xcd_remap", "options"]
    if a.get("kernel", 0) == 0:
        keys += ["lds", "reg_dims", "split_dims", "loop_dims"]
        keys += ["cells_per_wg"] if a.get("lds") else ["wg_size"]
    return all(a.get(k, 0) == b.get(k, 0) for k in keys)


def representative_case(d, k, target_dofs=1.5e8):
    dx, dv = W.SPLITS[d]
    n = k + 1
    c = max(2, int(round((target_dofs / n ** d) ** (1.0 / d))))
    cells = [c] * d
    if dx == dv:
        return W.phase_space_case("tune_d%dk%d" % (d, k), dx, dv, cells, k, 1)
    rng = np.random.default_rng(d * 10 + k)
    return W.Case("tune_d%dk%d" % (d, k), dx, dv, cells, [0.0] * d, [1.0] * d, k, "constant",
                  a=list(rng.uniform(-1, 1, d)))


def time_plans(case, precision, reps=2):
    import torch

    from .solver import Solver
    S = Solver(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
               precision=precision)
    if case.field == "sine":
        S.set_field_sine(case.amp)
    else:
        S.set_field_constant(case.a)
    S.init_state(case.ic, list(case.ic_params))
    dt = S.stable_dt(case.cfl)
    results = []
    for plan in candidate_plans(case.d, case.degree, case.dim_v, precision):
        try:
            S.set_plan(**plan)
        except Exception:
            continue
        for st in range(5):
            S.rk_stage(st, dt)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            for st in range(5):
                S.rk_stage(st, dt)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / (5 * reps)
        results.append((ms, plan))
    S.close()
    torch.cuda.empty_cache()
    results.sort(key=lambda r: r[0])
    return S.ndofs, results


def load_cache(path=DEFAULT_CACHE):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def lookup(d, k, precision, path=DEFAULT_CACHE, arch=None):
    cache = load_cache(path)
    if arch is None:
        arch = arch_name()
    entry = cache.get(key(arch, d, k, precision))
    return None if entry is None else entry["plan"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--dims", default="3,4,5,6")
    ap.add_argument("--degrees", default="2,3,4,5")
    ap.add_argument("--precisions", default="fp32,fp64")
    ap.add_argument("--target-dofs", type=float, default=1.5e8)
    args = ap.parse_args()
    arch = arch_name()
    cache = load_cache(args.out)
    for prec in args.precisions.split(","):
        for d in map(int, args.dims.split(",")):
            for k in map(int, args.degrees.split(",")):
                case = representative_case(d, k, args.target_dofs)
                ndofs, res = time_plans(case, prec)
                if not res:
                    continue
                best_ms, best = res[0]
                cache[key(arch, d, k, prec)] = {
                    "plan": best, "ms_per_stage": best_ms, "dofs": ndofs, "cells": case.cells,
                    "gdofs_per_s": ndofs / best_ms / 1e6,
                    "worst_ms": res[-1][0], "candidates": len(res)}
                print("%s d=%d k=%d: best %.3f ms (%.1f GDoF/s) %s; worst %.3f ms over %d plans"
                      % (prec, d, k, best_ms, ndofs / best_ms / 1e6, best, res[-1][0], len(res)),
                      file=sys.stderr, flush=True)
                with open(args.out, "w") as f:
                    json.dump(cache, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
