"""Benchmark of the fused DG advection RK stage on one MI355X.

Workload: 6D phase-space advection (3 x + 3 v dims), 8^6 cells, degree 3
(4096 DoFs per cell, 1,073,741,824 DoFs), a = (v, 0.1 sin(2 pi x)), the
perturbed-Maxwellian initial state, LSRK45 with CFL 0.2. A "step" is one
full RK step (5 fused stage launches) over the whole state, which is
resident in HBM before timing starts. The metric is DoF updates per second
per RK stage (N_DoF / t_stage, t_stage = t_step / 5); the headline value is
FP64, the FP32-operator mode is reported beside it.

Prints ONE JSON line (rank 0, N = 1).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0     # MI355X HBM3E peak
PAPER_GDOFS_PER_NODE = 1.12  # 6D k=3 32^6 DoFs per SuperMUC-NG node, context only
# Algorithmic bytes per DoF of the five fused stages: stage 1 reads u and
# writes du and u'; stages 2-4 read u, du and write du, u'; stage 5 reads u,
# du and writes u'. u is FP64, du has the operator precision.
def stage_bytes(psize):
    return [8 + psize + 8, 8 + 2 * psize + 8, 8 + 2 * psize + 8, 8 + 2 * psize + 8, 8 + psize + 8]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="6d", choices=["6d", "4d", "6d_small", "2d", "6d_k4", "6d_k5"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving trace in the default run")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="seconds of the headline-mesh cell sample (CPU baseline extra)")
    ap.add_argument("--precisions", default="fp64,fp32")
    ap.add_argument("--plan", default="", help="override plan, e.g. lds=1,reg_dims=1")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the library's default plan instead of timing the candidates "
                         "on the workload's mesh (profiled runs: no tuning launches)")
    ap.add_argument("--mode", default="bench",
                    choices=["bench", "stages", "copy", "batch", "serve", "vp", "gauss", "mapped"],
                    help="stages: only run --steps x 5 stage launches per precision (for "
                         "profilers); copy: a plain device copy of --copy-mib MiB (the "
                         "calibration kernel for the byte counters); batch: the 96-solve "
                         "mix; serve: a prefix of the seeded request trace; vp: the 6D "
                         "Vlasov-Poisson stage (self-consistent field each stage); gauss: "
                         "the workload with Gauss-Legendre quadrature beside collocation; "
                         "mapped: the workload on a deformed configuration mesh")
    ap.add_argument("--map-eps", type=float, default=0.02,
                    help="mapped: deformation amplitude of the configuration mesh")
    ap.add_argument("--stages-map-eps", type=float, default=0.0,
                    help="stages: deform the configuration mesh by this amplitude")
    ap.add_argument("--quadrature", default="gauss_lobatto",
                    choices=["gauss_lobatto", "gauss_legendre"],
                    help="stages: quadrature of the profiled run")
    ap.add_argument("--modes", type=int, default=4, help="vp: Fourier modes per x-dimension")
    ap.add_argument("--copy-mib", type=int, default=4096)
    ap.add_argument("--requests", type=int, default=24, help="serve: trace segment length")
    ap.add_argument("--start", type=int, default=0, help="serve: first request of the segment")
    ap.add_argument("--steps-scale", type=float, default=1.0,
                    help="serve: factor on each request's step count")
    ap.add_argument("--fill-dofs", type=float, default=1e8,
                    help="serve: DoFs a batched step aims to cover")
    ap.add_argument("--load", type=float, default=0.7,
                    help="serve: offered load of the second, stretched-arrival run (0: skip)")
    return ap.parse_args()


def run_stages(case, precision, steps, plan_override, quadrature="gauss_lobatto", map_eps=0.0):
    """Only the fused stage launches (5 per step), for counter collection."""
    import torch

    from paper_2002_08110_amd.solver import Solver
    S = Solver(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
               precision=precision)
    if map_eps:
        S.set_mapping(map_eps)  # before the field: node coordinates follow the mapping
    if case.field == "sine":
        S.set_field_sine(case.amp)
    else:
        S.set_field_constant(case.a)
    if plan_override:
        S.set_plan(**plan_override)
    if quadrature != "gauss_lobatto":
        S.set_quadrature(quadrature)
    S.init_state(case.ic, list(case.ic_params))
    dt = S.stable_dt(case.cfl)
    for _ in range(steps):
        for st in range(5):
            S.rk_stage(st, dt)
    torch.cuda.synchronize()
    print("# ran %d stage launches (%s, plan %s)" % (5 * steps, precision, S.get_plan()),
          file=sys.stderr, flush=True)
    S.close()


def run_copy(mib):
    """The library's plain streaming copy (hd_stream_copy) of a known size,
    three launches: the calibration kernel for the byte counters."""
    import ctypes

    import torch

    from paper_2002_08110_amd import _hd
    lib = _hd.load()
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(3):
        _hd.check(lib.hd_stream_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                     n, stream))
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    print("# hd_stream_copy %d MiB: %.3f ms, %.0f GB/s (read + write)"
          % (mib, ms, 2 * n * 8 / ms / 1e6), file=sys.stderr, flush=True)


def measure(case, precision, steps, warmup, plan_override, quadrature="gauss_lobatto",
            map_eps=0.0, tune=True):
    import torch

    from paper_2002_08110_amd.solver import Solver
    S = Solver(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
               precision=precision)
    if map_eps:
        S.set_mapping(map_eps)  # before the field: node coordinates follow the mapping
    if case.field == "sine":
        S.set_field_sine(case.amp)
    else:
        S.set_field_constant(case.a)
    if quadrature != "gauss_lobatto":
        S.set_quadrature(quadrature)
    S.init_state(case.ic, list(case.ic_params))
    dt = S.stable_dt(case.cfl)
    stream = torch.cuda.current_stream()
    # The launch plan: an explicit override, else the fastest candidate timed
    # on this very mesh (setup, before anything is measured; the collocation
    # kernels only - the sweep kernel has no plan choices).
    if plan_override:
        S.set_plan(**plan_override)
        plan_source = "override"
    elif quadrature == "gauss_lobatto" and not map_eps and tune:
        S.tune_plan(dt)
        plan_source = "tuned on this mesh"
    elif quadrature == "gauss_lobatto" and not map_eps:
        plan_source = "library default"
    else:
        plan_source = "none"
    torch.cuda.synchronize()
    m0, e0 = S.diagnostics()
    S.rk_step(dt, warmup)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t0.record(stream)
    S.rk_step(dt, steps)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = t0.elapsed_time(t1) / steps
    # Per-stage kernel durations: each stage launch bracketed by events on
    # the stream it runs on.
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    reps = max(2, min(steps, 5))
    stage_ms = np.zeros(5)
    for _ in range(reps):
        for st in range(5):
            evs[st].record(stream)
            S.rk_stage(st, dt)
        evs[5].record(stream)
        torch.cuda.synchronize()
        for st in range(5):
            stage_ms[st] += evs[st].elapsed_time(evs[st + 1])
    stage_ms /= reps
    m1, e1 = S.diagnostics()
    psize = 4 if precision == "fp32" else 8
    byts = np.array(stage_bytes(psize), dtype=float) * S.ndofs
    achieved = byts.sum() / (stage_ms.sum() * 1e-3) / 1e9
    res = dict(
        precision=precision, ndofs=S.ndofs, dt=dt, ms_per_step=ms_step, wall_s=wall,
        dof_updates_per_s=S.ndofs * 5 / (ms_step * 1e-3),
        stage_ms=[round(float(x), 4) for x in stage_ms],
        stage_kernel_GBps=achieved, algorithmic_bytes_per_dof=float(np.mean(stage_bytes(psize))),
        plan=S.get_plan(), plan_source=plan_source,
        quadrature=quadrature, mass_drift=(m1 - m0) / abs(m0), energy_ratio=e1 / e0,
    )
    S.close()
    del S
    torch.cuda.empty_cache()
    return res


def _make_solver(case, precision, tuned=False):
    from paper_2002_08110_amd.solver import Solver
    S = Solver(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
               precision=precision)
    if tuned:
        S.apply_tuned_plan()
    if case.field == "sine":
        S.set_field_sine(case.amp)
    else:
        S.set_field_constant(case.a)
    S.init_state(case.ic, list(case.ic_params))
    return S


def run_batch(steps, seq_steps):
    """The seeded mix of 96 uneven solves (6D and lower, degrees 2-5) advanced
    together, FP32 operator mode, the autotuned plan of each (d, k): one
    hipGraph replay per step, per RK stage one work-list launch per group of
    solves sharing a kernel variant and launch shape. Compared with the same
    solves, same plans, stepped one after another (FP32, then FP64). Prints
    one JSON line."""
    import torch

    from paper_2002_08110_amd import workloads as W
    from paper_2002_08110_amd.solver import Batch
    cases = W.batch_mix()
    total = sum(c.ndofs for c in cases)
    res = {"metric": "batched DoF-updates/s per RK stage (96-solve mix)", "unit": "DoF-updates/s",
           "solves": len(cases), "total_dofs": total, "steps": steps}

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3

    solvers = [_make_solver(c, "fp32", tuned=True) for c in cases]
    dts = [S.stable_dt(c.cfl) for S, c in zip(solvers, cases)]
    B = Batch(solvers)
    B.step(dts)
    B.step(dts)  # both solution-buffer parities captured
    t = timed(lambda: [B.step(dts) for _ in range(steps)])
    res["value"] = total * 5 * steps / t
    res["batched_fp32_s"] = t
    nlist, nown = B.launch_counts()
    res["launches_per_step"] = {"work_list": nlist, "single_solve": nown}
    t_seq = timed(lambda: [S.rk_step(dt, seq_steps) for S, dt in zip(solvers, dts)])
    res["sequential_fp32"] = total * 5 * seq_steps / t_seq
    B.close()
    del B, solvers
    torch.cuda.empty_cache()
    solvers = [_make_solver(c, "fp64", tuned=True) for c in cases]
    for S, dt in zip(solvers, dts):
        S.rk_step(dt, 1)
    t64 = timed(lambda: [S.rk_step(dt, seq_steps) for S, dt in zip(solvers, dts)])
    res["sequential_fp64"] = total * 5 * seq_steps / t64
    del solvers
    torch.cuda.empty_cache()
    print("# batch %.3e, sequential fp32 %.3e, sequential fp64 %.3e DoF-updates/s per stage"
          % (res["value"], res["sequential_fp32"], res["sequential_fp64"]), file=sys.stderr,
          flush=True)
    print(json.dumps(res), flush=True)


def run_serve(n_requests, steps_scale, load, fill, quiet=False, start=0):
    """n_requests consecutive requests (from index `start`) of the seeded serving trace (Poisson
    arrivals at 20 req/s; d in {4,5,6}, k in {2..5}, 1e6-2e9 DoFs), each
    request's step count scaled by steps_scale, served with continuous
    batching in FP32 operator mode, and one at a time in FP64 on the same
    arrivals. A second batched run stretches the arrivals to the offered
    load `load` (relative to the measured batched throughput; 0: skip).
    Returns the results; prints them as one JSON line unless quiet."""
    from paper_2002_08110_amd import serve
    from paper_2002_08110_amd import workloads as W
    trace = W.serve_trace()[start:start + n_requests]
    t_first = trace[0].arrival
    for q in trace:
        q.arrival -= t_first  # the segment starts at time 0
    for q in trace:
        q.case.steps = max(1, int(round(q.case.steps * steps_scale)))
    work = float(sum(q.case.ndofs * q.case.steps * 5 for q in trace))
    span = max(q.arrival for q in trace)

    def log(msg):
        if not quiet:
            print("# " + msg, file=sys.stderr, flush=True)

    out = {"metric": "served DoF-updates/s and completion latency (request trace)",
           "requests": len(trace), "first_request": start, "steps_scale": steps_scale,
           "work_dof_updates": work,
           "dofs_max": max(q.case.ndofs for q in trace),
           "dofs_mean": float(np.mean([q.case.ndofs for q in trace]))}
    _, b = serve.serve(trace, precision="fp32", batched=True, log=log, fill_dofs=fill)
    log("batched fp32: %s" % json.dumps(b))
    _, f = serve.serve(trace, precision="fp64", batched=False, log=log)
    log("one-at-a-time fp64: %s" % json.dumps(f))
    rho = work / b["dof_updates_per_s"] / span
    out.update({"batched_fp32": b, "one_at_a_time_fp64": f, "offered_load": rho})
    if load > 0:
        scale = rho / load
        _, c = serve.serve(trace, precision="fp32", batched=True, time_scale=scale, log=log,
                           fill_dofs=fill)
        out["stretched"] = {"offered_load": load, "time_scale": scale, "batched_fp32": c}
    if not quiet:
        print(json.dumps(out), flush=True)
    return out


# One Vlasov-Poisson RK stage of the 6D 8^6-cell k=3 run on one 48-core
# SuperMUC-NG node, read off the weak-scaling figure (Fig. vp:scalingprofile).
PAPER_VP_STAGE_S = 0.955


def run_vp(steps, warmup, precisions, modes):
    """6D Vlasov-Poisson (Sec. 6): Landau-damping initial state on 8^6
    cells, degree 3, x in [0, 4 pi]^3, v in [-6, 6]^3, the field solved from
    the density at every stage. Times the graph-captured RK step, the field
    pre-pass alone (density, transforms, E table) and the stage with the
    field frozen (the advection kernel alone). Prints one JSON line."""
    import torch

    from paper_2002_08110_amd import workloads as W
    from paper_2002_08110_amd.solver import Solver
    case = W.landau_case("6d_vlasov_poisson_8^6_k3", 3, [8] * 6, 3, steps, modes=modes)
    stream = torch.cuda.current_stream()

    def ev_ms(fn, reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"metric": "6D Vlasov-Poisson DoF-updates/s per RK stage (field solved each stage)",
           "unit": "DoF-updates/s", "workload": case.name, "ndofs": case.ndofs, "modes": modes,
           "paper_context": {"stage_s": PAPER_VP_STAGE_S,
                             "hardware": "1 SuperMUC-NG node (48 cores), FP64, multigrid "
                                         "Poisson"},
           "modes_result": {}}
    for prec in precisions:
        S = Solver(3, 3, case.cells, case.lo, case.hi, 3, precision=prec)
        S.apply_tuned_plan()
        S.set_field_vlasov_poisson(modes)
        S.init_state(case.ic, list(case.ic_params))
        torch.cuda.synchronize()
        dt = S.stable_dt(case.cfl)
        m0, _ = S.diagnostics()
        S.rk_step(dt, warmup)
        step_ms = ev_ms(lambda: S.rk_step(dt, steps), 1) / steps
        field_ms = ev_ms(lambda: S.compute_field(), 10)
        # the same stage kernels with the field frozen at the current state
        E = S.get_field()
        m1, _ = S.diagnostics()
        S.set_field_phase_space(E, -1.0)
        S.rk_step(dt, 1)
        adv_ms = ev_ms(lambda: S.rk_step(dt, steps), 1) / steps / 5
        S.close()
        del S
        torch.cuda.empty_cache()
        stage_ms = step_ms / 5
        gbps = 8.0 * case.ndofs / (field_ms * 1e-3) / 1e9
        out["modes_result"][prec] = {
            "dof_updates_per_s": case.ndofs / (stage_ms * 1e-3), "stage_ms": stage_ms,
            "field_ms": field_ms, "advection_stage_ms": adv_ms,
            "field_fraction": field_ms / stage_ms, "dt": dt, "mass_drift": (m1 - m0) / abs(m0),
            "field_pass_GBps": gbps, "speedup_vs_paper_node": PAPER_VP_STAGE_S / (stage_ms * 1e-3)}
        print("# vp %s: stage %.3f ms (field %.3f ms at %.0f GB/s of f, advection %.3f ms)"
              % (prec, stage_ms, field_ms, gbps, adv_ms), file=sys.stderr, flush=True)
    head = out["modes_result"].get("fp64") or next(iter(out["modes_result"].values()))
    out["value"] = head["dof_updates_per_s"]
    out["roofline"] = {"bound": "hbm", "kernel": "Vlasov-Poisson field pre-pass (reads f once)",
                       "achieved": head["field_pass_GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac": head["field_pass_GBps"] / HBM_PEAK_GBPS,
                       "algorithmic_bytes_per_dof": 8.0}
    print(json.dumps(out), flush=True)


def run_gauss(case, steps, warmup, precisions):
    """The workload with Gauss-Legendre quadrature (k+1 Gauss points per
    dimension: basis change to the points and back, the exact mass matrix)
    and, in the same run, with collocation. Prints one JSON line."""
    out = {"metric": "6D k=3 DoF-updates/s per RK stage, Gauss-Legendre quadrature",
           "unit": "DoF-updates/s", "workload": case.name, "modes": {},
           "paper_context": "on average 15% slower than collocation on CPUs while the "
                            "interpolated data stays in cache (Fig. performance:alternatives c)"}
    for prec in precisions:
        g = measure(case, prec, steps, warmup, {}, quadrature="gauss_legendre")
        c = measure(case, prec, steps, warmup, {})
        out["modes"][prec] = {
            "gauss_dof_updates_per_s": g["dof_updates_per_s"], "gauss_stage_ms": g["stage_ms"],
            "gauss_stage_kernel_GBps": g["stage_kernel_GBps"],
            "collocation_dof_updates_per_s": c["dof_updates_per_s"],
            "gauss_over_collocation_time": c["dof_updates_per_s"] / g["dof_updates_per_s"],
            "mass_drift": g["mass_drift"]}
        print("# %s: Gauss %.1f GDoF/s (%.0f GB/s), collocation %.1f GDoF/s, time ratio %.2f"
              % (prec, g["dof_updates_per_s"] / 1e9, g["stage_kernel_GBps"],
                 c["dof_updates_per_s"] / 1e9, out["modes"][prec]["gauss_over_collocation_time"]),
              file=sys.stderr, flush=True)
    head = out["modes"].get("fp64") or next(iter(out["modes"].values()))
    out["value"] = head["gauss_dof_updates_per_s"]
    gb = head["gauss_stage_kernel_GBps"]
    out["roofline"] = {"bound": "alu", "kernel": "stage_k3g_kernel<double>",
                       "achieved_hbm": gb, "peak_hbm": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac_hbm": gb / HBM_PEAK_GBPS, "algorithmic_bytes_per_dof": 28.8}
    print(json.dumps(out), flush=True)


def run_mapped(case, steps, warmup, precisions, eps):
    """The workload on a deformed configuration mesh (hd_set_mapping eps),
    with Gauss-Legendre quadrature (the paper's default discretization) and
    with collocation. Prints one JSON line."""
    n, dx = case.degree + 1, case.dim_x
    nxc = int(np.prod(case.cells[:dx]))
    metric_bytes = nxc * (n ** dx * (dx * dx + 1) + dx * 2 * n ** (dx - 1) * dx) * 8
    full_bytes = case.ndofs * (case.d ** 2 + 1) * 8
    out = {"metric": "6D k=3 DoF-updates/s per RK stage on a deformed configuration mesh",
           "unit": "DoF-updates/s", "workload": case.name, "map_eps": eps,
           "metric_table_bytes": metric_bytes, "per_dof_jacobian_bytes": full_bytes,
           "paper_context": {"value": PAPER_GDOFS_PER_NODE * 1e9, "unit": "DoF-updates/s",
                             "hardware": "1 SuperMUC-NG node, FP64, Gauss quadrature, "
                                         "deformed mesh"},
           "modes": {}}
    for prec in precisions:
        for quad in ("gauss_legendre", "gauss_lobatto"):
            r = measure(case, prec, steps, warmup, {}, quadrature=quad, map_eps=eps)
            out["modes"]["%s_%s" % (prec, quad)] = {
                k: r[k] for k in ("dof_updates_per_s", "ms_per_step", "stage_ms",
                                  "stage_kernel_GBps", "mass_drift")}
            print("# %s %s mapped: %.1f GDoF/s, stage ms %s, mass drift %.1e"
                  % (prec, quad, r["dof_updates_per_s"] / 1e9, r["stage_ms"], r["mass_drift"]),
                  file=sys.stderr, flush=True)
    head = out["modes"].get("fp64_gauss_legendre") or next(iter(out["modes"].values()))
    out["value"] = head["dof_updates_per_s"]
    out["vs_paper_node"] = head["dof_updates_per_s"] / (PAPER_GDOFS_PER_NODE * 1e9)
    gb = head["stage_kernel_GBps"]
    out["roofline"] = {"bound": "alu", "kernel": "stage_k3mg_kernel<double>",
                       "achieved_hbm": gb, "peak_hbm": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac_hbm": gb / HBM_PEAK_GBPS, "algorithmic_bytes_per_dof": 28.8}
    print(json.dumps(out), flush=True)


def profiled_kernel(precision, plan_override, plan):
    """The committed counter profile of the stage kernels (bytes per launch,
    VALU activity), or None if the kernel source changed since it was taken
    or the profiled run used another plan than `plan`."""
    if plan_override:
        return None
    from paper_2002_08110_amd import profiling
    path = os.path.join(ROOT, "profiles", "stage_6d_8x6_k3_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    if data.get("kernel_source_digest") != profiling.kernel_source_digest():
        return None
    # The fields that decide the 6D degree-3 kernel's launch (it ignores the
    # generic kernel's).
    keys = ("kernel", "options", "xcd_remap")
    prof_plan = data.get("plans", {}).get(precision)
    if not prof_plan or any(prof_plan.get(k) != plan.get(k) for k in keys):
        return None
    # The stage launches of one precision use up to three variants (first,
    # general, late-increment stage); their launch-weighted mean is the
    # traffic per stage launch.
    want = "stage_k3_kernel<double" if precision == "fp64" else "stage_k3_kernel<float"
    ks = [d for name, d in data["kernels"].items() if want in name]
    if not ks:
        return None
    n = sum(d["launches"] for d in ks)
    out = {"launches": n, "variants": len(ks),
           "bytes_per_launch": sum(d["launches"] * d["bytes_per_launch"] for d in ks) / n}
    if all("valu_busy_pct" in d for d in ks):
        out["valu_busy_pct"] = sum(d["launches"] * d["valu_busy_pct"] for d in ks) / n
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_problem(case):
    import oracle
    if case.field == "sine":
        return oracle.Problem(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
                              field="phase", sine_amp=case.amp)
    return oracle.Problem(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
                          field="constant", a=case.a)


def oracle_configs(precisions, sample_seconds):
    """The oracle (zero-skipping mode, FP64, OpenMP over cells on the host
    cores) run over each configuration that it finishes in about a minute:
    the 2D configuration (100 steps), the 4D configuration (16^4 cells, 20
    steps) and the 4^6-cell rerun of the 6D configuration (10 steps). Every
    stage (operator plus LSRK update) is timed; the CPU baseline is the
    median over the stages after the first (the warm-up). The final states
    are the references of the GPU runs of the same configurations, in each
    precision: the FP32 operator mode's error per configuration. A sample of
    the 8^6 headline mesh's cells (operator only) is timed as an extra."""
    import oracle
    import torch
    from paper_2002_08110_amd import workloads as W
    out = {"cores": oracle.num_threads(), "cpu_model": cpu_model(), "configs": {}}
    for case in (W.CONFIG_2D, W.CONFIG_4D, W.CONFIG_6D_SMALL):
        P = _oracle_problem(case)
        u = P.init_state(case.ic, list(case.ic_params))
        du = np.zeros_like(u)
        L = np.empty_like(u)
        dt = P.stable_dt(case.cfl)
        times = []
        w0 = time.perf_counter()
        for _ in range(case.steps):
            for st in range(5):
                t = time.perf_counter()
                P.rk_stage(u, du, L, dt, st)
                times.append(time.perf_counter() - t)
        med = float(np.median(times[1:]))
        rec = {"ndofs": P.ndofs, "steps": case.steps, "stages_timed": len(times) - 1,
               "oracle_stage_s_median": med, "oracle_dof_updates_per_s": P.ndofs / med,
               "oracle_run_s": time.perf_counter() - w0}
        e_ref = P.diagnostics(u)[1]
        for prec in precisions:
            S = _make_solver(case, prec)
            S.rk_step(dt, case.steps)
            got = S.get_state()
            S.close()
            rec[prec + "_rel_l2"] = float(np.linalg.norm(got - u) / np.linalg.norm(u))
            rec[prec + "_rel_l2_weighted"] = float(np.sqrt(P.diagnostics(got - u)[1] / e_ref))
        torch.cuda.empty_cache()
        out["configs"][case.name] = rec
        print("# oracle %s: %.3f s per stage (%.3e DoF-updates/s); GPU vs oracle %s"
              % (case.name, med, P.ndofs / med,
                 ", ".join("%s %.2e" % (p, rec[p + "_rel_l2"]) for p in precisions)),
              file=sys.stderr, flush=True)
        del u, du, L
    # Extra: a bounded random sample of the headline mesh's cells.
    case = W.CONFIG_6D
    P = _oracle_problem(case)
    nd = P.n ** P.d
    u = np.zeros(P.ndofs)  # pages the sample never touches stay unallocated
    rng = np.random.default_rng(5)
    sample = rng.choice(P.ncells, size=min(P.ncells, 64), replace=False).astype(np.int64)
    t = time.perf_counter()
    P.apply_cells(u, sample)
    per_cell = (time.perf_counter() - t) / len(sample)
    count = int(min(P.ncells, max(64, sample_seconds / max(per_cell, 1e-9))))
    sample = rng.choice(P.ncells, size=count, replace=False).astype(np.int64)
    t = time.perf_counter()
    P.apply_cells(u, sample)
    el = time.perf_counter() - t
    out["headline_cell_sample"] = {
        "value": count * nd / el, "unit": "DoF/s (operator only)",
        "sample": "%d of %d cells of %s, %.1f s" % (count, P.ncells, case.name, el)}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2002_08110_amd import _hd
    from paper_2002_08110_amd import workloads as W
    if not os.path.exists(_hd.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    case = {"6d": W.CONFIG_6D, "4d": W.CONFIG_4D, "6d_small": W.CONFIG_6D_SMALL,
            "2d": W.CONFIG_2D, "6d_k4": W.CONFIG_6D_K4, "6d_k5": W.CONFIG_6D_K5}[args.config]
    plan = {}
    if args.plan:
        for kv in args.plan.split(","):
            k, v = kv.split("=")
            plan[k] = int(v)
    if args.mode == "copy":
        run_copy(args.copy_mib)
        return
    if args.mode == "batch":
        run_batch(args.steps, max(1, args.steps // 5))
        return
    if args.mode == "serve":
        run_serve(args.requests, args.steps_scale, args.load, args.fill_dofs, start=args.start)
        return
    if args.mode == "vp":
        run_vp(args.steps, args.warmup, args.precisions.split(","), args.modes)
        return
    if args.mode == "gauss":
        run_gauss(case, args.steps, args.warmup, args.precisions.split(","))
        return
    if args.mode == "mapped":
        run_mapped(case, args.steps, args.warmup, args.precisions.split(","), args.map_eps)
        return
    if args.mode == "stages":
        for prec in args.precisions.split(","):
            run_stages(case, prec, args.steps, plan, args.quadrature, args.stages_map_eps)
        return
    results = {}
    for prec in args.precisions.split(","):
        results[prec] = measure(case, prec, args.steps, args.warmup, plan, tune=not args.no_tune)
        print("# %s: %.1f GDoF/s per stage, stage kernels %.0f GB/s, stages ms %s, plan %s"
              % (prec, results[prec]["dof_updates_per_s"] / 1e9,
                 results[prec]["stage_kernel_GBps"], results[prec]["stage_ms"],
                 results[prec]["plan"]), file=sys.stderr, flush=True)
    head = results.get("fp64") or next(iter(results.values()))
    achieved = head["stage_kernel_GBps"]
    prof = (profiled_kernel(head["precision"], plan, head["plan"]) if args.config == "6d"
            else None)
    line = {
        "metric": "6D k=3 DoF-updates/s per RK stage, FP64 vs FP32, % HBM peak; p99 latency",
        "value": head["dof_updates_per_s"],
        "unit": "DoF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head["precision"] == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": case.name, "cells": case.cells, "degree": case.degree,
                   "ndofs": head["ndofs"], "field": "a=(v, 0.1 sin(2 pi x))",
                   "initial_state": "(1+0.01 cos(2 pi x1)) Maxwellian(v)",
                   "rk": "LSRK45 (5 fused stages per step)", "cfl": case.cfl},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": prof["bytes_per_launch"] if prof else None,
                     "valu_busy_pct": prof.get("valu_busy_pct") if prof else None,
                     "kernel": ("stage_k3_kernel (6D degree-3 fused LSRK stage)"
                                if head["plan"].get("kernel") == 1
                                else "stage_kernel (fused LSRK stage)"),
                     "algorithmic_bytes_per_dof": head["algorithmic_bytes_per_dof"]},
        "pct_hbm_peak": 100.0 * achieved / HBM_PEAK_GBPS,
        "modes": {p: {k: r[k] for k in ("dof_updates_per_s", "ms_per_step", "stage_ms",
                                        "stage_kernel_GBps", "algorithmic_bytes_per_dof",
                                        "plan", "mass_drift", "energy_ratio")}
                  for p, r in results.items()},
        "paper_context": {"value": PAPER_GDOFS_PER_NODE * 1e9, "unit": "DoF-updates/s",
                          "hardware": "1 SuperMUC-NG node, 2x24-core Xeon 8174, FP64, "
                                      "Gauss quadrature, deformed mesh"},
    }
    if not args.no_serve and args.config == "6d":
        # The metric's latency part: the serving trace (batched FP32 against
        # one-at-a-time FP64), without the stretched-arrival run.
        sv = run_serve(args.requests, args.steps_scale, 0.0, args.fill_dofs, quiet=True)
        b, f = sv["batched_fp32"], sv["one_at_a_time_fp64"]
        line["serving"] = {
            "requests": sv["requests"], "offered_load": sv["offered_load"],
            "latency_p99_s": b["latency_p99_s"], "latency_p50_s": b["latency_p50_s"],
            "dof_updates_per_s": b["dof_updates_per_s"], "throughput_req_s": b["throughput_req_s"],
            "precision": "fp32 operator, batched",
            "one_at_a_time_fp64": {k: f[k] for k in ("latency_p99_s", "latency_p50_s",
                                                     "dof_updates_per_s", "throughput_req_s")}}
        print("# serving: p50 %.3f s, p99 %.3f s (one at a time FP64: %.3f / %.3f s)"
              % (b["latency_p50_s"], b["latency_p99_s"], f["latency_p50_s"], f["latency_p99_s"]),
              file=sys.stderr, flush=True)
        # A later segment of the same trace holding three requests of 1.2e9-1.5e9
        # DoFs (requests 24-47, step counts scaled by 1/4 to keep the run short).
        sv = run_serve(24, 0.25, 0.0, args.fill_dofs, quiet=True, start=24)
        b, f = sv["batched_fp32"], sv["one_at_a_time_fp64"]
        line["serving_large"] = {
            "requests": sv["requests"], "first_request": 24, "steps_scale": 0.25,
            "dofs_max": sv["dofs_max"], "offered_load": sv["offered_load"],
            "latency_p99_s": b["latency_p99_s"], "latency_p50_s": b["latency_p50_s"],
            "dof_updates_per_s": b["dof_updates_per_s"], "throughput_req_s": b["throughput_req_s"],
            "peak_bytes": b["peak_bytes"], "precision": "fp32 operator, batched",
            "one_at_a_time_fp64": {k: f[k] for k in ("latency_p99_s", "latency_p50_s",
                                                     "dof_updates_per_s", "throughput_req_s")}}
        print("# serving (segment with 1.5e9-DoF requests): p50 %.3f s, p99 %.3f s (one at a time "
              "FP64: %.3f / %.3f s)" % (b["latency_p50_s"], b["latency_p99_s"], f["latency_p50_s"],
                                         f["latency_p99_s"]), file=sys.stderr, flush=True)
    if not args.no_cpu_baseline and args.config == "6d":
        orc = oracle_configs(list(results), args.cpu_seconds)
        six = orc["configs"][W.CONFIG_6D_SMALL.name]
        line["cpu_baseline"] = {
            "value": six["oracle_dof_updates_per_s"], "unit": "DoF-updates/s",
            "cores": orc["cores"], "cpu_model": orc["cpu_model"], "kind": "oracle",
            "sample": "the 6D k=3 phase-space workload at 4^6 cells (its reduced rerun, %d DoFs): "
                      "median of %d full LSRK stages (operator + update) after one warm-up stage"
                      % (six["ndofs"], six["stages_timed"]),
            "per_config": {name: {k: r[k] for k in ("ndofs", "oracle_stage_s_median",
                                                    "oracle_dof_updates_per_s", "stages_timed")}
                           for name, r in orc["configs"].items()},
            "headline_cell_sample": orc["headline_cell_sample"]}
        line["fp32_error_vs_fp64_oracle"] = {
            name: {k: r[k] for k in r if k.endswith("rel_l2") or k.endswith("rel_l2_weighted")}
            | {"steps": r["steps"]} for name, r in orc["configs"].items()}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
