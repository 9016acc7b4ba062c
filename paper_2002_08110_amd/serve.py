"""Request serving with continuous batching.

Requests (advection solves: mesh, degree, field, initial state, number of
LSRK steps) arrive over time. The server admits them in arrival order as
soon as their device footprint (hd_required_bytes: two FP64 solution
buffers, the stage increment and the field table) fits the memory budget,
keeps their state resident on the GPU, and advances admitted requests one
LSRK step per iteration with one batched hipGraph replay (hd_batch_step).
Each step takes resident requests until their DoFs fill the GPU (fill_dofs,
at least one request), shortest remaining work first (order="shortest") or
in arrival order (order="arrival"): small requests share steps and overlap
on the device instead of queueing behind a large one, whose steps cost the
same whether or not it shares them. A request that arrives while others run
joins at the next step boundary; a finished request frees its memory at
once.
The loop is host bookkeeping only: every stage runs in the library's
kernels.

A request that can never run is rejected with a status and the server
goes on: its footprint exceeds the whole budget (status "rejected", code
HD_ERR_OOM), or the library refuses it at set-up (code: the library's
status). Every other request ends with status "done".

Times are wall-clock seconds from the start of the run; latency is
completion minus arrival, service time completion minus admission.
Latency statistics cover the completed requests.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

from . import _hd
from .solver import Batch, Solver



@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = float("nan")
    completed: float = float("nan")
    ndofs: int = 0
    steps: int = 0
    footprint: int = 0
    mass: float = float("nan")
    energy: float = float("nan")
    state: np.ndarray | None = None
    status: str = "pending"   # "done" or "rejected"
    code: int = 0             # hd_status of a rejection (0 otherwise)
    reason: str = ""

    @property
    def latency(self):
        return self.completed - self.arrival

    @property
    def service(self):
        return self.completed - self.admitted


def make_solver(case, precision, tuned=True, bind=True):
    s = Solver(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
               precision=precision, bind=bind)
    if tuned:
        s.apply_tuned_plan()
    return s


def setup(s, case):
    if case.field == "sine":
        s.set_field_sine(case.amp)
    elif case.field == "vlasov_poisson":
        s.set_field_vlasov_poisson(case.modes)
    else:
        s.set_field_constant(case.a)
    s.init_state(case.ic, list(case.ic_params))
    return s.stable_dt(case.cfl)


def footprint(case, precision):
    s = make_solver(case, precision, tuned=False, bind=False)
    b = s.device_bytes
    s.close()
    return b


def default_budget(reserve=16 << 30):
    free, total = torch.cuda.mem_get_info()
    return max(0, total - reserve)


class _Running:
    __slots__ = ("req", "solver", "dt", "left", "res")

    def __init__(self, req, solver, dt, res):
        self.req, self.solver, self.dt, self.res = req, solver, dt, res
        self.left = req.case.steps


def serve(requests, precision="fp32", budget=None, batched=True, keep_states=False,
          time_scale=1.0, tuned=True, log=None, fill_dofs=1e8, order="shortest"):
    """Run `requests` (workloads.Request, arrival-ordered) through the
    server. batched=False serves one request at a time (the baseline).
    time_scale multiplies the arrival times; fill_dofs is the DoF count a
    batched step aims to cover (None: every resident request steps each
    iteration); order picks which resident requests fill a step. Returns
    (results, stats)."""
    if order not in ("shortest", "arrival"):
        raise ValueError("order must be 'shortest' or 'arrival'")
    budget = default_budget() if budget is None else int(budget)
    reqs = sorted(requests, key=lambda r: r.arrival)
    results = {r.rid: Result(r.rid, r.arrival * time_scale, ndofs=r.case.ndofs,
                             steps=r.case.steps, footprint=footprint(r.case, precision))
               for r in reqs}
    waiting, running = [], []
    nxt = 0
    used = 0
    peak = 0
    batch, members = None, None
    steps_run = 0
    t_step = None  # wall time of the last batched step
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def now():
        return time.perf_counter() - t0

    def reject(r, code, reason):
        res = results[r.rid]
        res.status, res.code, res.reason = "rejected", code, reason
        res.completed = now()
        if log:
            log("request %d rejected (status %d): %s" % (r.rid, code, reason))

    while nxt < len(reqs) or waiting or running:
        t = now()
        while nxt < len(reqs) and reqs[nxt].arrival * time_scale <= t:
            r = reqs[nxt]
            nxt += 1
            if results[r.rid].footprint > budget:
                # It would never fit: reject at arrival, keep serving.
                reject(r, _hd.HD_ERR_OOM, "needs %d bytes, more than the budget %d"
                       % (results[r.rid].footprint, budget))
                continue
            waiting.append(r)
        # Admission in arrival order while the footprint fits.
        cap = None if batched else 1
        while waiting and (cap is None or len(running) < cap):
            r = waiting[0]
            fp = results[r.rid].footprint
            if used + fp > budget:
                break
            waiting.pop(0)
            try:
                s = make_solver(r.case, precision, tuned=tuned)
                dt = setup(s, r.case)
            except _hd.HDError as e:
                reject(r, e.status, str(e))
                continue
            used += fp
            peak = max(peak, used)
            results[r.rid].admitted = now()
            running.append(_Running(r, s, dt, results[r.rid]))
        if not running:
            if nxt < len(reqs):
                time.sleep(max(0.0, reqs[nxt].arrival * time_scale - now()))
            continue
        if batched:
            ids = [id(x.solver) for x in running]
            if members != ids:
                if batch is not None:
                    batch.close()
                batch = Batch([x.solver for x in running])
                members = ids
            # The stepping set: by the policy's order until the GPU is filled.
            pick = list(range(len(running)))
            if order == "shortest":
                pick.sort(key=lambda i: (running[i].res.ndofs * running[i].left, i))
            act, tot = [0] * len(running), 0
            for i in pick:
                if tot > 0 and fill_dofs is not None and tot >= fill_dofs:
                    break
                act[i] = 1
                tot += running[i].res.ndofs
            stepping = [x for x, a in zip(running, act) if a]
            # Several steps per check when no request finishes and none can
            # arrive before they are done: fewer host round trips.
            k = min(x.left for x in stepping)
            if waiting:
                k = 1
            elif nxt < len(reqs):
                gap = reqs[nxt].arrival * time_scale - now()
                k = min(k, int(gap / t_step) if t_step else 1)
            k = max(1, min(k, 64))
            ts = time.perf_counter()
            dts = [x.dt for x in running]
            for _ in range(k):
                batch.step(dts, active=act)
            for x in stepping:
                x.left -= k
            steps_run += k
        else:
            x = running[0]
            x.solver.rk_step(x.dt, x.left)
            x.left = 0
            steps_run += x.req.case.steps
        torch.cuda.synchronize()
        if batched:
            t_step = (time.perf_counter() - ts) / k
        done = [x for x in running if x.left == 0]
        if done:
            tc = now()
            for x in done:
                x.res.completed = tc
                x.res.status = "done"
                x.res.mass, x.res.energy = x.solver.diagnostics()
                if keep_states:
                    x.res.state = x.solver.get_state()
                x.solver.close()
                x.solver = None
                used -= x.res.footprint
                if log:
                    log("request %d done: %d DoFs x %d steps, latency %.3f s"
                        % (x.res.rid, x.res.ndofs, x.res.steps, x.res.latency))
            running = [x for x in running if x.left > 0]
            torch.cuda.empty_cache()
    if batch is not None:
        batch.close()
    makespan = now()
    res = [results[r.rid] for r in reqs]
    ok = [r for r in res if r.status == "done"]
    lat = np.array([r.latency for r in ok]) if ok else np.array([np.nan])
    svc = np.array([r.service for r in ok]) if ok else np.array([np.nan])
    work = float(sum(r.ndofs * r.steps * 5 for r in ok))
    stats = {
        "requests": len(res), "completed": len(ok), "rejected": len(res) - len(ok),
        "makespan_s": makespan,
        "throughput_req_s": len(ok) / makespan,
        "dof_updates_per_s": work / makespan,
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "service_p50_s": float(np.percentile(svc, 50)), "service_p99_s": float(np.percentile(svc, 99)),
        "peak_bytes": peak, "budget_bytes": budget, "batched": batched, "precision": precision,
        "fill_dofs": fill_dofs if batched else None, "order": order if batched else "arrival",
    }
    return res, stats
