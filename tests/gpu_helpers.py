"""Shared setup for the GPU parity tests: build the oracle problem and the
HIP solver for the same seeded workload. The two sides share only the
workload description (paper_2002_08110_amd.workloads) and the seeded input
arrays; each computes its own nodes, field tables and operator.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2002_08110_amd import workloads as W

# FP64 parity bar: relative L2 difference to the oracle (and the same bound on
# the max-norm relative to the reference's max) of at most 1e-12.
TOL_FP64 = 1e-12


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def rel_max(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def oracle_problem(case: W.Case, E=None, sign=1.0):
    if case.field == "constant":
        return oracle.Problem(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
                              field="constant", a=case.a)
    if case.field == "sine":
        return oracle.Problem(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
                              field="phase", sine_amp=case.amp, sign=sign)
    if case.field == "table":
        return oracle.Problem(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
                              field="phase", E=E, sign=sign)
    if case.field == "vlasov_poisson":
        return oracle.VlasovPoisson(case.dim_x, case.dim_v, case.cells, case.lo, case.hi,
                                    case.degree, case.modes)
    raise ValueError(case.field)


def gpu_solver(case: W.Case, precision="fp64", E=None, sign=1.0, plan=None):
    from paper_2002_08110_amd.solver import Solver
    s = Solver(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
               precision=precision)
    if case.field == "constant":
        s.set_field_constant(case.a)
    elif case.field == "sine":
        s.set_field_sine(case.amp, sign)
    elif case.field == "table":
        s.set_field_phase_space(E, sign)
    elif case.field == "vlasov_poisson":
        s.set_field_vlasov_poisson(case.modes)
    if plan:
        s.set_plan(**plan)
    return s


def x_table_size(case: W.Case):
    return int(np.prod(case.cells[: case.dim_x])) * (case.degree + 1) ** case.dim_x * case.dim_x


def all_plans(case: W.Case, precision="fp64"):
    """Every valid launch plan of the stage kernel for this case (the generic
    kernel's streaming option alternates over the plans)."""
    n = case.degree + 1
    d = case.d
    psize = 4 if precision == "fp32" else 8
    nd = n ** d
    plans = []
    for rd in (1, 2):
        if rd > case.dim_v:
            continue
        for sd in (1, 2):  # slab variants (degree >= 4, d >= 5)
            Ts = n ** (d - rd - sd)
            if n < 5 or d < 5 or rd + sd > case.dim_v or Ts > 1024:
                continue
            ub = n ** (d - sd) * psize
            for cpw in ([1] if Ts > 256 else sorted({1, max(1, 256 // Ts)})):
                if cpw * ub <= 160 * 1024:
                    plans.append(dict(lds=1, cells_per_wg=cpw, reg_dims=rd, split_dims=sd,
                                      xcd_remap=cpw % 2, wg_size=256, kernel=0))
        for sd in (0, 1, 2):  # looped-pencil variants (degree >= 4, d >= 5)
            nf = d - rd - sd
            if (n < 5 or d < 5 or rd + sd > case.dim_v or nf - 1 < case.dim_x
                    or n ** (nf - 1) > 1024 or n ** (d - sd) * psize > 160 * 1024):
                continue
            plans.append(dict(lds=1, cells_per_wg=1, reg_dims=rd, split_dims=sd, loop_dims=1,
                              xcd_remap=sd % 2, wg_size=256, kernel=0))
        T = n ** (d - rd)
        for xcd in (0, 1):
            for wg in (64, 256):
                plans.append(dict(lds=0, wg_size=wg, reg_dims=rd, xcd_remap=xcd, cells_per_wg=1,
                                  kernel=0, split_dims=0))
            if T <= 1024 and nd * psize <= 160 * 1024:
                cpws = [1] if T > 256 else sorted({1, max(1, 256 // T)})
                for cpw in cpws:
                    if cpw * nd * psize <= 160 * 1024:
                        plans.append(dict(lds=1, cells_per_wg=cpw, reg_dims=rd, xcd_remap=xcd,
                                          wg_size=256, kernel=0, split_dims=0))
    for i, p in enumerate(plans):
        p["options"] = i % 2
    if k3_eligible(case):
        for xcd in (0, 1):
            for opt in range(4):
                plans.append(dict(kernel=1, xcd_remap=xcd, reg_dims=2, options=opt, split_dims=0))
    full = dict(lds=0, cells_per_wg=1, wg_size=256, xcd_remap=0, reg_dims=1, kernel=0, options=0,
                split_dims=0, loop_dims=0)
    return [dict(full, **p) for p in plans]


def split_eligible(case: W.Case):
    """The dimension-split passes (plan kernel 2): 6D (3 x + 3 v) or 5D
    (3 x + 2 v) at degree 4 or 5, collocation on Cartesian cells."""
    return case.dim_x == 3 and case.dim_v in (2, 3) and case.degree in (4, 5)


def split_plans(case: W.Case):
    """Every launch plan of the dimension-split passes: both cell orders,
    with and without streaming stores."""
    if not split_eligible(case):
        return []
    full = dict(lds=0, cells_per_wg=1, wg_size=256, xcd_remap=0, reg_dims=1, kernel=2, options=0,
                split_dims=0, loop_dims=0)
    return [dict(full, xcd_remap=x, options=o) for x in (0, 1) for o in (0, 1)]


def k3_eligible(case: W.Case):
    """The specialised kernel: 6D (3 x + 3 v), degree 3, < 2^31 DoFs."""
    return case.dim_x == 3 and case.dim_v == 3 and case.degree == 3 and case.ndofs < 2 ** 31


def sample_cells(ncells, seed, count=24):
    """The corners of the periodic box (wrap-around neighbours), the middle
    cell and a seeded random sample."""
    rng = np.random.default_rng(seed)
    fixed = [0, ncells - 1, ncells // 2]
    return np.unique(np.concatenate([fixed, rng.integers(0, ncells, count)])).astype(np.int64)


def stages_sampled(S, problem_of, cells, dt, tol, mode=1):
    """One RK step of the GPU solver S, stage by stage as its launches run
    them, checked on the sampled cells: the increment is local to a cell, so
    before each stage the oracle problem of the current state
    (problem_of(host_state)) evaluates L on the samples from the full device
    state, and du and u are followed there (Sec. 5.4 update). Returns the
    largest relative L2 error over the stages."""
    import torch
    A, B, _ = oracle.lsrk45_coefficients()
    nd = (S.k + 1) ** S.d
    idx = (cells[:, None] * nd + np.arange(nd)[None, :]).reshape(-1)
    idx_t = torch.from_numpy(idx).to(S.device)
    host = np.empty(S.ndofs)
    du = np.zeros(len(idx))
    worst = 0.0
    for st in range(5):
        host[:] = S.state_tensor().cpu().numpy()
        us = host[idx]
        L = problem_of(host).apply_cells(host, cells, mode=mode)
        du = A[st] * du + dt * L
        S.rk_stage(st, dt)
        got = S.state_tensor()[idx_t].cpu().numpy()
        err = rel_l2(got - us, B[st] * du)
        assert err <= tol, (st, err)
        worst = max(worst, err)
    return worst
