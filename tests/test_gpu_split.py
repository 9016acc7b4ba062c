"""GPU parity of the dimension-split stage passes (plan kernel 2: pass x over
rows of x-nodes, pass v over column blocks with the RK update) against the
CPU oracle, through the C ABI.

Meshes hold one, two and three cells along different dimensions (self
neighbours and distinct left and right neighbours); the pass-x tiles of
degree 4 span two cells and the column blocks end ragged. Bars: FP64
relative L2 and max-norm differences <= 1e-12; the FP32 operator mode within
2e-6 (operator) and 1e-5 (RK steps) and reported.
"""
import json

import numpy as np
import pytest

from gpu_helpers import (TOL_FP64, gpu_solver, oracle_problem, rel_l2, rel_max, sample_cells,
                         split_plans, stages_sampled, x_table_size)
from paper_2002_08110_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(d, k, field):
    dx, dv = 3, d - 3
    cells = {(6, 4): [3, 2, 1, 1, 3, 2], (6, 5): [3, 1, 2, 1, 2, 3],
             (5, 4): [2, 3, 3, 3, 2], (5, 5): [3, 2, 3, 1, 3]}[(d, k)]
    if field == "constant":
        rng = np.random.default_rng(70 + 10 * d + k)
        a = list(rng.uniform(-1, 1, d))
        a[1] = 0.0  # a zero component: no flux through those faces
        lo = list(rng.uniform(-1, 0, d))
        hi = [l + w for l, w in zip(lo, rng.uniform(0.5, 2, d))]
        return W.Case("c", dx, dv, cells, lo, hi, k, "constant", a=a, steps=2)
    if field == "sine":
        return W.Case("s", dx, dv, cells, [0.0] * dx + [-6.0] * dv, [1.0] * dx + [6.0] * dv,
                      k, "sine", amp=0.3, steps=2)
    return W.Case("t", dx, dv, cells, [0.0] * dx + [-5.0] * dv, [1.0] * dx + [3.5] * dv, k,
                  "table", steps=2)


PARAMS = [(d, k, f) for d in (5, 6) for k in (4, 5)
          for f in (("constant", "sine", "table") if d == 6 else ("constant",))]


@pytest.mark.parametrize("d,k,field", PARAMS)
def test_split_apply_matches_oracle(d, k, field):
    case = _case(d, k, field)
    E = W.random_field_table(x_table_size(case), seed=7) if field == "table" else None
    sign = -1.0 if field == "table" else 1.0
    P = oracle_problem(case, E=E, sign=sign)
    u = W.random_state(P.ndofs, seed=d * 100 + k)
    ref = P.apply(u)
    ut = torch.from_numpy(u).cuda()
    S = gpu_solver(case, "fp64", E=E, sign=sign)
    S32 = gpu_solver(case, "fp32", E=E, sign=sign)
    outs = []
    for plan in split_plans(case):
        S.set_plan(**plan)
        out = S.apply(ut).cpu().numpy()
        assert rel_l2(out, ref) <= TOL_FP64, plan
        assert rel_max(out, ref) <= TOL_FP64, plan
        outs.append(out)
        S32.set_plan(**plan)
        o32 = S32.apply(ut)
        assert o32.dtype == torch.float32
        e32 = rel_l2(o32.double().cpu().numpy(), ref)
        assert e32 < 2e-6, (plan, e32)
    # No output depends on which workgroup computed it or on the stores.
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    S.close()
    S32.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("d,k,field", [(6, 4, "sine"), (6, 5, "table"), (5, 4, "constant"),
                                       (5, 5, "constant")])
def test_split_rk_steps_match_oracle(precision, d, k, field):
    case = _case(d, k, field)
    E = W.random_field_table(x_table_size(case), seed=8) if field == "table" else None
    sign = -1.0 if field == "table" else 1.0
    P = oracle_problem(case, E=E, sign=sign)
    S = gpu_solver(case, precision, E=E, sign=sign)
    dt = S.stable_dt(0.2)
    u0 = W.random_state(P.ndofs, seed=17)
    ref = P.rk_steps(u0, dt, case.steps)
    tol = TOL_FP64 if precision == "fp64" else 1e-5
    outs = []
    for plan in split_plans(case):
        S.set_plan(**plan)
        S.set_state(u0)
        S.rk_step(dt, case.steps)
        got = S.get_state()
        err = rel_l2(got, ref)
        assert err <= tol, (plan, err)
        outs.append(got)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    print(json.dumps({"split_rk": [d, k, field, precision], "rel_l2": err}))
    S.close()


@pytest.mark.parametrize("d,k", [(6, 4), (5, 5)])
def test_split_agrees_with_the_fused_kernel(d, k):
    # The same operator as the generic fused kernel, summed in the same
    # dimension order: agreement to rounding on an RK step.
    case = _case(d, k, "sine" if d == 6 else "constant")
    S = gpu_solver(case, "fp64")
    u0 = W.random_state(S.ndofs, seed=23)
    dt = S.stable_dt(0.2)
    S.set_state(u0)
    S.rk_step(dt, 1)
    fused = S.get_state()
    S.set_plan(**split_plans(case)[1])
    S.set_state(u0)
    S.rk_step(dt, 1)
    assert rel_max(S.get_state(), fused) <= 1e-14
    S.close()


def test_split_vlasov_poisson_matches_oracle():
    # The self-consistent field recomputed before every stage from the
    # stage's input (ragged x-boxes not at 0, asymmetric velocity box).
    case = W.Case("vp", 3, 3, [3, 1, 2, 2, 1, 1], [0.3, -1.0, 0.5, -5.0, -4.5, -6.0],
                  [0.3 + 2 * np.pi, 2.0, 1.7, 4.0, 5.5, 3.0], 4, "vlasov_poisson", steps=2,
                  modes=2)
    V = oracle_problem(case)
    u0 = np.abs(W.random_state(case.ndofs, 29)) + 0.5
    dt = V.stable_dt(u0, 0.2)
    ref = V.rk_steps(u0, dt, case.steps)
    for precision, tol in (("fp64", TOL_FP64), ("fp32", 1e-5)):
        S = gpu_solver(case, precision, plan=split_plans(case)[1])
        S.set_state(u0)
        S.rk_step(dt, case.steps)
        err = rel_l2(S.get_state(), ref)
        assert err <= tol, (precision, err)
        S.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_split_at_6d_k5_full_size_stages_sampled(precision):
    # The 6D 4^6-cell degree-5 mesh (1.9e8 DoFs), sine field, stage by stage
    # on sampled cells (corners with wrap-around neighbours among them).
    case = W.CONFIG_6D_K5
    S = gpu_solver(case, precision, plan=split_plans(case)[3])
    g = torch.Generator(device="cuda")
    g.manual_seed(41)
    S.set_state(torch.randn(S.ndofs, dtype=torch.float64, device="cuda", generator=g))
    dt = S.stable_dt(0.2)
    cells = sample_cells(int(np.prod(case.cells)), 3, count=12)
    P = oracle_problem(case)
    worst = stages_sampled(S, lambda host: P, cells, dt,
                           TOL_FP64 if precision == "fp64" else 5e-6)
    print(json.dumps({"split_full_size": precision, "worst_stage_rel_l2": worst}))
    S.close()


def test_split_plan_is_rejected_where_not_compiled():
    # Degree 3, or Gauss-Legendre quadrature: no dimension-split passes.
    from paper_2002_08110_amd import _hd
    S = gpu_solver(_case(5, 4, "constant"), "fp64")
    S.set_plan(kernel=2, xcd_remap=1, options=0)
    S.set_quadrature("gauss_legendre")  # the sweep kernel takes over
    with pytest.raises(_hd.HDError):
        S.set_plan(kernel=2, xcd_remap=0, options=0)
    S.close()
    case = W.Case("k3", 3, 3, [2, 1, 1, 1, 1, 2], [0.0] * 6, [1.0] * 6, 3, "constant",
                  a=[0.5] * 6)
    S = gpu_solver(case, "fp64")
    with pytest.raises(_hd.HDError):
        S.set_plan(kernel=2, xcd_remap=1, options=0)
    S.close()


def test_batch_with_split_plan_solves_equals_alone():
    # Split-plan solves take their own two launches per stage inside the
    # batch's step graph; beside work-list solves they step as alone.
    from paper_2002_08110_amd.solver import Batch
    cases = [(_case(6, 5, "sine"), "fp64", split_plans(_case(6, 5, "sine"))[1]),
             (_case(5, 4, "constant"), "fp32", split_plans(_case(5, 4, "constant"))[3]),
             (W.phase_space_case("k3", 3, 3, [2, 1, 2, 1, 1, 2], 3, 2), "fp64", None)]
    alone, batched = [], []
    for i, (case, prec, plan) in enumerate(cases):
        u0 = W.random_state(case.ndofs, 60 + i)
        for lst in (alone, batched):
            S = gpu_solver(case, prec, plan=plan)
            S.set_state(u0)
            lst.append(S)
    dts = [S.stable_dt(0.2) for S in alone]
    for S, dt in zip(alone, dts):
        S.rk_step(dt, 2)
    B = Batch(batched)
    B.step(dts)
    B.step(dts)
    torch.cuda.synchronize()
    assert B.launch_counts()[1] >= 10  # the split-plan solves' own stages
    for a, b in zip(alone, batched):
        assert np.array_equal(a.get_state(), b.get_state())
    B.close()
    for S in alone + batched:
        S.close()
