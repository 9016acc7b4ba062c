"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bar: FP64 relative L2 (and max-norm relative to the reference maximum)
difference <= 1e-12 against the oracle on the same seeded inputs; plans
(LDS/global, register dims, cells per workgroup, XCD remap) must agree
bitwise with each other; FP32 errors are bounded and reported.
"""
import numpy as np
import pytest

from gpu_helpers import (TOL_FP64, all_plans, gpu_solver, oracle_problem, rel_l2, rel_max,
                         x_table_size)
from paper_2002_08110_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MESHES = {
    # d: (cells for k <= 3, cells for k >= 4) - ragged, non-power-of-two,
    # with single-cell (self-neighbour) dimensions.
    2: ([5, 3], [3, 2]),
    3: ([3, 2, 5], [2, 3, 1]),
    4: ([3, 2, 1, 3], [2, 1, 2, 1]),
    5: ([2, 3, 1, 2, 3], [1, 2, 1, 1, 2]),
    6: ([2, 1, 3, 1, 2, 2], [1, 2, 1, 1, 2, 1]),
}


def small_case(d, k, field, seed=0):
    dx, dv = W.SPLITS[d]
    cells = MESHES[d][0 if k <= 3 else 1]
    rng = np.random.default_rng(1000 + 10 * d + k)
    if field == "constant":
        a = list(rng.uniform(-1, 1, d))
        a[d - 1] = 0.0  # a zero component: no flux through those faces
        lo = list(rng.uniform(-1, 0, d))
        hi = [l + w for l, w in zip(lo, rng.uniform(0.5, 2, d))]
        return W.Case("c", dx, dv, cells, lo, hi, k, "constant", a=a)
    if field == "sine":
        return W.Case("s", dx, dv, cells, [0.0] * dx + [-6.0] * dv, [1.0] * dx + [6.0] * dv,
                      k, "sine", amp=0.3)
    # a random prescribed E table on an asymmetric velocity box: mixed signs
    # of a inside cells
    return W.Case("t", dx, dv, cells, [0.0] * dx + [-5.0] * dv, [1.0] * dx + [3.5] * dv, k,
                  "table")


def _phase_ok(d):
    dx, dv = W.SPLITS[d]
    return dx == dv


PARAMS = [(d, k, f) for d in (2, 3, 4, 5, 6) for k in (1, 2, 3, 4, 5)
          for f in ("constant", "sine", "table") if f == "constant" or _phase_ok(d)]


@pytest.mark.parametrize("d,k,field", PARAMS)
def test_apply_matches_oracle_fp64(d, k, field):
    case = small_case(d, k, field)
    E = W.random_field_table(x_table_size(case), seed=7) if field == "table" else None
    P = oracle_problem(case, E=E, sign=-1.0 if field == "table" else 1.0)
    u = W.random_state(P.ndofs, seed=d * 100 + k)
    ref = P.apply(u)
    S = gpu_solver(case, "fp64", E=E, sign=-1.0 if field == "table" else 1.0)
    ut = torch.from_numpy(u).cuda()
    outs = {}
    for plan in all_plans(case):
        S.set_plan(**plan)
        out = S.apply(ut).cpu().numpy()
        assert rel_l2(out, ref) <= TOL_FP64, plan
        assert rel_max(out, ref) <= TOL_FP64, plan
        outs.setdefault((plan.get("kernel", 0), plan["reg_dims"], plan.get("loop_dims", 0)),
                        []).append(out)
    # Plans of one kernel with the same register dims (and looped-pencil
    # mode, whose loop the compiler contracts into FMAs differently) evaluate
    # each output with the same arithmetic whatever the schedule (LDS or
    # global reads, slabs, cells per workgroup, XCD remap, streaming), so
    # they agree bitwise; no output depends on which workgroup computed it.
    for group in outs.values():
        for o in group[1:]:
            assert np.array_equal(o, group[0])


@pytest.mark.parametrize("d,k", [(2, 3), (3, 2), (4, 3), (5, 2), (6, 3), (6, 5)])
def test_apply_fp32_error_is_small(d, k):
    case = small_case(d, k, "sine" if _phase_ok(d) else "constant")
    P = oracle_problem(case)
    u = W.random_state(P.ndofs, seed=5)
    ref = P.apply(u)
    S = gpu_solver(case, "fp32")
    ut = torch.from_numpy(u).cuda()
    for plan in all_plans(case, "fp32"):
        S.set_plan(**plan)
        out = S.apply(ut)
        assert out.dtype == torch.float32
        assert rel_l2(out.double().cpu().numpy(), ref) < 2e-6, plan


def test_config_2d_rk_matches_oracle_and_exact_solution():
    case = W.CONFIG_2D
    P = oracle_problem(case)
    S = gpu_solver(case, "fp64")
    dt = S.stable_dt(case.cfl)
    assert abs(dt - P.stable_dt(case.cfl)) <= 1e-15 * dt
    S.init_state(case.ic)
    u0 = P.init_state(case.ic)
    assert rel_max(S.get_state(), u0) <= 1e-14
    S.rk_step(dt, case.steps)
    ref = P.rk_steps(u0, dt, case.steps)
    got = S.get_state()
    assert rel_l2(got, ref) <= TOL_FP64
    X = P.node_coords()
    T = case.steps * dt
    exact = np.sin(2 * np.pi * (X[:, 0] - T)) * np.sin(2 * np.pi * (X[:, 1] - 0.5 * T))
    m_ref, e_ref = P.diagnostics(got - exact)
    err = np.sqrt(e_ref / P.diagnostics(exact)[1])
    assert 1e-6 < err < 1e-4
    m0, e0 = P.diagnostics(u0)
    m, e = S.diagnostics()
    assert abs(m - m0) < 1e-14 and e <= e0 * (1 + 1e-14)
    mo, eo = P.diagnostics(got)
    assert abs(m - mo) <= 1e-15 and abs(e - eo) <= 1e-13 * eo


@pytest.mark.parametrize("d,k,cells,steps", [(4, 3, [3, 2, 2, 3], 3), (6, 3, [2] * 6, 2),
                                             (2, 4, [5, 3], 4), (6, 2, [3, 2, 1, 2, 1, 3], 2)])
def test_phase_space_rk_matches_oracle(d, k, cells, steps):
    dx, dv = W.SPLITS[d]
    case = W.phase_space_case("p", dx, dv, cells, k, steps)
    P = oracle_problem(case)
    S = gpu_solver(case, "fp64")
    dt = S.stable_dt(case.cfl)
    assert abs(dt - P.stable_dt(case.cfl)) <= 1e-15 * dt
    S.init_state(case.ic, case.ic_params)
    u0 = P.init_state(case.ic, list(case.ic_params))
    assert rel_max(S.get_state(), u0) <= 1e-14
    u0 = u0 + 1e-3 * W.random_state(P.ndofs, seed=3)  # excite all modes
    S.set_state(u0)
    S.rk_step(dt, steps)
    ref = P.rk_steps(u0, dt, steps)
    assert rel_l2(S.get_state(), ref) <= TOL_FP64
    m, e = S.diagnostics()
    mo, eo = P.diagnostics(ref)
    assert abs(m - mo) <= 1e-13 * abs(mo) and abs(e - eo) <= 1e-12 * eo


@pytest.mark.parametrize("d,k,cells", [(5, 2, [2, 3, 1, 2, 3]), (3, 3, [4, 3, 5]), (5, 4, [1, 2, 1, 2, 2])])
def test_constant_field_rk_matches_oracle(d, k, cells):
    dx, dv = W.SPLITS[d]
    rng = np.random.default_rng(d + k)
    case = W.Case("c", dx, dv, cells, [0.0] * d, [1.0] * d, k, "constant",
                  a=list(rng.uniform(-1, 1, d)), ic=0, steps=3)
    P = oracle_problem(case)
    S = gpu_solver(case, "fp64")
    dt = S.stable_dt(case.cfl)
    u0 = W.random_state(P.ndofs, seed=4)
    S.set_state(u0)
    S.rk_step(dt, case.steps)
    ref = P.rk_steps(u0, dt, case.steps)
    assert rel_l2(S.get_state(), ref) <= TOL_FP64


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("d,k,cells", [(6, 3, [2, 1, 3, 2, 1, 2]), (4, 2, [3, 2, 2, 3]),
                                       (5, 4, [1, 2, 1, 2, 2]), (6, 3, [1, 2, 1, 1, 3, 1]),
                                       (6, 3, [1, 2, 1, 2, 4, 1]), (6, 3, [2, 1, 1, 2, 2, 2])])
def test_rk_steps_match_oracle_for_every_plan(precision, d, k, cells):
    # Every launch plan the autotuner may pick, in stage mode (the fused RK
    # update, streaming options of the 6D degree-3 kernel included).
    dx, dv = W.SPLITS[d]
    if dx == dv:
        case = W.phase_space_case("p", dx, dv, cells, k, 2)
    else:
        case = W.Case("c", dx, dv, cells, [0.0] * d, [1.0] * d, k, "constant",
                      a=list(np.random.default_rng(d).uniform(-1, 1, d)), steps=2)
    P = oracle_problem(case)
    S = gpu_solver(case, precision)
    dt = S.stable_dt(case.cfl)
    u0 = W.random_state(P.ndofs, seed=13)
    ref = P.rk_steps(u0, dt, case.steps)
    tol = TOL_FP64 if precision == "fp64" else 1e-5
    outs = {}
    for plan in all_plans(case, precision):
        S.set_plan(**plan)
        S.set_state(u0)
        S.rk_step(dt, case.steps)
        got = S.get_state()
        assert rel_l2(got, ref) <= tol, plan
        outs.setdefault((plan.get("kernel", 0), plan["reg_dims"], plan.get("loop_dims", 0)),
                        []).append(got)
    for group in outs.values():
        for o in group[1:]:
            assert np.array_equal(o, group[0])


def test_graph_replay_is_bitwise_equal_to_direct_stages():
    case = W.phase_space_case("p", 2, 2, [3, 2, 2, 3], 3, 3)
    u0 = W.random_state(case.ndofs, seed=9)
    A = gpu_solver(case, "fp64")
    B = gpu_solver(case, "fp64")
    A.set_state(u0)
    B.set_state(u0)
    dt = A.stable_dt(0.2)
    for rep in range(3):
        A.rk_step(dt, 2)
        for _ in range(2):
            for st in range(5):
                B.rk_stage(st, dt)
        torch.cuda.synchronize()
        assert np.array_equal(A.get_state(), B.get_state()), rep


def test_checkpoint_resume_is_bitwise():
    case = W.phase_space_case("p", 3, 3, [2, 1, 2, 1, 2, 1], 3, 2)
    u0 = W.random_state(case.ndofs, seed=11)
    A = gpu_solver(case, "fp64")
    A.set_state(u0)
    dt = A.stable_dt(0.2)
    A.rk_step(dt, 4)
    full = A.get_state()
    B = gpu_solver(case, "fp64")
    B.set_state(u0)
    B.rk_step(dt, 2)
    mid = B.get_state()
    C = gpu_solver(case, "fp64")
    C.set_state(mid)
    C.rk_step(dt, 2)
    assert np.array_equal(C.get_state(), full)


def test_diagnostics_are_deterministic_and_match_oracle():
    case = W.phase_space_case("p", 2, 2, [4, 3, 5, 2], 4, 1)
    P = oracle_problem(case)
    S = gpu_solver(case, "fp64")
    u = W.random_state(P.ndofs, seed=2)
    S.set_state(u)
    r1 = S.diagnostics()
    r2 = S.diagnostics()
    assert r1 == r2
    mo, eo = P.diagnostics(u)
    assert abs(r1[0] - mo) <= 1e-12 * (abs(mo) + 1) and abs(r1[1] - eo) <= 1e-13 * eo


def test_fp32_stage_keeps_fp64_solution():
    # FP32 operator mode: du and the operator in FP32, u stays FP64.
    case = W.phase_space_case("p", 2, 2, [3, 2, 2, 3], 3, 2)
    P = oracle_problem(case)
    S = gpu_solver(case, "fp32")
    u0 = P.init_state(case.ic, list(case.ic_params))
    S.set_state(u0)
    dt = S.stable_dt(0.2)
    S.rk_step(dt, 2)
    ref = P.rk_steps(u0, dt, 2)
    assert rel_l2(S.get_state(), ref) < 1e-6


def test_invalid_arguments_are_rejected_on_device_calls():
    from paper_2002_08110_amd._hd import HDError
    case = W.phase_space_case("p", 2, 2, [2, 2, 2, 2], 2, 1)
    S = gpu_solver(case, "fp64")
    with pytest.raises(HDError):
        S.rk_stage(5, 1e-3)
    with pytest.raises(HDError):
        S.set_plan(lds=1, cells_per_wg=100)
    with pytest.raises(HDError):
        S.set_plan(reg_dims=3)
    u = torch.zeros(S.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(HDError):
        S.apply(u, out=u)  # in and out must not alias


@pytest.mark.parametrize("d,k,precision", [(6, 3, "fp64"), (6, 3, "fp32"), (4, 2, "fp64")])
def test_tune_plan_keeps_the_state_and_steps_as_the_fixed_plan(d, k, precision):
    # Timing the candidate plans on the solver's own mesh must leave its
    # solution untouched; afterwards it steps exactly as a solver given the
    # chosen plan directly.
    case = small_case(d, k, "sine" if W.SPLITS[d][0] == W.SPLITS[d][1] else "constant")
    S = gpu_solver(case, precision)
    u0 = W.random_state(S.ndofs, seed=31)
    S.set_state(u0)
    dt = S.stable_dt(0.2)
    plan = S.tune_plan(dt)
    assert plan == S.get_plan()
    assert np.array_equal(S.get_state(), u0)
    S.rk_step(dt, 2)
    T = gpu_solver(case, precision, plan=plan)
    T.set_state(u0)
    T.rk_step(dt, 2)
    assert np.array_equal(S.get_state(), T.get_state())
    S.close()
    T.close()


def test_tune_plan_keeps_the_plan_it_had_within_the_margin():
    # A candidate replaces the plan the solver had only when it is faster by
    # more than the margin; with a margin of 1 none can be.
    case = small_case(6, 3, "sine")
    S = gpu_solver(case, "fp64")
    start = S.get_plan()
    u0 = W.random_state(S.ndofs, seed=37)
    S.set_state(u0)
    assert S.tune_plan(S.stable_dt(0.2), margin=1.0) == start
    assert S.get_plan() == start
    assert np.array_equal(S.get_state(), u0)
    S.close()
