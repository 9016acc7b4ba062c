"""Batched persistent stepping: each solve in the mix equals the same solve
stepped alone (bitwise with the same launch variant) and the oracle (FP64,
1e-12), inactive solves stay untouched, and per-solve time steps and outside
steps are honoured."""
import numpy as np
import pytest

from gpu_helpers import TOL_FP64, gpu_solver, oracle_problem, rel_l2
from paper_2002_08110_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MIX = [  # (d, k, cells, field)
    (2, 3, [5, 3], "constant"), (3, 2, [3, 2, 4], "constant"), (4, 3, [3, 2, 2, 3], "sine"),
    (4, 5, [2, 1, 2, 1], "sine"), (5, 2, [2, 3, 1, 2, 2], "constant"), (6, 3, [2, 1, 2, 2, 1, 2], "sine"),
    (6, 2, [2, 2, 1, 1, 2, 1], "constant"), (5, 4, [1, 2, 1, 1, 2], "constant"), (3, 5, [2, 2, 3], "constant"),
    (6, 3, [2, 2, 1, 1, 2, 2], "constant"),
]


def make_case(i, d, k, cells, field):
    dx, dv = W.SPLITS[d]
    rng = np.random.default_rng(100 + i)
    if field == "sine":
        return W.phase_space_case("m%d" % i, dx, dv, cells, k, 3)
    return W.Case("m%d" % i, dx, dv, cells, [0.0] * d, [1.0] * d, k, "constant",
                  a=list(rng.uniform(-1, 1, d)), steps=3)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_alone_and_oracle(precision):
    from paper_2002_08110_amd.solver import Batch, batch_plan
    cases = [make_case(i, *m) for i, m in enumerate(MIX)]
    states = [W.random_state(c.ndofs, seed=50 + i) for i, c in enumerate(cases)]
    mixed = [gpu_solver(c, precision) for c in cases]
    alone = [gpu_solver(c, precision, plan=batch_plan(c.d, c.degree, c.dim_v, precision))
             for c in cases]
    dts = []
    for s, a, u in zip(mixed, alone, states):
        s.set_state(u)
        a.set_state(u)
        dts.append(s.stable_dt(0.2))
    B = Batch(mixed)
    steps = 3
    for _ in range(steps):
        B.step(dts)
    for a, dt in zip(alone, dts):
        a.rk_step(dt, steps)
    torch.cuda.synchronize()
    for i, (c, s, a, u, dt) in enumerate(zip(cases, mixed, alone, states, dts)):
        got = s.get_state()
        assert np.array_equal(got, a.get_state()), (i, c.d, c.degree)
        if precision == "fp64":
            ref = oracle_problem(c).rk_steps(u, dt, steps)
            assert rel_l2(got, ref) <= TOL_FP64, (i, c.d, c.degree)
    B.close()


def test_batch_active_mask_dt_change_and_outside_steps():
    from paper_2002_08110_amd.solver import Batch, batch_plan
    cases = [make_case(i, *m) for i, m in enumerate(MIX[:4])]
    states = [W.random_state(c.ndofs, seed=70 + i) for i, c in enumerate(cases)]
    mixed = [gpu_solver(c, "fp64") for c in cases]
    alone = [gpu_solver(c, "fp64", plan=batch_plan(c.d, c.degree, c.dim_v, "fp64")) for c in cases]
    for s, a, u in zip(mixed, alone, states):
        s.set_state(u)
        a.set_state(u)
    dts = [s.stable_dt(0.2) for s in mixed]
    B = Batch(mixed)
    B.step(dts, active=[1, 0, 1, 1])
    alone[0].rk_step(dts[0])
    alone[2].rk_step(dts[2])
    alone[3].rk_step(dts[3])
    dts2 = [0.5 * x for x in dts]
    B.step(dts2, active=[0, 1, 1, 0])
    alone[1].rk_step(dts2[1])
    alone[2].rk_step(dts2[2])
    # a solve stepped outside the batch, then batched again
    mixed[3].rk_step(dts[3])
    alone[3].rk_step(dts[3])
    B.step(dts, active=[1, 1, 1, 1])
    for a, dt in zip(alone, dts):
        a.rk_step(dt)
    torch.cuda.synchronize()
    for i, (s, a) in enumerate(zip(mixed, alone)):
        assert np.array_equal(s.get_state(), a.get_state()), i
    B.close()


def test_batch_rejects_mixed_precision_and_unbound():
    from paper_2002_08110_amd._hd import HDError
    from paper_2002_08110_amd.solver import Batch, Solver
    c = make_case(0, *MIX[0])
    a = gpu_solver(c, "fp64")
    b = gpu_solver(c, "fp32")
    with pytest.raises(HDError):
        Batch([a, b])
    u = Solver(c.dim_x, c.dim_v, c.cells, c.lo, c.hi, c.degree, bind=False)
    with pytest.raises(HDError):
        Batch([a, u])
    with pytest.raises(HDError):
        Batch([a, a])
