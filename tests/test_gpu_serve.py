"""Serving with continuous batching: every request's result is the same
alone and in the mix (bitwise for the same plan and precision; FP64 also
against the oracle), admission respects the memory budget and arrival
order, and the one-at-a-time baseline gives the same results."""
import numpy as np
import pytest

from gpu_helpers import TOL_FP64, oracle_problem, rel_l2
from paper_2002_08110_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def small_trace(seed=5, count=10):
    # the serving mix (d in {4,5,6}, k in {2..5}, phase-space or constant
    # fields) at sizes the oracle handles, arriving 5 ms apart on average
    return W.serve_trace(seed=seed, count=count, rate=200.0, steps=(2, 5),
                         dof_range=(2e3, 6e4), cells_range=(1, 3))


def alone(case, precision):
    from paper_2002_08110_amd import serve
    s = serve.make_solver(case, precision)
    dt = serve.setup(s, case)
    s.rk_step(dt, case.steps)
    out = s.get_state()
    s.close()
    return out, dt


@pytest.mark.parametrize("precision,fill,order", [
    ("fp32", 1e8, "shortest"), ("fp64", 1e8, "shortest"), ("fp32", 3e4, "shortest"),
    ("fp32", 3e4, "arrival"), ("fp64", None, "arrival")])
def test_served_results_equal_alone(precision, fill, order):
    # fill: DoFs a step aims to cover (3e4: a few requests per step, the
    # rest resident and inactive; None: every resident request each step)
    from paper_2002_08110_amd import serve
    reqs = small_trace()
    res, stats = serve.serve(reqs, precision=precision, keep_states=True, fill_dofs=fill,
                             order=order)
    assert stats["requests"] == len(reqs)
    by_id = {r.rid: r for r in res}
    for q in reqs:
        got = by_id[q.rid].state
        ref, dt = alone(q.case, precision)
        assert np.array_equal(got, ref), (q.rid, q.case.d, q.case.degree)
        if precision == "fp64" and q.case.ndofs <= 2e4:
            P = oracle_problem(q.case)
            u0 = P.init_state(q.case.ic, list(q.case.ic_params))
            assert rel_l2(got, P.rk_steps(u0, dt, q.case.steps)) <= TOL_FP64, q.rid


def test_admission_respects_budget_and_order():
    from paper_2002_08110_amd import serve
    reqs = small_trace(seed=7, count=8)
    fps = [serve.footprint(q.case, "fp32") for q in reqs]
    budget = max(fps) + min(fps)  # at most a couple of requests at a time
    res, stats = serve.serve(reqs, precision="fp32", budget=budget)
    assert stats["peak_bytes"] <= budget
    assert all(np.isfinite(r.completed) for r in res)
    adm = [r.admitted for r in sorted(res, key=lambda r: r.arrival)]
    assert adm == sorted(adm)  # admitted in arrival order
    assert all(r.admitted >= r.arrival - 1e-9 for r in res)


def test_one_at_a_time_baseline_matches_batched():
    from paper_2002_08110_amd import serve
    reqs = small_trace(seed=9, count=6)
    a, sa = serve.serve(reqs, precision="fp64", keep_states=True)
    b, sb = serve.serve(reqs, precision="fp64", batched=False, keep_states=True)
    assert not sb["batched"]
    for x, y in zip(sorted(a, key=lambda r: r.rid), sorted(b, key=lambda r: r.rid)):
        assert np.array_equal(x.state, y.state)
        assert x.mass == y.mass and x.energy == y.energy


def test_over_budget_request_is_rejected_and_the_rest_are_served():
    # A budget below the largest request's footprint: that request is
    # rejected with a status (HD_ERR_OOM) when it arrives, and every other
    # request is served and equals the same request alone, bitwise.
    from paper_2002_08110_amd import _hd, serve
    reqs = small_trace(seed=11, count=6)
    fps = {q.rid: serve.footprint(q.case, "fp32") for q in reqs}
    big = max(fps, key=fps.get)
    budget = max(v for k, v in fps.items() if k != big)
    assert fps[big] > budget
    res, stats = serve.serve(reqs, precision="fp32", budget=budget, keep_states=True)
    by_id = {r.rid: r for r in res}
    assert by_id[big].status == "rejected" and by_id[big].code == _hd.HD_ERR_OOM
    assert by_id[big].state is None
    assert stats["rejected"] == 1 and stats["completed"] == len(reqs) - 1
    assert stats["peak_bytes"] <= budget
    for q in reqs:
        if q.rid == big:
            continue
        assert by_id[q.rid].status == "done"
        ref, _ = alone(q.case, "fp32")
        assert np.array_equal(by_id[q.rid].state, ref), q.rid
