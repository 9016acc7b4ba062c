"""GPU parity of the Gauss-Legendre quadrature variant (Sec. 2.5) against the
oracle's mode 2: the operator (d = 2..6, degrees 1..5 where the kernel
exists, constant, sine and random-table fields), RK steps, the
Vlasov-Poisson field, graph replay, the switch back to collocation and the
unsupported cases.

Bar: FP64 relative L2 and max-norm differences <= 1e-12; FP32 bounded.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import TOL_FP64, gpu_solver, oracle_problem, rel_l2, rel_max, x_table_size
from paper_2002_08110_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MESHES = {2: [5, 3], 3: [3, 2, 2], 4: [2, 1, 2, 3], 5: [1, 2, 1, 2, 1], 6: [1, 2, 1, 1, 2, 1]}


def case_of(d, k, field):
    dx, dv = W.SPLITS[d]
    cells = MESHES[d]
    rng = np.random.default_rng(200 + 10 * d + k)
    if field == "constant":
        a = list(rng.uniform(-1, 1, d))
        lo = list(rng.uniform(-1, 0, d))
        hi = [l + w for l, w in zip(lo, rng.uniform(0.5, 2, d))]
        return W.Case("c", dx, dv, cells, lo, hi, k, "constant", a=a)
    if field == "sine":
        return W.Case("s", dx, dv, cells, [0.0] * dx + [-6.0] * dv, [1.0] * dx + [6.0] * dv, k,
                      "sine", amp=0.3)
    return W.Case("t", dx, dv, cells, [0.0] * dx + [-5.0] * dv, [1.0] * dx + [3.5] * dv, k,
                  "table")


def supported(d, k, precision):
    n = k + 1
    dx = W.SPLITS[d][0]
    def padded(c):  # one element of padding per n^2
        return c + c // (n * n) + 1
    lds = (2 * padded(n ** d) + padded(n ** (d - 1)) + n ** dx * dx + 3 * n * n + 5 * n) * (
        8 if precision == "fp64" else 4)
    return lds + 1024 <= 160 * 1024


def _cost_ok(d, k, ncells):
    # the oracle's full-sum Gauss mode costs ~ (k+1)^(2d) per cell
    return ncells * (k + 1) ** (2 * d) <= 3e8


PARAMS = [(d, k, f) for d in (2, 3, 4, 5, 6) for k in (1, 2, 3, 4, 5)
          for f in ("constant", "sine", "table")
          if (f == "constant" or W.SPLITS[d][0] == W.SPLITS[d][1])
          and supported(d, k, "fp64") and _cost_ok(d, k, int(np.prod(MESHES[d])))]


def _solver(case, precision, E=None):
    S = gpu_solver(case, precision, E=E)
    S.set_quadrature("gauss_legendre")
    return S


@pytest.mark.parametrize("d,k,field", PARAMS)
def test_apply_matches_oracle_gauss_mode(d, k, field):
    case = case_of(d, k, field)
    E = W.random_field_table(x_table_size(case), seed=7) if field == "table" else None
    P = oracle_problem(case, E=E)
    u = W.random_state(P.ndofs, seed=3)
    ref = P.apply(u, mode=2)
    S = _solver(case, "fp64", E=E)
    out = S.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    assert rel_l2(out, ref) <= TOL_FP64
    assert rel_max(out, ref) <= TOL_FP64
    # differs from collocation
    assert rel_l2(out, P.apply(u, mode=1)) > 1e-6
    S.close()


@pytest.mark.parametrize("d,k", [(2, 3), (4, 2), (5, 3), (6, 2), (6, 4)])
def test_apply_fp32_error_is_small(d, k):
    case = case_of(d, k, "sine" if W.SPLITS[d][0] == W.SPLITS[d][1] else "constant")
    if d == 6 and k == 4:
        case.cells = [1, 1, 1, 1, 2, 1]
    P = oracle_problem(case)
    u = W.random_state(P.ndofs, seed=5)
    ref = P.apply(u, mode=2)
    S = _solver(case, "fp32")
    out = S.apply(torch.from_numpy(u).cuda())
    assert out.dtype == torch.float32
    assert rel_l2(out.double().cpu().numpy(), ref) < 5e-6
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("d,k,cells", [(2, 3, [4, 5]), (4, 3, [2, 1, 3, 2]), (6, 3, [1, 1, 1, 1, 2, 1]),
                                       (5, 2, [2, 1, 2, 1, 3])])
def test_rk_steps_match_oracle(precision, d, k, cells):
    dx, dv = W.SPLITS[d]
    if dx == dv:
        case = W.phase_space_case("p", dx, dv, cells, k, 2)
    else:
        case = W.Case("c", dx, dv, cells, [0.0] * d, [1.0] * d, k, "constant",
                      a=list(np.random.default_rng(d).uniform(-1, 1, d)), steps=2)
    P = oracle_problem(case)
    S = _solver(case, precision)
    dt = S.stable_dt(case.cfl)
    u0 = W.random_state(P.ndofs, seed=13)
    ref = P.rk_steps(u0, dt, case.steps, mode=2)
    S.set_state(u0)
    S.rk_step(dt, case.steps)
    tol = TOL_FP64 if precision == "fp64" else 1e-5
    assert rel_l2(S.get_state(), ref) <= tol
    S.close()


@pytest.mark.parametrize("dx,cells,k", [(1, [6, 4], 3), (2, [3, 2, 2, 3], 2), (3, [2, 1, 2, 1, 2, 1], 2),
                                       (3, [2, 1, 1, 1, 2, 1], 3)])
def test_vlasov_poisson_with_gauss_quadrature(dx, cells, k):
    lo = [0.0] * dx + [-5.0] * dx
    hi = [2 * np.pi] * dx + [4.0] * dx
    case = W.Case("vp", dx, dx, cells, lo, hi, k, "vlasov_poisson", steps=2, modes=2)
    V = oracle.VlasovPoisson(dx, dx, cells, lo, hi, k, 2)
    u0 = np.abs(W.random_state(case.ndofs, 17)) + 0.5
    dt = V.stable_dt(u0, 0.2)
    ref = V.rk_steps(u0, dt, 2, mode=2)
    S = _solver(case, "fp64")
    S.set_state(u0)
    S.rk_step(dt, 2)
    assert rel_l2(S.get_state(), ref) <= TOL_FP64
    S.close()


def test_graph_replay_and_switching_back_to_collocation():
    case = W.phase_space_case("p", 2, 2, [3, 2, 2, 3], 3, 3)
    u0 = W.random_state(case.ndofs, seed=9)
    A = _solver(case, "fp64")
    B = _solver(case, "fp64")
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
    # back to collocation: the same result as a solver that never switched
    C = gpu_solver(case, "fp64")
    A.set_quadrature("gauss_lobatto")
    for S in (A, C):
        S.set_state(u0)
        S.rk_step(dt, 2)
    assert np.array_equal(A.get_state(), C.get_state())
    for S in (A, B, C):
        S.close()


def test_unsupported_gauss_cases_raise():
    from paper_2002_08110_amd._hd import HDError
    for d, k, prec in [(6, 4, "fp64"), (6, 5, "fp32"), (6, 5, "fp64")]:
        dx, dv = W.SPLITS[d]
        case = W.Case("c", dx, dv, [1] * d, [0.0] * d, [1.0] * d, k, "constant", a=[1.0] * d)
        S = gpu_solver(case, prec)
        with pytest.raises(HDError):
            S.set_quadrature("gauss_legendre")
        S.close()


def test_batch_mixing_quadratures_and_mapped_cells_equals_alone():
    from paper_2002_08110_amd.solver import Batch
    cases = [W.phase_space_case("p", 2, 2, [3, 2, 2, 3], 3, 3),
             W.phase_space_case("q", 3, 3, [2, 1, 1, 1, 2, 1], 2, 3),
             W.phase_space_case("r", 1, 1, [6, 5], 4, 3),
             W.phase_space_case("s", 2, 2, [2, 3, 2, 2], 2, 3),
             W.phase_space_case("t", 3, 3, [1, 2, 1, 1, 2, 1], 3, 3),
             W.phase_space_case("v", 3, 3, [2, 1, 1, 2, 1, 1], 3, 3)]
    setups = [("gauss_lobatto", 0.0, "fp64"), ("gauss_legendre", 0.0, "fp64"),
              ("gauss_lobatto", 0.02, "fp64"), ("gauss_legendre", 0.03, "fp32"),
              ("gauss_legendre", 0.0, "fp64"), ("gauss_legendre", 0.0, "fp32")]

    def make(case, quad, eps, prec):
        S = gpu_solver(case, prec)
        if quad == "gauss_legendre":
            S.set_quadrature(quad)
        if eps:
            S.set_mapping(eps)
            S.set_field_sine(case.amp)
        S.init_state(case.ic, list(case.ic_params))
        return S

    alone, dts = [], []
    for c, (q, e, p) in zip(cases, setups):
        S = make(c, q, e, p)
        dt = S.stable_dt(0.2)
        dts.append(dt)
        S.rk_step(dt, 3)
        alone.append(S.get_state())
        S.close()
    solvers = [make(c, q, e, p) for c, (q, e, p) in zip(cases, setups)]
    B = Batch(solvers)
    for _ in range(3):
        B.step(dts)
    torch.cuda.synchronize()
    for S, a in zip(solvers, alone):
        assert np.array_equal(S.get_state(), a)
    B.close()
    for S in solvers:
        S.close()


@pytest.mark.parametrize("field", ["constant", "sine", "table"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_6d_k3_layout_and_sweep_kernels_match_the_oracle(field, precision):
    # 6D degree 3 has two Gauss-Legendre kernels: the collocation kernel's
    # thread layout (plan kernel 1, the default) and the sweep kernel
    # (kernel 0). Both against the oracle, on a mesh whose velocity cells
    # straddle v = 0 (inflow on both sides of x-faces) for the table field.
    case = case_of(6, 3, field)
    case.cells = [2, 1, 2, 1, 2, 2] if field != "table" else [1, 2, 1, 2, 1, 2]
    E = W.random_field_table(x_table_size(case), seed=11) if field == "table" else None
    P = oracle_problem(case, E=E)
    u = W.random_state(P.ndofs, seed=21)
    ref = P.apply(u, mode=2)
    outs = []
    for kernel in (1, 0):
        S = _solver(case, precision, E=E)
        S.set_plan(kernel=kernel)
        out = S.apply(torch.from_numpy(u).cuda()).double().cpu().numpy()
        tol = TOL_FP64 if precision == "fp64" else 5e-6
        assert rel_l2(out, ref) <= tol, kernel
        if precision == "fp64":
            assert rel_max(out, ref) <= TOL_FP64, kernel
        outs.append(out)
        S.close()
    assert rel_l2(outs[0], outs[1]) <= (1e-13 if precision == "fp64" else 5e-6)
