"""GPU parity on curved configuration cells (the tensor-product mapping of
Sec. 3.1/3.3, hd_set_mapping) against the oracle's mapped weak form: the
operator with collocation (oracle mode 0) and Gauss-Legendre quadrature
(mode 2) for d = 2..6, RK steps, mapped initial states and sine fields,
exact mass conservation with collocation, the return to Cartesian cells and
the unsupported cases.

Bar: FP64 relative L2 and max-norm differences <= 1e-12; FP32 bounded.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import TOL_FP64, gpu_solver, rel_l2, rel_max, x_table_size
from paper_2002_08110_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = 0.03
MESHES = {2: [5, 3], 3: [3, 2, 2], 4: [2, 2, 2, 1], 5: [2, 1, 2, 1, 1], 6: [2, 1, 1, 1, 2, 1]}


def case_of(d, k, field):
    dx, dv = W.SPLITS[d]
    cells = MESHES[d]
    rng = np.random.default_rng(300 + 10 * d + k)
    if field == "constant":
        a = list(rng.uniform(-1, 1, d))
        return W.Case("c", dx, dv, cells, [0.0] * d, list(rng.uniform(0.6, 1.5, d)), k, "constant",
                      a=a)
    if field == "sine":
        return W.Case("s", dx, dv, cells, [0.0] * dx + [-6.0] * dv, [1.0] * dx + [6.0] * dv, k,
                      "sine", amp=0.3)
    return W.Case("t", dx, dv, cells, [0.0] * dx + [-5.0] * dv, [1.0] * dx + [3.5] * dv, k,
                  "table")


def oracle_of(case, E=None, eps=EPS):
    kw = dict(map_eps=eps)
    if case.field == "constant":
        return oracle.Problem(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
                              field="constant", a=case.a, **kw)
    if case.field == "sine":
        return oracle.Problem(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
                              field="phase", sine_amp=case.amp, **kw)
    return oracle.Problem(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
                          field="phase", E=E, **kw)


def solver_of(case, precision, quadrature, E=None, eps=EPS):
    S = gpu_solver(case, precision, E=E)
    if quadrature == "gauss_legendre":
        S.set_quadrature(quadrature)
    S.set_mapping(eps)
    # fields given at node coordinates follow the mapping: set them after it
    if case.field == "sine":
        S.set_field_sine(case.amp)
    elif case.field == "table":
        S.set_field_phase_space(E)
    return S


def lds_ok(d, k, precision):
    n, dx = k + 1, W.SPLITS[d][0]

    def padded(c):
        return c + c // (n * n) + 1
    lds = 2 * padded(n ** d) + padded(n ** (d - 1)) + n ** dx * dx + 3 * n * n + 6 * n
    if precision == "fp32":  # the metric is staged in LDS in FP32 only
        lds += n ** dx * (dx * dx + 1) + dx * 2 * n ** (dx - 1) * dx
    return lds * (8 if precision == "fp64" else 4) + 1024 <= 160 * 1024 and not (d == 5 and k == 5)


def _cost_ok(d, k):
    return int(np.prod(MESHES[d])) * (k + 1) ** (2 * d) <= 1.2e8


PARAMS = [(d, k, f, q) for d in (2, 3, 4, 5, 6) for k in (1, 2, 3, 4, 5)
          for f in ("constant", "sine", "table") for q in ("gauss_lobatto", "gauss_legendre")
          if (f == "constant" or W.SPLITS[d][0] == W.SPLITS[d][1]) and lds_ok(d, k, "fp64")
          and _cost_ok(d, k) and (f != "table" or k in (2, 3))]


@pytest.mark.parametrize("d,k,field,quadrature", PARAMS)
def test_apply_matches_oracle_on_mapped_cells(d, k, field, quadrature):
    case = case_of(d, k, field)
    E = W.random_field_table(x_table_size(case), seed=7) if field == "table" else None
    P = oracle_of(case, E)
    u = W.random_state(P.ndofs, seed=3)
    ref = P.apply(u, mode=0 if quadrature == "gauss_lobatto" else 2)
    S = solver_of(case, "fp64", quadrature, E)
    out = S.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    assert rel_l2(out, ref) <= TOL_FP64
    assert rel_max(out, ref) <= TOL_FP64
    S.close()


@pytest.mark.parametrize("quadrature", ["gauss_lobatto", "gauss_legendre"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("d,k,cells", [(2, 3, [5, 4]), (4, 2, [2, 2, 3, 2]), (6, 2, [2, 1, 1, 1, 2, 1])])
def test_rk_steps_match_oracle_on_mapped_cells(quadrature, precision, d, k, cells):
    dx, dv = W.SPLITS[d]
    case = W.phase_space_case("p", dx, dv, cells, k, 2)
    P = oracle_of(case)
    S = solver_of(case, precision, quadrature)
    S.init_state(case.ic, list(case.ic_params))
    u0 = P.init_state(case.ic, list(case.ic_params))
    assert rel_max(S.get_state(), u0) <= 1e-14  # nodal values at mapped coordinates
    dt = P.stable_dt(case.cfl)
    ref = P.rk_steps(u0, dt, case.steps, mode=0 if quadrature == "gauss_lobatto" else 2)
    S.rk_step(dt, case.steps)
    tol = TOL_FP64 if precision == "fp64" else 1e-5
    assert rel_l2(S.get_state(), ref) <= tol
    S.close()


def test_sine_table_follows_the_mapping():
    case = case_of(4, 2, "sine")
    P = oracle_of(case)
    S = solver_of(case, "fp64", "gauss_lobatto")
    np.testing.assert_allclose(S.get_field(), P.sine_table(case.amp), rtol=0, atol=1e-15)
    S.close()


def test_mass_is_conserved_with_collocation_on_mapped_cells():
    case = W.phase_space_case("p", 2, 2, [3, 2, 3, 2], 3, 10)
    S = solver_of(case, "fp64", "gauss_lobatto")
    S.init_state(case.ic, list(case.ic_params))
    m0, _ = S.diagnostics()
    P = oracle_of(case)
    mo, _ = P.diagnostics(P.init_state(case.ic, list(case.ic_params)))
    assert abs(m0 / mo - 1) <= 1e-13
    S.rk_step(S.stable_dt(0.2), case.steps)
    m1, _ = S.diagnostics()
    assert abs(m1 - m0) <= 1e-13 * abs(m0)
    S.close()


def test_zero_deformation_returns_to_the_cartesian_kernels():
    case = W.phase_space_case("p", 3, 3, [2, 1, 2, 1, 2, 1], 3, 2)
    u0 = W.random_state(case.ndofs, seed=5)
    A = gpu_solver(case, "fp64")
    B = gpu_solver(case, "fp64")
    B.set_mapping(EPS)
    B.set_mapping(0.0)
    dt = A.stable_dt(0.2)
    for S in (A, B):
        S.set_state(u0)
        S.rk_step(dt, 2)
    assert np.array_equal(A.get_state(), B.get_state())
    A.close()
    B.close()


def test_invalid_mappings_are_rejected():
    from paper_2002_08110_amd._hd import HDError
    case = W.phase_space_case("p", 1, 1, [4, 4], 2, 1)
    S = gpu_solver(case, "fp64")
    with pytest.raises(HDError):
        S.set_mapping(0.2)
    S.set_field_vlasov_poisson(2)
    with pytest.raises(HDError):
        S.set_mapping(0.01)
    S.close()
    T = gpu_solver(W.phase_space_case("p", 1, 1, [4, 4], 2, 1), "fp64")
    T.set_mapping(0.01)
    with pytest.raises(HDError):
        T.set_field_vlasov_poisson(2)
    T.close()
    U = gpu_solver(W.Case("c", 3, 2, [1] * 5, [0.0] * 5, [1.0] * 5, 5, "constant", a=[1.0] * 5),
                   "fp32")
    with pytest.raises(HDError):
        U.set_mapping(0.01)
    U.close()


@pytest.mark.parametrize("field", ["constant", "sine", "table"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_6d_k3_collocation_layout_and_sweep_kernels_match_the_oracle(field, precision):
    # Mapped 6D degree 3 with collocation has two kernels: the collocation
    # kernel's thread layout (plan kernel 1, the default) and the sweep
    # kernel (kernel 0). Both against the oracle's mapped collocation.
    case = case_of(6, 3, field)
    case.cells = [2, 1, 2, 1, 1, 2]
    E = W.random_field_table(x_table_size(case), seed=13) if field == "table" else None
    P = oracle_of(case, E)
    u = W.random_state(P.ndofs, seed=41)
    ref = P.apply(u, mode=0)
    outs = []
    for kernel in (1, 0):
        S = solver_of(case, precision, "gauss_lobatto", E)
        S.set_plan(kernel=kernel)
        out = S.apply(torch.from_numpy(u).cuda()).double().cpu().numpy()
        tol = TOL_FP64 if precision == "fp64" else 5e-6
        assert rel_l2(out, ref) <= tol, kernel
        if precision == "fp64":
            assert rel_max(out, ref) <= TOL_FP64, kernel
        outs.append(out)
        S.close()
    assert rel_l2(outs[0], outs[1]) <= (1e-13 if precision == "fp64" else 5e-6)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_6d_k3_collocation_rk_steps_on_mapped_cells(precision):
    case = W.phase_space_case("p", 3, 3, [2, 1, 1, 1, 2, 1], 3, 2)
    P = oracle_of(case)
    S = solver_of(case, precision, "gauss_lobatto")
    assert S.get_plan()["kernel"] == 1
    u0 = W.random_state(P.ndofs, seed=43)
    dt = P.stable_dt(case.cfl)
    ref = P.rk_steps(u0, dt, case.steps, mode=0)
    S.set_state(u0)
    S.rk_step(dt, case.steps)
    assert rel_l2(S.get_state(), ref) <= (TOL_FP64 if precision == "fp64" else 1e-5)
    S.close()


@pytest.mark.parametrize("field,precision,cells", [
    (f, p, [2, 1, 2, 1, 1, 2]) for f in ("constant", "sine", "table") for p in ("fp64", "fp32")] + [
    ("sine", "fp64", [1, 2, 1, 2, 2, 2]), ("sine", "fp32", [1, 2, 1, 2, 2, 2])])
def test_6d_k3_gauss_legendre_layout_and_sweep_kernels_match_the_oracle(field, precision, cells):
    # Mapped 6D degree 3 with Gauss-Legendre quadrature: the kernel in the
    # collocation kernel's thread layout (plan kernel 1, the default) and the
    # sweep kernel (kernel 0), both against the oracle's mapped Gauss mode.
    # With one velocity cell over [-6, 6] in v1 and v2, x-faces mix inflow
    # and outflow points; a constant field gives faces of one sign, and
    # velocity cells split at v = 0 give both kinds.
    case = case_of(6, 3, field)
    case.cells = cells
    E = W.random_field_table(x_table_size(case), seed=17) if field == "table" else None
    P = oracle_of(case, E)
    u = W.random_state(P.ndofs, seed=47)
    ref = P.apply(u, mode=2)
    outs = []
    for kernel in (1, 0):
        S = solver_of(case, precision, "gauss_legendre", E)
        S.set_plan(kernel=kernel)
        out = S.apply(torch.from_numpy(u).cuda()).double().cpu().numpy()
        tol = TOL_FP64 if precision == "fp64" else 5e-6
        assert rel_l2(out, ref) <= tol, kernel
        if precision == "fp64":
            assert rel_max(out, ref) <= TOL_FP64, kernel
        outs.append(out)
        S.close()
    assert rel_l2(outs[0], outs[1]) <= (1e-13 if precision == "fp64" else 5e-6)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_6d_k3_gauss_legendre_rk_steps_on_mapped_cells(precision):
    case = W.phase_space_case("p", 3, 3, [2, 1, 1, 2, 1, 1], 3, 2)
    P = oracle_of(case)
    S = solver_of(case, precision, "gauss_legendre")
    assert S.get_plan()["kernel"] == 1
    u0 = W.random_state(P.ndofs, seed=53)
    dt = P.stable_dt(case.cfl)
    ref = P.rk_steps(u0, dt, case.steps, mode=2)
    S.set_state(u0)
    S.rk_step(dt, case.steps)
    assert rel_l2(S.get_state(), ref) <= (TOL_FP64 if precision == "fp64" else 1e-5)
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("quadrature,field", [("gauss_lobatto", "sine"), ("gauss_lobatto", "table"),
                                              ("gauss_legendre", "sine"),
                                              ("gauss_legendre", "table")])
def test_6d_k3_mapped_kernels_with_distinct_neighbours(quadrature, field, precision):
    # Three cells in every dimension: each cell's left and right neighbours
    # are distinct cells, different from itself, so the upwind choice of the
    # neighbour side and the cell order of the launch are exercised. The
    # default kernels of mapped 6D degree 3 (collocation and Gauss-Legendre
    # layouts) on sampled cells against the oracle, and in FP64 one RK step
    # stage by stage.
    from gpu_helpers import sample_cells, stages_sampled
    case = case_of(6, 3, field)
    case.cells = [3] * 6
    E = W.random_field_table(x_table_size(case), seed=19) if field == "table" else None
    P = oracle_of(case, E)
    mode = 0 if quadrature == "gauss_lobatto" else 2
    S = solver_of(case, precision, quadrature, E)
    assert S.get_plan()["kernel"] == 1
    u = W.random_state(P.ndofs, seed=61)
    cells = sample_cells(P.ncells, seed=63, count=9)
    ref = P.apply_cells(u, cells, mode=mode)
    nd = 4 ** 6
    idx = (cells[:, None] * nd + np.arange(nd)[None, :]).reshape(-1)
    out = S.apply(torch.from_numpy(u).cuda()).double().cpu().numpy()[idx]
    tol = TOL_FP64 if precision == "fp64" else 5e-6
    assert rel_l2(out, ref) <= tol
    if precision == "fp64":
        assert rel_max(out, ref) <= TOL_FP64
        S.set_state(u)
        stages_sampled(S, lambda host: P, cells[:6], S.stable_dt(0.2), TOL_FP64, mode=mode)
    S.close()
