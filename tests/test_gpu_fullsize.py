"""Parity at the headline size (6D phase space, 8^6 cells, k = 3, 1.07e9
DoFs) in the launch configuration the benchmark times: the whole operator
runs on the GPU, the oracle recomputes a seeded sample of cells one by one
from the same input and the outputs are compared cell by cell.
"""
import numpy as np
import pytest

from gpu_helpers import (TOL_FP64, gpu_solver, oracle_problem, rel_l2, rel_max, sample_cells,
                         stages_sampled)
from paper_2002_08110_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _sample_cells(ncells, seed, count=24):
    rng = np.random.default_rng(seed)
    # corners of the periodic box (wrap-around neighbours) plus random cells
    fixed = [0, ncells - 1, ncells // 2]
    return np.unique(np.concatenate([fixed, rng.integers(0, ncells, count)])).astype(np.int64)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_headline_operator_and_stage_sampled(precision):
    case = W.CONFIG_6D
    nd = (case.degree + 1) ** case.d
    ncells = int(np.prod(case.cells))
    S = gpu_solver(case, precision)
    P = oracle_problem(case)
    g = torch.Generator(device="cuda")
    g.manual_seed(6086)
    u = torch.randn(case.ndofs, dtype=torch.float64, device="cuda", generator=g)
    u_host = u.cpu().numpy()
    out = S.apply(u)
    cells = _sample_cells(ncells, seed=17)
    ref = P.apply_cells(u_host, cells).reshape(len(cells), nd)
    idx = (cells[:, None] * nd + np.arange(nd)[None, :]).reshape(-1)
    got = out[torch.from_numpy(idx).cuda()].double().cpu().numpy().reshape(len(cells), nd)
    tol = TOL_FP64 if precision == "fp64" else 2e-6
    assert rel_l2(got, ref) <= tol
    if precision == "fp64":
        assert rel_max(got, ref) <= tol
    # First RK stage on the same state: du = dt L(u), u1 = u + B_1 du.
    S.set_state(u)
    dt = S.stable_dt(case.cfl)
    S.rk_stage(0, dt)
    u1 = S.state_tensor()[torch.from_numpy(idx).cuda()].cpu().numpy().reshape(len(cells), nd)
    import oracle
    _, B, _ = oracle.lsrk45_coefficients()
    want = u_host[idx].reshape(len(cells), nd) + B[0] * (dt * ref)
    assert rel_l2(u1 - u_host[idx].reshape(len(cells), nd),
                  want - u_host[idx].reshape(len(cells), nd)) <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_headline_full_step_stage_by_stage_sampled(precision):
    # The five stages of one step at the headline size, launched as the
    # benchmark launches them (first-stage, general and last-stage kernel
    # variants). The increment is local to a cell, so the sampled cells'
    # du and u can be followed exactly: after each stage the oracle
    # evaluates L(u_s) on the samples from the full device state.
    import oracle
    A, B, _ = oracle.lsrk45_coefficients()
    case = W.CONFIG_6D
    nd = (case.degree + 1) ** case.d
    ncells = int(np.prod(case.cells))
    S = gpu_solver(case, precision)
    P = oracle_problem(case)
    g = torch.Generator(device="cuda")
    g.manual_seed(2020)
    u = torch.randn(case.ndofs, dtype=torch.float64, device="cuda", generator=g)
    S.set_state(u)
    del u
    dt = S.stable_dt(case.cfl)
    cells = _sample_cells(ncells, seed=29, count=12)
    idx = (cells[:, None] * nd + np.arange(nd)[None, :]).reshape(-1)
    idx_t = torch.from_numpy(idx).cuda()
    host = np.empty(case.ndofs)
    du = np.zeros(len(idx))
    tol = TOL_FP64 if precision == "fp64" else 5e-6  # FP32 increments, chained
    for st in range(5):
        host[:] = S.state_tensor().cpu().numpy()
        us = host[idx]
        L = P.apply_cells(host, cells)
        du = A[st] * du + dt * L
        S.rk_stage(st, dt)
        got = S.state_tensor()[idx_t].cpu().numpy()
        assert rel_l2(got - us, B[st] * du) <= tol, st
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_headline_gauss_legendre_operator_sampled(precision):
    # The 6D degree-3 Gauss-Legendre kernel at the headline size.
    case = W.CONFIG_6D
    nd = (case.degree + 1) ** case.d
    ncells = int(np.prod(case.cells))
    S = gpu_solver(case, precision)
    S.set_quadrature("gauss_legendre")
    P = oracle_problem(case)
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    u = torch.randn(case.ndofs, dtype=torch.float64, device="cuda", generator=g)
    out = S.apply(u)
    cells = _sample_cells(ncells, seed=31, count=6)
    ref = P.apply_cells(u.cpu().numpy(), cells, mode=2).reshape(len(cells), nd)
    idx = (cells[:, None] * nd + np.arange(nd)[None, :]).reshape(-1)
    got = out[torch.from_numpy(idx).cuda()].double().cpu().numpy().reshape(len(cells), nd)
    tol = TOL_FP64 if precision == "fp64" else 5e-6
    assert rel_l2(got, ref) <= tol
    if precision == "fp64":
        assert rel_max(got, ref) <= tol
    S.close()


def _random_state_on(S, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    u = torch.randn(S.ndofs, dtype=torch.float64, device="cuda", generator=g)
    S.set_state(u)
    return u


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("quadrature", ["gauss_lobatto", "gauss_legendre"])
def test_headline_mapped_cells_sampled(quadrature, precision):
    # The 6D degree-3 kernels on deformed configuration cells at the
    # headline size, in the benchmark's launch configuration (collocation:
    # stage_k3m_kernel, always one slab per XCD; Gauss-Legendre:
    # stage_k3mg_kernel): the operator on sampled cells against the
    # oracle's mapped weak form (mode 0 collocation, mode 2 Gauss), and in
    # FP64 one whole step stage by stage.
    import oracle
    case = W.CONFIG_6D
    eps = 0.02
    mode = 0 if quadrature == "gauss_lobatto" else 2
    S = gpu_solver(case, precision)
    if quadrature == "gauss_legendre":
        S.set_quadrature(quadrature)
    S.set_mapping(eps)
    S.set_field_sine(case.amp)
    assert S.get_plan()["kernel"] == 1
    P = oracle.Problem(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
                       field="phase", sine_amp=case.amp, map_eps=eps)
    u = _random_state_on(S, 4242 + mode)
    nd = (case.degree + 1) ** case.d
    cells = sample_cells(S.ndofs // nd, seed=37 + mode, count=5)
    out = S.apply(u)
    ref = P.apply_cells(u.cpu().numpy(), cells, mode=mode).reshape(len(cells), nd)
    idx = (cells[:, None] * nd + np.arange(nd)[None, :]).reshape(-1)
    got = out[torch.from_numpy(idx).cuda()].double().cpu().numpy().reshape(len(cells), nd)
    del out, u
    tol = TOL_FP64 if precision == "fp64" else 5e-6
    assert rel_l2(got, ref) <= tol
    if precision == "fp64":
        assert rel_max(got, ref) <= tol
        dt = S.stable_dt(case.cfl)
        stages_sampled(S, lambda host: P, cells[:4], dt, TOL_FP64, mode=mode)
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_headline_vlasov_poisson_stages_sampled(precision):
    # The self-consistent field at the headline size: the first stage of a
    # step takes the density from the state, the later ones from the
    # velocity moments the previous stage kernel wrote with its output. After
    # each stage the oracle computes the density and field of the full
    # device state (Sec. 6 steps 1-3) and the operator on sampled cells.
    import oracle
    case = W.landau_case("landau_6d_8^6_k3", 3, [8] * 6, 3, 1, modes=4)
    S = gpu_solver(case, precision)
    assert S.get_plan()["kernel"] == 1
    S.init_state(case.ic, list(case.ic_params))
    # a seeded perturbation on top of the Landau state (density of full
    # entropy in every velocity cell)
    g = torch.Generator(device="cuda")
    g.manual_seed(808)
    st = S.state_tensor()
    st += 1e-3 * torch.randn(S.ndofs, dtype=torch.float64, device="cuda", generator=g)
    del st
    vp = oracle.VlasovPoisson(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree,
                              case.modes)
    nd = (case.degree + 1) ** case.d
    cells = sample_cells(S.ndofs // nd, seed=55, count=10)
    dt = S.stable_dt(case.cfl)
    tol = TOL_FP64 if precision == "fp64" else 5e-6
    worst = stages_sampled(S, vp.advection, cells, dt, tol)
    print("vlasov-poisson 8^6 stages: worst rel-L2 %.3e (%s)" % (worst, precision))
    S.close()
