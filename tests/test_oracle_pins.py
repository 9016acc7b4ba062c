"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
not by the oracle itself (closed forms, invariants, exact solutions, brute
force). A plausible mistake anywhere in the oracle (a dropped face term, a
wrong sign, a wrong neighbour, a transposed derivative matrix, a wrong RK
coefficient) fails at least one of these.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle_helpers import (butcher_from_2n, cell_axis, golden_gl, golden_lines,
                            golden_lsrk, grid_view, integrate, node_axis,
                            weights_view)

RNG = np.random.default_rng(20020811)


# --------------------------------------------------------------------------
# 1D rule (Sec. 2.3 nodes, Sec. 2.5 Gauss-Lobatto quadrature)
# --------------------------------------------------------------------------

def test_gl_rule_matches_closed_forms():
    for k, (xi_ref, w_ref) in golden_gl().items():
        xi, w = oracle.gl_rule(k)
        np.testing.assert_allclose(xi, xi_ref, rtol=0, atol=2e-16 * 4)
        np.testing.assert_allclose(w, w_ref, rtol=0, atol=2e-16 * 4)


@pytest.mark.parametrize("k", range(1, 9))
def test_gl_rule_exact_to_degree_2k_minus_1_only(k):
    xi, w = oracle.gl_rule(k)
    assert abs(w.sum() - 1.0) < 1e-15
    for p in range(0, 2 * k):
        assert abs((w * xi ** p).sum() - 1.0 / (p + 1)) < 1e-14, p
    # Gauss-Lobatto with k+1 points is not exact for degree 2k (Sec. 2.5).
    assert abs((w * xi ** (2 * k)).sum() - 1.0 / (2 * k + 1)) > 1e-10


@pytest.mark.parametrize("k", range(1, 7))
def test_lagrange_basis_cardinal_and_derivative_exact(k):
    xi, _ = oracle.gl_rule(k)
    for m in range(k + 1):
        for q in range(k + 1):
            assert oracle.lagrange(k, xi, m, xi[q]) == (1.0 if m == q else 0.0)
    # Differentiating the interpolant of any degree-<=k polynomial is exact.
    for _ in range(3):
        coef = RNG.standard_normal(k + 1)
        dcoef = np.polyder(coef)
        for x in RNG.uniform(0, 1, 4):
            interp = sum(np.polyval(coef, xi[m]) * oracle.lagrange(k, xi, m, x) for m in range(k + 1))
            deriv = sum(np.polyval(coef, xi[m]) * oracle.lagrange_deriv(k, xi, m, x) for m in range(k + 1))
            assert abs(interp - np.polyval(coef, x)) < 1e-12
            assert abs(deriv - np.polyval(dcoef, x)) < 1e-10 * max(1, abs(np.polyval(dcoef, x)))


def test_dofs_per_cell_match_paper_table():
    splits = {2: (1, 1), 3: (2, 1), 4: (2, 2), 5: (3, 2), 6: (3, 3)}
    for line in golden_lines("dofs_per_cell.txt"):
        k, d, nd = map(int, line.split())
        dx, dv = splits[d]
        P = oracle.Problem(dx, dv, [1] * d, [0] * d, [1] * d, k, field="constant", a=[1] * d)
        assert P.ndofs == nd
        P2 = oracle.Problem(dx, dv, [2, 3] + [1] * (d - 2), [0] * d, [1] * d, k,
                            field="constant", a=[1] * d)
        assert P2.ndofs == 6 * nd  # N = |C| (k+1)^d, Sec. 2.3


# --------------------------------------------------------------------------
# Runge-Kutta scheme (Sec. 5.4)
# --------------------------------------------------------------------------

def test_lsrk_coefficients_are_the_published_ones():
    A, B, C = oracle.lsrk45_coefficients()
    gA, gB, gC = golden_lsrk()
    np.testing.assert_allclose(A, [float(x) for x in gA], rtol=1e-16, atol=0)
    np.testing.assert_allclose(B, [float(x) for x in gB], rtol=1e-16, atol=0)
    np.testing.assert_allclose(C, [float(x) for x in gC], rtol=1e-16, atol=0)


def test_lsrk_scheme_has_order_four():
    A, B, C = golden_lsrk()
    a, b, c = butcher_from_2n(A, B)
    S = len(b)
    one = [Fraction(1)] * S

    def mv(M, v):
        return [sum(M[i][j] * v[j] for j in range(S)) for i in range(S)]

    def dot(x, y):
        return sum(p * q for p, q in zip(x, y))

    Ac = mv(a, c)
    conds = [
        (dot(b, one), Fraction(1)),
        (dot(b, c), Fraction(1, 2)),
        (dot(b, [x * x for x in c]), Fraction(1, 3)),
        (dot(b, Ac), Fraction(1, 6)),
        (dot(b, [x ** 3 for x in c]), Fraction(1, 4)),
        (dot(b, [x * y for x, y in zip(c, Ac)]), Fraction(1, 8)),
        (dot(b, mv(a, [x * x for x in c])), Fraction(1, 12)),
        (dot(b, mv(a, Ac)), Fraction(1, 24)),
    ]
    for got, want in conds:
        assert abs(float(got - want)) < 1e-15
    # The stage times of the published C are the row sums of the tableau.
    for ci, Ci in zip(c, C):
        assert abs(float(ci - Ci)) < 1e-15


def _dense(P, mode=1):
    N = P.ndofs
    Lmat = np.zeros((N, N))
    e = np.zeros(N)
    for col in range(N):
        e[:] = 0
        e[col] = 1
        Lmat[:, col] = P.apply(e, mode)
    return Lmat


@pytest.mark.parametrize("field", ["constant", "phase"])
def test_rk_step_is_the_scheme_stability_polynomial(field):
    # One step of any 5-stage explicit RK on a linear ODE u' = L u is
    # R(dt L) u with R(z) = sum_m z^m b^T a^(m-1) 1; for order 4 the first
    # five coefficients are 1/m!.
    if field == "constant":
        P = oracle.Problem(1, 1, [3, 2], [0, 0], [1, 1], 2, field="constant", a=[0.7, -0.4])
    else:
        P = oracle.Problem(1, 1, [3, 2], [0, -3], [1, 3], 2, field="phase")
    Lmat = _dense(P)
    A, B, _ = golden_lsrk()
    a, b, _ = butcher_from_2n(A, B)
    S = len(b)
    coeffs = [Fraction(1)]
    vec = [Fraction(1)] * S
    for m in range(1, S + 1):
        coeffs.append(sum(bi * vi for bi, vi in zip(b, vec)))
        vec = [sum(a[i][j] * vec[j] for j in range(S)) for i in range(S)]
    for m, fact in enumerate([1, 1, 2, 6, 24]):
        assert abs(float(coeffs[m]) - 1.0 / fact) < 1e-15
    dt = P.stable_dt(0.9)
    u0 = RNG.standard_normal(P.ndofs)
    want = np.zeros_like(u0)
    term = u0.copy()
    for m in range(S + 1):
        want += float(coeffs[m]) * term
        term = dt * (Lmat @ term)
    got = P.rk_steps(u0, dt, 1)
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)


# --------------------------------------------------------------------------
# Operator (Sec. 1.3 weak form, Algorithm 2)
# --------------------------------------------------------------------------

CASES = [
    # dx, dv, k, cells, field
    (1, 1, 1, [3, 4], "constant"),
    (1, 1, 3, [4, 3], "phase"),
    (1, 1, 5, [2, 3], "constant"),
    (2, 1, 2, [3, 2, 2], "constant"),
    (2, 1, 4, [2, 2, 3], "constant"),
    (2, 2, 3, [2, 3, 2, 2], "phase"),
    (2, 2, 2, [3, 2, 2, 3], "constant"),
    (3, 2, 2, [2, 2, 1, 2, 3], "constant"),
    (3, 3, 1, [2, 1, 2, 2, 1, 3], "phase"),
    (3, 3, 2, [1, 2, 1, 1, 2, 1], "constant"),
]


def make(dx, dv, k, cells, field, seed=0):
    rng = np.random.default_rng(seed)
    d = dx + dv
    if field == "constant":
        a = rng.uniform(-1, 1, d)
        lo = rng.uniform(-1, 0, d)
        hi = lo + rng.uniform(0.5, 2, d)
        return oracle.Problem(dx, dv, cells, lo, hi, k, field="constant", a=a)
    lo = [0.0] * dx + [-6.0] * dv
    hi = [1.0] * dx + [6.0] * dv
    return oracle.Problem(dx, dv, cells, lo, hi, k, field="phase", sine_amp=0.3)


@pytest.mark.parametrize("case", CASES)
def test_full_basis_equals_zero_skipping(case):
    P = make(*case)
    u = RNG.standard_normal(P.ndofs)
    full = P.apply(u, mode=0)
    skip = P.apply(u, mode=1)
    assert np.linalg.norm(full - skip) <= 1e-13 * np.linalg.norm(skip)


@pytest.mark.parametrize("case", CASES)
def test_mass_is_conserved(case):
    # Summing the weak form over all test functions (sum_i phi_i = 1): the
    # volume term vanishes and the fluxes of each interior face cancel.
    P = make(*case)
    u = RNG.standard_normal(P.ndofs)
    L = P.apply(u)
    assert abs(integrate(P, L)) <= 1e-13 * integrate(P, np.abs(L))


@pytest.mark.parametrize("case", CASES)
def test_constants_are_steady(case):
    # div(a) = 0 for both fields, so f = 1 is a steady state.
    P = make(*case)
    L = P.apply(np.ones(P.ndofs))
    scale = sum(abs(P.field.a[j]) / ((P.hi[j] - P.lo[j]) / P.cells[j]) for j in range(P.d)) + 10
    assert np.abs(L).max() <= 1e-12 * scale * (P.k + 1) ** 2


def _field_at_nodes(P):
    """a_j at every DoF, computed from the node coordinates (closed forms of
    the two fields, not the oracle's table lookup)."""
    X = P.node_coords()
    if P.field.kind == 0:
        return np.tile(np.array([P.field.a[j] for j in range(P.d)]), (P.ndofs, 1))
    a = np.empty_like(X)
    a[:, : P.dim_x] = X[:, P.dim_x:]
    span = np.array(P.hi[: P.dim_x]) - np.array(P.lo[: P.dim_x])
    sine = np.sin(2 * np.pi * (X[:, : P.dim_x] - np.array(P.lo[: P.dim_x])) / span)
    a[:, P.dim_x:] = P.field.sign * P.sine_amp * sine
    return a


@pytest.mark.parametrize("case", CASES)
def test_energy_identity(case):
    # For fields with a_j independent of x_j (both fields here) the upwind
    # scheme satisfies 2 u^T W L(u) = - sum_faces W_f |a.n| [[u]]^2, the
    # discrete analogue of d/dt ||f||^2 = -(upwind jump dissipation).
    P = make(*case)
    u = RNG.standard_normal(P.ndofs)
    L = P.apply(u)
    xi, w = oracle.gl_rule(P.k)
    d, n = P.d, P.n
    h = [(P.hi[j] - P.lo[j]) / P.cells[j] for j in range(d)]
    lhs = 2 * integrate(P, u * L)
    a = _field_at_nodes(P)
    g = grid_view(u, P.cells, n)
    rhs = 0.0
    for j in range(d):
        aj = grid_view(a[:, j], P.cells, n)
        own = np.take(g, n - 1, axis=node_axis(d, j))
        nbr = np.take(np.roll(g, -1, axis=cell_axis(d, j)), 0, axis=node_axis(d, j))
        an = np.take(aj, n - 1, axis=node_axis(d, j))
        hf = [h[m] if m != j else 1.0 for m in range(d)]
        wf = weights_view(w, hf, d)
        Wf = np.take(wf, n - 1, axis=d - 1 - j) / w[n - 1]
        rhs -= float((Wf * np.abs(an) * (own - nbr) ** 2).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    assert lhs <= 1e-12 * abs(rhs)


# Small meshes of every (dx, dv) split for the dense checks (at most ~650
# DoFs, so every case runs).
DENSE_CASES = [
    (1, 1, 1, [3, 4], "constant"),
    (1, 1, 3, [4, 3], "phase"),
    (1, 1, 5, [2, 3], "constant"),
    (2, 1, 2, [3, 2, 2], "constant"),
    (2, 1, 4, [1, 2, 1], "constant"),
    (2, 2, 1, [2, 3, 2, 2], "phase"),
    (2, 2, 2, [2, 1, 2, 2], "constant"),
    (3, 2, 1, [2, 1, 2, 2, 1], "constant"),
    (3, 3, 1, [1, 2, 1, 1, 2, 1], "phase"),
]


@pytest.mark.parametrize("case", DENSE_CASES)
def test_dense_operator_spectrum_is_stable(case):
    P = make(*case)
    assert P.ndofs <= 700
    Lm = _dense(P)
    ev = np.linalg.eigvals(Lm)
    rho = np.abs(ev).max()
    assert ev.real.max() <= 1e-10 * rho
    # W L + (W L)^T is negative semidefinite (energy stability).
    Wvec = integrate_weights(P)
    S = Wvec[:, None] * Lm
    S = S + S.T
    assert np.linalg.eigvalsh(S).max() <= 1e-10 * np.abs(S).max()


@pytest.mark.parametrize("k,rho_want", [(2, 5.420), (3, 9.648), (4, 14.730), (5, 20.598)])
def test_dense_1d_upwind_spectral_radius(k, rho_want):
    # The periodic 1D upwind operator of Sec. 1.3 with N = 16 cells, a = 1,
    # h = 1 has spectral radius 5.420, 9.648, 14.730, 20.598 for k = 2..5
    # (values computed independently of this oracle). The oracle works in
    # d >= 2: with a = (1, 0) on 16 x 1 cells (x-width 1 each) the operator
    # is the 1D one acting on each of the k+1 velocity node lines, so its
    # spectrum is the 1D spectrum, each eigenvalue k+1 times.
    P = oracle.Problem(1, 1, [16, 1], [0.0, 0.0], [16.0, 1.0], k, field="constant",
                       a=[1.0, 0.0])
    ev = np.linalg.eigvals(_dense(P))
    rho = np.abs(ev).max()
    assert abs(rho - rho_want) <= 5e-4 * rho_want
    assert ev.real.max() <= 1e-10 * rho
    # The radius is attained on the negative real axis (the most damped,
    # cell-scale mode); a central flux would put the spectrum on the
    # imaginary axis instead.
    assert abs(ev.real.min() + rho_want) <= 5e-4 * rho_want


def integrate_weights(P):
    xi, w = oracle.gl_rule(P.k)
    h = [(P.hi[j] - P.lo[j]) / P.cells[j] for j in range(P.d)]
    Wn = weights_view(w, h, P.d)  # node axes in (n_d..n_1) order
    return np.tile(Wn.reshape(-1), P.ncells)


@pytest.mark.parametrize("dx,dv,k,field", [(1, 1, 3, "constant"), (1, 1, 5, "phase"),
                                           (2, 1, 2, "constant"), (2, 2, 2, "phase"),
                                           (2, 2, 3, "constant")])
def test_polynomials_are_differentiated_exactly(dx, dv, k, field):
    # For u a tensor polynomial of degree <= k per variable (continuous, so
    # all interior jumps vanish), M^{-1}A(u) = -a . grad u at the nodes of
    # every cell that does not touch the periodic seam.
    d = dx + dv
    cells = [3] * d
    P = make(dx, dv, k, cells, field, seed=3)
    X = P.node_coords()
    rng = np.random.default_rng(5)
    coefs = [rng.standard_normal(k + 1) for _ in range(d)]
    vals = np.stack([np.polyval(c, X[:, j]) for j, c in enumerate(coefs)], 1)
    ders = np.stack([np.polyval(np.polyder(c), X[:, j]) for j, c in enumerate(coefs)], 1)
    u = np.prod(vals, 1)
    grad = np.empty_like(vals)
    for j in range(d):
        grad[:, j] = ders[:, j] * np.prod(np.delete(vals, j, 1), 1)
    a = _field_at_nodes(P)
    want = -(a * grad).sum(1)
    L = P.apply(u)
    g_got = grid_view(L, cells, P.n)
    g_want = grid_view(want, cells, P.n)
    inner = tuple([slice(None)] * 0 + [slice(1, 2)] * d)
    assert np.abs(g_got[inner] - g_want[inner]).max() <= 1e-10 * np.abs(g_want).max()


def test_upwind_uses_only_the_inflow_neighbour():
    # a = (+1, 0): the flux at a cell's right face is its own trace (outflow),
    # at its left face the left neighbour's trace (inflow).
    P = oracle.Problem(1, 1, [4, 3], [0, 0], [1, 1], 3, field="constant", a=[1.0, 0.0])
    nd = P.n ** 2
    u = RNG.standard_normal(P.ndofs)
    base = P.apply(u)
    c = 1 + 4 * 1  # cell (1,1)
    down = u.copy()
    down[(c + 1) * nd:(c + 2) * nd] += 1.0  # cell (2,1): downwind
    assert np.array_equal(P.apply(down)[c * nd:(c + 1) * nd], base[c * nd:(c + 1) * nd])
    up = u.copy()
    up[(c - 1) * nd:c * nd] += 1.0  # cell (0,1): upwind
    diff = P.apply(up)[c * nd:(c + 1) * nd] - base[c * nd:(c + 1) * nd]
    assert np.abs(diff).max() > 1.0
    # Only the left-face nodes (i_1 = 0) of the cell feel the inflow.
    diff = diff.reshape(P.n, P.n)
    assert np.abs(diff[:, 1:]).max() == 0.0


@pytest.mark.parametrize("dx,dv,k", [(1, 1, 3), (2, 1, 2), (2, 2, 2)])
def test_cyclic_shift_commutes(dx, dv, k):
    # Constant field on a periodic box: L commutes with shifting cells.
    d = dx + dv
    cells = [3, 4, 2, 3][:d]
    P = make(dx, dv, k, cells, "constant", seed=11)
    u = RNG.standard_normal(P.ndofs)
    L = P.apply(u)
    for j in range(d):
        su = np.roll(grid_view(u, cells, P.n), 1, axis=cell_axis(d, j)).reshape(-1)
        sL = np.roll(grid_view(L, cells, P.n), 1, axis=cell_axis(d, j)).reshape(-1)
        assert np.abs(P.apply(su) - sL).max() <= 1e-13 * np.abs(L).max()


@pytest.mark.parametrize("j", [0, 1])
def test_reflection_symmetry_phase_space(j):
    # x box [0,1], velocity box symmetric about 0, E_j = amp sin(2 pi x_j):
    # the joint reflection (x_j, v_j) -> (1 - x_j, -v_j) maps the equation
    # df/dt + v . grad_x f + E . grad_v f = 0 to itself (v_j d/dx_j and
    # E_j d/dv_j both keep their sign), and maps the mesh and its nodes to
    # themselves, so the discrete operator commutes with it: L(R u) = R L(u).
    # A wrong upwind side, neighbour direction or velocity sign breaks this.
    P = oracle.Problem(2, 2, [3, 2, 4, 3], [0, 0, -6, -6], [1, 1, 6, 6], 2, field="phase",
                       sine_amp=0.3)
    d = P.d
    u = RNG.standard_normal(P.ndofs)
    L = P.apply(u)

    def R(x):
        g = grid_view(x, P.cells, P.n)
        for m in (j, P.dim_x + j):
            g = np.flip(np.flip(g, axis=cell_axis(d, m)), axis=node_axis(d, m))
        return g.reshape(-1)

    assert np.abs(P.apply(R(u)) - R(L)).max() <= 1e-12 * np.abs(L).max()
    # Reflecting x_j alone is not a symmetry (v_j d/dx_j changes sign).
    def Rx(x):
        g = grid_view(x, P.cells, P.n)
        g = np.flip(np.flip(g, axis=cell_axis(d, j)), axis=node_axis(d, j))
        return g.reshape(-1)

    assert np.abs(P.apply(Rx(u)) - Rx(L)).max() > 1e-3 * np.abs(L).max()


@pytest.mark.parametrize("j", [0, 1, 2])
def test_single_cell_is_its_own_periodic_neighbour(j):
    # A mesh with one cell in dim j equals a mesh with two cells in dim j and
    # the state repeated: both represent the same periodic function.
    dx, dv, k = 2, 1, 2
    d = 3
    cells1 = [2, 3, 2]
    cells1[j] = 1
    cells2 = list(cells1)
    cells2[j] = 2
    lo = [0.0, 0.0, -1.0]
    hi1 = [1.0, 1.0, 1.0]
    hi2 = list(hi1)
    hi2[j] = lo[j] + 2 * (hi1[j] - lo[j])
    a = [0.6, -0.8, 0.3]
    P1 = oracle.Problem(dx, dv, cells1, lo, hi1, k, field="constant", a=a)
    P2 = oracle.Problem(dx, dv, cells2, lo, hi2, k, field="constant", a=a)
    u1 = RNG.standard_normal(P1.ndofs)
    g1 = grid_view(u1, cells1, P1.n)
    u2 = np.concatenate([g1, g1], axis=cell_axis(d, j)).reshape(-1)
    L1 = P1.apply(u1)
    L2 = grid_view(P2.apply(u2), cells2, P2.n)
    first = np.take(L2, [0], axis=cell_axis(d, j)).reshape(-1)
    np.testing.assert_allclose(first, L1, rtol=0, atol=1e-13 * np.abs(L1).max())


# --------------------------------------------------------------------------
# Exact solutions, initial states, diagnostics, time step
# --------------------------------------------------------------------------

def _config1(N, k=3):
    return oracle.Problem(1, 1, [N, N], [0, 0], [1, 1], k, field="constant", a=[1.0, 0.5])


def _rel_err_vs_exact(P, T, dt, nsteps):
    u = P.rk_steps(P.init_state(0), dt, nsteps)
    X = P.node_coords()
    ex = np.sin(2 * np.pi * (X[:, 0] - 1.0 * T)) * np.sin(2 * np.pi * (X[:, 1] - 0.5 * T))
    return np.sqrt(integrate(P, (u - ex) ** 2) / integrate(P, ex ** 2))


def test_constant_advection_matches_exact_solution_with_order_k_plus_1():
    # Translation u0(x - a t) is the exact solution for constant a (Sec. 1.2).
    errs = []
    for N in (8, 16, 32):
        P = _config1(N)
        dt0 = P.stable_dt(0.2)
        nsteps = int(np.ceil(0.25 / dt0))
        errs.append(_rel_err_vs_exact(P, 0.25, 0.25 / nsteps, nsteps))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 1e-5
    assert rates.min() > 3.7  # DG of degree k converges at order k+1 = 4


def test_config_2d_100_steps_error_and_invariants():
    P = _config1(16)
    dt = P.stable_dt(0.2)
    assert abs(dt - 0.2 / (7 * (16 + 8))) < 1e-18
    u0 = P.init_state(0)
    u = P.rk_steps(u0, dt, 100)
    err = _rel_err_vs_exact(P, 100 * dt, dt, 100)
    # The discretization error of this configuration at t = 100 dt = 0.11905,
    # computed independently of this oracle (a separate 1D-per-direction
    # nodal DG script with the same scheme): 3.264e-5.
    assert abs(err - 3.264e-5) <= 0.01 * 3.264e-5
    m0, e0 = P.diagnostics(u0)
    m1, e1 = P.diagnostics(u)
    assert abs(m1 - m0) < 1e-15
    assert e1 <= e0 * (1 + 1e-14)


def test_energy_never_increases_over_steps():
    P = oracle.Problem(1, 1, [6, 5], [0, -6], [1, 6], 3, field="phase")
    u = P.init_state(1, [0.01])
    u = u + 0.1 * RNG.standard_normal(P.ndofs)
    dt = P.stable_dt(0.2)
    e_prev = P.diagnostics(u)[1]
    for _ in range(5):
        u = P.rk_steps(u, dt, 1)
        e = P.diagnostics(u)[1]
        assert e <= e_prev * (1 + 1e-14)
        e_prev = e


def test_node_coordinates_and_initial_states():
    P = oracle.Problem(2, 2, [2, 3, 2, 2], [0, 0, -6, -6], [1, 1, 6, 6], 3, field="phase")
    X = P.node_coords()
    xi_ref, _ = golden_gl()[3]
    g = [grid_view(X[:, j], P.cells, P.n) for j in range(P.d)]
    for j in range(P.d):
        h = (P.hi[j] - P.lo[j]) / P.cells[j]
        idx_c = np.arange(P.cells[j])
        idx_n = np.arange(P.n)
        shape_c = [1] * (2 * P.d)
        shape_c[cell_axis(P.d, j)] = P.cells[j]
        shape_n = [1] * (2 * P.d)
        shape_n[node_axis(P.d, j)] = P.n
        want = P.lo[j] + (idx_c.reshape(shape_c) + xi_ref[idx_n].reshape(shape_n)) * h
        np.testing.assert_allclose(g[j], np.broadcast_to(want, g[j].shape), rtol=0, atol=1e-14)
    u1 = P.init_state(1, [0.01])
    v2 = (X[:, 2:] ** 2).sum(1)
    want1 = (1 + 0.01 * np.cos(2 * np.pi * X[:, 0])) * np.exp(-v2 / 2) / (2 * np.pi)
    np.testing.assert_allclose(u1, want1, rtol=1e-14, atol=1e-300)
    u0 = P.init_state(0)
    want0 = np.prod([np.sin(2 * np.pi * (X[:, j] - P.lo[j]) / (P.hi[j] - P.lo[j]))
                     for j in range(P.d)], axis=0)
    np.testing.assert_allclose(u0, want0, rtol=0, atol=1e-14)


def test_diagnostics_integrate_polynomials_exactly():
    k = 3
    P = oracle.Problem(1, 2, [2, 3, 2], [0, 0, -1], [2, 1, 1], k, field="constant",
                       a=[1, 1, 1])
    X = P.node_coords()
    # Degree 2k-1 = 5 per variable is integrated exactly by the GL rule.
    u = X[:, 0] ** 5 * (1 + X[:, 1] ** 2) * X[:, 2] ** 4
    exact = (2 ** 6 / 6) * (1 + 1 / 3) * (2 / 5)
    m, e = P.diagnostics(u)
    assert abs(m - exact) < 1e-12
    assert abs(e - integrate(P, u * u)) < 1e-12 * e


def test_stable_dt_phase_space_values():
    # Sec. 8c reading: dt = CFL / ((2k+1) sum_j max|a_j|/h_j). For the 6D
    # 8^6 configuration |v|max = 6 and |E|max = 0.1 sin(2 pi xi) at a node.
    P = oracle.Problem(3, 3, [8] * 6, [0, 0, 0, -6, -6, -6], [1, 1, 1, 6, 6, 6], 3,
                       field="phase", sine_amp=0.1)
    xi, _ = oracle.gl_rule(3)
    xs = (np.arange(8)[:, None] + xi[None, :]) / 8
    emax = 0.1 * np.abs(np.sin(2 * np.pi * xs)).max()
    want = 0.2 / (7 * (3 * 6 / (1 / 8) + 3 * emax / 1.5))
    assert abs(P.stable_dt(0.2) - want) < 1e-18


def test_rk_stage_by_stage_equals_rk_steps():
    # The per-stage entry (used to time one stage) composes to the same step,
    # bitwise.
    P = oracle.Problem(1, 1, [3, 4], [0, -6], [1, 6], 3, field="phase", sine_amp=0.2)
    u0 = RNG.standard_normal(P.ndofs)
    dt = P.stable_dt(0.2)
    u = u0.copy()
    du = np.full(P.ndofs, np.nan)  # stage 0 must not read it
    L = np.empty(P.ndofs)
    for _ in range(2):
        for st in range(5):
            P.rk_stage(u, du, L, dt, st)
    assert np.array_equal(u, P.rk_steps(u0, dt, 2))
