"""Pins of the oracle on mapped cells (the tensor-product mapping of Sec.
3.1/3.3 with a curved configuration mesh): with the deformation x_m = X_m +
eps L_m prod_k sin(2 pi (X_k - lo_k) / L_k) the weak form carries the
metric terms (contravariant flux |J| J^{-1} a, mass with |J|). Pinned by
what does not depend on the implementation: the general evaluation agrees
with the Kronecker-structured Gauss mode without a mapping, mass is
conserved with |J| computed here independently, constant advection
converges at order k+1 to the exact translated solution on the curved mesh,
and the operator depends continuously on eps."""
import numpy as np
import pytest

import oracle


def _problem(dx, cells, k, eps, a=None, field="constant", box=1.0):
    d = 2 * dx
    lo = [0.0] * d
    hi = [box] * d
    if field == "constant":
        return oracle.Problem(dx, dx, cells, lo, hi, k, field="constant", a=a, map_eps=eps)
    return oracle.Problem(dx, dx, cells, lo, [1.0] * dx + [3.0] * dx, k, field="phase",
                          sine_amp=0.3, map_eps=eps)


def _detJx(P, X):
    """det(dx/dX) of the deformation at box points X (n x d), by central
    differences of the mapping formula (step 1e-6, error ~1e-12)."""
    dx = P.dim_x
    L = np.array(P.hi[:dx]) - np.array(P.lo[:dx])

    def phi(Y):
        th = 2 * np.pi * (Y[:, :dx] - np.array(P.lo[:dx])) / L
        prod = np.prod(np.sin(th), axis=1)
        return Y[:, :dx] + P.map_eps * L[None, :] * prod[:, None]

    h = 1e-6
    J = np.zeros((len(X), dx, dx))
    for kk in range(dx):
        Xp, Xm = X.copy(), X.copy()
        Xp[:, kk] += h
        Xm[:, kk] -= h
        J[:, :, kk] = (phi(Xp) - phi(Xm)) / (2 * h)
    return np.linalg.det(J)


def _box_nodes(P):
    """Box (unmapped) coordinates of the nodes."""
    Q = oracle.Problem(P.dim_x, P.dim_v, P.cells, P.lo, P.hi, P.k, field="constant",
                       a=[0.0] * P.d)
    return Q.node_coords()


@pytest.mark.parametrize("dx,cells,k", [(1, [4, 3], 3), (2, [2, 3, 2, 1], 2)])
def test_general_gauss_evaluation_equals_kronecker_gauss_without_mapping(dx, cells, k):
    for field in ("constant", "phase"):
        P = _problem(dx, cells, k, 0.0, a=[0.7, -0.3, 0.4, 0.2][: 2 * dx], field=field)
        u = np.random.default_rng(1).standard_normal(P.ndofs)
        ref = P.apply(u, mode=2)
        got = P.apply(u, mode=3)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("dx,cells,k", [(1, [5, 4], 3), (2, [3, 2, 2, 2], 2)])
def test_mass_is_conserved_on_mapped_cells(mode, dx, cells, k):
    P = _problem(dx, cells, k, 0.04, field="phase")
    u = np.random.default_rng(2).standard_normal(P.ndofs)
    Lu = P.apply(u, mode=mode)
    n, d = k + 1, P.d
    xi, w = oracle.gl_rule(k)
    g, wg = oracle.gauss_rule(k)
    pts, wts = (xi, w) if mode == 0 else (g, wg)
    # reference weights and the quadrature points of every cell, box coords
    B = np.array([[oracle.lagrange(k, xi, m, x) for m in range(n)] for x in pts])
    h = (np.array(P.hi) - np.array(P.lo)) / np.array(P.cells)
    cells_mi = np.array(np.unravel_index(np.arange(P.ncells), P.cells[::-1])[::-1]).T
    nodes_mi = np.array(np.unravel_index(np.arange(n ** d), [n] * d)[::-1]).T
    total = 0.0
    Lc = Lu.reshape(P.ncells, -1)
    for c in range(P.ncells):
        X = np.array(P.lo) + (cells_mi[c][None, :] + pts[nodes_mi]) * h[None, :]
        W = np.prod(wts[nodes_mi], axis=1) * np.prod(h)
        # L(u) at the quadrature points: B along every dimension
        v = Lc[c].reshape([n] * d)  # axis order: dim d ... dim 1 (C order)
        for ax in range(d):
            v = np.moveaxis(np.tensordot(B, v, axes=([1], [ax])), 0, ax)
        total += np.sum(W * _detJx(P, X) * v.reshape(-1))
    scale = np.abs(Lu).max() * np.prod(np.array(P.hi) - np.array(P.lo))
    assert abs(total) < 1e-10 * scale


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("k", [2, 3])
def test_constant_advection_on_a_stretched_1d_mesh_converges_at_order_k_plus_1(mode, k):
    a, t_end = [1.0, 0.5], 0.1
    errs = []
    for N in (8, 16, 32):
        P = _problem(1, [N, N], k, 0.04, a=a)
        u0 = P.init_state(0)
        dt = P.stable_dt(0.2)
        steps = int(np.ceil(t_end / dt))
        u = P.rk_steps(u0, t_end / steps, steps, mode=mode)
        X = P.node_coords()
        ex = np.sin(2 * np.pi * (X[:, 0] - a[0] * t_end)) * np.sin(2 * np.pi * (X[:, 1] - a[1] * t_end))
        errs.append(np.sqrt(np.mean((u - ex) ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > k + 0.5 and rates.min() > k - 0.3, (errs, rates)


@pytest.mark.parametrize("mode", [0, 2])
def test_constant_advection_on_a_curved_2d_mesh_converges_at_order_k_plus_1(mode):
    # a v-independent wave on a curved 2D configuration mesh (one velocity
    # cell per dimension, a_v = 0): u = sin(2 pi x1) sin(2 pi x2) moves with
    # (1, 0.5) in physical coordinates.
    k, a, t_end = 2, [1.0, 0.5, 0.0, 0.0], 0.05
    errs = []
    for N in (8, 16, 32):
        P = _problem(2, [N, N, 1, 1], k, 0.04, a=a)
        X = P.node_coords()
        u0 = np.sin(2 * np.pi * X[:, 0]) * np.sin(2 * np.pi * X[:, 1])
        dt = P.stable_dt(0.2)
        steps = int(np.ceil(t_end / dt))
        u = P.rk_steps(u0, t_end / steps, steps, mode=mode)
        ex = np.sin(2 * np.pi * (X[:, 0] - a[0] * t_end)) * np.sin(2 * np.pi * (X[:, 1] - a[1] * t_end))
        errs.append(np.sqrt(np.mean((u - ex) ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > k + 0.5, (errs, rates)


def test_operator_is_continuous_in_eps_and_mode_1_refuses_a_mapping():
    u = np.random.default_rng(4).standard_normal(_problem(1, [4, 3], 2, 0.0, a=[1, 1]).ndofs)
    base = _problem(1, [4, 3], 2, 0.0, a=[1.0, 0.5]).apply(u, mode=0)
    d1 = np.abs(_problem(1, [4, 3], 2, 1e-3, a=[1.0, 0.5]).apply(u, mode=0) - base).max()
    d2 = np.abs(_problem(1, [4, 3], 2, 2e-3, a=[1.0, 0.5]).apply(u, mode=0) - base).max()
    assert 0 < d1 < d2 < 3 * d1
    with pytest.raises(RuntimeError):
        _problem(1, [4, 3], 2, 0.01, a=[1.0, 0.5]).apply(u, mode=1)
    with pytest.raises(ValueError):
        _problem(1, [4, 3], 2, 0.2, a=[1.0, 0.5])
