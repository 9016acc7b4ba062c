"""Pins of the oracle's Gauss-Legendre quadrature mode (mode 2; Sec. 2.5,
the paper's default rule): the 1D rule against closed forms and its exact
degree, and the whole operator against the exact Galerkin operator assembled
here independently from exactly integrated 1D polynomial matrices (every
integrand is a polynomial of degree <= 2k+1 per dimension for the fields
used, which k+1 Gauss points integrate exactly), plus invariants and
convergence for a field where exactness does not hold."""
import math
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "gauss_legendre.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, xe, we = line.split()
        env = {"sqrt": math.sqrt}
        rows.setdefault(int(n), []).append((eval(xe, env), eval(we, env)))
    return rows


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_gauss_rule_matches_closed_forms(n):
    g, w = oracle.gauss_rule(n - 1)
    ref = _golden()[n]
    np.testing.assert_allclose(g, [r[0] for r in ref], atol=1e-15)
    np.testing.assert_allclose(w, [r[1] for r in ref], atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_gauss_rule_degree_is_exactly_2n_minus_1(k):
    g, w = oracle.gauss_rule(k)
    n = k + 1
    for p in range(2 * n):
        assert abs(np.dot(w, g ** p) - 1.0 / (p + 1)) < 1e-14, p
    assert abs(np.dot(w, g ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12


# --- exact Galerkin operator, assembled independently ------------------------

def _one_d(k, weight=(1.0,)):
    """Exact reference-cell matrices with a polynomial weight w(xi) (power
    coefficients): G[a][b] = int l_a w l_b, K[i][b] = int l_i' w l_b over
    [0, 1], integrated by mpmath at 40 digits (its own quadrature, exact for
    these polynomials to that precision; a float power basis loses ~1e-11 at
    k = 5)."""
    import mpmath as mp
    mp.mp.dps = 40
    xi, _ = oracle.gl_rule(k)
    X = [mp.mpf(x) for x in xi]
    n = k + 1

    def l(m, x):
        v = mp.mpf(1)
        for r in range(n):
            if r != m:
                v *= (x - X[r]) / (X[m] - X[r])
        return v

    def dl(m, x):
        return mp.diff(lambda y: l(m, y), x)

    def wt(x):
        return sum(mp.mpf(c) * x ** e for e, c in enumerate(weight))

    G = np.array([[float(mp.quad(lambda x: l(a, x) * wt(x) * l(b, x), [0, 1]))
                   for b in range(n)] for a in range(n)])
    K = np.array([[float(mp.quad(lambda x: dl(i, x) * wt(x) * l(b, x), [0, 1]))
                   for b in range(n)] for i in range(n)])
    return G, K


def _adv_1d(k, C, sign, K):
    """Global 1D DG advection matrix per unit speed (volume K, upwind faces)
    on C periodic cells, index c * n + i, for a field of the given sign."""
    n = k + 1
    A = np.zeros((C * n, C * n))
    for c in range(C):
        A[c * n:(c + 1) * n, c * n:(c + 1) * n] += K
        if sign > 0:
            A[c * n + k, c * n + k] -= 1.0                      # outflow, right face
            A[c * n + 0, ((c - 1) % C) * n + k] += 1.0          # inflow from the left
        else:
            A[c * n + 0, c * n + 0] += 1.0                      # outflow, left face
            A[c * n + k, ((c + 1) % C) * n + 0] -= 1.0          # inflow from the right
    return A


def _perm(cells, k):
    """Canonical DoF index of each Kronecker index (dim d slowest, (c_j, i_j)
    per dim with c_j slow)."""
    d = len(cells)
    n = k + 1
    sizes = [c * n for c in cells]
    out = np.empty(int(np.prod(sizes)), dtype=np.int64)
    cs = np.cumprod([1] + list(cells[:-1]))
    for flat in range(len(out)):
        r = flat
        idx = []
        for j in reversed(range(d)):
            s = int(np.prod(sizes[:j]))
            idx.append(r // s)
            r %= s
        idx = idx[::-1]
        cell = sum((idx[j] // n) * cs[j] for j in range(d))
        node = sum((idx[j] % n) * n ** j for j in range(d))
        out[flat] = cell * n ** d + node
    return out


def _kron(mats):
    """Kronecker product with dim 1 fastest (mats[0] acts on dim 1)."""
    out = np.ones((1, 1))
    for m in mats:
        out = np.kron(m, out)
    return out


def _block(M, C, k):
    n = k + 1
    return np.kron(np.eye(C), M)


def exact_operator_constant(cells, lo, hi, k, a):
    d = len(cells)
    h = [(hi[j] - lo[j]) / cells[j] for j in range(d)]
    G, K = _one_d(k)
    mass = [h[j] * _block(G, cells[j], k) for j in range(d)]
    R = 0
    for j in range(d):
        if a[j] == 0:
            continue
        mats = list(mass)
        mats[j] = a[j] * _adv_1d(k, cells[j], np.sign(a[j]), K)
        R = R + _kron(mats)
    Mfull = _kron(mass)
    L = np.linalg.solve(Mfull, R)
    p = _perm(cells, k)
    out = np.zeros_like(L)
    out[np.ix_(p, p)] = L
    return out


def exact_operator_phase_2d(cells, lo, hi, k, E_cell):
    """a = (v, E(x)) in 1x + 1v with E affine in each x-cell (E_cell[c] =
    (E at the cell's left end, E at its right end)), E > 0, and velocity
    cells not straddling v = 0."""
    (Cx, Cv), n = cells, k + 1
    hx, hv = (hi[0] - lo[0]) / Cx, (hi[1] - lo[1]) / Cv
    G, K = _one_d(k)
    Mx = hx * _block(G, Cx, k)
    Mv = hv * _block(G, Cv, k)
    R = np.zeros((Cx * n * Cv * n,) * 2)
    # x-transport: speed v, upwind side by the sign of the velocity cell
    for cv in range(Cv):
        v0 = lo[1] + cv * hv
        assert v0 >= 0 or v0 + hv <= 0
        sgn = 1.0 if v0 >= 0 else -1.0
        Gv, _ = _one_d(k, weight=(v0, hv))                  # int l_a (v0 + hv xi) l_b
        Pv = np.zeros((Cv * n, Cv * n))
        Pv[cv * n:(cv + 1) * n, cv * n:(cv + 1) * n] = hv * Gv
        R += _kron([_adv_1d(k, Cx, sgn, K), Pv])
    # v-transport: speed E(x) > 0 (affine per x-cell)
    Ax = np.zeros((Cx * n, Cx * n))
    for cx in range(Cx):
        e0, e1 = E_cell[cx]
        Gx, _ = _one_d(k, weight=(e0, e1 - e0))             # int l_a E l_b
        Ax[cx * n:(cx + 1) * n, cx * n:(cx + 1) * n] = hx * Gx
    R += _kron([Ax, _adv_1d(k, Cv, 1.0, K)])
    L = np.linalg.solve(_kron([Mx, Mv]), R)
    p = _perm(cells, k)
    out = np.zeros_like(L)
    out[np.ix_(p, p)] = L
    return out


def _dense(P, mode):
    N = P.ndofs
    cols = [P.apply(e, mode=mode) for e in np.eye(N)]
    return np.array(cols).T


@pytest.mark.parametrize("cells,k,a", [([4, 3], 2, [0.7, -0.4]), ([3, 2], 3, [-1.1, 0.3]),
                                       ([2, 3], 5, [0.5, 0.9]), ([2, 1, 2], 2, [0.3, -0.6, 0.8]),
                                       ([2, 2, 1, 2], 1, [0.4, 0.0, -0.7, 0.2])])
def test_gauss_mode_is_the_exact_galerkin_operator_constant_field(cells, k, a):
    d = len(cells)
    lo = [0.1 * j for j in range(d)]
    hi = [l + 1.0 + 0.3 * j for j, l in enumerate(lo)]
    dx = (d + 1) // 2
    P = oracle.Problem(dx, d - dx, cells, lo, hi, k, field="constant", a=a)
    ref = exact_operator_constant(cells, lo, hi, k, a)
    got = _dense(P, 2)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
    # collocation (modes 0/1) integrates the mass matrix inexactly: it differs
    assert np.abs(_dense(P, 1) - ref).max() > 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_gauss_mode_is_the_exact_galerkin_operator_phase_space(k):
    cells, lo, hi = [3, 4], [0.0, -2.0], [1.5, 2.0]
    n = k + 1
    xi, _ = oracle.gl_rule(k)
    rng = np.random.default_rng(k)
    E_cell = [(1.0 + rng.uniform(0, 1), 1.0 + rng.uniform(0, 1)) for _ in range(cells[0])]
    # the E table at the x-nodes of the affine-per-cell field
    E = np.array([e0 + (e1 - e0) * xi[q] for (e0, e1) in E_cell for q in range(n)])
    P = oracle.Problem(1, 1, cells, lo, hi, k, field="phase", E=E, sign=1.0)
    ref = exact_operator_phase_2d(cells, lo, hi, k, E_cell)
    got = _dense(P, 2)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_gauss_mode_invariants_for_a_sine_field():
    # E = 0.3 sin(2 pi x) is not a polynomial: no exactness, but the
    # discrete mass (with the exact Gauss mass matrix) is conserved and
    # constants are steady.
    for dx, cells, k in [(1, [5, 4], 3), (2, [2, 3, 2, 2], 2)]:
        P = oracle.Problem(dx, dx, cells, [0.0] * dx + [-3.0] * dx, [1.0] * dx + [3.0] * dx, k,
                           field="phase", sine_amp=0.3)
        assert np.abs(P.apply(np.ones(P.ndofs), mode=2)).max() < 1e-12
        u = np.random.default_rng(3).standard_normal(P.ndofs)
        Lu = P.apply(u, mode=2)
        # mass of L(u): with the Gauss mass matrix M = kron(h MG),
        # 1^T M L(u) = sum over cells of the exactly integrated L(u)_h
        g, w = oracle.gauss_rule(k)
        xi, _ = oracle.gl_rule(k)
        B = np.array([[oracle.lagrange(k, xi, m, x) for m in range(k + 1)] for x in g])
        col = w @ B   # integral of each 1D basis function
        d = 2 * dx
        wn = col
        for _ in range(d - 1):
            wn = np.kron(col, wn)
        vol = np.prod([(P.hi[j] - P.lo[j]) / P.cells[j] for j in range(d)])
        mass = vol * (Lu.reshape(P.ncells, -1) @ wn).sum()
        assert abs(mass) < 1e-11 * np.abs(Lu).max() * vol * P.ncells


@pytest.mark.parametrize("k", [2, 3])
def test_gauss_mode_converges_at_order_k_plus_1(k):
    # constant advection of sin(2 pi x) sin(2 pi v) on the unit square: the
    # error at t = 0.25 drops by about 2^(k+1) per mesh doubling.
    errs = []
    for N in (4, 8, 16):
        P = oracle.Problem(1, 1, [N, N], [0, 0], [1, 1], k, field="constant", a=[1.0, 0.5])
        u0 = P.init_state(0)
        dt = P.stable_dt(0.2)
        steps = int(round(0.25 / dt))
        dt = 0.25 / steps
        u = P.rk_steps(u0, dt, steps, mode=2)
        X = P.node_coords()
        ex = np.sin(2 * np.pi * (X[:, 0] - 0.25)) * np.sin(2 * np.pi * (X[:, 1] - 0.125))
        errs.append(np.sqrt(np.mean((u - ex) ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > k + 0.6, (errs, rates)
