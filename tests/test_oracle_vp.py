"""Pins of the oracle's Vlasov-Poisson field (Sec. 6): the velocity moment
is the exact integral of the DG polynomial, the spectral Poisson solve
reproduces closed-form fields, mass is conserved, and the linearized
dynamics damps the electric field at the Landau rate, i.e. the root of the
plasma dispersion relation (computed here from the Faddeeva function), not
a number taken from any code."""
import numpy as np
import pytest

import oracle


def _vp(dx, cells, k, modes, L=1.0, vmax=6.0):
    return oracle.VlasovPoisson(dx, dx, cells, [0.0] * dx + [-vmax] * dx,
                                [L] * dx + [vmax] * dx, k, modes)


def _nodal(vp, fn):
    X = oracle.Problem(vp.dim_x, vp.dim_v, vp.cells, vp.lo, vp.hi, vp.k,
                       field="phase").node_coords()
    return fn(X)


@pytest.mark.parametrize("dx", [1, 2, 3])
def test_density_is_the_exact_velocity_integral(dx):
    # f = (1 + 0.3 cos 2 pi x1) (1 + v1^2 + 0.5 v_dx): GL quadrature with k+1
    # points integrates the degree-2 velocity polynomial exactly on [-6, 6]^dv.
    cells = [2] * dx + [3] * dx
    vp = _vp(dx, cells, 3, 2)
    u = _nodal(vp, lambda X: (1 + 0.3 * np.cos(2 * np.pi * X[:, 0]))
               * (1 + X[:, dx] ** 2 + 0.5 * X[:, 2 * dx - 1]))
    rho = vp.density(u)
    vol_v = 12.0 ** dx
    exact_v = vol_v + vol_v / 12.0 * 144.0  # int 1 + int v1^2 (the odd term vanishes)
    xs = vp.x_coords()
    np.testing.assert_allclose(rho, (1 + 0.3 * np.cos(2 * np.pi * xs[:, 0])) * exact_v,
                               rtol=1e-13)


def test_field_of_a_cosine_density_1d():
    # rho = 1 + a cos(k x) gives E = -(a / k) sin(k x) on [0, 4 pi] (k = 0.5).
    k, a = 0.5, 0.01
    vp = oracle.VlasovPoisson(1, 1, [16, 4], [0, -6], [4 * np.pi, 6], 5, 4)
    x = vp.x_coords()[:, 0]
    E = vp.field(1 + a * np.cos(k * x))
    np.testing.assert_allclose(E, -(a / k) * np.sin(k * x), atol=1e-12)


def test_field_of_a_product_density_2d():
    # rho = 1 + a cos(k1 x1) cos(k2 x2): phi = -a cos cos / |k|^2 and
    # E = -grad phi = -(a / |k|^2) (k1 sin cos, k2 cos sin).
    a = 0.2
    vp = oracle.VlasovPoisson(2, 2, [6, 5, 1, 1], [0, 0, -1, -1], [1, 2, 1, 1], 5, 3)
    X = vp.x_coords()
    k1, k2 = 2 * np.pi * 2 / 1.0, 2 * np.pi * 1 / 2.0
    rho = 1 + a * np.cos(k1 * X[:, 0]) * np.cos(k2 * X[:, 1])
    E = vp.field(rho).reshape(-1, 2)
    kk = k1 ** 2 + k2 ** 2
    np.testing.assert_allclose(E[:, 0], -a / kk * k1 * np.sin(k1 * X[:, 0]) * np.cos(k2 * X[:, 1]),
                               atol=1e-9)
    np.testing.assert_allclose(E[:, 1], -a / kk * k2 * np.cos(k1 * X[:, 0]) * np.sin(k2 * X[:, 1]),
                               atol=1e-9)


def test_field_of_a_uniform_density_vanishes_and_modes_truncate():
    vp = oracle.VlasovPoisson(1, 1, [8, 2], [0, -1], [1, 1], 4, 2)
    x = vp.x_coords()[:, 0]
    assert np.abs(vp.field(np.full(len(x), 3.7))).max() < 1e-14
    # a mode beyond M = 2 is not represented
    assert np.abs(vp.field(1 + np.cos(2 * np.pi * 3 * x))).max() < 1e-12


@pytest.mark.parametrize("C", [2, 3, 5])
def test_constant_density_aliases_only_onto_multiples_of_the_cell_count(C):
    # On C uniform cells, sum_c exp(-2 pi i m c / C) vanishes unless C | m:
    # a constant density (every cell alike) has rho_hat_m = 0 for the other
    # m != 0, and a nonzero field exactly when some |m| <= M is a multiple of C.
    for M in (1, 2, 3, 4):
        vp = oracle.VlasovPoisson(1, 1, [C, 2], [0.5, -1], [2.5, 1], 3, M)
        E = vp.field(np.full(C * 4, 2.0))
        if M >= C:
            assert np.abs(E).max() > 1e-3, (C, M)
        else:
            assert np.abs(E).max() < 1e-14, (C, M)


@pytest.mark.parametrize("dx,cells,k", [(1, [6, 8], 3), (2, [3, 2, 4, 3], 2)])
def test_vp_steps_conserve_mass(dx, cells, k):
    vp = _vp(dx, cells, k, 3, L=2 * np.pi)
    u0 = vp.init_state(1, [0.05])
    dt = vp.stable_dt(u0)
    u = vp.rk_steps(u0, dt, 20)
    m0, e0 = vp.diagnostics(u0)
    m1, e1 = vp.diagnostics(u)
    assert abs(m1 - m0) <= 1e-13 * abs(m0)
    assert not np.allclose(u, u0)


def _landau_root(k):
    """Root of the Maxwellian dielectric function 1 + (1 + z Z(z)) / k^2,
    z = omega / (sqrt(2) k), Z(z) = i sqrt(pi) w(z), by Newton's method."""
    from scipy.special import wofz

    def eps(om):
        z = om / (np.sqrt(2) * k)
        return 1 + (1 + z * 1j * np.sqrt(np.pi) * wofz(z)) / k ** 2

    om = 1.4 - 0.15j
    for _ in range(50):
        h = 1e-7
        step = eps(om) / ((eps(om + h) - eps(om - h)) / (2 * h))
        om -= step
        if abs(step) < 1e-13:
            break
    return om


def test_linear_landau_damping_rate():
    # f0 = (1 + 0.01 cos(0.5 x)) M(v) on [0, 4 pi] x [-6, 6]: the electric
    # energy oscillates at 2 Re(omega) and decays at 2 Im(omega).
    k = 0.5
    om = _landau_root(k)
    assert abs(om.real - 1.4156) < 1e-3 and abs(om.imag + 0.1533) < 1e-3
    vp = oracle.VlasovPoisson(1, 1, [16, 32], [0, -6], [4 * np.pi, 6], 3, 4)
    u = vp.init_state(1, [0.01])
    dt = vp.stable_dt(u)
    T, chunk = 18.0, 20
    ts, W = [0.0], [vp.electric_energy(vp.field(vp.density(u)))]
    while ts[-1] < T:
        u = vp.rk_steps(u, dt, chunk)
        ts.append(ts[-1] + chunk * dt)
        W.append(vp.electric_energy(vp.field(vp.density(u))))
    ts, W = np.array(ts), np.array(W)
    # local maxima of the energy after the first period
    peaks = [i for i in range(1, len(W) - 1) if W[i] > W[i - 1] and W[i] >= W[i + 1]
             and ts[i] > 2.0]
    assert len(peaks) >= 4
    slope = np.polyfit(ts[peaks], np.log(W[peaks]), 1)[0]
    assert abs(slope / (2 * om.imag) - 1) < 0.05, (slope, 2 * om.imag)
    period = np.mean(np.diff(ts[peaks]))
    assert abs(period / (np.pi / om.real) - 1) < 0.05, (period, np.pi / om.real)
