"""Seeded synthetic workloads shared by the tests, the benchmark and the
serving loop. This module only describes inputs (meshes, degrees, fields,
initial-state kinds, step counts, seeded random states, batch mixes and
request traces); it contains none of the method's arithmetic.

The paper's runs are synthetic too: boxes meshed with Cartesian cells, a
constant velocity (Sec. 5.1) and the phase-space field a = (v, E(x))
(Sec. 6). No dataset is involved.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# x/v split of d (Sec. 5.1): 2=1+1, 3=2+1, 4=2+2, 5=3+2, 6=3+3.
SPLITS = {2: (1, 1), 3: (2, 1), 4: (2, 2), 5: (3, 2), 6: (3, 3)}


@dataclasses.dataclass
class Case:
    name: str
    dim_x: int
    dim_v: int
    cells: list
    lo: list
    hi: list
    degree: int
    field: str          # "constant", "sine" (a = (v, amp sin(2 pi x))),
                        # "table" (a given E) or "vlasov_poisson" (a = (v, -E[f]))
    a: list | None = None
    amp: float = 0.1
    ic: int = 0         # 0: prod sin(2 pi x); 1: perturbed Maxwellian
    ic_params: tuple = (0.0,)
    steps: int = 1
    cfl: float = 0.2
    modes: int = 4      # Fourier modes per x-dimension of the Poisson solve

    @property
    def d(self):
        return self.dim_x + self.dim_v

    @property
    def ndofs(self):
        return int(np.prod(self.cells)) * (self.degree + 1) ** self.d


def phase_space_case(name, dx, dv, cells, degree, steps, vmax=6.0, amp=0.1):
    return Case(name, dx, dv, list(cells), [0.0] * dx + [-vmax] * dv,
                [1.0] * dx + [vmax] * dv, degree, "sine", amp=amp, ic=1,
                ic_params=(0.01,), steps=steps)


def landau_case(name, dx, cells, degree, steps, modes=4, alpha=0.01, kx=0.5, vmax=6.0):
    """Linear Landau damping (Sec. 6): f0 = (1 + alpha cos(kx x_1)) times the
    unit Maxwellian, x in [0, 2 pi / kx]^dx, v in [-vmax, vmax]^dx, with the
    self-consistent Vlasov-Poisson field."""
    L = 2.0 * math.pi / kx
    return Case(name, dx, dx, list(cells), [0.0] * dx + [-vmax] * dx, [L] * dx + [vmax] * dx,
                degree, "vlasov_poisson", ic=1, ic_params=(alpha,), steps=steps, modes=modes)


# Configuration 1: 2D constant advection, exact solution u0(x - a t).
CONFIG_2D = Case("2d_const_16x16_k3", 1, 1, [16, 16], [0, 0], [1, 1], 3, "constant",
                 a=[1.0, 0.5], ic=0, steps=100)
# Configuration 2: 4D phase space, 16^4 cells, k = 3 (16.8M DoFs).
CONFIG_4D = phase_space_case("4d_phase_16^4_k3", 2, 2, [16] * 4, 3, 20)
# Configuration 3: 6D phase space, 8^6 cells, k = 3 (1.07e9 DoFs) - headline.
CONFIG_6D = phase_space_case("6d_phase_8^6_k3", 3, 3, [8] * 6, 3, 10)
# Its reduced rerun for the FP32-vs-FP64 error: 4^6 cells (16.8M DoFs).
CONFIG_6D_SMALL = phase_space_case("6d_phase_4^6_k3", 3, 3, [4] * 6, 3, 10)
# The same phase-space workload at degrees 4 and 5 (about 1.6e8 / 1.9e8 DoFs):
# the degrees that dominate the batched mix and the served requests.
CONFIG_6D_K4 = phase_space_case("6d_phase_5^4x4^2_k4", 3, 3, [5, 5, 5, 5, 4, 4], 4, 10)
CONFIG_6D_K5 = phase_space_case("6d_phase_4^6_k5", 3, 3, [4] * 6, 5, 10)


def random_state(n, seed):
    """Seeded standard-normal FP64 state of n DoFs."""
    return np.random.default_rng(seed).standard_normal(n)


def random_field_table(n, seed, scale=1.0):
    """Seeded E table entries (an arbitrary prescribed field E(x) at x-nodes)."""
    return scale * np.random.default_rng(seed).uniform(-1.0, 1.0, n)


# ---------------------------------------------------------------------------
# Batched mix (configuration 4) and serving trace (configuration 5)
# ---------------------------------------------------------------------------

def _cells_for_target(rng, d, n, target, lo_cells, hi_cells):
    """Cells per dim (anisotropic allowed) with prod(cells) * n^d near target."""
    per_cell = n ** d
    want = max(1.0, target / per_cell)
    base = want ** (1.0 / d)
    cells = []
    for j in range(d):
        c = int(round(base * rng.uniform(0.8, 1.25)))
        cells.append(min(hi_cells, max(lo_cells, c)))
    return cells


def batch_mix(seed=2002, count=96, dims=(3, 4, 5, 6), degrees=(2, 3, 4, 5),
              dof_range=(1e6, 2e8), cells_range=(4, 16), d3_cells_max=40,
              steps=50, max_tries=1000):
    """96 seeded solves of uneven dimension, degree and size. d = 3 cannot
    reach 1M DoFs with <= 16 cells per dim, so its range extends to 40. Even
    solves get a constant field, odd ones the phase-space field where the
    split allows it (d_x = d_v), a constant field otherwise."""
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(count):
        for _ in range(max_tries):
            d = int(rng.choice(dims))
            k = int(rng.choice(degrees))
            target = math.exp(rng.uniform(math.log(dof_range[0]), math.log(dof_range[1])))
            hi_c = d3_cells_max if d == 3 else cells_range[1]
            cells = _cells_for_target(rng, d, k + 1, target, cells_range[0], hi_c)
            nd = int(np.prod(cells)) * (k + 1) ** d
            if dof_range[0] <= nd <= dof_range[1]:
                break
        dx, dv = SPLITS[d]
        # Odd d (2+1, 3+2) has no phase-space field a = (v, E(x)): constant there.
        if i % 2 == 0 or dx != dv:
            a = list(rng.uniform(-1, 1, d))
            cases.append(Case("batch%02d" % i, dx, dv, cells, [0.0] * d, [1.0] * d, k,
                              "constant", a=a, ic=0, steps=steps))
        else:
            c = phase_space_case("batch%02d" % i, dx, dv, cells, k, steps)
            cases.append(c)
    return cases


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float      # seconds
    case: Case


def serve_trace(seed=811, count=2000, rate=20.0, dims=(4, 5, 6), degrees=(2, 3, 4, 5),
                steps=(10, 500), dof_range=(1e6, 2e9), cells_range=(4, 16)):
    """Poisson arrivals (exponential gaps of mean 1/rate) of seeded solves."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        for _ in range(1000):
            d = int(rng.choice(dims))
            k = int(rng.choice(degrees))
            target = math.exp(rng.uniform(math.log(dof_range[0]), math.log(dof_range[1])))
            cells = _cells_for_target(rng, d, k + 1, target, *cells_range)
            nd = int(np.prod(cells)) * (k + 1) ** d
            if dof_range[0] <= nd <= dof_range[1]:
                break
        nsteps = int(rng.integers(steps[0], steps[1] + 1))
        dx, dv = SPLITS[d]
        if i % 2 == 0 or dx != dv:
            case = Case("req%04d" % i, dx, dv, cells, [0.0] * d, [1.0] * d, k, "constant",
                        a=list(rng.uniform(-1, 1, d)), ic=0, steps=nsteps)
        else:
            case = phase_space_case("req%04d" % i, dx, dv, cells, k, nsteps)
        out.append(Request(i, t, case))
    return out
