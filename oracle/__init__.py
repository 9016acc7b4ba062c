"""ctypes binding of the plain CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg. The product package never imports it.

The oracle evaluates the DG advection operator of the paper (hyper.deal,
arXiv 2002.08110: Sec. 1.3 weak form, Sec. 2.3/2.5 Gauss-Lobatto nodes and
collocated quadrature, Algorithm 2 cell + face evaluation) by direct
evaluation of the d-dimensional basis, plus the low-storage RK scheme of
Sec. 5.4. See oracle.h for the per-function citations.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, -O2, FP64)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, src, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Mesh(ctypes.Structure):
    _fields_ = [("dim_x", ctypes.c_int), ("dim_v", ctypes.c_int),
                ("cells", ctypes.c_int * 6), ("lo", ctypes.c_double * 6),
                ("hi", ctypes.c_double * 6), ("map_eps", ctypes.c_double)]


class Field(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("a", ctypes.c_double * 6),
                ("E", ctypes.POINTER(ctypes.c_double)), ("sign", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        d = ctypes.c_double
        i64 = ctypes.c_int64
        lib.or_gl_rule.argtypes = [ctypes.c_int, P(d), P(d)]
        lib.or_gauss_rule.argtypes = [ctypes.c_int, P(d), P(d)]
        lib.or_lagrange.argtypes = [ctypes.c_int, P(d), ctypes.c_int, d]
        lib.or_lagrange.restype = d
        lib.or_lagrange_deriv.argtypes = [ctypes.c_int, P(d), ctypes.c_int, d]
        lib.or_lagrange_deriv.restype = d
        lib.or_num_dofs.argtypes = [P(Mesh), ctypes.c_int]
        lib.or_num_dofs.restype = i64
        lib.or_node_coords.argtypes = [P(Mesh), ctypes.c_int, P(d)]
        lib.or_apply_cells.argtypes = [P(Mesh), ctypes.c_int, P(Field), ctypes.c_int,
                                       P(d), P(i64), i64, P(d)]
        lib.or_apply.argtypes = [P(Mesh), ctypes.c_int, P(Field), ctypes.c_int, P(d), P(d)]
        lib.or_lsrk45_coefficients.argtypes = [P(d), P(d), P(d)]
        lib.or_lsrk45_coefficients.restype = None
        lib.or_rk_steps.argtypes = [P(Mesh), ctypes.c_int, P(Field), ctypes.c_int, d,
                                    ctypes.c_int, P(d)]
        lib.or_rk_stage.argtypes = [P(Mesh), ctypes.c_int, P(Field), ctypes.c_int, d,
                                    ctypes.c_int, P(d), P(d), P(d)]
        lib.or_stable_dt.argtypes = [P(Mesh), ctypes.c_int, P(Field), d]
        lib.or_stable_dt.restype = d
        lib.or_init_state.argtypes = [P(Mesh), ctypes.c_int, ctypes.c_int, P(d), P(d)]
        lib.or_field_sine_table.argtypes = [P(Mesh), ctypes.c_int, d, P(d)]
        lib.or_diagnostics.argtypes = [P(Mesh), ctypes.c_int, P(d), P(d), P(d)]
        lib.or_num_threads.argtypes = []
        lib.or_vp_density.argtypes = [P(Mesh), ctypes.c_int, P(d), P(d)]
        lib.or_vp_field.argtypes = [P(Mesh), ctypes.c_int, ctypes.c_int, P(d), P(d)]
        lib.or_vp_rk_steps.argtypes = [P(Mesh), ctypes.c_int, ctypes.c_int, ctypes.c_int, d,
                                       ctypes.c_int, P(d)]
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_mesh(dim_x, dim_v, cells, lo, hi, map_eps=0.0) -> Mesh:
    d = dim_x + dim_v
    m = Mesh()
    m.dim_x, m.dim_v = dim_x, dim_v
    m.map_eps = float(map_eps)
    for j in range(d):
        m.cells[j] = int(cells[j])
        m.lo[j] = float(lo[j])
        m.hi[j] = float(hi[j])
    return m


class Problem:
    """A mesh, a degree and a field; holds the E table alive for ctypes."""

    def __init__(self, dim_x, dim_v, cells, lo, hi, k, field="constant", a=None,
                 E=None, sign=1.0, sine_amp=None, map_eps=0.0):
        self.lib = _load()
        self.dim_x, self.dim_v, self.k = dim_x, dim_v, k
        self.d = dim_x + dim_v
        self.n = k + 1
        self.cells = [int(c) for c in cells]
        self.lo = [float(x) for x in lo]
        self.hi = [float(x) for x in hi]
        self.map_eps = float(map_eps)
        self.mesh = make_mesh(dim_x, dim_v, cells, lo, hi, map_eps)
        self.ndofs = int(self.lib.or_num_dofs(ctypes.byref(self.mesh), k))
        if self.ndofs < 0:
            raise ValueError("invalid mesh/degree")
        self.ncells = self.ndofs // self.n ** self.d
        self.field = Field()
        self._E = None
        self.sine_amp = None
        if field == "constant":
            self.field.kind = 0
            for j in range(self.d):
                self.field.a[j] = float(a[j])
        elif field == "phase":
            self.field.kind = 1
            self.field.sign = float(sign)
            if E is None:
                self.sine_amp = 0.1 if sine_amp is None else float(sine_amp)
                E = self.sine_table(self.sine_amp)
            self._E = np.ascontiguousarray(E, dtype=np.float64)
            self.field.E = _dp(self._E)
        else:
            raise ValueError(field)

    def nx_nodes(self):
        nxc = int(np.prod(self.cells[: self.dim_x]))
        return nxc * self.n ** self.dim_x

    def sine_table(self, amp):
        E = np.zeros(self.nx_nodes() * self.dim_x)
        r = self.lib.or_field_sine_table(ctypes.byref(self.mesh), self.k, amp, _dp(E))
        assert r == 0
        return E

    def apply(self, u, mode=1):
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.empty_like(u)
        r = self.lib.or_apply(ctypes.byref(self.mesh), self.k, ctypes.byref(self.field),
                              mode, _dp(u), _dp(out))
        if r:
            raise RuntimeError("or_apply failed")
        return out

    def apply_cells(self, u, cells, mode=1):
        u = np.ascontiguousarray(u, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty(len(cells) * self.n ** self.d)
        r = self.lib.or_apply_cells(ctypes.byref(self.mesh), self.k, ctypes.byref(self.field),
                                    mode, _dp(u),
                                    cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    len(cells), _dp(out))
        if r:
            raise RuntimeError("or_apply_cells failed")
        return out

    def rk_steps(self, u, dt, nsteps, mode=1):
        u = np.array(u, dtype=np.float64, copy=True)
        r = self.lib.or_rk_steps(ctypes.byref(self.mesh), self.k, ctypes.byref(self.field),
                                 mode, dt, nsteps, _dp(u))
        if r:
            raise RuntimeError("or_rk_steps failed")
        return u

    def rk_stage(self, u, du, L, dt, stage, mode=1):
        """One RK stage in place on the float64 arrays u and du (N values
        each; du is not read at stage 0); L is scratch of N values."""
        for a in (u, du, L):
            assert a.dtype == np.float64 and a.flags.c_contiguous and a.size == self.ndofs
        r = self.lib.or_rk_stage(ctypes.byref(self.mesh), self.k, ctypes.byref(self.field),
                                 mode, dt, stage, _dp(u), _dp(du), _dp(L))
        if r:
            raise RuntimeError("or_rk_stage failed")

    def stable_dt(self, cfl=0.2):
        return float(self.lib.or_stable_dt(ctypes.byref(self.mesh), self.k,
                                           ctypes.byref(self.field), cfl))

    def init_state(self, kind, params=None):
        u = np.empty(self.ndofs)
        p = np.ascontiguousarray(params if params is not None else [0.0], dtype=np.float64)
        r = self.lib.or_init_state(ctypes.byref(self.mesh), self.k, kind, _dp(p), _dp(u))
        assert r == 0
        return u

    def node_coords(self):
        X = np.empty(self.ndofs * self.d)
        r = self.lib.or_node_coords(ctypes.byref(self.mesh), self.k, _dp(X))
        assert r == 0
        return X.reshape(self.ndofs, self.d)

    def diagnostics(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        m = ctypes.c_double()
        e = ctypes.c_double()
        r = self.lib.or_diagnostics(ctypes.byref(self.mesh), self.k, _dp(u),
                                    ctypes.byref(m), ctypes.byref(e))
        assert r == 0
        return m.value, e.value


class VlasovPoisson:
    """The Vlasov-Poisson system of Sec. 6 on a periodic x-box times a
    periodic v-box (dim_x == dim_v): f_t + v.grad_x f - E.grad_v f = 0,
    -Laplace phi = 1 - rho, E = -grad phi, rho = int f dv, with the field
    solved spectrally from the modes |m_j| <= modes (see oracle.h)."""

    def __init__(self, dim_x, dim_v, cells, lo, hi, k, modes):
        if dim_x != dim_v:
            raise ValueError("Vlasov-Poisson needs dim_x == dim_v")
        self.lib = _load()
        self.dim_x, self.dim_v, self.k, self.modes = dim_x, dim_v, k, int(modes)
        self.d = dim_x + dim_v
        self.n = k + 1
        self.cells = [int(c) for c in cells]
        self.lo = [float(x) for x in lo]
        self.hi = [float(x) for x in hi]
        self.mesh = make_mesh(dim_x, dim_v, cells, lo, hi)
        self.ndofs = int(self.lib.or_num_dofs(ctypes.byref(self.mesh), k))
        self.npoints = int(np.prod(self.cells[:dim_x])) * self.n ** dim_x

    def density(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        rho = np.empty(self.npoints)
        assert self.lib.or_vp_density(ctypes.byref(self.mesh), self.k, _dp(u), _dp(rho)) == 0
        return rho

    def field(self, rho):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        E = np.empty(self.npoints * self.dim_x)
        assert self.lib.or_vp_field(ctypes.byref(self.mesh), self.k, self.modes, _dp(rho),
                                    _dp(E)) == 0
        return E

    def advection(self, u):
        """The advection problem a = (v, -E) with the field of state u."""
        return Problem(self.dim_x, self.dim_v, self.cells, self.lo, self.hi, self.k,
                       field="phase", E=self.field(self.density(u)), sign=-1.0)

    def apply(self, u, mode=1):
        return self.advection(u).apply(u, mode)

    def rk_steps(self, u, dt, nsteps, mode=1):
        u = np.array(u, dtype=np.float64, copy=True)
        r = self.lib.or_vp_rk_steps(ctypes.byref(self.mesh), self.k, self.modes, mode, dt,
                                    nsteps, _dp(u))
        if r:
            raise RuntimeError("or_vp_rk_steps failed")
        return u

    def stable_dt(self, u, cfl=0.2):
        return self.advection(u).stable_dt(cfl)

    def x_weights(self):
        """GL quadrature weight of each x-point (E table order)."""
        xi, w = gl_rule(self.k)
        W = np.ones(self.npoints)
        p = np.arange(self.npoints)
        nxn = self.n ** self.dim_x
        xc, xn = p // nxn, p % nxn
        for j in range(self.dim_x):
            h = (self.hi[j] - self.lo[j]) / self.cells[j]
            W = W * h * w[xn % self.n]
            xc //= self.cells[j]
            xn //= self.n
        return W

    def x_coords(self):
        """Coordinates of the x-points, shape (npoints, dim_x)."""
        xi, w = gl_rule(self.k)
        p = np.arange(self.npoints)
        nxn = self.n ** self.dim_x
        xc, xn = p // nxn, p % nxn
        X = np.empty((self.npoints, self.dim_x))
        for j in range(self.dim_x):
            h = (self.hi[j] - self.lo[j]) / self.cells[j]
            X[:, j] = self.lo[j] + (xc % self.cells[j] + xi[xn % self.n]) * h
            xc //= self.cells[j]
            xn //= self.n
        return X

    def electric_energy(self, E):
        """1/2 int |E|^2 dx by GL quadrature over the x-points."""
        E = np.asarray(E).reshape(self.npoints, self.dim_x)
        return 0.5 * float(np.sum(self.x_weights()[:, None] * E * E))

    def init_state(self, kind, params=None):
        return Problem(self.dim_x, self.dim_v, self.cells, self.lo, self.hi, self.k,
                       field="phase").init_state(kind, params)

    def diagnostics(self, u):
        return Problem(self.dim_x, self.dim_v, self.cells, self.lo, self.hi, self.k,
                       field="phase").diagnostics(u)


def gl_rule(k):
    lib = _load()
    xi = np.zeros(k + 1)
    w = np.zeros(k + 1)
    if lib.or_gl_rule(k, _dp(xi), _dp(w)):
        raise ValueError(k)
    return xi, w


def gauss_rule(k):
    """Gauss-Legendre points and weights (k+1 of them) on [0, 1]."""
    lib = _load()
    g = np.zeros(k + 1)
    w = np.zeros(k + 1)
    if lib.or_gauss_rule(k, _dp(g), _dp(w)):
        raise ValueError(k)
    return g, w


def lagrange(k, xi, m, x):
    return _load().or_lagrange(k, _dp(np.ascontiguousarray(xi, dtype=np.float64)), m, x)


def lagrange_deriv(k, xi, m, x):
    return _load().or_lagrange_deriv(k, _dp(np.ascontiguousarray(xi, dtype=np.float64)), m, x)


def lsrk45_coefficients():
    lib = _load()
    A = np.zeros(5)
    B = np.zeros(5)
    C = np.zeros(5)
    lib.or_lsrk45_coefficients(_dp(A), _dp(B), _dp(C))
    return A, B, C


def num_threads():
    return int(_load().or_num_threads())
