"""Thin object wrapper over the C ABI: a Solver owns an hd_solver handle and
a torch device tensor as its workspace. Only marshalling happens here; every
computation is a HIP kernel in libhd.so. PyTorch supplies device memory and
the current stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _hd
from ._hd import check, hd_mesh, hd_plan

_ALIGN = 256


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_mesh(dim_x, dim_v, cells, lo, hi) -> hd_mesh:
    m = hd_mesh()
    m.dim_x, m.dim_v = int(dim_x), int(dim_v)
    for j in range(dim_x + dim_v):
        m.cells[j] = int(cells[j])
        m.lo[j] = float(lo[j])
        m.hi[j] = float(hi[j])
    return m


class Solver:
    """hd_create + hd_bind over torch-allocated state and workspace buffers
    on `device`."""

    def __init__(self, dim_x, dim_v, cells, lo, hi, degree, precision="fp64",
                 device="cuda:0", bind=True):
        self.lib = _hd.load()
        self.dim_x, self.dim_v, self.k = int(dim_x), int(dim_v), int(degree)
        self.d = self.dim_x + self.dim_v
        self.cells = [int(c) for c in cells[: self.d]]
        self.lo = [float(x) for x in lo[: self.d]]
        self.hi = [float(x) for x in hi[: self.d]]
        self.precision = precision
        self.prec = _hd.HD_FP32_OP_FP64_ACC if precision == "fp32" else _hd.HD_FP64
        self.device = torch.device(device)
        self.mesh = make_mesh(dim_x, dim_v, cells, lo, hi)
        h = ctypes.c_void_p()
        check(self.lib.hd_create(ctypes.byref(self.mesh), self.k, self.prec, ctypes.byref(h)))
        self.h = h
        n = ctypes.c_int64()
        check(self.lib.hd_num_dofs(self.h, ctypes.byref(n)))
        self.ndofs = n.value
        sb = ctypes.c_size_t()
        wb = ctypes.c_size_t()
        check(self.lib.hd_required_bytes(self.h, ctypes.byref(sb), ctypes.byref(wb)))
        self.state_bytes = sb.value
        self.workspace_bytes = wb.value
        self.state = None
        self.workspace = None
        if bind:
            self.bind()

    @property
    def device_bytes(self) -> int:
        """Device memory of a bound solver: state and workspace buffers
        (with their alignment slack)."""
        return self.state_bytes + self.workspace_bytes + 2 * _ALIGN

    # -- memory -----------------------------------------------------------
    def bind(self, state: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
        """hd_bind over two torch uint8 device buffers (allocated here if not
        given): the state (two FP64 solution vectors) and the workspace."""
        def aligned(buf, nbytes):
            if buf is None:
                buf = torch.empty(nbytes + _ALIGN, dtype=torch.uint8, device=self.device)
            off = (-buf.data_ptr()) % _ALIGN
            assert buf.numel() - off >= nbytes, "buffer too small"
            return buf, buf[off: off + nbytes]
        self._st_raw, self.state = aligned(state, self.state_bytes)
        self._ws_raw, self.workspace = aligned(workspace, self.workspace_bytes)
        check(self.lib.hd_bind(self.h, ctypes.c_void_p(self.state.data_ptr()), self.state_bytes,
                               ctypes.c_void_p(self.workspace.data_ptr()), self.workspace_bytes))

    def state_ptr(self) -> int:
        p = ctypes.c_void_p()
        check(self.lib.hd_state_ptr(self.h, ctypes.byref(p)))
        return p.value

    def state_tensor(self) -> torch.Tensor:
        """A float64 view of the current solution inside the state buffer."""
        off = self.state_ptr() - self.state.data_ptr()
        return self.state[off: off + 8 * self.ndofs].view(torch.float64)

    # -- field ------------------------------------------------------------
    def set_field_constant(self, a):
        arr = (ctypes.c_double * 6)(*([float(x) for x in a] + [0.0] * (6 - len(a))))
        check(self.lib.hd_set_field_constant(self.h, arr))

    def set_field_sine(self, amp=0.1, sign=1.0):
        check(self.lib.hd_set_field_sine(self.h, float(amp), float(sign)))

    def set_field_phase_space(self, E, sign=1.0):
        E = np.ascontiguousarray(E, dtype=np.float64)
        check(self.lib.hd_set_field_phase_space(
            self.h, E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(sign)))

    def set_field_vlasov_poisson(self, modes=4):
        """a = (v, -E) with E solved from the density of every stage's input
        (modes per x-dimension, at most 16)."""
        check(self.lib.hd_set_field_vlasov_poisson(self.h, int(modes)))

    @property
    def field_entries(self):
        n = self.dim_x
        for j in range(self.dim_x):
            n *= self.cells[j] * (self.k + 1)
        return n

    def get_field(self, stream=None) -> np.ndarray:
        """The E table (x-points x dim_x, FP64); for the Vlasov-Poisson field
        that of the current state."""
        out = np.empty(self.field_entries, dtype=np.float64)
        check(self.lib.hd_get_field(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    _stream(stream)))
        return out

    def set_quadrature(self, quadrature="gauss_lobatto"):
        """'gauss_lobatto' (collocation, the default) or 'gauss_legendre'
        (k+1 Gauss points per dimension)."""
        q = {"gauss_lobatto": 0, "gauss_legendre": 1}[quadrature]
        check(self.lib.hd_set_quadrature(self.h, q))

    def set_mapping(self, eps):
        """Deform the configuration mesh (0: Cartesian); see hd_set_mapping."""
        check(self.lib.hd_set_mapping(self.h, float(eps)))

    def compute_field(self, stream=None):
        """Recompute the device E table of the Vlasov-Poisson field from the
        current state (asynchronous; no-op for prescribed fields)."""
        check(self.lib.hd_compute_field(self.h, _stream(stream)))

    # -- state ------------------------------------------------------------
    def set_state(self, u, stream=None):
        if isinstance(u, torch.Tensor):
            assert u.dtype == torch.float64 and u.is_contiguous() and u.numel() == self.ndofs
            if u.is_cuda:
                check(self.lib.hd_set_state(self.h, ctypes.c_void_p(u.data_ptr()), 1,
                                            _stream(stream)))
                return
            u = u.numpy()
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert u.size == self.ndofs
        check(self.lib.hd_set_state(self.h, ctypes.c_void_p(u.ctypes.data), 0, _stream(stream)))
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()

    def init_state(self, kind, params=None, stream=None):
        p = (ctypes.c_double * 1)(float(params[0]) if params else 0.0)
        check(self.lib.hd_init_state(self.h, int(kind), p, _stream(stream)))

    def get_state(self, stream=None) -> np.ndarray:
        out = np.empty(self.ndofs, dtype=np.float64)
        check(self.lib.hd_get_state(self.h, ctypes.c_void_p(out.ctypes.data), _stream(stream)))
        return out

    # -- operator and time stepping ---------------------------------------
    def apply(self, inp: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        assert inp.dtype == torch.float64 and inp.is_cuda and inp.is_contiguous()
        assert inp.numel() == self.ndofs
        odt = torch.float32 if self.prec == _hd.HD_FP32_OP_FP64_ACC else torch.float64
        if out is None:
            out = torch.empty(self.ndofs, dtype=odt, device=inp.device)
        assert out.dtype == odt and out.is_contiguous() and out.numel() == self.ndofs
        check(self.lib.hd_apply(self.h, ctypes.c_void_p(inp.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def stable_dt(self, cfl=0.2) -> float:
        dt = ctypes.c_double()
        check(self.lib.hd_stable_dt(self.h, float(cfl), ctypes.byref(dt)))
        return dt.value

    def rk_stage(self, stage, dt, stream=None):
        check(self.lib.hd_rk_stage(self.h, int(stage), float(dt), _stream(stream)))

    def rk_step(self, dt, nsteps=1, stream=None):
        check(self.lib.hd_rk_step(self.h, float(dt), int(nsteps), _stream(stream)))

    def diagnostics(self, stream=None):
        m = ctypes.c_double()
        e = ctypes.c_double()
        check(self.lib.hd_diagnostics(self.h, ctypes.byref(m), ctypes.byref(e), _stream(stream)))
        return m.value, e.value

    # -- plan -------------------------------------------------------------
    def get_plan(self) -> dict:
        p = hd_plan()
        check(self.lib.hd_get_plan(self.h, ctypes.byref(p)))
        return p.as_dict()

    def set_plan(self, **kw):
        p = hd_plan()
        check(self.lib.hd_get_plan(self.h, ctypes.byref(p)))
        for k, v in kw.items():
            setattr(p, k, int(v))
        check(self.lib.hd_set_plan(self.h, ctypes.byref(p)))

    def tune_plan(self, dt, reps=2, stream=None, margin=0.01) -> dict:
        """Time every candidate plan of this (d, k, precision) on this
        solver's own mesh and field - `reps` RK steps each, after one untimed
        step - and keep the fastest. The cell order that suits the caches
        depends on the mesh, not only on (d, k). The plan the solver had
        stays unless another is faster by more than `margin` (a fraction):
        candidates within the timing noise of each other do not flip the
        choice from run to run. The solution is restored from a device copy
        afterwards (one extra state vector of memory for the duration); the
        stage increment is left undefined, which the next step's first stage
        never reads. Returns the chosen plan."""
        from . import autotune
        st = torch.cuda.current_stream() if stream is None else stream
        saved = self.state_tensor().clone()
        start = self.get_plan()
        start_ms = None
        best = None
        for plan in autotune.candidate_plans(self.d, self.k, self.dim_v, self.precision):
            try:
                self.set_plan(**plan)
            except _hd.HDError:
                continue
            self.rk_step(dt, 1, stream=st)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            self.rk_step(dt, reps, stream=st)
            e1.record(st)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            if autotune.same_launch(self.get_plan(), start):
                start_ms = ms if start_ms is None else min(start_ms, ms)
            if best is None or ms < best[0]:
                best = (ms, self.get_plan())
        if best is None:
            raise RuntimeError("no candidate plan is valid for this solver")
        if start_ms is not None and best[0] > (1.0 - margin) * start_ms:
            best = (start_ms, start)
        self.set_plan(**best[1])
        self.set_state(saved, stream=st)
        st.synchronize()
        del saved
        return best[1]

    def apply_tuned_plan(self, cache=None, arch=None) -> bool:
        """Set the plan the autotuner measured fastest for this (d, k,
        precision) on this GPU architecture, if the cache holds one."""
        from . import autotune
        plan = autotune.lookup(self.d, self.k, self.precision,
                               path=cache or autotune.DEFAULT_CACHE, arch=arch)
        if plan is None:
            return False
        self.set_plan(**plan)
        return True

    def close(self):
        """Destroy the handle and drop the workspace (device memory returns
        to torch's allocator)."""
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.hd_destroy(self.h)
            self.h = ctypes.c_void_p()
        self.state = None
        self.workspace = None
        self._st_raw = None
        self._ws_raw = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """hd_batch over bound Solvers (any d, degree, size, precision, plan):
    one hipGraph replay per step advances every active solve; per RK stage,
    one work-list launch per kernel-variant group (hd_batch_step)."""

    def __init__(self, solvers):
        self.lib = _hd.load()
        self.solvers = list(solvers)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = ctypes.c_void_p()
        check(self.lib.hd_batch_create(arr, len(self.solvers), ctypes.byref(h)))
        self.h = h

    def step(self, dts, active=None, stream=None):
        n = len(self.solvers)
        dt = (ctypes.c_double * n)(*[float(x) for x in dts])
        act = None if active is None else (ctypes.c_int * n)(*[int(bool(a)) for a in active])
        check(self.lib.hd_batch_step(self.h, dt, act, _stream(stream)))

    def launch_counts(self):
        """(work-list launches, single-solve stage launches) of the most
        recently captured step."""
        a, b = ctypes.c_int(), ctypes.c_int()
        check(self.lib.hd_batch_launch_counts(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.hd_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
