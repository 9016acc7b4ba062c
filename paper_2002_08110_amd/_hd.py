"""ctypes declarations of the C ABI in include/hd.h (same names, same
arguments). Argument marshalling only: every step of the method runs in the
HIP kernels of libhd.so. There is no fallback: if libhd.so is missing or
fails to load, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhd.so")

HD_OK = 0
HD_ERR_INVALID = -1
HD_ERR_UNSUPPORTED = -2
HD_ERR_OOM = -3
HD_ERR_HIP = -4
HD_ERR_STATE = -5
HD_FP64 = 0
HD_FP32_OP_FP64_ACC = 1

# Every symbol include/hd.h declares.
SYMBOLS = (
    "hd_create", "hd_destroy", "hd_num_dofs", "hd_required_bytes", "hd_bind",
    "hd_set_field_constant", "hd_set_field_phase_space", "hd_set_field_sine",
    "hd_set_field_vlasov_poisson", "hd_get_field", "hd_compute_field", "hd_set_quadrature",
    "hd_set_mapping",
    "hd_set_state", "hd_init_state", "hd_state_ptr", "hd_get_state", "hd_apply",
    "hd_stable_dt", "hd_rk_stage", "hd_rk_step", "hd_diagnostics", "hd_get_plan",
    "hd_set_plan", "hd_last_error", "hd_batch_create", "hd_batch_destroy",
    "hd_batch_step", "hd_stream_copy", "hd_diagnostics_noalloc", "hd_batch_launch_counts",
)


class hd_mesh(ctypes.Structure):
    _fields_ = [("dim_x", ctypes.c_int), ("dim_v", ctypes.c_int),
                ("cells", ctypes.c_int * 6), ("lo", ctypes.c_double * 6),
                ("hi", ctypes.c_double * 6)]


class hd_plan(ctypes.Structure):
    _fields_ = [("lds", ctypes.c_int), ("cells_per_wg", ctypes.c_int),
                ("wg_size", ctypes.c_int), ("xcd_remap", ctypes.c_int),
                ("reg_dims", ctypes.c_int), ("kernel", ctypes.c_int),
                ("options", ctypes.c_int), ("split_dims", ctypes.c_int),
                ("loop_dims", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class HDError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("hd status %d: %s" % (status, message))
        self.status = status


_lib = None


def load():
    """Load libhd.so and declare every entry point; raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhd.so is not built (%s); build it with "
                          "paper_2002_08110_amd.build.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    d = ctypes.c_double
    i = ctypes.c_int
    st = ctypes.c_int
    sig = {
        "hd_create": ([P(hd_mesh), i, i, P(vp)], st),
        "hd_destroy": ([vp], st),
        "hd_num_dofs": ([vp, P(ctypes.c_int64)], st),
        "hd_required_bytes": ([vp, P(ctypes.c_size_t), P(ctypes.c_size_t)], st),
        "hd_bind": ([vp, vp, ctypes.c_size_t, vp, ctypes.c_size_t], st),
        "hd_set_field_constant": ([vp, P(d)], st),
        "hd_set_field_phase_space": ([vp, P(d), d], st),
        "hd_set_field_sine": ([vp, d, d], st),
        "hd_set_field_vlasov_poisson": ([vp, i], st),
        "hd_get_field": ([vp, P(d), vp], st),
        "hd_compute_field": ([vp, vp], st),
        "hd_set_quadrature": ([vp, i], st),
        "hd_set_mapping": ([vp, d], st),
        "hd_set_state": ([vp, vp, i, vp], st),
        "hd_init_state": ([vp, i, P(d), vp], st),
        "hd_state_ptr": ([vp, P(vp)], st),
        "hd_get_state": ([vp, vp, vp], st),
        "hd_apply": ([vp, vp, vp, vp], st),
        "hd_stable_dt": ([vp, d, P(d)], st),
        "hd_rk_stage": ([vp, i, d, vp], st),
        "hd_rk_step": ([vp, d, i, vp], st),
        "hd_diagnostics": ([vp, P(d), P(d), vp], st),
        "hd_get_plan": ([vp, P(hd_plan)], st),
        "hd_set_plan": ([vp, P(hd_plan)], st),
        "hd_last_error": ([], ctypes.c_char_p),
        "hd_batch_create": ([P(vp), i, P(vp)], st),
        "hd_batch_destroy": ([vp], st),
        "hd_batch_step": ([vp, P(d), P(i), vp], st),
        "hd_stream_copy": ([vp, vp, ctypes.c_size_t, vp], st),
        "hd_diagnostics_noalloc": ([vp, vp, vp, vp], st),
        "hd_batch_launch_counts": ([vp, P(i), P(i)], st),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status):
    if status != HD_OK:
        msg = _lib.hd_last_error().decode() if _lib is not None else ""
        raise HDError(status, msg)
    return status
