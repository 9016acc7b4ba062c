"""MI355X (gfx950) matrix-free upwind Gauss-Lobatto DG advection in 2-6
dimensions on a tensor product of configuration and velocity meshes, with a
fused five-stage low-storage Runge-Kutta integrator (hyper.deal, arXiv
2002.08110). The compute path is the HIP library libhd.so behind the C ABI of
include/hd.h; this package is its Python binding."""
from ._hd import HD_FP32_OP_FP64_ACC, HD_FP64, HDError, load  # noqa: F401

__all__ = ["HDError", "load", "Solver", "HD_FP32_OP_FP64_ACC", "HD_FP64"]


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    raise AttributeError(name)
