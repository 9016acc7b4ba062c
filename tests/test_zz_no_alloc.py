"""The allocation-free diagnostics entry point (hd_diagnostics_noalloc),
called through the C ABI: its mass and energy equal those of
hd_diagnostics on the same vector bitwise (the same kernels in the same
order, partial sums in the library's own device array), on two calls in a
row, the second on a smaller mesh, and on a deformed mesh."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import gpu_solver
from paper_2002_08110_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _noalloc(S, u):
    from paper_2002_08110_amd import _hd
    res = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _hd.check(S.lib.hd_diagnostics_noalloc(S.h, ctypes.c_void_p(u.data_ptr()),
                                           ctypes.c_void_p(res.data_ptr()), stream))
    torch.cuda.synchronize()
    return res.cpu().numpy()


def test_noalloc_diagnostics_equal_the_workspace_ones_on_two_calls():
    big = W.phase_space_case("big", 3, 3, [4, 3, 4, 3, 4, 2], 3, 1)
    small = W.Case("small", 2, 1, [3, 2, 5], [0.0] * 3, [1.0, 2.0, 1.5], 2, "constant",
                   a=[0.3, -0.7, 0.2])
    for case, seed in ((big, 3), (small, 4)):
        S = gpu_solver(case, "fp64")
        u = torch.from_numpy(W.random_state(case.ndofs, seed) + 0.5).cuda()
        S.set_state(u)
        m, e = S.diagnostics()
        got = _noalloc(S, u)
        assert got[0] == m and got[1] == e, (case.name, got, m, e)
        S.close()


def test_noalloc_diagnostics_on_a_mapped_mesh_and_an_unbound_solver():
    from paper_2002_08110_amd.solver import Solver
    case = W.phase_space_case("mapped", 2, 2, [3, 4, 2, 3], 3, 1)
    S = gpu_solver(case, "fp64")
    S.set_mapping(0.03)
    u = torch.from_numpy(W.random_state(case.ndofs, 5)).cuda()
    S.set_state(u)
    m, e = S.diagnostics()
    U = Solver(case.dim_x, case.dim_v, case.cells, case.lo, case.hi, case.degree, bind=False)
    U.set_mapping(0.03)
    got = _noalloc(U, u)
    assert got[0] == m and got[1] == e
    S.close()
    U.close()
