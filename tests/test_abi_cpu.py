"""CPU-only checks of the C ABI library: it loads without a GPU, exports every
entry point include/hd.h declares, and rejects invalid descriptors. No
compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2002_08110_amd import _hd
    if not os.path.exists(_hd.LIB_PATH):
        from paper_2002_08110_amd import build
        build.build()
    return _hd.load()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hd.h")).read()
    return sorted(set(re.findall(r"\b(hd_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib()
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    from paper_2002_08110_amd._hd import SYMBOLS
    assert sorted(SYMBOLS) == names


def _mesh(dx, dv, cells, lo=None, hi=None):
    from paper_2002_08110_amd._hd import hd_mesh
    m = hd_mesh()
    m.dim_x, m.dim_v = dx, dv
    d = dx + dv
    for j in range(d):
        m.cells[j] = cells[j]
        m.lo[j] = 0.0 if lo is None else lo[j]
        m.hi[j] = 1.0 if hi is None else hi[j]
    return m


@pytest.mark.parametrize("dx,dv,cells,k,prec,status", [
    (0, 1, [1, 1], 3, 0, -1), (1, 4, [1] * 5, 3, 0, -1), (1, 1, [0, 2], 3, 0, -1),
    (1, 1, [2, 2], 0, 0, -1), (1, 1, [2, 2], 6, 0, -2), (1, 1, [2, 2], 3, 7, -1),
    (1, 2, [2, 2, 2], 3, 0, -2), (3, 3, [8] * 6, 3, 0, 0), (3, 3, [8] * 6, 5, 1, 0),
])
def test_create_validates_descriptors(dx, dv, cells, k, prec, status):
    lib = _lib()
    m = _mesh(dx, dv, cells)
    h = ctypes.c_void_p()
    r = lib.hd_create(ctypes.byref(m), k, prec, ctypes.byref(h))
    assert r == status, lib.hd_last_error()
    if r == 0:
        lib.hd_destroy(h)
    else:
        assert lib.hd_last_error()


def test_lo_ge_hi_rejected_and_sizes():
    lib = _lib()
    m = _mesh(1, 1, [2, 2], lo=[0, 1], hi=[1, 1])
    h = ctypes.c_void_p()
    assert lib.hd_create(ctypes.byref(m), 2, 0, ctypes.byref(h)) == -1
    m = _mesh(3, 3, [8] * 6)
    assert lib.hd_create(ctypes.byref(m), 3, 0, ctypes.byref(h)) == 0
    n = ctypes.c_int64()
    sb = ctypes.c_size_t()
    b = ctypes.c_size_t()
    assert lib.hd_num_dofs(h, ctypes.byref(n)) == 0 and n.value == 8 ** 6 * 4 ** 6
    assert lib.hd_required_bytes(h, ctypes.byref(sb), ctypes.byref(b)) == 0
    # state: two FP64 solution buffers; workspace: FP64 du (the third vector
    # of Sec. 5.4) + small tables and the Vlasov-Poisson scratch (density
    # partial sums over <= 2^20 threads, transform buffers for 33^3 modes,
    # and for the 6D degree-3 kernel one velocity moment per 16 DoFs)
    assert sb.value == 2 * 8 * n.value
    mom = 8 * (n.value // 16)
    assert 8 * n.value + mom <= b.value < 8 * n.value + mom + (1 << 24)
    # a missing output pointer is rejected
    assert lib.hd_required_bytes(h, ctypes.byref(sb), None) == -1
    # calls that need bound memory fail cleanly before hd_bind
    dt = ctypes.c_double()
    assert lib.hd_rk_step(h, ctypes.c_double(1e-3), 1, None) == -1
    assert lib.hd_stable_dt(h, ctypes.c_double(0.2), ctypes.byref(dt)) == -1  # zero field
    lib.hd_destroy(h)
    m = _mesh(3, 3, [8] * 6)
    assert lib.hd_create(ctypes.byref(m), 3, 1, ctypes.byref(h)) == 0
    assert lib.hd_required_bytes(h, ctypes.byref(sb), ctypes.byref(b)) == 0
    assert sb.value == 2 * 8 * n.value
    assert 4 * n.value + mom <= b.value < 4 * n.value + mom + (1 << 24)  # FP32 du
    lib.hd_destroy(h)


def test_plan_validation_without_gpu():
    from paper_2002_08110_amd._hd import hd_plan
    lib = _lib()
    m = _mesh(3, 3, [8] * 6)
    h = ctypes.c_void_p()
    assert lib.hd_create(ctypes.byref(m), 3, 0, ctypes.byref(h)) == 0
    p = hd_plan()
    assert lib.hd_get_plan(h, ctypes.byref(p)) == 0
    assert p.reg_dims in (1, 2)
    q = hd_plan(lds=1, cells_per_wg=2, wg_size=256, xcd_remap=1, reg_dims=1)
    assert lib.hd_set_plan(h, ctypes.byref(q)) == -1  # 2 x 1024 threads
    q = hd_plan(lds=0, cells_per_wg=1, wg_size=100, xcd_remap=1, reg_dims=1)
    assert lib.hd_set_plan(h, ctypes.byref(q)) == -1
    q = hd_plan(lds=0, cells_per_wg=1, wg_size=128, xcd_remap=0, reg_dims=2)
    assert lib.hd_set_plan(h, ctypes.byref(q)) == 0
    lib.hd_destroy(h)


@pytest.mark.parametrize("d,k,precision", [(d, k, p) for d in (2, 3, 4, 5, 6) for k in (1, 2, 3, 4, 5)
                                           for p in ("fp64", "fp32")])
def test_autotune_candidates_are_valid_plans(d, k, precision):
    # Every plan the autotuner times passes the library's plan validation.
    _lib()
    from paper_2002_08110_amd import autotune
    from paper_2002_08110_amd import workloads as W
    from paper_2002_08110_amd.solver import Solver
    dx, dv = W.SPLITS[d]
    S = Solver(dx, dv, [2] * d, [0.0] * d, [1.0] * d, k, precision=precision, bind=False)
    plans = autotune.candidate_plans(d, k, dv, precision)
    assert plans
    default = S.get_plan()
    for plan in plans:
        S.set_plan(**plan)
    S.close()
    assert any(autotune.same_launch(default, p) for p in plans)


def test_autotune_cache_lookup(tmp_path):
    import json
    from paper_2002_08110_amd import autotune
    path = tmp_path / "plans.json"
    plan = dict(kernel=0, options=0, lds=1, cells_per_wg=4, reg_dims=1, xcd_remap=1, wg_size=256)
    path.write_text(json.dumps({autotune.key("gfx950", 4, 3, "fp32"): {"plan": plan}}))
    assert autotune.lookup(4, 3, "fp32", path=str(path), arch="gfx950") == plan
    assert autotune.lookup(4, 3, "fp64", path=str(path), arch="gfx950") is None
    assert autotune.lookup(4, 3, "fp32", path=str(tmp_path / "none.json"), arch="gfx950") is None


def declared_signatures():
    """name -> parameter list (text) of every function include/hd.h declares."""
    text = open(os.path.join(ROOT, "include", "hd.h")).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(hd_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", text):
        params = [p.strip() for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
        out[m.group(1)] = params
    return out


def test_binding_argument_counts_match_the_header():
    # The ctypes declarations marshal exactly the header's parameters.
    lib = _lib()
    sigs = declared_signatures()
    assert set(sigs) == set(declared_symbols())
    for name, params in sigs.items():
        assert len(getattr(lib, name).argtypes) == len(params), (name, params)


def test_boundary_signatures():
    # State and workspace are separate caller-owned buffers; the FP32 mode is
    # named for what it computes (FP32 operator, FP64 accumulation).
    sigs = declared_signatures()
    assert sigs["hd_required_bytes"] == ["const hd_solver *s", "size_t *state_bytes",
                                         "size_t *workspace_bytes"]
    assert sigs["hd_bind"] == ["hd_solver *s", "void *state_dev", "size_t state_bytes",
                               "void *workspace_dev", "size_t workspace_bytes"]
    text = open(os.path.join(ROOT, "include", "hd.h")).read()
    assert re.search(r"HD_FP64\s*=\s*0\s*,\s*HD_FP32_OP_FP64_ACC\s*=\s*1", text)
    from paper_2002_08110_amd import _hd
    assert _hd.HD_FP64 == 0 and _hd.HD_FP32_OP_FP64_ACC == 1


def test_bind_rejects_bad_buffers_without_gpu():
    # Argument checks of hd_bind run before any device call.
    lib = _lib()
    m = _mesh(1, 1, [2, 2])
    h = ctypes.c_void_p()
    assert lib.hd_create(ctypes.byref(m), 2, 0, ctypes.byref(h)) == 0
    sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.hd_required_bytes(h, ctypes.byref(sb), ctypes.byref(wb)) == 0
    base = 1 << 40  # never dereferenced: every case fails its checks first
    S, W = ctypes.c_void_p(base), ctypes.c_void_p(base + (1 << 30))
    assert lib.hd_bind(h, None, sb.value, W, wb.value) == -1
    assert lib.hd_bind(h, S, sb.value - 8, W, wb.value) == -1
    assert lib.hd_bind(h, S, sb.value, W, wb.value - 8) == -1
    assert lib.hd_bind(h, ctypes.c_void_p(base + 8), sb.value, W, wb.value) == -1
    assert lib.hd_bind(h, S, sb.value, ctypes.c_void_p(base + 256), wb.value) == -1  # overlap
    assert b"overlap" in lib.hd_last_error()
    lib.hd_destroy(h)


def test_noalloc_diagnostics_rejects_null_and_oversized_meshes_before_any_device_call():
    # Both checks return before the entry point touches a device.
    lib = _lib()
    h = ctypes.c_void_p()
    m = _mesh(3, 3, [32, 32, 32, 32, 32, 1])
    assert lib.hd_create(ctypes.byref(m), 5, 0, ctypes.byref(h)) == 0
    n = ctypes.c_int64()
    assert lib.hd_num_dofs(h, ctypes.byref(n)) == 0 and n.value > 2 ** 40
    fake = ctypes.c_void_p(256)
    assert lib.hd_diagnostics_noalloc(h, fake, fake, None) == -1
    assert b"2^40" in lib.hd_last_error()
    assert lib.hd_diagnostics_noalloc(h, None, fake, None) == -1
    assert lib.hd_diagnostics_noalloc(h, fake, None, None) == -1
    assert lib.hd_diagnostics_noalloc(None, fake, fake, None) == -1
    lib.hd_destroy(h)
