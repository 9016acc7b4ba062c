"""The dimension-split stage passes (plan kernel 2: pass x over rows of
x-nodes, pass v over column blocks, csrc/stage_split.h) compiled for the
host (tests/native/emu_stage.cpp with EMU_SPLIT: one host thread per GPU
thread, __syncthreads a barrier) under AddressSanitizer and
UndefinedBehaviorSanitizer.

Cases: 6D (3 x + 3 v) at degrees 4 and 5 and 5D (3 x + 2 v) at degrees 4
and 5, on meshes with one, two and three cells along different dimensions
(self-neighbours, and distinct left and right neighbours), with the sine
phase-space field (mixed-sign speeds) or a constant field, in both
precisions; an operator application and each of the five LSRK stages. For
each: no access leaves its buffer or the launch's dynamic LDS, and the
result matches the oracle (FP64 within 1e-12 relative L2; FP32 within 2e-6).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2002_08110_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "tests"))
from gpu_helpers import oracle_problem  # noqa: E402
from test_kernel_emulation_cpu import CXX, SRC, _write_spec  # noqa: E402

CASES = [
    ("fp64", W.phase_space_case("s6k5", 3, 3, [3, 1, 2, 1, 2, 3], 5, 1)),
    ("fp32", W.phase_space_case("s6k5", 3, 3, [2, 3, 1, 3, 1, 2], 5, 1)),
    ("fp64", W.Case("s6k4", 3, 3, [3, 2, 1, 1, 3, 2], [0.0] * 6, [1.0] * 6, 4, "constant",
                    a=[0.7, -0.4, 0.3, -0.9, 0.5, -0.2])),
    ("fp32", W.phase_space_case("s6k4", 3, 3, [1, 3, 2, 2, 1, 3], 4, 1)),
    ("fp64", W.Case("s5k5", 3, 2, [3, 2, 3, 1, 3], [0.0] * 5, [1.0] * 5, 5, "constant",
                    a=[-0.6, 0.8, 0.2, 0.45, -0.75])),
    ("fp32", W.Case("s5k4", 3, 2, [2, 3, 3, 3, 2], [0.0] * 5, [1.0] * 5, 4, "constant",
                    a=[0.3, -0.5, 0.9, -0.35, 0.6])),
]


def _variant(case, precision):
    return dict(D=case.d, N=case.degree + 1, DX=case.dim_x, RD=1,
                P="float" if precision == "fp32" else "double", LDS="false", SD=0,
                OPT=1 if case.degree == 5 else 0, LD=0)


@pytest.fixture(scope="module")
def binaries(tmp_path_factory):
    if not os.path.exists(CXX):
        pytest.skip("clang++ of the ROCm toolchain not available")
    out = tmp_path_factory.mktemp("emu_split")
    variants = {}
    for precision, case in CASES:
        v = _variant(case, precision)
        variants[tuple(sorted(v.items()))] = v

    def build(v):
        exe = str(out / ("split_" + "_".join(str(v[k]) for k in sorted(v))))
        cmd = [CXX, "-std=c++20", "-O1", "-g", "-pthread", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "tests", "native", "emu"),
               "-I" + os.path.join(ROOT, "paper_2002_08110_amd", "csrc"),
               "-I" + os.path.join(ROOT, "include"), "-DEMU_SPLIT"]
        cmd += ["-DEMU_%s=%s" % (k, v[k]) for k in sorted(v)] + [SRC, "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True)
        return exe

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 2)) as ex:
        exes = dict(zip(variants, ex.map(build, variants.values())))
    return exes, out


@pytest.mark.parametrize("precision,case", CASES,
                         ids=["%s-%s" % (c[0], c[1].name) for c in CASES])
def test_split_passes_on_the_host(binaries, precision, case):
    exes, out = binaries
    exe = exes[tuple(sorted(_variant(case, precision).items()))]
    d = str(out / ("%s_%s" % (precision, case.name)))
    os.makedirs(d, exist_ok=True)
    P = oracle_problem(case)
    pt = np.float32 if precision == "fp32" else np.float64
    u = W.random_state(P.ndofs, 5)
    du = W.random_state(P.ndofs, 6).astype(pt)
    u.tofile(os.path.join(d, "u.bin"))
    du.tofile(os.path.join(d, "du.bin"))
    if case.field != "constant":
        P.sine_table(case.amp).astype(pt).tofile(os.path.join(d, "E.bin"))
    A, B, _ = oracle.lsrk45_coefficients()
    dt = P.stable_dt(0.2)
    L = P.apply(u)
    tol = 1e-12 if precision == "fp64" else 2e-6
    scale = np.linalg.norm(L)
    plan = dict(cells_per_wg=1, wg_size=256, xcd_remap=1)
    for mode, stage in [(0, 0)] + [(1, s) for s in range(5)]:
        _write_spec(d, case, plan, mode, stage, dt, A, B)
        r = subprocess.run([exe, d], capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
        if mode == 0:
            got = np.fromfile(os.path.join(d, "out.bin"), dtype=pt).astype(np.float64)
            assert np.linalg.norm(got - L) <= tol * scale, (mode, stage)
        else:
            got_u = np.fromfile(os.path.join(d, "out_u.bin"), dtype=np.float64)
            got_du = np.fromfile(os.path.join(d, "out_du.bin"), dtype=pt).astype(np.float64)
            want_du = dt * L + (A[stage] * du.astype(np.float64) if stage > 0 else 0.0)
            want_u = u + B[stage] * want_du
            ref = np.linalg.norm(want_du)
            if stage < 4:
                assert np.linalg.norm(got_du - want_du) <= tol * ref, (mode, stage)
            assert (np.linalg.norm(got_u - want_u)
                    <= tol * abs(B[stage]) * ref + 1e-15 * np.linalg.norm(u)), (mode, stage)
