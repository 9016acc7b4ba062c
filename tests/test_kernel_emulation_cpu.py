"""The generic stage kernel compiled for the host (tests/native/emu_stage.cpp:
one host thread per GPU thread, __syncthreads a barrier, workgroups one after
another) under AddressSanitizer and UndefinedBehaviorSanitizer, in both its
own launch form and its batched work-list form.

Cases: the ten mixed-dimension solves of the batched-stepping GPU tests with
the launch plans that the three plan-varied parameter sets draw (the sets
kept off the GPU: an earlier work-list design faulted on them), in both
precisions, in operator mode and in each of the five stage variants. For each
case: no access leaves its buffer or the launch's dynamic LDS, the work-list
form (two slots) equals the own launch bitwise, and the result matches the
oracle (FP64 within 1e-12 relative L2; FP32 within 2e-6). Among them is the
6D degree-3 kernel (cross-lane moves exchanged between the threads of a
64-lane wave) in each of its three stage variants.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2002_08110_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "tests"))
from gpu_helpers import all_plans, oracle_problem  # noqa: E402
from test_gpu_batch import MIX, make_case  # noqa: E402

CXX = "/opt/rocm/llvm/bin/clang++"
SRC = os.path.join(ROOT, "tests", "native", "emu_stage.cpp")


def _variant(case, plan, precision):
    if plan.get("kernel", 0) == 1:
        # The 6D degree-3 kernel: FP64 uses option bit 0 only, FP32 both bits.
        opt = plan.get("options", 0) & (3 if precision == "fp32" else 1)
        return dict(K3=1, D=6, N=4, DX=3, RD=2, P="float" if precision == "fp32" else "double",
                    LDS="true", SD=0, OPT=opt, LD=0)
    return dict(K3=0, D=case.d, N=case.degree + 1, DX=case.dim_x, RD=plan["reg_dims"],
                P="float" if precision == "fp32" else "double",
                LDS="true" if plan["lds"] else "false", SD=plan.get("split_dims", 0),
                OPT=plan.get("options", 0) & 1, LD=plan.get("loop_dims", 0))


def _cases():
    out = []
    for precision in ("fp64", "fp32"):
        for i, m in enumerate(MIX):
            case = make_case(i, *m)
            plans = all_plans(case, precision)
            plan = plans[(7 * i) % len(plans)]
            out.append((precision, i, case, plan))
    return out


CASES = _cases()


@pytest.fixture(scope="module")
def binaries(tmp_path_factory):
    if not os.path.exists(CXX):
        pytest.skip("clang++ of the ROCm toolchain not available")
    out = tmp_path_factory.mktemp("emu")
    variants = {}
    for precision, i, case, plan in CASES:
        v = _variant(case, plan, precision)
        variants[tuple(sorted(v.items()))] = v

    def build(v):
        name = "emu_" + "_".join(str(v[k]) for k in sorted(v))
        exe = str(out / name)
        cmd = [CXX, "-std=c++20", "-O1", "-g", "-pthread", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "tests", "native", "emu"),
               "-I" + os.path.join(ROOT, "paper_2002_08110_amd", "csrc"),
               "-I" + os.path.join(ROOT, "include")]
        cmd += ["-DEMU_%s=%s" % (k, v[k]) for k in sorted(v) if k != "K3"]
        cmd += (["-DEMU_K3"] if v["K3"] else []) + [SRC, "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True)
        return exe

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 2)) as ex:
        exes = dict(zip(variants, ex.map(build, variants.values())))
    return exes, out


def _write_spec(d, case, plan, mode, stage, dt, A, B):
    lines = [" ".join(str(c) for c in case.cells), " ".join(repr(float(x)) for x in case.lo),
             " ".join(repr(float(x)) for x in case.hi)]
    if case.field == "constant":
        lines += ["0", " ".join(repr(float(x)) for x in case.a)]
    else:
        lines += ["1", "1.0"]
    lines.append("%d %d %d %d %d %r %r %r" % (plan.get("cells_per_wg", 1), plan.get("wg_size", 256),
                                           plan.get("xcd_remap", 0), mode, stage, float(dt),
                                           float(A[stage]), float(B[stage])))
    with open(os.path.join(d, "spec.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


@pytest.mark.parametrize("precision,i,case,plan", CASES,
                         ids=["%s-%d" % (c[0], c[1]) for c in CASES])
def test_plan_varied_kernels_on_the_host(binaries, precision, i, case, plan):
    exes, out = binaries
    exe = exes[tuple(sorted(_variant(case, plan, precision).items()))]
    d = str(out / ("%s_%d" % (precision, i)))
    os.makedirs(d, exist_ok=True)
    P = oracle_problem(case)
    pt = np.float32 if precision == "fp32" else np.float64
    u = W.random_state(P.ndofs, 11 + i)
    du = W.random_state(P.ndofs, 21 + i).astype(pt)
    u.tofile(os.path.join(d, "u.bin"))
    du.tofile(os.path.join(d, "du.bin"))
    if case.field != "constant":
        P.sine_table(case.amp).astype(pt).tofile(os.path.join(d, "E.bin"))
    A, B, _ = oracle.lsrk45_coefficients()
    dt = P.stable_dt(0.2)
    L = P.apply(u)
    tol = 1e-12 if precision == "fp64" else 2e-6
    scale = np.linalg.norm(L)
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
