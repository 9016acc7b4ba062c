"""The even-odd line transforms of the Gauss-Legendre sweep kernel
(csrc/stage_gauss.h, Sec. 2.6 sum factorization) compiled for the host
(tests/native/evenodd_check.cpp, AddressSanitizer + UBSan): equal to the
dense products to rounding for random centro-symmetric and
centro-antisymmetric matrices of sizes 2..6 and for the library's own
interpolation and derivative tables at degrees 1..5, whose (anti)symmetry
the even-odd form assumes is checked too."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CXX = "/opt/rocm/llvm/bin/clang++"


def test_even_odd_transforms_equal_dense_products(tmp_path):
    if not os.path.exists(CXX):
        pytest.skip("clang++ of the ROCm toolchain not available")
    exe = str(tmp_path / "evenodd_check")
    subprocess.run([CXX, "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "tests", "native", "emu"),
                    "-I" + os.path.join(ROOT, "paper_2002_08110_amd", "csrc"),
                    "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "native", "evenodd_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert r.stdout.strip().endswith("all ok")
    assert r.stdout.count(" ok") >= 30
