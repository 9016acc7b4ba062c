"""The batched launch's work list (csrc/work_list.h) on the host: built and
checked for seeded scenarios and edge cases, then every item of the grid
walked as the kernels walk it (bisection over item0), under AddressSanitizer
and UndefinedBehaviorSanitizer. Each (solve, tile) pair is visited exactly
once, item0 is strictly increasing in steps of whole XCD rounds (8 items),
padding stays below 8 items per solve, and lists that do not fit one grid,
empty lists and solves without tiles are rejected."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_08110_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "native", "worklist_check.cpp")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("wl") / "worklist_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I" + CSRC, SRC, "-o", exe], check=True)
    return exe


def run(exe, scenarios):
    text = "".join("%d %s\n" % (len(t), " ".join(str(int(x)) for x in t)) for t in scenarios)
    r = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    return r.stdout.split("\n")[: len(scenarios)]


def test_seeded_scenarios_are_walked_exactly_once(checker):
    rng = np.random.default_rng(2002)
    scenarios = [[1], [8], [9], [7, 1, 16, 3]]
    for _ in range(200):
        n = int(rng.integers(1, 40))
        scenarios.append(list(rng.integers(1, 3000, n)))
    scenarios.append(list(rng.integers(1, 20, 1024)))  # the largest batch
    out = run(checker, scenarios)
    for t, line in zip(scenarios, out):
        assert line.startswith("ok "), line
        want = sum((x + 7) // 8 * 8 for x in t)
        assert int(line.split()[1]) == want


def test_batch_mix_tile_counts(checker):
    # Tile counts of the seeded 96-solve mix under one workgroup per cell
    # (and per 8 cells), as its tuned plans give them.
    from paper_2002_08110_amd import workloads as W
    cases = W.batch_mix()
    cells = [int(np.prod(c.cells)) for c in cases]
    out = run(checker, [cells, [(c + 7) // 8 for c in cells]])
    assert all(line.startswith("ok ") for line in out), out


def test_lists_beyond_one_grid_and_empty_solves_are_rejected(checker):
    out = run(checker, [[2 ** 31 - 8, 16], [5, 0, 3], [2 ** 32 - 1]])
    assert all(line.startswith("rejected") for line in out), out
