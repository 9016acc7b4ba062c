"""Error of the FP32 operator mode (and of the FP64 path) against the FP64
oracle for each configuration: the 2D and 4D configurations and the 6D
configuration's 4^6-cell rerun, each over its configured number of LSRK
steps from the configured initial state. Prints one JSON line per
configuration; run on a GPU host:

  python tests/fp32_error_report.py [--configs 2d,4d,6d_small]

Errors are relative L2 norms, weighted by the quadrature (sqrt of the
oracle's energy of the difference over that of the reference) and plain
(unweighted vector norms).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))

from gpu_helpers import gpu_solver, oracle_problem, rel_l2  # noqa: E402
from paper_2002_08110_amd import workloads as W  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", default="2d,4d,6d_small")
    args = ap.parse_args()
    cases = {"2d": W.CONFIG_2D, "4d": W.CONFIG_4D, "6d_small": W.CONFIG_6D_SMALL}
    for name in args.configs.split(","):
        case = cases[name]
        P = oracle_problem(case)
        u0 = P.init_state(case.ic, list(case.ic_params))
        dt = P.stable_dt(case.cfl)
        t0 = time.time()
        ref = P.rk_steps(u0, dt, case.steps)
        t_oracle = time.time() - t0
        e_ref = P.diagnostics(ref)[1]
        out = {"config": case.name, "ndofs": P.ndofs, "steps": case.steps, "dt": dt,
               "oracle_s": t_oracle}
        for prec in ("fp64", "fp32"):
            S = gpu_solver(case, prec)
            S.init_state(case.ic, list(case.ic_params))
            S.rk_step(dt, case.steps)
            got = S.get_state()
            S.close()
            out[prec + "_rel_l2_weighted"] = float(np.sqrt(P.diagnostics(got - ref)[1] / e_ref))
            out[prec + "_rel_l2"] = rel_l2(got, ref)
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
