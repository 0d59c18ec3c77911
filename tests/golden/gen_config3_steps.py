"""Write tests/golden/config3_400_oracle.json: the oracle's run of the 2D
Riemann configuration 3 at 400 x 400 to T = 0.8 with CFL 0.45, the setting of
the CPU timing table of Section 4.4 (which reports 3497 RK steps for
WENO-ZA6).

Only the oracle runs here (about 9 minutes on 8 host threads); the stored
step count is what the GPU test must reproduce, and the CPU test compares it
with the paper's 3497.

Usage:  python tests/golden/gen_config3_steps.py [threads]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2603_26272_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "config3_400_oracle.json")


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    oracle.set_threads(threads)
    P, q0, T = W.riemann_config3(400)
    dt0 = oracle.cfl_dt(P, q0)
    # the first 200 steps alone, for a quick reproducibility check
    _, n200, t200, st200 = oracle.solve(P, q0, T, 200)
    assert st200 == 0 and n200 == 200, (st200, n200)
    t0 = time.time()
    q, steps, t, st = oracle.solve(P, q0, T)
    wall = time.time() - t0
    assert st == 0, st
    rho = q[0]
    rec = {
        "what": "oracle, 2D Riemann configuration 3, 400x400 on [0,1]^2, transmissive, "
                "T = 0.8, CFL 0.45, dt = CFL / (max(|u|+c)/dx + max(|v|+c)/dy), SSP-RK3, WENO-ZA6 FP64",
        "paper_steps": 3497,
        "paper_source": "Section 4.4, CPU timing table (WENO-ZA6 row)",
        "steps": int(steps),
        "t": float(t),
        "first_dt": float(dt0),
        "t_after_200_steps": float(t200),
        "rho_min": float(rho.min()),
        "rho_max": float(rho.max()),
        "mass": float(rho.sum()) / (400 * 400),
        "oracle_wall_s": wall,
        "oracle_threads": threads,
    }
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
