"""Writes ch_long_parity.json: the oracle's Cahn-Hilliard state after many
steps, sampled, for the long-horizon GPU parity test.

Runs only the oracle (oracle.ch_run, the ADI step of Sec. 5.1 in double
precision) from the seeded initial data of workloads.ch_initial (seed 2,
0.1 U(-1, 1), the deep quench of Sec. 5.3) on the periodic square (0, 2 pi)^2
with dt = 0.1 dx^2, D = 1, gamma = 0.01 and the start rule C^{-1} = C^0:

* 1024 x 1024 for 1000 steps,
* 4096 x 4096 for 20 steps.

For each case it stores max |C| and the plain sum of the final C^n over the
whole grid, every value of one row and one column, and 2048 seeded random
points (seed 11).  One run takes about 9 minutes (1024^2) and 3 minutes
(4096^2) single-threaded; the two cases run in separate processes.

    python tests/golden/make_ch_long.py
"""
import json
import math
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

CASES = ((1024, 1000), (4096, 20))
NSAMPLE = 2048
D, GAMMA = 1.0, 0.01


def run_case(case):
    import oracle
    from paper_1902_09931_amd import workloads as wl

    n, steps = case
    c0 = wl.ch_initial(n, n, seed=2)
    dx = 2 * math.pi / n
    _, c = oracle.ch_run(c0, c0, steps, dx, dx, 0.1 * dx * dx, D, GAMMA)
    rng = np.random.default_rng(11)
    jj = rng.integers(0, n, NSAMPLE)
    ii = rng.integers(0, n, NSAMPLE)
    row, col = n // 3, (2 * n) // 5
    return {
        "n": n,
        "steps": steps,
        "dt": 0.1 * dx * dx,
        "max_abs": float(np.abs(c).max()),
        "sum": float(oracle.mass(c)),
        "sum_abs_c0": float(np.abs(c0).sum()),
        "row": row,
        "row_values": c[row].tolist(),
        "col": col,
        "col_values": c[:, col].tolist(),
        "points_j": jj.tolist(),
        "points_i": ii.tolist(),
        "points_values": c[jj, ii].tolist(),
    }


def main():
    with ProcessPoolExecutor(len(CASES)) as ex:
        results = list(ex.map(run_case, CASES))
    out = {
        "citation": "Sec. 5.1 (ADI scheme), Sec. 5.3 (random initial data); values from the oracle",
        "writer": "tests/golden/make_ch_long.py",
        "D": D,
        "gamma": GAMMA,
        "cases": results,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ch_long_parity.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
