"""Writes ch_long_parity.json: the oracle's Cahn-Hilliard state after many
steps, sampled, and the oracle's own rounding spread over the same run, for
the long-horizon GPU parity test.

Runs only the oracle (oracle.ch_run, the ADI step of Sec. 5.1 in double
precision) from the seeded initial data of workloads.ch_initial (seed 2,
0.1 U(-1, 1), the deep quench of Sec. 5.3) on the periodic square (0, 2 pi)^2
with dt = 0.1 dx^2, D = 1, gamma = 0.01 and the start rule C^{-1} = C^0:

* 1024 x 1024 to 1000 steps (checkpoints 3, 10, 30, 100, 300, 1000),
* 4096 x 4096 to 20 steps (checkpoints 2, 5, 10, 20).

Rounding spread.  On a square grid (dx = dy) the x and y line operators of
the scheme are the same matrix acting along the two axes, so they commute,
and the 13-point biharmonic and 5-point Laplacian windows are symmetric under
exchanging x and y and under reflecting either axis (Sec. 5.1).  The exact
run started from the transposed field C^0^T is therefore the transpose of
the run from C^0, and the run from the field reflected in both axes is the
reflection of the run from C^0.  In double precision these runs round
differently: the transposed run swaps the order of the two sweeps, and the
reflected run accumulates every stencil sum in the opposite order along
both axes and eliminates every line from its other end, much as a second
implementation would.  Both keep the oracle's own rounded coefficients,
though: the window weights and band values, rounded once and used at every
step.  A second implementation rounds them its own way (the weights of the
13-point window as products or as quotients), and that difference, repeated
at every step, makes two runs drift apart linearly in n where the
transposed and reflected runs do not.  The third alternative run measures
it: every nonzero window weight and band value moved by one unit in the
last place, up or down by a seeded sequence (oracle.ch_run_nudged, seed 1).

The spread at step n is max |C_n - (alternative run, mapped back)| over the
whole grid, the largest of the three: how far two equally valid double
evaluations of the scheme drift apart after n steps.  The GPU test allows a
stated small multiple of it.

For each checkpoint the file stores the three spreads and their maximum,
max |C| and the plain sum of C^n, every value of one row and one column, and
2048 seeded random points (seed 11).  The eight runs (four per grid) go to
separate processes; the slowest (1024^2, 1000 steps) takes about 9 minutes
single-threaded.

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

CASES = ((1024, (3, 10, 30, 100, 300, 1000)), (4096, (2, 5, 10, 20)))
NSAMPLE = 2048
D, GAMMA = 1.0, 0.01


def run(args):
    """The oracle run of one grid, from C^0 or from its transpose; returns
    the state C^n at every checkpoint (transposed back for the second)."""
    import oracle
    from paper_1902_09931_amd import workloads as wl

    n, checkpoints, mode = args
    # the map applied to the initial field, and its inverse for the results
    fwd = {"direct": lambda a: a, "transposed": lambda a: a.T, "reflected": lambda a: a[::-1, ::-1],
           "nudged": lambda a: a}[mode]
    c0 = np.ascontiguousarray(fwd(wl.ch_initial(n, n, seed=2)))
    dx = 2 * math.pi / n
    cp, cc = c0.copy(), c0.copy()
    done, states = 0, {}
    for k in checkpoints:
        if mode == "nudged":
            cp, cc = oracle.ch_run_nudged(cp, cc, k - done, dx, dx, 0.1 * dx * dx, 1, D, GAMMA)
        else:
            cp, cc = oracle.ch_run(cp, cc, k - done, dx, dx, 0.1 * dx * dx, D, GAMMA)
        done = k
        states[k] = np.ascontiguousarray(fwd(cc))   # both maps are their own inverse
    return states


def main():
    import oracle
    from paper_1902_09931_amd import workloads as wl

    modes = ("direct", "transposed", "reflected", "nudged")
    jobs = [(n, cps, m) for n, cps in CASES for m in modes]
    with ProcessPoolExecutor(len(jobs)) as ex:
        results = list(ex.map(run, jobs))
    cases = []
    for ci, (n, cps) in enumerate(CASES):
        ref, alt, refl, ndg = results[4 * ci: 4 * ci + 4]
        c0 = wl.ch_initial(n, n, seed=2)
        dx = 2 * math.pi / n
        rng = np.random.default_rng(11)
        jj = rng.integers(0, n, NSAMPLE)
        ii = rng.integers(0, n, NSAMPLE)
        row, col = n // 3, (2 * n) // 5
        checks = []
        for k in cps:
            c = ref[k]
            st = float(np.abs(c - alt[k]).max())
            sr = float(np.abs(c - refl[k]).max())
            sn = float(np.abs(c - ndg[k]).max())
            checks.append({
                "steps": k,
                "spread": max(st, sr, sn),
                "spread_transposed": st,
                "spread_reflected": sr,
                "spread_nudged": sn,
                "max_abs": float(np.abs(c).max()),
                "sum": float(oracle.mass(c)),
                "row_values": c[row].tolist(),
                "col_values": c[:, col].tolist(),
                "points_values": c[jj, ii].tolist(),
            })
        cases.append({
            "n": n,
            "dt": 0.1 * dx * dx,
            "max_abs_c0": float(np.abs(c0).max()),
            "sum_abs_c0": float(np.abs(c0).sum()),
            "row": row,
            "col": col,
            "points_j": jj.tolist(),
            "points_i": ii.tolist(),
            "checkpoints": checks,
        })
    out = {
        "citation": "Sec. 5.1 (ADI scheme), Sec. 5.3 (random initial data); values from the oracle",
        "writer": "tests/golden/make_ch_long.py",
        "D": D,
        "gamma": GAMMA,
        "cases": cases,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ch_long_parity.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f)
    os.replace(path + ".tmp", path)
    for c in cases:
        print(c["n"], [(k["steps"], k["spread"], k["max_abs"]) for k in c["checkpoints"]])
    print("wrote", path)


if __name__ == "__main__":
    main()
