#!/usr/bin/env python3
"""Write the oracle's full-size reference trajectories (tests/golden/fullsize_n*.npz).

The full-size parity tests step the workloads' full-spectrum fields (every degree l <= N - 1)
in the configuration bench.py times: polynomial starting iterate from the run's midpoints
(degree 3; the third and fourth steps from the midpoints and the states), W_{n+1} = W_n +
h (A - A^H), tol 1e-12.  The oracle needs minutes for that at
N = 2048 and 4096 (the full eigenvector basis of every diagonal, then dense FP64 products),
so this script runs it once and stores what the tests compare against: every entry of a few
rows and a seeded random sample of entries, of W_0 and of the state after the stored step
counts, with the evaluation counts, residuals, Frobenius norms and Casimirs of each state.

Only ``oracle`` and the seeded coefficient generator of ``workloads`` are called.

    python tests/golden/make_fullsize_reference.py [--n 2048 4096] [--workers 8]
"""

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import WORKLOADS, omega_coeffs  # noqa: E402

# (workload, stored step counts): n4096 as timed (20 steps) and its configuration's 10
PLANS = {4096: ("n4096", (10, 20)), 2048: ("n2048", (20,))}
SAMPLE_ENTRIES = 2048


def sample_points(N):
    rng = np.random.default_rng(7000 + N)
    rows = np.array([0, N // 2, N - 1])
    r = rng.integers(0, N, SAMPLE_ENTRIES)
    c = rng.integers(0, N, SAMPLE_ENTRIES)
    return rows, r, c


def make(N, workers):
    wname, counts = PLANS[N]
    cfg = WORKLOADS[wname]
    seed = cfg["seeds"][0]
    rows, r, c = sample_points(N)
    t0 = time.time()
    W0 = oracle.assemble(N, omega_coeffs(N, seed, cfg["law"]), workers=workers)
    print(f"N={N}: W_0 assembled in {time.time() - t0:.0f} s", flush=True)
    out = {"N": N, "h": cfg["h"], "tol": cfg["tol"], "maxit": cfg["maxit"], "seed": seed,
           "law": cfg["law"], "degree": 3, "solution_differences": True,
           "update": "difference", "steps": np.array(counts),
           "rows": rows, "sample_r": r, "sample_c": c}

    def store(tag, W):
        out[f"{tag}_rows"] = W[rows]
        out[f"{tag}_sample"] = W[r, c]
        out[f"{tag}_fro"] = np.linalg.norm(W)
        out[f"{tag}_casimirs"] = oracle.casimirs(W, 4)

    store("W0", W0)

    def on_step(n, W):
        if n in counts:
            store(f"W{n}", W)
            print(f"N={N}: step {n} stored ({time.time() - t0:.0f} s)", flush=True)

    _, iters, res = oracle.isomp_run(W0, cfg["h"], max(counts), cfg["tol"], cfg["maxit"],
                                     extrapolate=True, degree=3, update="difference",
                                     on_step=on_step, solution_differences=True)
    out["iters"] = np.array(iters)
    out["resid"] = np.array(res)
    path = os.path.join(HERE, f"fullsize_n{N}.npz")
    np.savez(path, **out)
    print(f"N={N}: iterations {iters}, wrote {path} ({time.time() - t0:.0f} s)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[2048, 4096])
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    a = ap.parse_args()
    for N in a.n:
        make(N, a.workers)


if __name__ == "__main__":
    main()
