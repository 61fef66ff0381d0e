"""Write precision_tier_fp64.json: the float64 oracle's trajectory on the
precision-tier workload (8192 x 32768, planted rank r in {32, 128, 256}, seed
1003 + r, U(0,1) start seed 2003 + r), 200 iterations of Algorithm 1 (NNMF),
Sec. 3.1.

Stored per rank: the objective f_k (Sec. 3.1 eq. nnmf-objfn) at the
checkpoints k in CHECKPOINTS, the Frobenius norms of W_k and H_k at k = 10
and k = 200, and the values of W_200 and H_200 at SAMPLE seeded positions.
The GPU tiers are compared against these numbers by the benchmark (error of
every result against float64) and by the tests.

Only the oracle and the seeded generators are called.  Run from the
repository root:  python tests/golden/make_precision_tier_fp64.py [ranks...]
(about 4 minutes for the three ranks on 8 cores).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import nmf_oracle as oracle  # noqa: E402
from synth import generators as gen  # noqa: E402

OUT = os.path.join(HERE, "precision_tier_fp64.json")
CHECKPOINTS = (0, 1, 2, 5, 10, 20, 50, 100, 150, 200)
SAMPLE = 256
SAMPLE_SEED = 77


def sample_positions(rows, cols, count=SAMPLE, seed=SAMPLE_SEED):
    """Seeded (row, col) positions, shared by the writer and the readers."""
    rng = np.random.default_rng(seed)
    return (rng.integers(0, rows, size=count).tolist(), rng.integers(0, cols, size=count).tolist())


def trajectory(r):
    V, W0, H0 = gen.precision_tier(r)
    p, n = V.shape
    V = V.astype(np.float64)
    W, H = W0.astype(np.float64), H0.astype(np.float64)
    f = {0: oracle.objective(V, W, H)}
    norms = {}
    for k in range(1, CHECKPOINTS[-1] + 1):
        W, H = oracle.step(V, W, H)
        if k in CHECKPOINTS:
            f[k] = oracle.objective(V, W, H)
        if k in (10, 200):
            norms[k] = (float(np.linalg.norm(W)), float(np.linalg.norm(H)))
    wi, wk = sample_positions(p, r)
    hk, hj = sample_positions(r, n)
    return {
        "p": p, "n": n, "r": r,
        "data_norm2": float(np.sum(V * V)),
        "f": {str(k): v for k, v in f.items()},
        "norm_W": {str(k): v[0] for k, v in norms.items()},
        "norm_H": {str(k): v[1] for k, v in norms.items()},
        "W200_sample": [float(W[i, k]) for i, k in zip(wi, wk)],
        "H200_sample": [float(H[k, j]) for k, j in zip(hk, hj)],
    }


def main(ranks):
    data = {}
    if os.path.exists(OUT):
        data = json.load(open(OUT))
    data["about"] = ("float64 oracle (oracle/nmf_oracle.py, numpy BLAS) on the precision-tier "
                     "workload: synth.generators.precision_tier(r), 200 iterations; written by "
                     "tests/golden/make_precision_tier_fp64.py")
    data["checkpoints"] = list(CHECKPOINTS)
    data["sample"] = {"count": SAMPLE, "seed": SAMPLE_SEED}
    data.setdefault("ranks", {})
    for r in ranks:
        t0 = time.perf_counter()
        data["ranks"][str(r)] = trajectory(r)
        print(f"r={r}: f_200 = {data['ranks'][str(r)]['f']['200']:.12g} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
            fh.write("\n")


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [32, 128, 256])
