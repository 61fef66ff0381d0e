"""The stored float64 trajectory of the precision tier
(tests/golden/precision_tier_fp64.json) against what fixes it without
re-running 200 iterations: the objective of the seeded start recomputed by
the oracle, the descent property of the method (the objective never
increases, Sec. 3.1), nonnegative factors, and a gap that decreased."""
import json
import os

import numpy as np

from oracle import nmf_oracle as O
from synth import generators as g

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "precision_tier_fp64.json")


def test_precision_tier_fixture_is_a_descent_trajectory():
    d = json.load(open(GOLDEN))
    assert sorted(d["ranks"]) == ["128", "256", "32"]
    for r, rr in d["ranks"].items():
        f = [rr["f"][str(k)] for k in d["checkpoints"]]
        assert all(b <= a * (1 + 1e-13) for a, b in zip(f, f[1:])), r
        assert f[-1] / rr["data_norm2"] < 0.05 < f[0] / rr["data_norm2"]
        assert min(rr["W200_sample"]) >= 0 and min(rr["H200_sample"]) >= 0
        assert len(rr["W200_sample"]) == len(rr["H200_sample"]) == d["sample"]["count"]


def test_precision_tier_fixture_start_matches_the_generator():
    """f_0 and ||V||^2 of the rank-32 case recomputed from the seeded
    generator (the stored numbers belong to the workload they name)."""
    d = json.load(open(GOLDEN))["ranks"]["32"]
    V, W0, H0 = g.precision_tier(32)
    V64 = V.astype(np.float64)
    assert abs(float(np.sum(V64 * V64)) - d["data_norm2"]) <= 1e-12 * d["data_norm2"]
    f0 = O.objective(V64, W0, H0)
    assert abs(f0 - d["f"]["0"]) <= 1e-12 * f0
