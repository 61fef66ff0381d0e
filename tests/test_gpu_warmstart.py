"""Warm-start pipeline on a small stream of matrices sharing a dictionary:
the trained network's start reaches the objective gap in fewer iterations
than a cold start, and every run still reaches the tolerance."""
import numpy as np
import pytest
import torch

from synth import generators as g

pytestmark = pytest.mark.gpu


def test_warm_start_pipeline_small(gpu_lib):
    from paper_1003_3272_amd import nmf, warmstart as ws
    p, n, r = 256, 512, 8
    Wb = g.warm_start_base(p=p, r=r, seed=77)
    mats = [torch.from_numpy(g.warm_start_matrix(Wb, m, n=n)[0]).cuda() for m in range(44)]
    train, test = mats[:40], mats[40:]
    Wbar = ws.mean_dictionary(train[:8], r, iters=400)
    norms = torch.linalg.vector_norm(Wbar, dim=0).cpu().numpy()
    assert np.allclose(norms, 1.0, atol=1e-5)
    Hs = ws.fit_targets(train, Wbar, iters=200)
    net = ws.make_network(g.mlp_init(p, 128, r, 5), Hs, max_batch=128)
    losses = ws.train(net, train, Hs, epochs=12, lr=1e-3, batch=128)
    # the float64 oracle with bf16 products, run through the same schedule,
    # goes from about 3e-2 to 2e-3 (a constant predictor scores 8.5e-2)
    print("training loss per epoch:", ["%.3e" % x for x in losses])
    assert losses[-1] < 0.2 * losses[0] and losses[-1] < 1e-2
    res = {k: [] for k in ("cold", "wbar", "net")}
    for i, V in enumerate(test):
        res["cold"].append(ws.solve_to_gap(V, "cold", tol=2e-3, precision="fp32", seed=9000 + i,
                                           Wbar=Wbar))
        res["wbar"].append(ws.solve_to_gap(V, "wbar", tol=2e-3, precision="bf16", Wbar=Wbar))
        res["net"].append(ws.solve_to_gap(V, "net", tol=2e-3, precision="bf16", Wbar=Wbar,
                                          net=net))
    for k, v in res.items():
        assert all(x["converged"] and x["gap"] <= 2e-3 for x in v), (k, v)
    it = {k: np.median([x["iters"] for x in v]) for k, v in res.items()}
    print("median iterations to gap 2e-3:", it)
    assert it["net"] < it["cold"]
    net.close()
