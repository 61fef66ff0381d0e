"""Learned warm start for the multiplicative NMF solver: data pipeline,
training and time-to-tolerance runs.

Every numerical step runs in the HIP library:
- solves: nmf.Nmf (multiplicative updates, FP32 or BF16 tier);
- gauge fixing: nmf.normalize_gauge;
- the network: nmf.Mlp (bf16 matrix-core products, Adam).
This module only schedules those calls and moves tensors between them.

Pipeline (for a stream of matrices V_m that share a dictionary):
1. mean dictionary W-bar: a joint factorization of the column-wise
   concatenation of a few training matrices, columns scaled to unit norm;
2. targets: each training matrix is factored starting from W = W-bar (to
   the same gap tolerance the solves use, or for a fixed iteration count),
   and the result is put in the unit-norm-column gauge, so that its H
   columns h_j are expressed in (nearly) W-bar's basis;
3. the network is trained on the pairs (v_j, h_j);
4. a new matrix starts from H0 = network(V) and W0 = W-bar ("net"), or W0 =
   the least-squares dictionary for H0 clipped to a positive floor
   (nmf_refit_w, "net_ls"), and is refined by the multiplicative updates
   (which never increase the objective).
"""
from __future__ import annotations

import time

from . import nmf


def _sync():
    import torch
    torch.cuda.synchronize()


def mean_dictionary(Vs, r, iters, precision="bf16", seed=1):
    """Unit-norm-column W-bar (p x r) from a joint factorization of the
    column-wise concatenation of the matrices in Vs."""
    import torch
    Vcat = torch.cat(list(Vs), dim=1).contiguous()
    p, n = Vcat.shape
    W = torch.empty((p, r), dtype=torch.float32, device=Vcat.device)
    H = torch.empty((r, n), dtype=torch.float32, device=Vcat.device)
    with nmf.Nmf(Vcat, W, H, precision=precision, seed=seed) as ctx:
        ctx.step(iters)
    nmf.normalize_gauge(W, H)
    _sync()
    del Vcat, H
    return W


def fit_targets(Vs, Wbar, iters=None, precision="bf16", tol=None, check_every=50,
                max_iters=20000):
    """For each V: factor from (W-bar, constant H) and return H in the
    unit-norm-column gauge (r x n tensors).  With tol: run to the gap
    f / ||V||^2 <= tol (the solver-converged factors); else `iters`
    iterations."""
    import torch
    out = []
    r = Wbar.shape[1]
    for V in Vs:
        W = Wbar.clone()
        H = torch.full((r, V.shape[1]), 1.0 / r, dtype=torch.float32, device=V.device)
        if tol is not None:
            with nmf.Nmf(V, W, H, precision=precision, tol_kind="gap", tol=tol,
                         check_every=check_every) as ctx:
                ctx.solve(max_iters)
        else:
            with nmf.Nmf(V, W, H, precision=precision) as ctx:
                ctx.step(iters)
        nmf.normalize_gauge(W, H)
        out.append(H)
    _sync()
    return out


def output_bias(Hs):
    """Starting output bias: softplus^-1 of the mean target entry, so that the
    untrained network already predicts the targets' mean.  (With a zero bias
    the first Adam steps push the softplus deep into its flat negative range,
    where its slope, and with it every gradient, all but vanishes.)"""
    import math
    tot = sum(float(H.sum()) for H in Hs)
    cnt = sum(H.numel() for H in Hs)
    mean = max(tot / cnt, 1e-6)
    return math.log(math.expm1(mean))


def make_network(params, Hs, max_batch):
    """nmf.Mlp from initial [M1, b1, M2, b2] (numpy or torch) with b2 set by
    output_bias(Hs)."""
    import numpy as np
    M1, b1, M2, b2 = (np.array(x, dtype=np.float32, copy=True) for x in params)
    b2[:] = output_bias(Hs)
    return nmf.Mlp([M1, b1, M2, b2], max_batch=max_batch)


def inference_copy(net, max_batch):
    """A copy of a trained network (and of its stored dictionary) whose
    buffers take max_batch columns at once, so a whole matrix is predicted
    in one pass instead of in chunks of the training batch."""
    out = nmf.Mlp(net.params(), max_batch=max_batch)
    if getattr(net, "_wbar", None) is not None:
        out.set_dictionary(net._wbar)
    return out


def train(net, Vs, Hs, epochs, lr, batch=512, decay=0.9, seed=0, log=None):
    """Adam epochs over the (V_m, H_m) pairs in minibatches of `batch`
    columns, run by the library's training loop (nmf_ws_train: matrices in
    a seeded random order each epoch, the learning rate scaled by `decay`
    after each epoch).  Returns the mean minibatch loss of each epoch."""
    losses = net.train_loop(Vs, Hs, epochs, lr, batch, decay=decay, seed=seed)
    if log:
        rate = lr
        for ep, loss in enumerate(losses):
            log(f"epoch {ep}: loss {loss:.4e} lr {rate:.2e}")
            rate *= decay
    return losses


def solve_to_gap(V, start, tol=1e-4, precision="fp32", check_every=10, max_iters=20000,
                 net=None, Wbar=None, seed=None, ls_floor=1e-3, hfit=20, qn=0):
    """Time to reach f / ||V||_F^2 <= tol from a given start (V already on
    the device).  start: "cold" (device U(0,1) draw keyed by `seed`),
    "wbar" (W-bar and a constant H), "net" (nmf_ws_predict: the network's
    stored W-bar and H0 = net(V)),
    "net_ls" (H0 = net(V), W0 refit to H0 by least squares) or "hfit_ls"
    (no network: H fitted to W-bar by `hfit` H-only multiplicative updates
    from a constant H, then W0 refit to that H).
    qn > 0 refines with the QN(qn)-accelerated solver (nmf_solve_qn)
    instead of plain multiplicative updates; iterations then count map
    evaluations (two per QN iteration).
    The clock covers everything after V is resident: the start, context
    set-up (casts, copies), every iteration and every objective check.
    Returns a dict with seconds, iterations, final gap and convergence."""
    import torch
    p, n = V.shape
    r = Wbar.shape[1] if Wbar is not None else net.r
    _sync()
    t0 = time.perf_counter()
    if start == "cold":
        if not seed:
            raise ValueError("a cold start needs a nonzero seed")
        W = torch.empty((p, r), dtype=torch.float32, device=V.device)
        H = torch.empty((r, n), dtype=torch.float32, device=V.device)
        ctx = nmf.Nmf(V, W, H, precision=precision, tol_kind="gap", tol=tol,
                      check_every=check_every, seed=seed)
    else:
        if start in ("net", "net_ls"):
            W, H = net.ws_predict(V)       # W0 = the network's W-bar, H0 = network(V)
        elif start in ("wbar", "hfit_ls"):
            W = Wbar.clone()
            H = torch.full((r, n), 1.0 / r, dtype=torch.float32, device=V.device)
        else:
            raise ValueError(f"unknown start {start!r}")
        ctx = nmf.Nmf(V, W, H, precision=precision, tol_kind="gap", tol=tol,
                      check_every=check_every)
        if start == "hfit_ls":
            for _ in range(hfit):
                ctx.update_h()
        if start in ("net_ls", "hfit_ls"):
            ctx.refit_w(ls_floor)
    accepted = None
    if qn > 0:
        conv, iters, accepted, f, _ = ctx.solve_qn(max_iters, q=qn)
    else:
        conv, iters, f, _ = ctx.solve(max_iters)
    _sync()
    seconds = time.perf_counter() - t0
    gap = f / ctx.data_norm2()
    ctx.close()
    out = {"seconds": seconds, "iters": iters, "gap": gap, "converged": bool(conv)}
    if accepted is not None:
        out["qn_accepted"] = accepted
    return out
