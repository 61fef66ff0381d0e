"""Plain FP64 CPU oracle for the Poisson (Kullback-Leibler) variant of
multiplicative NMF, Sec. 3.1 (last two displays).

TEST INFRASTRUCTURE ONLY.  Only the test suite may import this module.  The
GPU path (the library's NMF_LOSS_POISSON update) never calls it, and nothing
here is shared with the HIP path.

Letters as in nmf_oracle: data V (p x n) <- paper's X, W (p x r) <- paper's
V, H (r x n) <- paper's W.  The objective, to be maximized, is the Poisson
log-likelihood without its constant terms,

    L(W, H) = sum_ij [ v_ij ln b_ij - b_ij ],   b_ij = sum_k w_ik h_kj,

with 0 ln 0 = 0 for v_ij = 0.

Readings of points the paper leaves open:
  * the second update of the display carries garbled indices; it is read as
    the mirror image of the first:
        w_{n+1,ik} = w_ik sqrt( sum_j v_ij h_kj / b_ij  /  sum_j h_kj )
        h_{n+1,kj} = h_kj sqrt( sum_i v_ij w_ik / b_ij  /  sum_i w_ik )
    with every quantity on the right (w, h and b) from iteration n: one
    iteration updates W and H simultaneously, as displayed.  This is the
    maximizer of the minorizer in `surrogate` (Jensen's inequality on the
    logarithm with weights w_ik h_kj / b_ij, and v w <= (v_n w_n / 2)
    ((v / v_n)^2 + (w / w_n)^2) on the subtracted products), which separates
    every parameter; hence the square roots, and L never decreases;
  * a zero denominator sum_j h_kj (or sum_i w_ik) keeps the entry unchanged,
    as in the Euclidean oracle;
  * b_ij must be positive wherever v_ij > 0 (positive starting factors).
"""
from __future__ import annotations

import numpy as np


def _f64(x):
    return np.asarray(x, dtype=np.float64)


def objective(V, W, H) -> float:
    """L(W,H) = sum_ij [v_ij ln (WH)_ij - (WH)_ij], Sec. 3.1 (the Poisson
    objective), 0 ln 0 = 0."""
    V, W, H = _f64(V), _f64(W), _f64(H)
    B = W @ H
    logs = np.zeros_like(B)
    pos = V > 0
    logs[pos] = V[pos] * np.log(B[pos])
    return float(np.sum(logs - B))


def _ratio(V, B):
    """v_ij / b_ij, zero where v_ij = 0."""
    R = np.zeros_like(B)
    pos = V > 0
    R[pos] = V[pos] / B[pos]
    return R


def step(V, W, H):
    """One iteration of the square-root MM update (Sec. 3.1, last display),
    W and H both from iteration n."""
    V, W, H = _f64(V), _f64(W), _f64(H)
    R = _ratio(V, W @ H)
    num_w = R @ H.T                      # sum_j v_ij h_kj / b_ij   (p x r)
    den_w = np.sum(H, axis=1)[None, :]   # sum_j h_kj               (1 x r)
    num_h = W.T @ R                      # sum_i v_ij w_ik / b_ij   (r x n)
    den_h = np.sum(W, axis=0)[:, None]   # sum_i w_ik               (r x 1)
    Wn = W.copy()
    ok = np.broadcast_to(den_w > 0, W.shape)
    Wn[ok] = W[ok] * np.sqrt(num_w[ok] / np.broadcast_to(den_w, W.shape)[ok])
    Hn = H.copy()
    ok = np.broadcast_to(den_h > 0, H.shape)
    Hn[ok] = H[ok] * np.sqrt(num_h[ok] / np.broadcast_to(den_h, H.shape)[ok])
    return Wn, Hn


def run(V, W0, H0, iters):
    """`iters` iterations from (W0, H0); returns (W, H, trace) with
    trace[k] = L(W_k, H_k), k = 0..iters."""
    V = _f64(V)
    W, H = _f64(W0).copy(), _f64(H0).copy()
    trace = [objective(V, W, H)]
    for _ in range(iters):
        W, H = step(V, W, H)
        trace.append(objective(V, W, H))
    return W, H, np.array(trace)


def surrogate(V, W, H, Wn, Hn) -> float:
    """The minorizer g(W, H | Wn, Hn) of L at (Wn, Hn) that the update
    maximizes:

        sum_ij v_ij sum_k c_ijk [ln w_ik + ln h_kj - ln c_ijk]
      - sum_ijk (wn_ik hn_kj / 2) [(w_ik / wn_ik)^2 + (h_kj / hn_kj)^2],

    c_ijk = wn_ik hn_kj / bn_ij.  g <= L everywhere (Jensen on the concave
    logarithm; AM-GM on each product), with equality at (Wn, Hn)."""
    V, W, H, Wn, Hn = (_f64(x) for x in (V, W, H, Wn, Hn))
    Bn = Wn @ Hn
    C = Wn[:, :, None] * Hn[None, :, :] / Bn[:, None, :]          # (p, r, n)
    logt = np.log(W)[:, :, None] + np.log(H)[None, :, :] - np.log(C)
    first = np.sum(V[:, None, :] * C * logt)
    prod = Wn[:, :, None] * Hn[None, :, :] / 2.0
    second = np.sum(prod * ((W / Wn)[:, :, None] ** 2 + (H / Hn)[None, :, :] ** 2))
    return float(first - second)


def gradients(V, W, H):
    """dL/dW = (V / B - 1) H^T and dL/dH = W^T (V / B - 1)."""
    V, W, H = _f64(V), _f64(W), _f64(H)
    E = _ratio(V, W @ H) - 1.0
    return E @ H.T, W.T @ E
