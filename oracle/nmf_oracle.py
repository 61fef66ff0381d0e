"""Plain FP64 CPU oracle for multiplicative-update Euclidean NMF.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this module.  The GPU library never
calls it, and it shares no code with the HIP path.

Notation.  The paper (Zhou, Lange & Suchard, "Graphics Processing Units and
High-Dimensional Optimization", Sec. 3.1) factors a nonnegative p x q matrix X
as V W.  This code uses the more common letters

    data    V  (p x n)     <- paper's X
    left    W  (p x r)     <- paper's V  (per-row coefficients)
    right   H  (r x n)     <- paper's W  (basis rows)

so the objective is f(W, H) = ||V - W H||_F^2 (Sec. 3.1, eq. nnmf-objfn) and
one iteration of Algorithm 1 (NNMF) updates W first and then H with the new W
(block relaxation, Sec. 3.1).

Every array is promoted to float64 on entry; nothing is blocked, fused or
reordered beyond the definitions cited at each function.  Matrix products use
numpy's matmul (a library primitive).

Readings of points the paper leaves open:
  * denominators use the Gram association W (H H^T) and (W^T W) H, which is
    algebraically the paper's V_n W_n W_n^t and V_{n+1}^t V_{n+1} W_n;
  * a zero (or non-positive) denominator keeps the entry unchanged, a valid
    "merely decrease the surrogate" MM step (Sec. 2, remark after the ascent
    proof): the surrogate does not depend on that coordinate;
  * one iteration = W half-step then H half-step; f_0 is taken at the start;
  * the BF16 emulation rounds every operand of a product to bfloat16 with
    round-to-nearest-even and accumulates in float64.
"""
from __future__ import annotations

import numpy as np

REL_CHANGE = 0
GAP_NORMALIZED = 1


def _f64(x):
    return np.asarray(x, dtype=np.float64)


# ----------------------------------------------------------------------------
# Objective
# ----------------------------------------------------------------------------
def objective(V, W, H) -> float:
    """f(W,H) = sum_ij (v_ij - sum_k w_ik h_kj)^2, Sec. 3.1 eq. nnmf-objfn.

    Direct residual form (no trace identity), accumulated in float64.
    """
    V, W, H = _f64(V), _f64(W), _f64(H)
    R = V - W @ H
    return float(np.sum(R * R))


def gap_normalized(f, V) -> float:
    """Objective gap (f - f*) / ||V||_F^2 with f* = 0 (a reading: the planted
    generators are noiseless, so W*H* attains f = 0)."""
    V = _f64(V)
    return float(f) / float(np.sum(V * V))


def rel_change(f_new, f_old) -> float:
    """|f_n - f_{n-1}| / (|f_{n-1}| + 1), the stopping statistic of Sec. 3
    (introduction of the numerical examples)."""
    return abs(float(f_new) - float(f_old)) / (abs(float(f_old)) + 1.0)


# ----------------------------------------------------------------------------
# BF16 round-to-nearest-even emulation (for the precision tier)
# ----------------------------------------------------------------------------
def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even) and return
    them as float32.  Works on the IEEE-754 binary32 bit patterns: bfloat16 is
    the upper 16 bits of a binary32.  NaN stays NaN; overflow goes to inf."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    rounded = (u + 0x7FFF + lsb) >> 16 << 16
    out = rounded.astype(np.uint32).view(np.float32).copy()
    nan = np.isnan(a)
    if nan.any():
        out[nan] = np.float32(np.nan)
    return out.reshape(np.shape(x))


def _prep(x, bf16):
    """Operand of a product: float64 view of x, or of bf16(float32(x))."""
    if bf16:
        return _f64(bf16_round(np.asarray(x, dtype=np.float32)))
    return _f64(x)


# ----------------------------------------------------------------------------
# Multiplicative MM half-steps
# ----------------------------------------------------------------------------
def _guarded_ratio(x, num, den):
    """x * num / den where den > 0; x unchanged where den <= 0."""
    out = x.copy()
    ok = den > 0
    out[ok] = x[ok] * (num[ok] / den[ok])
    return out


def update_w(V, W, H, bf16=False):
    """One W half-step, Sec. 3.1 eq. nnmf_v_update (the paper's V update):

        w_ik <- w_ik * (V H^T)_ik / (W H H^T)_ik

    numerator sum_j v_ij h_kj, denominator sum_j b_ij h_kj with
    b_ij = sum_l w_il h_lj, associated as W (H H^T).
    With bf16=True every product operand is bfloat16-rounded first; the ratio
    itself uses the unrounded W (the master copy).
    """
    V, W, H = _f64(V), _f64(W), _f64(H)
    Vb, Wb, Hb = _prep(V, bf16), _prep(W, bf16), _prep(H, bf16)
    A = Vb @ Hb.T                      # p x r
    G = Hb @ Hb.T                      # r x r
    B = Wb @ _prep(G, bf16)            # p x r
    return _guarded_ratio(W, A, B)


def update_h(V, W, H, bf16=False):
    """One H half-step, Sec. 3.1 eq. nnmf_w_update (the paper's W update),
    using the W already updated in this iteration:

        h_kj <- h_kj * (W^T V)_kj / (W^T W H)_kj

    numerator sum_i v_ij w_ik, denominator sum_i c_ij w_ik with
    c_ij = sum_l w_il h_lj, associated as (W^T W) H.
    """
    V, W, H = _f64(V), _f64(W), _f64(H)
    Vb, Wb, Hb = _prep(V, bf16), _prep(W, bf16), _prep(H, bf16)
    S = Wb.T @ Vb                      # r x n
    G = Wb.T @ Wb                      # r x r
    D = _prep(G, bf16) @ Hb            # r x n
    return _guarded_ratio(H, S, D)


def step(V, W, H, bf16=False):
    """One iteration of Algorithm 1 (NNMF): W half-step, then H half-step
    with the new W."""
    W1 = update_w(V, W, H, bf16)
    H1 = update_h(V, W1, H, bf16)
    return W1, H1


def run(V, W0, H0, iters, bf16=False, half=False):
    """Run `iters` iterations from (W0, H0).

    Returns (W, H, trace) with trace[k] = f(W_k, H_k), k = 0..iters.  With
    half=True also returns the half-step values f(W_{k+1}, H_k), k < iters.
    """
    V = _f64(V)
    W, H = _f64(W0).copy(), _f64(H0).copy()
    trace = [objective(V, W, H)]
    halves = []
    for _ in range(iters):
        W = update_w(V, W, H, bf16)
        if half:
            halves.append(objective(V, W, H))
        H = update_h(V, W, H, bf16)
        trace.append(objective(V, W, H))
    if half:
        return W, H, np.array(trace), np.array(halves)
    return W, H, np.array(trace)


def solve(V, W0, H0, max_iters, tol, tol_kind=REL_CHANGE, check_every=1,
          bf16=False):
    """Iterate until the stopping rule holds or max_iters is reached.

    REL_CHANGE (Sec. 3 introduction): stop at the first check where
    |f_k - f_prev| / (|f_prev| + 1) < tol, f_prev being the objective at the
    previous check (with check_every=1 this is the paper's rule).
    GAP_NORMALIZED: stop at the first check where f_k / ||V||_F^2 <= tol.
    Checks happen after every `check_every` iterations and at max_iters.

    Returns (W, H, iters_done, f, trace) with trace the checked objectives,
    trace[0] = f_0.
    """
    V = _f64(V)
    W, H = _f64(W0).copy(), _f64(H0).copy()
    f_prev = objective(V, W, H)
    trace = [f_prev]
    nv2 = float(np.sum(V * V))
    k = 0
    while k < max_iters:
        todo = min(check_every, max_iters - k)
        for _ in range(todo):
            W, H = step(V, W, H, bf16)
        k += todo
        f = objective(V, W, H)
        trace.append(f)
        if tol_kind == REL_CHANGE:
            done = rel_change(f, f_prev) < tol
        else:
            done = f / nv2 <= tol
        f_prev = f
        if done:
            break
    return W, H, k, trace[-1], np.array(trace)


# ----------------------------------------------------------------------------
# Surrogate (majorization) of Sec. 3.1 eq. frobenius_majorization
# ----------------------------------------------------------------------------
def surrogate(V, Wv, Hv, Wn, Hn) -> float:
    """g(W, H | W_n, H_n) = sum_ijk (a_ikj / b_ij) (v_ij - (b_ij / a_ikj) w_ik h_kj)^2
    with a_ikj = wn_ik hn_kj and b_ij = sum_k a_ikj (Sec. 3.1).

    Written term by term over (i, j, k); terms with a_ikj = 0 are dropped
    (the convexity weights a/b are then 0 and the term is absent).
    """
    V, Wv, Hv, Wn, Hn = map(_f64, (V, Wv, Hv, Wn, Hn))
    p, n = V.shape
    r = Wn.shape[1]
    total = 0.0
    for i in range(p):
        for j in range(n):
            a = Wn[i, :] * Hn[:, j]
            b = a.sum()
            for k in range(r):
                if a[k] == 0.0:
                    continue
                t = V[i, j] - (b / a[k]) * Wv[i, k] * Hv[k, j]
                total += (a[k] / b) * t * t
    return total


# ----------------------------------------------------------------------------
# KKT (natural complementarity) residual
# ----------------------------------------------------------------------------
def gradients(V, W, H):
    """Gradient of f: grad_W = -2 (V - W H) H^T, grad_H = -2 W^T (V - W H)."""
    V, W, H = _f64(V), _f64(W), _f64(H)
    R = V - W @ H
    return -2.0 * R @ H.T, -2.0 * W.T @ R


def kkt_residual(V, W, H):
    """max(|min(W, grad_W f)|, |min(H, grad_H f)|): zero exactly at KKT points of
    min f subject to W, H >= 0 (natural-map complementarity residual)."""
    gW, gH = gradients(V, W, H)
    return max(float(np.max(np.abs(np.minimum(_f64(W), gW)))),
               float(np.max(np.abs(np.minimum(_f64(H), gH)))))


def ls_dictionary(V, H, floor_rel=1e-3):
    """Least-squares dictionary for a given H: the warm-start refit of W (an
    addition to the method: Algorithm 1 only needs some positive start, and
    the multiplicative updates refine whatever start they get).

        W = max(V H^T (H H^T + delta I)^{-1}, floor)
        delta = 1e-6 tr(H H^T) / r,  floor = floor_rel * max(0, max W),
        floor at least the smallest normal float32,

    i.e. the ridge-regularized unconstrained minimizer of ||V - W H||_F^2 over
    W, clipped to a positive floor so that every entry is a valid start for
    the multiplicative updates."""
    V, H = _f64(V), _f64(H)
    r = H.shape[0]
    G = H @ H.T
    tr = float(np.trace(G))
    delta = 1e-6 * tr / r if tr > 0 else 1e-300
    W = np.linalg.solve(G + delta * np.eye(r), (V @ H.T).T).T
    floor = max(floor_rel * max(float(W.max()), 0.0), float(np.finfo(np.float32).tiny))
    return np.maximum(W, floor)
