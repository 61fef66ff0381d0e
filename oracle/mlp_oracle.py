"""Plain FP64 CPU oracle for the warm-start network.

TEST INFRASTRUCTURE ONLY (see nmf_oracle).  Shares no code with the GPU path.

The network maps one column v of V (p values) to a starting column h0 of H
(r values): h0 = softplus(M2 relu(M1 v + b1) + b2).  It is trained on pairs
(v_j, h_j) where h_j is a column of a converged H, with the mean squared
error over the r outputs and the batch, and Adam (Kingma & Ba 2015) updates.

Rows of every array are examples (batch-major): X is B x p, targets T are
B x r.  Parameters: M1 (d x p), b1 (d), M2 (r x d), b2 (r).

With bf16=True every operand of a matrix product (X, M1, the hidden
activations, M2 and the back-propagated errors) is rounded to bfloat16
(round to nearest even) before the product, matching the GPU kernels, which
feed bfloat16 to the matrix cores and accumulate in float32; everything else
stays in float64.
"""
from __future__ import annotations

import numpy as np

from oracle.nmf_oracle import bf16_round


def _f64(x):
    return np.asarray(x, dtype=np.float64)


def _q(x, bf16):
    """Operand of a matrix product."""
    return _f64(bf16_round(np.asarray(x, dtype=np.float32))) if bf16 else _f64(x)


def softplus(z):
    """log(1 + e^z), computed without overflow."""
    z = _f64(z)
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    z = _f64(z)
    out = np.empty_like(z)
    pos = z >= 0
    out[pos] = 1.0 / (1.0 + np.exp(-z[pos]))
    e = np.exp(z[~pos])
    out[~pos] = e / (1.0 + e)
    return out


def forward(params, X, bf16=False):
    """Returns (Y, cache): Y = softplus(relu(X M1^T + b1) M2^T + b2)."""
    M1, b1, M2, b2 = (_f64(a) for a in params)
    Z1 = _q(X, bf16) @ _q(M1, bf16).T + b1
    A1 = np.maximum(Z1, 0.0)
    Z2 = _q(A1, bf16) @ _q(M2, bf16).T + b2
    Y = softplus(Z2)
    return Y, (X, Z1, A1, Z2)


def mse(Y, T):
    """Mean over all B * r entries of (Y - T)^2."""
    D = _f64(Y) - _f64(T)
    return float(np.mean(D * D))


def backward(params, cache, Y, T, bf16=False):
    """Gradients of mse(forward(X), T) with respect to (M1, b1, M2, b2)."""
    M1, b1, M2, b2 = (_f64(a) for a in params)
    X, Z1, A1, Z2 = cache
    B, r = np.shape(Y)
    dY = 2.0 * (_f64(Y) - _f64(T)) / (B * r)
    dZ2 = dY * sigmoid(Z2)                      # d softplus / dz = sigmoid
    gM2 = _q(dZ2, bf16).T @ _q(A1, bf16)
    gb2 = dZ2.sum(axis=0)
    dA1 = _q(dZ2, bf16) @ _q(M2, bf16)
    dZ1 = dA1 * (Z1 > 0)
    gM1 = _q(dZ1, bf16).T @ _q(X, bf16)
    gb1 = dZ1.sum(axis=0)
    return gM1, gb1, gM2, gb2


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) of every parameter.

    m, v: lists of first and second moment arrays (updated and returned);
    t: the step number after this update (1 for the first)."""
    new_p, new_m, new_v = [], [], []
    for p_, g_, m_, v_ in zip(params, grads, m, v):
        g_ = _f64(g_)
        m_ = beta1 * _f64(m_) + (1.0 - beta1) * g_
        v_ = beta2 * _f64(v_) + (1.0 - beta2) * g_ * g_
        mhat = m_ / (1.0 - beta1 ** t)
        vhat = v_ / (1.0 - beta2 ** t)
        new_p.append(_f64(p_) - lr * mhat / (np.sqrt(vhat) + eps))
        new_m.append(m_)
        new_v.append(v_)
    return new_p, new_m, new_v
