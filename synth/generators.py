"""Seeded synthetic inputs for NMF tests and benchmarks.

This module only draws random matrices; it holds none of the factorization's
arithmetic and is shared by the oracle-side tests and the GPU-side tests and
benchmark.  All draws use numpy's PCG64 Generator (numpy.random.default_rng).

Recipes (sizes are the workloads the library is measured on):

  uniform_planted  W* ~ U(0,1)^{p x r}, H* ~ U(0,1)^{r x n},
                   V = W* H* + |N(0, sigma^2)|          (256 x 512, r=10)
  sparse_planted   W* ~ Gamma(shape 2, scale 0.5)^{p x r},
                   H* = Exp(1) * Bernoulli(0.3) mask (70% zeros),
                   V = W* H* / max(W* H*)               (image-like, in [0,1])
  uniform_init     W0 ~ U(0,1)^{p x r}, H0 ~ U(0,1)^{r x n}, exact zeros
                   redrawn (the start is drawn on the open interval (0,1)).
  batch_shapes     512 triples p ~ U{64..1024}, n ~ U{128..4096}, r ~ U{4..64};
                   problem b: sparse_planted seed 100000 + b, start seed 200000 + b
  warm_start       W_base ~ Gamma(2, 0.5)^{1024 x 48}; matrix m uses
                   W_m = W_base * LogNormal(0, 0.1), H_m sparse Exp,
                   V_m = W_m H_m / max.
"""
from __future__ import annotations

import numpy as np


def _open_uniform(rng, shape):
    x = rng.uniform(0.0, 1.0, size=shape)
    zero = x == 0.0
    while zero.any():
        x[zero] = rng.uniform(0.0, 1.0, size=int(zero.sum()))
        zero = x == 0.0
    return x


def uniform_init(p, n, r, seed, dtype=np.float32):
    """(W0, H0) ~ U(0,1), W0 drawn first."""
    rng = np.random.default_rng(seed)
    W0 = _open_uniform(rng, (p, r))
    H0 = _open_uniform(rng, (r, n))
    return W0.astype(dtype), H0.astype(dtype)


def uniform_planted(p, n, r, seed, sigma=0.01, dtype=np.float32):
    """V = W* H* + |N(0, sigma^2)| with W*, H* ~ U(0,1); returns (V, W*, H*)."""
    rng = np.random.default_rng(seed)
    Ws = rng.uniform(0.0, 1.0, size=(p, r))
    Hs = rng.uniform(0.0, 1.0, size=(r, n))
    V = Ws @ Hs + np.abs(rng.normal(0.0, sigma, size=(p, n)))
    return V.astype(dtype), Ws, Hs


def sparse_factor(rng, r, n, keep=0.3):
    """H* = Exp(1) entries kept with probability `keep` (else exactly 0)."""
    vals = rng.exponential(1.0, size=(r, n))
    mask = rng.uniform(0.0, 1.0, size=(r, n)) < keep
    return vals * mask


def sparse_planted(p, n, r, seed, dtype=np.float32):
    """Image-like V = W* H* / max with W* ~ Gamma(2, 0.5), H* sparse Exp.

    Returns (V, W*, H*) where W* H* / max(W* H*) == V up to the cast; the
    1/max scale is folded into H* so that W* H* reproduces V.
    """
    rng = np.random.default_rng(seed)
    Ws = rng.gamma(2.0, 0.5, size=(p, r))
    Hs = sparse_factor(rng, r, n)
    V = Ws @ Hs
    m = float(V.max())
    if m > 0:
        V /= m
        Hs = Hs / m
    return V.astype(dtype), Ws, Hs


def batch_shapes(count=512, seed=4000):
    """Shapes of the batched workload, drawn in the order (p, n, r)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        p = int(rng.integers(64, 1024, endpoint=True))
        n = int(rng.integers(128, 4096, endpoint=True))
        r = int(rng.integers(4, 64, endpoint=True))
        out.append((p, n, r))
    return out


def batch_problem(b, p, n, r, dtype=np.float32):
    """Problem b of the batched workload: sparse planted V (seed 100000 + b)
    and a U(0,1) start (seed 200000 + b); returns (V, W0, H0)."""
    V, _, _ = sparse_planted(p, n, r, seed=100000 + b, dtype=dtype)
    W0, H0 = uniform_init(p, n, r, seed=200000 + b, dtype=dtype)
    return V, W0, H0


def warm_start_base(p=1024, r=48, seed=5000):
    rng = np.random.default_rng(seed)
    return rng.gamma(2.0, 0.5, size=(p, r))


def warm_start_matrix(W_base, m, n=4096, dtype=np.float32):
    """Matrix m of the warm-start stream (seed 300000 + m); returns (V, W_m, H_m)."""
    rng = np.random.default_rng(300000 + m)
    p, r = W_base.shape
    Wm = W_base * rng.lognormal(0.0, 0.1, size=(p, r))
    Hm = sparse_factor(rng, r, n)
    V = Wm @ Hm
    mx = float(V.max())
    if mx > 0:
        V /= mx
        Hm = Hm / mx
    return V.astype(dtype), Wm, Hm


# Named workloads ------------------------------------------------------------
def small_uniform():
    """256 x 512, planted rank 10 + |N(0, 0.01^2)| noise; init seed 2001."""
    V, _, _ = uniform_planted(256, 512, 10, seed=1001)
    W0, H0 = uniform_init(256, 512, 10, seed=2001)
    return V, W0, H0


def image_like(p=4096, n=16384, r=64, seed=1002, init_seed=2002):
    """Image-like sparse planted V (default 4096 x 16384, rank 64)."""
    V, _, _ = sparse_planted(p, n, r, seed=seed)
    W0, H0 = uniform_init(p, n, r, seed=init_seed)
    return V, W0, H0


def precision_tier(r, p=8192, n=32768):
    """8192 x 32768 planted rank r, seed 1003 + r, init seed 2003 + r."""
    return image_like(p, n, r, seed=1003 + r, init_seed=2003 + r)


def mlp_init(p, d, r, seed):
    """Warm-start network parameters [M1 (d x p), b1, M2 (r x d), b2]:
    He-uniform M1, Glorot-uniform M2, zero biases, float32."""
    rng = np.random.default_rng(seed)
    a1 = np.sqrt(6.0 / p)
    a2 = np.sqrt(6.0 / (d + r))
    M1 = rng.uniform(-a1, a1, size=(d, p)).astype(np.float32)
    M2 = rng.uniform(-a2, a2, size=(r, d)).astype(np.float32)
    return [M1, np.zeros(d, np.float32), M2, np.zeros(r, np.float32)]
