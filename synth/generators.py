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


# PET (the paper's second demonstration, Sec. 3.2) ----------------------------
def pet_geometry(grid=64, detectors=64, step=0.05):
    """System matrix of a ring of `detectors` detectors around a grid x grid
    image: one line of flight per detector pair (64 detectors: 2016 lines),
    e_ij = length of line i inside pixel j (unit pixels, image centred on the
    ring's centre, ring radius = 1.05 x the image's half diagonal), measured
    by sampling each chord every `step` pixels.  Returns E (d x p, float32,
    row-major, pixels in row-major order)."""
    rad = 1.05 * grid / np.sqrt(2.0)
    ang = 2.0 * np.pi * np.arange(detectors) / detectors
    pts = np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)
    pairs = [(a, b) for a in range(detectors) for b in range(a + 1, detectors)]
    E = np.zeros((len(pairs), grid * grid), dtype=np.float64)
    for i, (a, b) in enumerate(pairs):
        p0, p1 = pts[a], pts[b]
        L = float(np.linalg.norm(p1 - p0))
        m = int(np.ceil(L / step))
        t = (np.arange(m) + 0.5) / m
        xy = p0[None, :] + t[:, None] * (p1 - p0)[None, :]
        col = np.floor(xy[:, 0] + grid / 2).astype(np.int64)
        row = np.floor(grid / 2 - xy[:, 1]).astype(np.int64)
        ok = (col >= 0) & (col < grid) & (row >= 0) & (row < grid)
        np.add.at(E[i], row[ok] * grid + col[ok], L / m)
    return E.astype(np.float32)


def pet_phantom(grid=64):
    """Emission intensities of a synthetic phantom (grid x grid, row-major):
    a disc of intensity 1 with two hot ellipses (4 and 2.5) and a cold one
    (0.2)."""
    yy, xx = np.mgrid[0:grid, 0:grid]
    x = (xx + 0.5) / grid * 2.0 - 1.0
    y = 1.0 - (yy + 0.5) / grid * 2.0
    lam = np.where(x ** 2 + y ** 2 <= 0.85 ** 2, 1.0, 0.0)
    for cx, cy, ax, ay, v in ((-0.3, 0.25, 0.18, 0.12, 4.0), (0.35, -0.2, 0.1, 0.2, 2.5),
                              (0.1, 0.45, 0.12, 0.08, 0.2)):
        lam = np.where(((x - cx) / ax) ** 2 + ((y - cy) / ay) ** 2 <= 1.0, v, lam)
    return lam.ravel()


def pet_counts(E, lam, mean_count=50.0, seed=6000):
    """Coincidence counts y_i ~ Poisson(s (E lam)_i) with s chosen so that the
    mean count per line is mean_count (float32 holding integers)."""
    rng = np.random.default_rng(seed)
    mu = np.asarray(E, np.float64) @ np.asarray(lam, np.float64)
    s = mean_count / max(float(mu.mean()), 1e-300)
    return rng.poisson(s * mu).astype(np.float32)


def pet_problem(grid=64, detectors=64, seed=6000):
    """(E, y, true intensities): the 64 x 64 image interrogated by 2016 lines
    of flight (the paper's PET problem size)."""
    E = pet_geometry(grid, detectors)
    lam = pet_phantom(grid)
    return E, pet_counts(E, lam, seed=seed), lam
