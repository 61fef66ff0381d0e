"""Pins of the Poisson (KL) variant's oracle (Sec. 3.1, last displays)
against what the method fixes: the minorizer it maximizes, monotone ascent,
exact fixed points, gauge equivariance, stationarity at convergence, and a
brute-force objective.  CPU only."""
import itertools

import numpy as np

from oracle import kl_oracle as k


def _problem(p, n, r, seed, exact=False):
    rng = np.random.default_rng(seed)
    Ws = rng.gamma(2.0, 0.5, size=(p, r))
    Hs = rng.exponential(1.0, size=(r, n))
    V = Ws @ Hs
    if not exact:
        V = rng.poisson(3.0 * V).astype(np.float64) / 3.0   # counts, some zeros
    W0 = rng.uniform(0.1, 1.0, size=(p, r))
    H0 = rng.uniform(0.1, 1.0, size=(r, n))
    return V, W0, H0, Ws, Hs


def test_objective_brute_force():
    V, W, H, _, _ = _problem(4, 5, 2, seed=1)
    V[0, 0] = 0.0                           # 0 ln 0 = 0
    ref = 0.0
    for i, j in itertools.product(range(4), range(5)):
        b = sum(W[i, t] * H[t, j] for t in range(2))
        ref += (V[i, j] * np.log(b) if V[i, j] > 0 else 0.0) - b
    assert abs(k.objective(V, W, H) - ref) <= 1e-12 * abs(ref)


def test_monotone_ascent():
    for seed in range(5):
        V, W0, H0, _, _ = _problem(30, 40, 4, seed=10 + seed)
        _, _, tr = k.run(V, W0, H0, 60)
        assert np.all(np.diff(tr) >= -1e-12 * np.abs(tr[1:])), seed
        assert tr[-1] > tr[0]


def test_exact_factorization_is_fixed_point():
    V, _, _, Ws, Hs = _problem(12, 15, 3, seed=3, exact=True)
    W1, H1 = k.step(V, Ws, Hs)
    assert np.allclose(W1, Ws, rtol=1e-12) and np.allclose(H1, Hs, rtol=1e-12)


def test_surrogate_minorizes_and_touches():
    rng = np.random.default_rng(4)
    V, Wn, Hn, _, _ = _problem(6, 7, 3, seed=4)
    Ln = k.objective(V, Wn, Hn)
    assert abs(k.surrogate(V, Wn, Hn, Wn, Hn) - Ln) <= 1e-10 * abs(Ln)
    for _ in range(50):
        W = Wn * np.exp(rng.normal(0, 0.5, Wn.shape))
        H = Hn * np.exp(rng.normal(0, 0.5, Hn.shape))
        assert k.surrogate(V, W, H, Wn, Hn) <= k.objective(V, W, H) + 1e-10 * abs(Ln)


def test_update_maximizes_surrogate():
    """The update is the argmax of the minorizer: every small multiplicative
    perturbation of (W1, H1) lowers it (so the square roots and the
    iteration-n quantities on both sides are pinned)."""
    rng = np.random.default_rng(5)
    V, Wn, Hn, _, _ = _problem(6, 7, 3, seed=5)
    W1, H1 = k.step(V, Wn, Hn)
    g1 = k.surrogate(V, W1, H1, Wn, Hn)
    for _ in range(100):
        W = W1 * np.exp(rng.normal(0, 1e-3, W1.shape))
        H = H1 * np.exp(rng.normal(0, 1e-3, H1.shape))
        assert k.surrogate(V, W, H, Wn, Hn) <= g1
    # and so the update never decreases L
    assert k.objective(V, W1, H1) >= k.objective(V, Wn, Hn)


def test_gauge_equivariance():
    V, W0, H0, _, _ = _problem(8, 9, 3, seed=6)
    c = np.array([0.5, 2.0, 3.0])
    W1, H1 = k.step(V, W0, H0)
    W2, H2 = k.step(V, W0 * c[None, :], H0 / c[:, None])
    assert np.allclose(W2, W1 * c[None, :], rtol=1e-12)
    assert np.allclose(H2, H1 / c[:, None], rtol=1e-12)


def test_stationarity_at_convergence():
    """On an exactly factorable positive V the iteration reaches a
    stationary point of L: W o dL/dW and H o dL/dH vanish (KKT
    complementarity) relative to the scale of V."""
    V, W0, H0, _, _ = _problem(10, 12, 2, seed=7, exact=True)
    W, H, tr = k.run(V, W0, H0, 4000)
    gW, gH = k.gradients(V, W, H)
    scale = np.sum(V)
    assert np.max(np.abs(W * gW)) < 1e-6 * scale
    assert np.max(np.abs(H * gH)) < 1e-6 * scale
