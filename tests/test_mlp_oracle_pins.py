"""Pins for the FP64 warm-start network oracle: finite differences, closed
forms of softplus and of Adam's first step, and explicit loops."""
import math

import numpy as np

from oracle import mlp_oracle as mo
from synth import generators as g


def _tiny(seed=3, B=6, p=5, d=4, r=3):
    rng = np.random.default_rng(seed)
    params = g.mlp_init(p, d, r, seed)
    params = [x.astype(np.float64) for x in params]
    params[1] = rng.uniform(-0.3, 0.3, size=d)
    params[3] = rng.uniform(-0.3, 0.3, size=r)
    X = rng.uniform(0, 1, size=(B, p))
    T = rng.uniform(0, 1, size=(B, r))
    return params, X, T


def test_softplus_closed_forms():
    z = np.array([-50.0, -3.0, -1e-3, 0.0, 2.0, 40.0, 800.0])
    sp = mo.softplus(z)
    assert abs(mo.softplus(np.array([0.0]))[0] - math.log(2.0)) < 1e-15
    np.testing.assert_allclose(sp - mo.softplus(-z), z, rtol=1e-13, atol=1e-13)
    assert sp[-1] == 800.0 and np.all(sp > 0)
    h = 1e-6
    fd = (mo.softplus(z + h) - mo.softplus(z - h)) / (2 * h)
    np.testing.assert_allclose(fd[:-1], mo.sigmoid(z)[:-1], rtol=1e-7, atol=1e-12)


def test_forward_matches_loops():
    params, X, _ = _tiny()
    M1, b1, M2, b2 = params
    Y, _ = mo.forward(params, X)
    for b in range(X.shape[0]):
        hid = [max(0.0, sum(M1[k, i] * X[b, i] for i in range(X.shape[1])) + b1[k])
               for k in range(M1.shape[0])]
        for o in range(M2.shape[0]):
            z = sum(M2[o, k] * hid[k] for k in range(M1.shape[0])) + b2[o]
            assert abs(Y[b, o] - math.log1p(math.exp(z))) < 1e-14


def test_gradients_match_central_differences():
    params, X, T = _tiny()
    _, cache = mo.forward(params, X)
    assert np.min(np.abs(cache[1])) > 1e-4      # no ReLU kink within the step
    Y, _ = mo.forward(params, X)
    grads = mo.backward(params, cache, Y, T)
    h = 1e-6
    for pi, (P, G) in enumerate(zip(params, grads)):
        it = np.nditer(P, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            plus = [q.copy() for q in params]
            minus = [q.copy() for q in params]
            plus[pi][idx] += h
            minus[pi][idx] -= h
            fd = (mo.mse(mo.forward(plus, X)[0], T) - mo.mse(mo.forward(minus, X)[0], T)) / (2 * h)
            assert abs(fd - G[idx]) <= 1e-7 * max(1.0, abs(fd)), (pi, idx, fd, G[idx])


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so every entry
    moves by -lr g / (|g| + eps)."""
    params, X, T = _tiny()
    Y, cache = mo.forward(params, X)
    grads = mo.backward(params, cache, Y, T)
    zeros = [np.zeros_like(q) for q in params]
    new, m, v = mo.adam_step(params, grads, zeros, zeros, 1, lr=0.01, eps=1e-8)
    for P0, P1, G in zip(params, new, grads):
        np.testing.assert_allclose(P1 - P0, -0.01 * G / (np.abs(G) + 1e-8), rtol=1e-12, atol=1e-15)


def test_bf16_forward_equals_fp64_on_representable_inputs():
    rng = np.random.default_rng(4)
    X = rng.integers(0, 3, size=(5, 6)).astype(np.float64)
    M1 = rng.integers(-2, 3, size=(4, 6)).astype(np.float64)
    M2 = rng.integers(-2, 3, size=(3, 4)).astype(np.float64) / 4
    params = [M1, np.zeros(4), M2, np.zeros(3)]
    a, _ = mo.forward(params, X, bf16=True)
    b, _ = mo.forward(params, X)
    assert np.array_equal(a, b)


def test_adam_decreases_loss():
    """Regressing onto a teacher network of the same shape is learnable: 200
    Adam steps cut the loss at least in half."""
    params, X, _ = _tiny(B=32)
    teacher, _, _ = _tiny(seed=9, B=32)
    T, _ = mo.forward(teacher, X)
    m = [np.zeros_like(q) for q in params]
    v = [np.zeros_like(q) for q in params]
    losses = []
    for t in range(1, 201):
        Y, cache = mo.forward(params, X)
        losses.append(mo.mse(Y, T))
        grads = mo.backward(params, cache, Y, T)
        params, m, v = mo.adam_step(params, grads, m, v, t, lr=1e-2)
    assert losses[-1] < 0.5 * losses[0]
