"""Pins for the precision-tier emulation and the gradient helpers of the FP64
oracles, each against something fixed outside the oracle's own code:

* the bf16 half-steps against rational arithmetic on hand-rounded operands,
  with an independent round-to-nearest-even written on fractions;
* the ratio of a bf16 half-step uses the float32 master factor, not its
  bf16 copy (a perturbation inside one bf16 rounding cell must scale the
  result by exactly the perturbation);
* the gradients of the Euclidean and Poisson objectives against central
  finite differences of those objectives;
* the warm-start network's bf16 backward against its float64 backward on
  exactly representable inputs, and its rounding of each product operand by
  perturbations inside one rounding cell.
CPU only."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import kl_oracle as kl
from oracle import mlp_oracle as mo
from oracle import nmf_oracle as o


# ---------------------------------------------------------------------------
# bfloat16 round-to-nearest-even on exact rationals (8 significant bits)
# ---------------------------------------------------------------------------
def rne8(x: Fraction) -> Fraction:
    """Nearest number with 8 significant bits (bfloat16 in its normal range),
    ties to an even last bit.  Written on fractions, independently of the
    oracle's bit-pattern rounding."""
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = 0
    while a >= 2:
        a /= 2
        e += 1
    while a < 1:
        a *= 2
        e -= 1
    # a in [1, 2): mantissa a * 2^7 in [128, 256)
    m = a * 128
    lo = m.numerator // m.denominator
    frac = m - lo
    if frac > Fraction(1, 2) or (frac == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    return sign * Fraction(lo, 128) * (Fraction(2) ** e)


def test_rne8_reference_points():
    """Spot values of the fraction rounding itself: exact bf16 values stay,
    1 + 2^-8 is a tie that goes to the even 1, 1 + 3 2^-8 a tie that goes to
    1 + 2^-6, and 1 + 0.75 2^-7 rounds up to 1 + 2^-7."""
    F = Fraction
    assert rne8(F(3, 2)) == F(3, 2)
    assert rne8(1 + F(1, 256)) == 1
    assert rne8(1 + F(3, 256)) == 1 + F(1, 64)
    assert rne8(1 + F(3, 512)) == 1 + F(1, 128)
    assert rne8(F(-5, 3)) == -rne8(F(5, 3))
    # agreement with the oracle's bit-pattern rounding on float32 inputs
    rng = np.random.default_rng(40)
    xs = rng.uniform(0.01, 100.0, size=200).astype(np.float32)
    got = o.bf16_round(xs)
    for x, g in zip(xs, got):
        assert Fraction(float(g)) == rne8(Fraction(float(x)))


def _mat(rows):
    return [[Fraction(v) for v in row] for row in rows]


def _mm(A, B):
    return [[sum(A[i][t] * B[t][j] for t in range(len(B))) for j in range(len(B[0]))]
            for i in range(len(A))]


def _T(A):
    return [list(r) for r in zip(*A)]


def _q(A):
    return [[rne8(v) for v in row] for row in A]


def _arr(A):
    return np.array([[float(v) for v in row] for row in A], dtype=np.float64)


# Operands with one entry that bfloat16 cannot hold exactly (each rounds to a
# different neighbour), and Grams whose entries need more than 8 bits.
F = Fraction
_V = [[1 + F(3, 512), F(5, 2)], [F(3, 4), F(7, 4)]]          # 1 + 3 2^-9 -> 1 + 2^-7
_W = [[F(9, 8), F(1, 2) + F(1, 1024)], [F(3, 2), F(5, 4)]]   # 1/2 + 2^-10 -> 1/2
_H = [[1 + F(1, 128), F(3, 2)], [F(5, 4), 3 + F(5, 256)]]    # 3 + 5 2^-8 -> 3 + 2^-6


def _exact_bf16_update_w(V, W, H):
    """W half-step of the precision tier in exact arithmetic: every product
    operand (V, W, H and the Gram H H^T) rounded to bf16, the ratio applied
    to the unrounded master W."""
    Vb, Wb, Hb = _q(V), _q(W), _q(H)
    A = _mm(Vb, _T(Hb))
    G = _q(_mm(Hb, _T(Hb)))
    B = _mm(Wb, G)
    return [[W[i][k] * A[i][k] / B[i][k] for k in range(len(W[0]))] for i in range(len(W))]


def _exact_bf16_update_h(V, W, H):
    Vb, Wb, Hb = _q(V), _q(W), _q(H)
    S = _mm(_T(Wb), Vb)
    G = _q(_mm(_T(Wb), Wb))
    D = _mm(G, Hb)
    return [[H[k][j] * S[k][j] / D[k][j] for j in range(len(H[0]))] for k in range(len(H))]


def test_operands_of_the_rational_case_need_rounding():
    """Every operand, and both Grams, differ from their bf16 rounding, so
    dropping any one rounding changes the exact result."""
    W1 = _exact_bf16_update_w(_V, _W, _H)
    for M in (_V, _W, _H, _mm(_q(_H), _T(_q(_H))), _mm(_T(_q(W1)), _q(W1))):
        assert _q(M) != M


def test_bf16_update_w_matches_rational_arithmetic():
    expect = _arr(_exact_bf16_update_w(_V, _W, _H))
    got = o.update_w(_arr(_V), _arr(_W), _arr(_H), bf16=True)
    np.testing.assert_allclose(got, expect, rtol=4e-16, atol=0)


def test_bf16_update_h_matches_rational_arithmetic():
    # the H half-step takes the new W, which has many significant bits
    W1 = _exact_bf16_update_w(_V, _W, _H)
    W1f = [[Fraction(float(v)) for v in row] for row in W1]   # the oracle's float64 W
    expect = _arr(_exact_bf16_update_h(_V, W1f, _H))
    got = o.update_h(_arr(_V), _arr(W1f), _arr(_H), bf16=True)
    np.testing.assert_allclose(got, expect, rtol=4e-16, atol=0)


def test_bf16_step_matches_rational_arithmetic():
    W1 = _exact_bf16_update_w(_V, _W, _H)
    W1f = [[Fraction(float(v)) for v in row] for row in W1]
    H1 = _exact_bf16_update_h(_V, W1f, _H)
    Wg, Hg = o.step(_arr(_V), _arr(_W), _arr(_H), bf16=True)
    np.testing.assert_allclose(Wg, _arr(W1), rtol=4e-16, atol=0)
    np.testing.assert_allclose(Hg, _arr(H1), rtol=4e-16, atol=0)


@pytest.mark.parametrize("half", ["w", "h"])
def test_bf16_ratio_uses_the_master_factor(half):
    """Scale the updated factor by 1 + 2^-12, which stays inside its bf16
    rounding cell: every product sees the same bf16 operands, so the update
    of eq. nnmf_v_update / nnmf_w_update must scale by exactly 1 + 2^-12
    (it would not move at all if the ratio used the bf16 copy)."""
    rng = np.random.default_rng(41)
    V = rng.uniform(0.1, 1.0, size=(12, 17)).astype(np.float32)
    W = o.bf16_round(rng.uniform(0.1, 1.0, size=(12, 3)).astype(np.float32))
    H = o.bf16_round(rng.uniform(0.1, 1.0, size=(3, 17)).astype(np.float32))
    s = 1.0 + 2.0 ** -12
    if half == "w":
        Wp = (W.astype(np.float64) * s).astype(np.float32)
        assert np.array_equal(o.bf16_round(Wp), W)
        a = o.update_w(V, W, H, bf16=True)
        b = o.update_w(V, Wp, H, bf16=True)
    else:
        Hp = (H.astype(np.float64) * s).astype(np.float32)
        assert np.array_equal(o.bf16_round(Hp), H)
        a = o.update_h(V, W, H, bf16=True)
        b = o.update_h(V, W, Hp, bf16=True)
    np.testing.assert_allclose(b / a, s, rtol=4e-16, atol=0)


# ---------------------------------------------------------------------------
# gradients against central differences
# ---------------------------------------------------------------------------
def _central(fun, X, h):
    G = np.zeros_like(X)
    for idx in np.ndindex(X.shape):
        Xp, Xm = X.copy(), X.copy()
        Xp[idx] += h
        Xm[idx] -= h
        G[idx] = (fun(Xp) - fun(Xm)) / (2 * h)
    return G


def test_euclidean_gradients_match_central_differences():
    """grad_W f and grad_H f of f = ||V - W H||_F^2 (eq. nnmf-objfn): the
    objective is quadratic in each block, so central differences are exact up
    to rounding."""
    rng = np.random.default_rng(42)
    V = rng.uniform(0, 1, size=(5, 6))
    W = rng.uniform(0.1, 1, size=(5, 3))
    H = rng.uniform(0.1, 1, size=(3, 6))
    gW, gH = o.gradients(V, W, H)
    fW = _central(lambda X: o.objective(V, X, H), W, 1e-4)
    fH = _central(lambda X: o.objective(V, W, X), H, 1e-4)
    np.testing.assert_allclose(gW, fW, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(gH, fH, rtol=1e-8, atol=1e-10)


def test_poisson_gradients_match_central_differences():
    """dL/dW and dL/dH of the Poisson log-likelihood (Sec. 3.1), including a
    zero count (0 ln 0 = 0)."""
    rng = np.random.default_rng(43)
    V = rng.poisson(2.0, size=(5, 6)).astype(np.float64)
    V[1, 2] = 0.0
    W = rng.uniform(0.2, 1, size=(5, 3))
    H = rng.uniform(0.2, 1, size=(3, 6))
    gW, gH = kl.gradients(V, W, H)
    fW = _central(lambda X: kl.objective(V, X, H), W, 1e-6)
    fH = _central(lambda X: kl.objective(V, W, X), H, 1e-6)
    np.testing.assert_allclose(gW, fW, rtol=1e-7, atol=1e-8)
    np.testing.assert_allclose(gH, fH, rtol=1e-7, atol=1e-8)


# ---------------------------------------------------------------------------
# warm-start network: bf16 backward
# ---------------------------------------------------------------------------
def _representable_net():
    """A network whose every product operand is exact in bf16 in the forward
    and the backward pass: integer X, M1, M2; hidden rows with a constant
    sum per output block, so that Z2 = 0 for every example (sigmoid(0) = 1/2
    exactly); targets chosen so that Y - T is a short dyadic number; B r = 8
    so the mean's 2 / (B r) is a power of two."""
    X = np.array([[1, 3, 3, 1], [2, 2, 2, 2], [3, 1, 1, 3], [1, 3, 1, 3]], dtype=np.float64)
    M1 = np.eye(4)
    b1 = np.zeros(4)
    M2 = np.array([[1, 1, 0, 0], [0, 0, 1, 1]], dtype=np.float64)
    b2 = np.array([-4.0, -4.0])
    params = [M1, b1, M2, b2]
    Y, _ = mo.forward(params, X)
    assert np.all(Y == Y[0, 0])                       # softplus(0) everywhere
    d = np.array([[0.25, -0.125], [0.1875, 0.0625], [-0.25, 0.375], [0.5, -0.28125]])
    T = Y - d                                         # exact: every T lies in [1/8, 1)
    assert np.array_equal(Y - T, d)
    return params, X, T


def test_mlp_bf16_backward_equals_fp64_on_representable_inputs():
    params, X, T = _representable_net()
    Yb, cb = mo.forward(params, X, bf16=True)
    Yd, cd = mo.forward(params, X)
    assert np.array_equal(Yb, Yd)
    gb = mo.backward(params, cb, Yb, T, bf16=True)
    gd = mo.backward(params, cd, Yd, T)
    for a, b in zip(gb, gd):
        assert np.array_equal(a, b)
    assert all(np.any(g != 0) for g in gd)


def _perturbed(params, X, T, which):
    """Move one quantity inside its bf16 rounding cell (or, for the targets,
    by an amount that leaves the rounded output error unchanged)."""
    params = [p.copy() for p in params]
    X = X.copy()
    T = T.copy()
    s = 1.0 + 2.0 ** -12
    if which == "X":
        X *= s
    elif which == "M1":
        params[0] = params[0] * s
    elif which == "M2":
        params[2] = params[2] * s
    elif which == "A1":
        params[1] = params[1] + 2.0 ** -12          # hidden pre-activations 1..3 move by 2^-12
    elif which == "T":
        T = T - 2.0 ** -14                          # output errors move inside their cells
    return params, X, T


@pytest.mark.parametrize("which", ["X", "M1", "M2", "A1", "T"])
def test_mlp_bf16_backward_rounds_each_operand(which):
    """Each product operand of the bf16 network (X, M1, the hidden activation
    A1, M2, the output error dZ2) is rounded before its products: moving it
    inside its rounding cell leaves every rounded product, and so every weight
    gradient, bit-identical, while the float64 network moves.  The bias
    gradient of the output layer sums the unrounded error, so it moves with
    the targets; the hidden layer's error is formed from the rounded output
    error, so its bias gradient does not."""
    params, X, T = _representable_net()
    P2, X2, T2 = _perturbed(params, X, T, which)
    Ya, ca = mo.forward(params, X, bf16=True)
    Yb, cb = mo.forward(P2, X2, bf16=True)
    ga = mo.backward(params, ca, Ya, T, bf16=True)
    gb = mo.backward(P2, cb, Yb, T2, bf16=True)
    assert np.array_equal(Ya, Yb)
    assert np.array_equal(ga[0], gb[0]) and np.array_equal(ga[2], gb[2])
    if which == "T":
        # the hidden error comes from the rounded output error, so gb1 stays
        assert np.array_equal(ga[1], gb[1])
        assert not np.array_equal(ga[3], gb[3])
    else:
        assert np.array_equal(ga[1], gb[1]) and np.array_equal(ga[3], gb[3])
    # the same perturbation does move the float64 network
    Yc, cc = mo.forward(params, X)
    Yd, cd = mo.forward(P2, X2)
    gc = mo.backward(params, cc, Yc, T)
    gd = mo.backward(P2, cd, Yd, T2)
    assert any(not np.array_equal(a, b) for a, b in zip(gc, gd)) or not np.array_equal(Yc, Yd)


def test_mlp_bf16_weight_gradient_of_one_hot_inputs_is_bf16():
    """With one-hot input rows the first layer's weight gradient copies
    entries of the rounded hidden error dZ1 (one term per sum), so every
    entry must be a bf16 number although dZ1 itself is not."""
    rng = np.random.default_rng(44)
    B, p, d, r = 8, 8, 16, 4
    X = np.eye(B, p)
    M1 = rng.uniform(-1, 1, size=(d, p))
    b1 = rng.uniform(0.5, 1.0, size=d)
    M2 = rng.uniform(-1, 1, size=(r, d))
    b2 = rng.uniform(-0.5, 0.5, size=r)
    T = rng.uniform(0, 1, size=(B, r))
    params = [M1, b1, M2, b2]
    Y, cache = mo.forward(params, X, bf16=True)
    gM1, _, _, _ = mo.backward(params, cache, Y, T, bf16=True)
    Yd, cd = mo.forward(params, X)
    gM1d = mo.backward(params, cd, Yd, T)[0]
    q = o.bf16_round(gM1.astype(np.float32)).astype(np.float64)
    assert np.array_equal(gM1, q)
    assert not np.array_equal(gM1d, o.bf16_round(gM1d.astype(np.float32)).astype(np.float64))
