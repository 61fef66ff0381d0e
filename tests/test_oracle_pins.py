"""Pins for the FP64 oracle: each test checks the oracle against something the
paper or the mathematics fixes, not against a retyped copy of its own code."""
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import nmf_oracle as o
from synth import generators as g

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rand(rng, shape, lo=0.1, hi=1.0):
    return rng.uniform(lo, hi, size=shape)


# ---------------------------------------------------------------- objective
def test_objective_matches_triple_loop():
    """Sec. 3.1 eq. nnmf-objfn written as explicit sums over i, j, k."""
    rng = np.random.default_rng(7)
    V, W, H = _rand(rng, (4, 5)), _rand(rng, (4, 3)), _rand(rng, (3, 5))
    tot = 0.0
    for i in range(4):
        for j in range(5):
            s = 0.0
            for k in range(3):
                s += W[i, k] * H[k, j]
            tot += (V[i, j] - s) ** 2
    assert abs(o.objective(V, W, H) - tot) <= 1e-14 * tot


def test_objective_zero_at_exact_factorization():
    rng = np.random.default_rng(8)
    W, H = _rand(rng, (6, 2)), _rand(rng, (2, 7))
    assert o.objective(W @ H, W, H) <= 1e-28


# ----------------------------------------------- updates in exact arithmetic
def _exact_updates(V, W, H):
    """Both half-steps of Algorithm 1 in rational arithmetic, with the
    denominators in the paper's direct association: b_ij = sum_k w_ik h_kj,
    den_ik = sum_j b_ij h_kj (eq. nnmf_v_update) and, with the new W,
    c_ij = sum_k w'_ik h_kj, den_kj = sum_i c_ij w'_ik (eq. nnmf_w_update)."""
    p, n = len(V), len(V[0])
    r = len(W[0])
    b = [[sum(W[i][k] * H[k][j] for k in range(r)) for j in range(n)] for i in range(p)]
    W1 = [[W[i][k] * sum(V[i][j] * H[k][j] for j in range(n))
           / sum(b[i][j] * H[k][j] for j in range(n)) for k in range(r)] for i in range(p)]
    c = [[sum(W1[i][k] * H[k][j] for k in range(r)) for j in range(n)] for i in range(p)]
    H1 = [[H[k][j] * sum(V[i][j] * W1[i][k] for i in range(p))
           / sum(c[i][j] * W1[i][k] for i in range(p)) for j in range(n)] for k in range(r)]
    return W1, H1


def test_one_iteration_matches_exact_rational_arithmetic():
    rng = np.random.default_rng(11)
    Vi = rng.integers(0, 9, size=(4, 5))
    Wi = rng.integers(1, 5, size=(4, 2))
    Hi = rng.integers(1, 5, size=(2, 5))
    F = lambda a: [[Fraction(int(x)) for x in row] for row in a]
    W1x, H1x = _exact_updates(F(Vi), F(Wi), F(Hi))
    W1, H1 = o.step(Vi, Wi, Hi)
    W1x = np.array([[float(x) for x in row] for row in W1x])
    H1x = np.array([[float(x) for x in row] for row in H1x])
    np.testing.assert_allclose(W1, W1x, rtol=1e-14)
    np.testing.assert_allclose(H1, H1x, rtol=1e-14)


# ----------------------------------------------------------------- surrogate
def test_surrogate_tangent_at_anchor():
    """g(theta_n | theta_n) = f(theta_n) (Sec. 2, eq. minorization_definition1,
    applied to minimization)."""
    rng = np.random.default_rng(12)
    V, W, H = _rand(rng, (4, 5)), _rand(rng, (4, 3)), _rand(rng, (3, 5))
    f = o.objective(V, W, H)
    assert abs(o.surrogate(V, W, H, W, H) - f) <= 1e-13 * f


def test_surrogate_majorizes_objective():
    """g(W, H | W_n, H_n) >= f(W, H) for all W, H >= 0 (Sec. 3.1)."""
    rng = np.random.default_rng(13)
    V, Wn, Hn = _rand(rng, (4, 5)), _rand(rng, (4, 3)), _rand(rng, (3, 5))
    for _ in range(200):
        Wv = rng.uniform(0, 2, size=(4, 3))
        Hv = rng.uniform(0, 2, size=(3, 5))
        assert o.surrogate(V, Wv, Hv, Wn, Hn) >= o.objective(V, Wv, Hv) - 1e-12


def test_w_update_minimizes_surrogate():
    """The W update is the minimizer of g(., H_n | W_n, H_n) (Sec. 3.1,
    stationarity condition for the paper's V block): no perturbation beats it."""
    rng = np.random.default_rng(14)
    V, Wn, Hn = _rand(rng, (4, 5)), _rand(rng, (4, 3)), _rand(rng, (3, 5))
    W1 = o.update_w(V, Wn, Hn)
    g1 = o.surrogate(V, W1, Hn, Wn, Hn)
    for _ in range(300):
        Wp = np.maximum(W1 + rng.normal(0, 0.05, size=W1.shape), 0.0)
        assert o.surrogate(V, Wp, Hn, Wn, Hn) >= g1 - 1e-12
    # coordinatewise: the surrogate is a parabola in each w_ik with vertex at w1_ik
    for (i, k) in [(0, 0), (2, 1), (3, 2)]:
        for d in (1e-3, -1e-3):
            Wp = W1.copy()
            Wp[i, k] += d
            assert o.surrogate(V, Wp, Hn, Wn, Hn) > g1


def test_h_update_minimizes_surrogate():
    """The H update minimizes g(W_{n+1}, . | W_{n+1}, H_n) (Sec. 3.1)."""
    rng = np.random.default_rng(15)
    V, Wn, Hn = _rand(rng, (4, 5)), _rand(rng, (4, 3)), _rand(rng, (3, 5))
    W1 = o.update_w(V, Wn, Hn)
    H1 = o.update_h(V, W1, Hn)
    g1 = o.surrogate(V, W1, H1, W1, Hn)
    for _ in range(300):
        Hp = np.maximum(H1 + rng.normal(0, 0.05, size=H1.shape), 0.0)
        assert o.surrogate(V, W1, Hp, W1, Hn) >= g1 - 1e-12


# ------------------------------------------------------------------- descent
@pytest.mark.parametrize("which", ["uniform", "sparse"])
def test_descent_every_half_step(which):
    """MM descent (Sec. 2): f never increases, after either half-step."""
    if which == "uniform":
        V, W0, H0 = g.small_uniform()
    else:
        V, _, _ = g.sparse_planted(120, 200, 4, seed=31)
        W0, H0 = g.uniform_init(120, 200, 4, seed=32)
    W, H, tr, hv = o.run(V, W0, H0, 60, half=True)
    tol = 1e-13 * tr[0]
    assert np.all(hv <= tr[:-1] + tol)
    assert np.all(tr[1:] <= hv + tol)
    assert np.all(W >= 0) and np.all(H >= 0)


def test_positivity_preserved_without_zero_rows_or_columns():
    V, W0, H0 = g.small_uniform()
    W, H, _ = o.run(V, W0, H0, 20)
    assert np.all(W > 0) and np.all(H > 0)


# -------------------------------------------------------- fixed points, rank 1
def test_exact_factorization_is_fixed_point():
    rng = np.random.default_rng(21)
    Ws, Hs = _rand(rng, (30, 4)), _rand(rng, (4, 40))
    V = Ws @ Hs
    W1, H1 = o.step(V, Ws, Hs)
    assert np.max(np.abs(W1 - Ws) / Ws) < 1e-14
    assert np.max(np.abs(H1 - Hs) / Hs) < 1e-14


def test_rank_one_recovered_in_one_iteration():
    """For V = u v^T and r = 1 the W step gives w proportional to u exactly."""
    rng = np.random.default_rng(22)
    u, v = _rand(rng, (17, 1)), _rand(rng, (1, 23))
    V = u @ v
    W0, H0 = _rand(rng, (17, 1)), _rand(rng, (1, 23))
    W1, H1 = o.step(V, W0, H0)
    assert o.objective(V, W1, H1) / np.sum(V * V) < 1e-28


def test_rank_one_is_alternating_power_iteration():
    """With r = 1 the updates are w <- V h / |h|^2, h <- V^T w / |w|^2; the
    limit attains ||V||_F^2 - sigma_1^2 (Eckart-Young; Perron-Frobenius keeps
    the leading singular pair nonnegative)."""
    rng = np.random.default_rng(23)
    V = rng.uniform(0, 1, size=(6, 8))
    W0, H0 = g.uniform_init(6, 8, 1, seed=24)
    W, H, tr = o.run(V, W0, H0, 200)
    s = np.linalg.svd(V, compute_uv=False)
    target = np.sum(V * V) - s[0] ** 2
    assert abs(tr[-1] - target) <= 1e-12 * np.sum(V * V)


# ---------------------------------------------------------------- symmetries
def test_power_of_two_scaling_is_exact():
    """V -> 4V maps W_k -> 4 W_k and leaves H_k unchanged, bit for bit."""
    V, W0, H0 = g.small_uniform()
    V = V.astype(np.float64)
    Wa, Ha, tra = o.run(V, W0, H0, 5)
    Wb, Hb, trb = o.run(4.0 * V, W0, H0, 5)
    assert np.array_equal(Wb, 4.0 * Wa)
    assert np.array_equal(Hb, Ha)
    assert np.array_equal(trb[1:], 16.0 * tra[1:])


def test_transpose_duality():
    """The W half-step on V is the H half-step on V^T with W, H swapped."""
    rng = np.random.default_rng(25)
    V, W, H = _rand(rng, (9, 13)), _rand(rng, (9, 3)), _rand(rng, (3, 13))
    a = o.update_w(V, W, H)
    b = o.update_h(V.T, H.T, W.T).T
    np.testing.assert_allclose(a, b, rtol=1e-14)


# ----------------------------------------------------------------------- KKT
@pytest.mark.slow
def test_kkt_at_interior_limit():
    """At a limit with all entries positive the natural complementarity
    residual min(x, grad) vanishes (stationarity, Sec. 2 condition (d))."""
    rng = np.random.default_rng(26)
    Ws, Hs = _rand(rng, (8, 2), 0.5, 1.0), _rand(rng, (2, 10), 0.5, 1.0)
    V = Ws @ Hs + rng.uniform(0.0, 0.05, size=(8, 10))
    W0, H0 = g.uniform_init(8, 10, 2, seed=27)
    gW, gH = o.gradients(V, W0.astype(np.float64), H0.astype(np.float64))
    scale = max(np.max(np.abs(gW)), np.max(np.abs(gH)))
    W, H = W0.astype(np.float64), H0.astype(np.float64)
    for _ in range(30000):
        W, H = o.step(V, W, H)
    assert min(W.min(), H.min()) > 1e-3          # interior limit
    assert o.kkt_residual(V, W, H) <= 1e-8 * scale


# --------------------------------------------------------------- zero guards
def test_zero_row_and_column_stay_finite():
    """A zero column of V drives its H column to 0, after which the
    denominator is 0; the guard keeps the entry (no 0/0)."""
    rng = np.random.default_rng(28)
    V = rng.uniform(0, 1, size=(10, 12))
    V[:, 3] = 0.0
    V[5, :] = 0.0
    W0, H0 = g.uniform_init(10, 12, 3, seed=29)
    W, H, tr = o.run(V, W0, H0, 10)
    assert np.all(np.isfinite(W)) and np.all(np.isfinite(H))
    assert np.all(H[:, 3] == 0.0) and np.all(W[5, :] == 0.0)
    assert np.all(np.diff(tr) <= 1e-13 * tr[0])


# ----------------------------------------------------------------- stop rule
def test_stopping_rule_limits():
    V, W0, H0 = g.small_uniform()
    _, _, k, _, tr = o.solve(V, W0, H0, 7, tol=0.0)
    assert k == 7 and len(tr) == 8
    _, _, k, _, tr = o.solve(V, W0, H0, 50, tol=1e300)
    assert k == 1


def test_gap_stop_agrees_with_plain_run():
    V, W0, H0 = g.small_uniform()
    _, _, tr = o.run(V, W0, H0, 60)
    nv2 = float(np.sum(V.astype(np.float64) ** 2))
    tol = float(tr[40] / nv2)
    first = int(np.argmax(tr / nv2 <= tol))
    _, _, k, f, _ = o.solve(V, W0, H0, 100, tol=tol, tol_kind=o.GAP_NORMALIZED)
    assert k == first and f == tr[first]


# ----------------------------------------------------------------- BF16 RNE
def test_bf16_round_matches_torch():
    rng = np.random.default_rng(30)
    x = np.concatenate([
        rng.normal(0, 1, 10000).astype(np.float32),
        rng.uniform(0, 1e-38, 1000).astype(np.float32),     # subnormals
        np.array([0.0, -0.0, 1.0, 3.0e38, -3.4e38, np.inf, -np.inf], np.float32),
        # exact ties: 1 + 2^-8 (to even: 1), 1 + 3*2^-8 (to even: 1 + 2^-6)
        np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20], np.float32),
    ])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = o.bf16_round(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert np.isnan(o.bf16_round(np.array([np.nan], np.float32))[0])
    assert got[-3] == 1.0 and got[-2] == np.float32(1 + 2 ** -6)


def test_bf16_path_equals_fp64_on_representable_inputs():
    """With small-integer inputs every operand and Gram is exact in bfloat16,
    so the emulated precision tier reproduces the FP64 step exactly."""
    rng = np.random.default_rng(31)
    V = rng.integers(0, 4, size=(5, 6)).astype(np.float64)
    W = rng.integers(1, 3, size=(5, 2)).astype(np.float64)
    H = rng.integers(1, 3, size=(2, 6)).astype(np.float64)
    a = o.update_w(V, W, H, bf16=True)
    b = o.update_w(V, W, H)
    assert np.array_equal(a, b)
    Hb = np.round(H)   # H half-step from integer W
    assert np.array_equal(o.update_h(V, W, Hb, bf16=True), o.update_h(V, W, Hb))


def test_bf16_path_close_to_fp64():
    V, W0, H0 = g.small_uniform()
    a = o.update_w(V, W0, H0, bf16=True)
    b = o.update_w(V, W0, H0)
    assert np.max(np.abs(a - b) / b) < 2 * 2 ** -8


def test_rel_change_statistic_values():
    """|f_n - f_{n-1}| / (|f_{n-1}| + 1): the +1 keeps it finite at f = 0."""
    assert o.rel_change(3.0, 1.0) == 1.0
    assert o.rel_change(0.5, 0.0) == 0.5
    assert o.rel_change(1.0, 3.0) == 0.5


def test_rel_change_stop_agrees_with_plain_run():
    V, W0, H0 = g.small_uniform()
    _, _, tr = o.run(V, W0, H0, 80)
    stat = np.abs(np.diff(tr)) / (np.abs(tr[:-1]) + 1.0)
    tol = float(stat[50]) * 1.0000001
    first = int(np.argmax(stat < tol)) + 1
    _, _, k, f, _ = o.solve(V, W0, H0, 200, tol=tol)
    assert k == first and f == tr[first]


# ---- least-squares warm-start dictionary ------------------------------------

def test_ls_dictionary_recovers_exact_factor():
    """V = W* H with W* > 0 and H of full row rank: the least-squares W is W*
    (up to the 1e-6 relative ridge), and nothing is clipped."""
    rng = np.random.default_rng(31)
    Ws = rng.uniform(0.5, 1.5, size=(40, 6))
    H = rng.uniform(0.0, 1.0, size=(6, 90))
    W = o.ls_dictionary(Ws @ H, H)
    assert np.linalg.norm(W - Ws) / np.linalg.norm(Ws) < 1e-4


def test_ls_dictionary_normal_equations():
    """Interior solution: the residual satisfies the ridge normal equations
    (V - W H) H^T = delta W with delta = 1e-6 tr(H H^T) / r."""
    rng = np.random.default_rng(32)
    H = rng.uniform(0.0, 1.0, size=(5, 70))
    V = rng.uniform(0.5, 1.0, size=(30, 5)) @ H + 0.01 * rng.uniform(size=(30, 70))
    W = o.ls_dictionary(V, H)
    delta = 1e-6 * np.trace(H @ H.T) / 5
    lhs = (V - W @ H) @ H.T
    assert np.allclose(lhs, delta * W, atol=1e-9 * np.abs(V @ H.T).max())


def test_ls_dictionary_scaling_and_floor():
    """Rescaling the rows of H by D rescales the columns of W by D^-1 (the
    ridge scales with tr, so only to its order); an unconstrained solution
    with negative entries is clipped to floor_rel * max(W) and stays positive."""
    rng = np.random.default_rng(33)
    H = rng.uniform(0.0, 1.0, size=(4, 60))
    Ws = rng.uniform(0.5, 1.5, size=(25, 4))
    V = Ws @ H
    D = np.array([2.0, 0.5, 4.0, 1.0])
    W1 = o.ls_dictionary(V, H)
    W2 = o.ls_dictionary(V, D[:, None] * H)
    assert np.allclose(W2 * D, W1, rtol=1e-4)
    # a data column pattern that needs a negative coefficient: V = W* H with
    # one column of W* negative
    Wn = Ws.copy()
    Wn[:, 2] = -0.3
    W3 = o.ls_dictionary(Wn @ H, H, floor_rel=1e-2)
    assert W3.min() > 0
    assert np.allclose(W3[:, 2], 1e-2 * W3.max())
    assert np.allclose(W3[:, [0, 1, 3]], Wn[:, [0, 1, 3]], rtol=1e-4)
