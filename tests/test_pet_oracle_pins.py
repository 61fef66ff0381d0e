"""Pins of the penalized PET MM oracle (oracle/pet_oracle.py; Sec. 3.2,
Algorithm 2) against what the method fixes: the objective by explicit loops,
the surrogate minorizing f and touching it at the current point, the update
solving the surrogate's stationarity equation (eq. next-lambda), monotone
ascent, the mu = 0 case equal to the classical EM update written from its
own definition (eq. PET_algorithm), and noiseless data being a fixed point
of EM.  CPU only."""
import numpy as np

from oracle import pet_oracle as P
from synth import generators as g


def _tiny(seed=1, d=12, rows=3, cols=4):
    rng = np.random.default_rng(seed)
    E = rng.uniform(0.0, 1.0, size=(d, rows * cols)) * (rng.uniform(size=(d, rows * cols)) < 0.6)
    lam = rng.uniform(0.5, 2.0, size=rows * cols)
    y = rng.poisson(3.0 * (E @ lam)).astype(np.float64)
    return E, y, lam, P.neighbour_pairs(rows, cols)


def test_neighbour_pairs_of_a_grid():
    pairs = P.neighbour_pairs(2, 3)
    assert sorted(map(tuple, pairs)) == [(0, 1), (0, 3), (1, 2), (1, 4), (2, 5), (3, 4), (4, 5)]
    count, s = P.neighbour_sums(np.arange(6.0), pairs, 6)
    assert list(count) == [2, 3, 2, 2, 3, 2]
    assert list(s) == [1 + 3, 0 + 2 + 4, 1 + 5, 0 + 4, 1 + 3 + 5, 2 + 4]


def test_objective_by_loops():
    E, y, lam, pairs = _tiny()
    y[0] = 0.0
    mu = 0.3
    ref = 0.0
    for i in range(E.shape[0]):
        b = sum(E[i, j] * lam[j] for j in range(E.shape[1]))
        ref += (y[i] * np.log(b) if y[i] > 0 else 0.0) - b
    ref -= 0.5 * mu * sum((lam[j] - lam[k]) ** 2 for j, k in pairs)
    assert abs(P.objective(E, y, lam, mu, pairs) - ref) <= 1e-12 * abs(ref)


def test_surrogate_minorizes_and_touches():
    E, y, lam_n, pairs = _tiny(seed=2)
    Es = P.scale_columns(E)
    mu = 0.2
    f_n = P.objective(Es, y, lam_n, mu, pairs)
    assert abs(P.surrogate(Es, y, lam_n, lam_n, mu, pairs) - f_n) <= 1e-12 * abs(f_n)
    rng = np.random.default_rng(3)
    for _ in range(200):
        lam = lam_n * rng.uniform(0.2, 3.0, size=lam_n.shape)
        assert P.surrogate(Es, y, lam, lam_n, mu, pairs) <= P.objective(Es, y, lam, mu, pairs) + 1e-12


def test_update_solves_the_stationarity_equation():
    """d g / d lambda_j = sum_i [y_i w_ij / lambda_j - e_ij]
    - mu sum_{k in N_j} (2 lambda_j - lambda_nj - lambda_nk) vanishes at the
    update, and the update maximizes g (perturbations lower it)."""
    E, y, lam_n, pairs = _tiny(seed=4)
    Es = P.scale_columns(E)
    mu = 0.4
    lam = P.step(Es, y, lam_n, mu, pairs)
    assert np.all(lam > 0)
    B = Es @ lam_n
    ratio = np.where(y > 0, y / np.where(B > 0, B, 1.0), 0.0)
    c = lam_n * (Es.T @ ratio)
    count, nsum = P.neighbour_sums(lam_n, pairs, len(lam_n))
    deriv = c / lam - Es.sum(axis=0) - mu * (2.0 * count * lam - count * lam_n - nsum)
    assert np.max(np.abs(deriv)) <= 1e-10 * np.max(np.abs(c / lam))
    g0 = P.surrogate(Es, y, lam, lam_n, mu, pairs)
    rng = np.random.default_rng(5)
    for _ in range(50):
        assert P.surrogate(Es, y, lam * rng.uniform(0.9, 1.1, size=lam.shape), lam_n, mu,
                           pairs) <= g0 + 1e-12


def test_monotone_ascent_on_the_phantom_problem():
    E, y, _ = g.pet_problem(grid=16, detectors=24)
    pairs = P.neighbour_pairs(16, 16)
    for mu in (0.0, 1e-3, 1e-1):
        lam, tr = P.run(E, y, np.ones(256), mu, pairs, 60)
        assert np.all(np.diff(tr) >= -1e-12 * np.abs(tr[1:])), mu
        assert tr[-1] > tr[0] and np.all(lam >= 0)


def test_mu_zero_is_the_em_update():
    """lambda_{n+1,j} = sum_i y_i w_nij / sum_i e_ij (eq. PET_algorithm),
    written with explicit loops, equals the oracle's mu = 0 step, and the
    small-mu root tends to it."""
    E, y, lam, pairs = _tiny(seed=6)
    Es = P.scale_columns(E)
    d, p = Es.shape
    em = np.zeros(p)
    for j in range(p):
        num = 0.0
        for i in range(d):
            b = sum(Es[i, k] * lam[k] for k in range(p))
            if y[i] > 0:
                num += y[i] * Es[i, j] * lam[j] / b
        em[j] = num / Es[:, j].sum()
    assert np.allclose(P.step(Es, y, lam, 0.0, pairs), em, rtol=1e-12)
    assert np.allclose(P.step(Es, y, lam, 1e-9, pairs), em, rtol=1e-6)


def test_noiseless_data_is_a_fixed_point_of_em():
    E, _, lam, pairs = _tiny(seed=7)
    Es = P.scale_columns(E)
    y = Es @ lam
    assert np.allclose(P.step(Es, y, lam, 0.0, pairs), lam, rtol=1e-13)


def _small_ring(mu):
    """A 16 x 16 image seen by the lines of a 24-detector ring."""
    E = g.pet_geometry(grid=16, detectors=24)
    lam = g.pet_phantom(16)
    y = g.pet_counts(E, lam, mean_count=30.0, seed=6200).astype(np.float64)
    return E.astype(np.float64), y, P.neighbour_pairs(16, 16)


def _maximum_by_lbfgsb(Es, y, mu, pairs):
    """max f over lambda >= 0 by a different method: scipy's bound-
    constrained L-BFGS-B on -f with the analytic gradient
    d f / d lambda_j = sum_i e_ij (y_i / B_i - 1) - mu sum_{k in N_j}
    (lambda_j - lambda_k)."""
    from scipy.optimize import minimize
    p = Es.shape[1]
    pos = y > 0

    def negf(lam):
        B = Es @ lam
        f = np.sum(y[pos] * np.log(B[pos])) - B.sum() \
            - 0.5 * mu * np.sum((lam[pairs[:, 0]] - lam[pairs[:, 1]]) ** 2)
        ratio = np.zeros_like(B)
        ratio[pos] = y[pos] / B[pos]
        count, nsum = P.neighbour_sums(lam, pairs, p)
        grad = Es.T @ ratio - Es.sum(axis=0) - mu * (count * lam - nsum)
        return -f, -grad

    res = minimize(negf, np.ones(p), jac=True, method="L-BFGS-B", bounds=[(1e-12, None)] * p,
                   options=dict(maxiter=100000, maxfun=200000, ftol=1e-16, gtol=1e-12))
    return -res.fun


def test_qn_reaches_the_maximum_with_fewer_evaluations():
    """f is concave (a Poisson log-likelihood of a linear model minus a
    convex quadratic): QN(10) must end at the maximum that an independent
    optimizer finds, and reach it (to 1e-9) in far fewer map evaluations
    than plain MM, with f never decreasing."""
    mu = 1e-2
    E, y, pairs = _small_ring(mu)
    Es = P.scale_columns(E)
    fstar = _maximum_by_lbfgsb(Es, y, mu, pairs)
    lam0 = np.ones(E.shape[1])
    x, ev, f, trace, acc = P.solve_qn(E, y, lam0, mu, pairs, 10, 200000, tol=1e-13)
    assert abs(f - fstar) <= 1e-9 * abs(fstar) and acc > 0
    assert (np.diff(trace) >= -1e-12 * np.abs(trace[1:])).all()
    near = trace >= fstar - 1e-9 * abs(fstar)
    qn_evals = 2 * int(np.argmax(near))
    lam, k = lam0, 0
    while P.objective(Es, y, lam, mu, pairs) < fstar - 1e-9 * abs(fstar):
        lam = P.step(Es, y, lam, mu, pairs)
        k += 1
    assert near.any() and qn_evals < k / 4, (qn_evals, k)


def test_qn_keeps_a_fixed_point():
    """Noiseless data (y = E_s lambda) with mu = 0: lambda maximizes f (the
    fitted values equal the counts) and is a fixed point of EM.  A QN
    iteration from it may only move along the flat directions of f (d < p
    here), so f and the fitted values E_s lambda stay where they are."""
    E, _, lam, pairs = _tiny(seed=7)
    Es = P.scale_columns(E)
    y = Es @ lam
    f_star = P.objective(Es, y, lam, 0.0, pairs)
    x, ev, f, trace, _ = P.solve_qn(E, y, lam, 0.0, pairs, 10, 8)
    assert ev == 8
    assert f >= f_star - 1e-12 * abs(f_star)
    assert np.linalg.norm(Es @ x - y) <= 1e-10 * np.linalg.norm(y)


def test_qn_plain_fallback_equals_two_mm_steps():
    """With no usable secant system (the first QN iteration from a start
    where q = 0 pairs precede it still has one pair: so use kappa = 1, which
    projects every extrapolation onto F(x) itself and can only take a point
    no better than F(F(x))): the accepted iterates are MM iterates."""
    mu = 1e-3
    E, y, pairs = _small_ring(mu)
    Es = P.scale_columns(E)
    lam0 = np.ones(E.shape[1])
    x, ev, f, trace, acc = P.solve_qn(E, y, lam0, mu, pairs, 4, 6, kappa=1.0)
    ref = lam0
    for _ in range(6):
        ref = P.step(Es, y, ref, mu, pairs)
    if acc == 0:
        assert np.array_equal(x, ref)
    assert f >= P.objective(Es, y, ref, mu, pairs) - 1e-12 * abs(f)


def test_qn_lands_on_the_fixed_point_of_a_linear_contraction():
    """For F(x) = x* + m (x - x*) the secant pair gives v = m u, and one QN(1)
    iteration is x* exactly: F(x) + v (u.u - u.v)^-1 u.u = x1 + v / (1 - m)
    (the Steffensen point).  Checks how the PET driver feeds the scheme."""
    rng = np.random.default_rng(11)
    xs = rng.uniform(1.0, 2.0, size=40)
    m = 0.9
    F = lambda v: xs + m * (v - xs)                     # noqa: E731
    obj = lambda v: -float(np.sum((v - xs) ** 2))       # noqa: E731
    x0 = xs * rng.uniform(0.9, 1.1, size=40)
    x, ev, f, trace, acc = P.solve_qn(None, None, x0, 0.0, None, 1, 2, kappa=0.5,
                                      step_fn=F, objective_fn=obj)
    assert acc == 1 and ev == 2
    assert np.allclose(x, xs, rtol=1e-12, atol=0.0)
