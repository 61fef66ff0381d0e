"""Plain FP64 CPU oracle of the penalized PET reconstruction MM algorithm,
Sec. 3.2 (Algorithm 2, PET image recovering).

TEST INFRASTRUCTURE ONLY.  Only the test suite and the benchmark's CPU
baseline may import this module; the GPU library never calls it and shares
no code with it.

Problem: Poisson emission intensities lambda (p pixels on a grid) seen
through d lines of flight with geometry constants e_ij (E, d x p) and
counts y (d).  Maximize the penalized log-likelihood (eq. PET-objpen)

    f(lambda) = sum_i [y_i ln (E lambda)_i - (E lambda)_i]
                - (mu / 2) sum_{{j,k} in N} (lambda_j - lambda_k)^2,

N the pairs of spatially adjacent pixels (here the 4-neighbour pairs of the
grid).  Algorithm 2: scale E to unit l1 column norms, then repeat for every
pixel j in parallel

    z_ij  = y_i e_ij lambda_j / (E lambda)_i
    b_j   = mu (|N_j| lambda_j + sum_{k in N_j} lambda_k) - 1
    c_j   = sum_i z_ij
    a_j   = -2 mu |N_j|
    lambda_j <- (-b_j - sqrt(b_j^2 - 4 a_j c_j)) / (2 a_j),

the positive root of the quadratic that setting the surrogate's partial
derivative (eq. next-lambda) to zero gives after multiplying by lambda_j.

Readings of points the paper leaves open:
  * the text's formula for b_nj omits the factor mu; Algorithm 2 and the
    derivative (eq. next-lambda) both carry it, so b_j includes mu;
  * mu = 0 (a_j = 0, where the root formula divides by zero) is the EM
    update of eq. PET_algorithm, lambda_j <- c_j (the limit of the root as
    mu -> 0, with unit column sums);
  * terms with y_i = 0 contribute nothing to c (0 / 0 read as 0 for a line
    that crosses no positive intensity), and 0 ln 0 = 0 in f;
  * a pixel whose column of E is zero keeps a zero column (no scaling).

solve_qn accelerates Algorithm 2 with the quasi-Newton scheme QN(q) of Zhou,
Alexander & Lange (Table 3, columns QN(10)), the same steps as
oracle/qn_oracle.py with the map F one iteration of Algorithm 2 on
x = lambda and the test turned round for a maximization: the projected
point max(x_qn, kappa F(x)) is taken when the q x q system is regular, it
is feasible and f(x_qn) >= f(F(F(x))).
"""
from __future__ import annotations

import numpy as np

from oracle import qn_oracle


def _f64(x):
    return np.asarray(x, dtype=np.float64)


def scale_columns(E):
    """E with unit l1 column norms (Algorithm 2, first step)."""
    E = _f64(E)
    s = E.sum(axis=0)
    out = E.copy()
    nz = s > 0
    out[:, nz] = E[:, nz] / s[nz]
    return out


def neighbour_pairs(rows, cols):
    """The 4-neighbour pairs {j, k} of a rows x cols grid (row-major pixel
    index), each pair once."""
    pairs = []
    for r in range(rows):
        for c in range(cols):
            j = r * cols + c
            if c + 1 < cols:
                pairs.append((j, j + 1))
            if r + 1 < rows:
                pairs.append((j, j + cols))
    return np.array(pairs, dtype=np.int64)


def neighbour_sums(lam, pairs, p):
    """|N_j| and sum_{k in N_j} lambda_k for every pixel j."""
    lam = _f64(lam)
    count = np.zeros(p)
    s = np.zeros(p)
    np.add.at(count, pairs[:, 0], 1.0)
    np.add.at(count, pairs[:, 1], 1.0)
    np.add.at(s, pairs[:, 0], lam[pairs[:, 1]])
    np.add.at(s, pairs[:, 1], lam[pairs[:, 0]])
    return count, s


def objective(E, y, lam, mu, pairs):
    """f(lambda) of eq. PET-objpen (E already scaled or not: f uses E as
    given)."""
    E, y, lam = _f64(E), _f64(y), _f64(lam)
    B = E @ lam
    logs = np.zeros_like(B)
    pos = y > 0
    logs[pos] = y[pos] * np.log(B[pos])
    pen = np.sum((lam[pairs[:, 0]] - lam[pairs[:, 1]]) ** 2)
    return float(np.sum(logs - B) - 0.5 * mu * pen)


def step(Es, y, lam, mu, pairs):
    """One iteration of Algorithm 2 on the column-scaled Es."""
    Es, y, lam = _f64(Es), _f64(y), _f64(lam)
    p = lam.shape[0]
    B = Es @ lam
    ratio = np.zeros_like(B)
    pos = y > 0
    ratio[pos] = y[pos] / B[pos]
    c = lam * (Es.T @ ratio)                 # c_j = sum_i z_ij
    count, nsum = neighbour_sums(lam, pairs, p)
    if mu == 0.0:
        return c                              # EM update (eq. PET_algorithm)
    b = mu * (count * lam + nsum) - 1.0
    a = -2.0 * mu * count
    out = c.copy()
    has = a != 0.0
    out[has] = (-b[has] - np.sqrt(b[has] ** 2 - 4.0 * a[has] * c[has])) / (2.0 * a[has])
    return out


def run(E, y, lam0, mu, pairs, iters):
    """Scale E, then `iters` iterations from lam0; returns (lambda, trace)
    with trace[k] = f(lambda_k) on the scaled E."""
    Es = scale_columns(E)
    lam = _f64(lam0).copy()
    trace = [objective(Es, y, lam, mu, pairs)]
    for _ in range(iters):
        lam = step(Es, y, lam, mu, pairs)
        trace.append(objective(Es, y, lam, mu, pairs))
    return lam, np.array(trace)


def surrogate(Es, y, lam, lam_n, mu, pairs):
    """g(lambda | lambda_n) = Q(lambda | lambda_n) - (mu / 4) sum_{{j,k}}
    [(2 lambda_j - lambda_nj - lambda_nk)^2 + (2 lambda_k - lambda_nj -
    lambda_nk)^2], Q the Jensen minorizer of L with weights
    w_ij = e_ij lambda_nj / (E lambda_n)_i (Sec. 3.2), written term by term."""
    Es, y, lam, lam_n = _f64(Es), _f64(y), _f64(lam), _f64(lam_n)
    d, p = Es.shape
    Bn = Es @ lam_n
    q = 0.0
    for i in range(d):
        for j in range(p):
            if Es[i, j] == 0.0:
                continue
            if y[i] > 0:
                w = Es[i, j] * lam_n[j] / Bn[i]
                q += y[i] * w * np.log(Es[i, j] * lam[j] / w)
            q -= Es[i, j] * lam[j]
    pen = 0.0
    for j, k in pairs:
        m = lam_n[j] + lam_n[k]
        pen += (2.0 * lam[j] - m) ** 2 + (2.0 * lam[k] - m) ** 2
    return q - 0.25 * mu * pen


def rel_change(f, f_prev):
    """The stopping statistic of Sec. 3: |f - f_prev| / (|f_prev| + 1)."""
    return abs(f - f_prev) / (abs(f_prev) + 1.0)


def solve(E, y, lam0, mu, pairs, max_iters, tol, check_every=1):
    """Algorithm 2 from lam0 until the relative change of f between checks
    (every check_every iterations) is below tol, or max_iters.  Returns
    (lambda, iterations, f, converged)."""
    Es = scale_columns(E)
    lam = _f64(lam0).copy()
    f_prev = objective(Es, y, lam, mu, pairs)
    k = 0
    while k < max_iters:
        todo = min(check_every, max_iters - k)
        for _ in range(todo):
            lam = step(Es, y, lam, mu, pairs)
        k += todo
        f = objective(Es, y, lam, mu, pairs)
        if rel_change(f, f_prev) < tol:
            return lam, k, f, True
        f_prev = f
    return lam, k, f_prev, False


def solve_qn(E, y, lam0, mu, pairs, q, max_evals, tol=None, check_every=2, kappa=0.5,
             step_fn=None, objective_fn=None):
    """QN(q)-accelerated Algorithm 2 from lam0, float64.  Each QN iteration
    evaluates the map twice; the stopping rule (relative change below tol)
    is tested on the accepted objective every check_every evaluations
    (check_every / 2 QN iterations, at least one).  Returns (lambda, evals,
    f, trace, accepted) with trace[0] = f(lam0) and then f after every QN
    iteration.  step_fn(x) and objective_fn(x) replace Algorithm 2's map
    and f (to check the scheme on maps whose fixed point is known)."""
    Es = scale_columns(E) if E is not None else None
    F = step_fn or (lambda v: step(Es, y, v, mu, pairs))
    obj = objective_fn or (lambda v: objective(Es, y, v, mu, pairs))
    x = _f64(lam0).copy()
    f = obj(x)
    trace = [f]
    Us, Vs = [], []
    evals = accepted = it = 0
    chunk = max(1, check_every // 2)
    f_prev = f
    while evals + 2 <= max_evals:
        x1 = F(x)
        x2 = F(x1)
        evals += 2
        Us.append(x1 - x)
        Vs.append(x2 - x1)
        if len(Us) > q:
            Us.pop(0)
            Vs.pop(0)
        f2 = obj(x2)
        xq = qn_oracle.qn_step(np.stack(Us, axis=1), np.stack(Vs, axis=1), x, x1)
        if xq is not None and kappa > 0.0:
            xq = qn_oracle.project(xq, x1, kappa)
        take = False
        if xq is not None and qn_oracle.feasible(xq, x1):
            fq = obj(xq)
            take = fq >= f2
        if take:
            x, f = xq, fq
            accepted += 1
        else:
            x, f = x2, f2
        trace.append(f)
        it += 1
        if tol is not None and it % chunk == 0:
            done = rel_change(f, f_prev) < tol
            f_prev = f
            if done:
                break
    return x, evals, f, np.array(trace), accepted
