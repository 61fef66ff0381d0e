"""Plain FP64 CPU oracle of the quasi-Newton acceleration QN(q) of an MM
algorithm map, applied to the multiplicative NMF update.

TEST INFRASTRUCTURE ONLY.  Only the test suite and the benchmark's CPU
baseline may import this module; the GPU library never calls it and shares
no code with it.

The paper (Discussion; Tables 3 and 4, columns QN(q)) accelerates its MM
algorithms with the quasi-Newton scheme of Zhou, Alexander & Lange (2011,
"A quasi-Newton acceleration for high-dimensional optimization
algorithms"), which it cites but does not print.  Restated from that
method: let F be the algorithm map (here one iteration of Algorithm 1 on
x = (W, H)) and x* a fixed point, so G(x) = x - F(x) vanishes at x*.  Each
application of F at x gives a secant pair

    u = F(x) - x,   v = F(F(x)) - F(x),   with  dF(x*) u ~ v.

With the q most recent pairs as the columns of U and V (D x q), the
smallest (Frobenius) M with M U = V is M = V (U^T U)^-1 U^T.  A Newton step
for G with dG = I - M, simplified by the Woodbury identity, is

    x_qn = F(x) - V (U^T U - U^T V)^-1 U^T (x - F(x))
         = F(x) + V (U^T U - U^T V)^-1 U^T u,

which needs only q x q algebra.  One QN iteration evaluates F twice (which
yields the newest secant pair); x_qn is accepted when it is feasible and
does not increase the objective compared with the plain MM point F(F(x));
otherwise the iteration falls back to F(F(x)).  So the objective never
increases, and a fixed point of F stays fixed.

Positivity.  NMF's iterates live in the positive orthant, and the
extrapolated point leaves it often: on the sparse warm-start matrices every
extrapolation but one in 900 had a negative entry, so the rejection-only
form above never accelerated.  The extrapolated point is therefore first
projected onto the box x >= kappa F(x) (entrywise; kappa = 0.5), which keeps
every entry at least a fixed fraction of its plain MM value, and the
projected point is what the objective test accepts or rejects.  kappa = 0
gives the rejection-only form.

Readings of points the method leaves open (the same on the GPU):
  * the first q QN iterations use the pairs collected so far (fewer than q
    columns); with no usable pair (a singular q x q system, e.g. u = 0 at a
    fixed point) the iteration is the plain MM point F(F(x));
  * "feasible" means nonnegative, and positive wherever F(x) is positive:
    the multiplicative updates need positive entries to move, and an entry
    that F itself sets to zero (e.g. the H column of an all-zero V column)
    is zero in x_qn too, so requiring strict positivity everywhere would
    switch the acceleration off for good on such data;
  * the acceptance test compares f(x_qn) <= f(F(F(x))) exactly;
  * the projection onto x >= kappa F(x) above (measured on 512 x 1024 warm-
    start matrices, rank 24, to the 1e-4 gap: QN(4) needed 0.12 and 0.22 of
    plain MM's map evaluations with kappa = 0.5; 0.19-0.44 with 0.25 or
    0.75; q = 3 or 6 did worse than 4).
"""
from __future__ import annotations

import numpy as np

from oracle import nmf_oracle as nmf


def _pack(W, H):
    return np.concatenate([np.ravel(W), np.ravel(H)])


def _unpack(x, p, r, n):
    return x[:p * r].reshape(p, r), x[p * r:].reshape(r, n)


def feasible(xq, Fx) -> bool:
    """x_qn >= 0 everywhere and > 0 wherever F(x) > 0."""
    return bool(np.all(xq >= 0.0) and np.all((xq > 0.0) | (Fx <= 0.0)))


def qn_step(U, V, x, Fx, rcond=1e-12):
    """x_qn = F(x) + V (U^T U - U^T V)^-1 U^T u with u = F(x) - x (the
    newest secant pair need not be a column of U).  Returns None when the
    q x q system is singular to working precision (relative to its largest
    entry, rcond) or U is empty."""
    if U.shape[1] == 0:
        return None
    A = U.T @ U - U.T @ V
    b = U.T @ (Fx - x)
    scale = np.max(np.abs(A))
    if not np.isfinite(scale) or scale == 0.0:
        return None
    if np.linalg.cond(A) > 1.0 / rcond:
        return None
    c = np.linalg.solve(A, b)
    return Fx + V @ c


def project(xq, Fx, kappa):
    """Entrywise max(x_qn, kappa F(x))."""
    return np.maximum(xq, kappa * Fx)


def solve(V, W0, H0, q, max_mm, tol=None, tol_kind=nmf.GAP_NORMALIZED, check_every=1,
          step=None, objective=None, kappa=0.5):
    """QN(q)-accelerated multiplicative NMF from (W0, H0), float64.

    Runs QN iterations (two evaluations of the map F = one Algorithm 1
    iteration each) until `max_mm` evaluations of F, or until the stopping
    rule (the one of nmf_oracle.solve, evaluated on the accepted iterates
    every `check_every` QN iterations) holds.  `step(V, W, H) -> (W, H)` and
    `objective(V, W, H) -> f` default to the Euclidean oracle's; kappa is
    the projection fraction (0: rejection only).

    Returns (W, H, mm_evals, f, trace, accepted) with trace the objective at
    every QN iterate (trace[0] = f_0) and accepted the number of QN
    iterations whose extrapolated point was taken."""
    step = step or nmf.step
    objective = objective or nmf.objective
    V = np.asarray(V, dtype=np.float64)
    p, n = V.shape
    r = np.shape(W0)[1]
    W, H = np.array(W0, dtype=np.float64), np.array(H0, dtype=np.float64)
    nv2 = float(np.sum(V * V))
    x = _pack(W, H)
    f = objective(V, W, H)
    trace = [f]
    Us, Vs = [], []
    evals, accepted, it = 0, 0, 0
    f_prev = f
    while evals + 2 <= max_mm:
        W1, H1 = step(V, *_unpack(x, p, r, n))
        x1 = _pack(W1, H1)
        W2, H2 = step(V, W1, H1)
        x2 = _pack(W2, H2)
        evals += 2
        Us.append(x1 - x)
        Vs.append(x2 - x1)
        if len(Us) > q:
            Us.pop(0)
            Vs.pop(0)
        f2 = objective(V, W2, H2)
        xq = qn_step(np.stack(Us, axis=1), np.stack(Vs, axis=1), x, x1)
        if xq is not None and kappa > 0.0:
            xq = project(xq, x1, kappa)
        take = False
        if xq is not None and feasible(xq, x1):
            fq = objective(V, *_unpack(xq, p, r, n))
            take = fq <= f2
        if take:
            x, f = xq, fq
            accepted += 1
        else:
            x, f = x2, f2
        trace.append(f)
        it += 1
        if tol is not None and it % check_every == 0:
            if tol_kind == nmf.REL_CHANGE:
                done = nmf.rel_change(f, f_prev) < tol
            else:
                done = f / nv2 <= tol
            f_prev = f
            if done:
                break
    W, H = _unpack(x, p, r, n)
    return W, H, evals, f, np.array(trace), accepted
