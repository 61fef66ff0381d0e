"""GPU parity of the Poisson (KL) square-root multiplicative update (Sec.
3.1, last display) against the float64 oracle oracle/kl_oracle.py, on the
same float32 inputs, through the C ABI (nmf_init with loss =
NMF_LOSS_POISSON).

Bars (float32 products against float64): the objective L within 1e-5
relative (of |L|) at every one of the first 20 iterations, the factors
within 1e-4 relative (Frobenius) after 10; L non-decreasing over 100
iterations (float32 slack 1e-6 |L|); bit-identical results for graph replay
and direct launches."""
import numpy as np
import pytest
import torch

from oracle import kl_oracle as K
from synth import generators as g

pytestmark = pytest.mark.gpu

# ragged p, n; every padded-rank class (16, 32, 64) with r = 1 and r = 64
SHAPES = [(37, 129, 1), (100, 300, 5), (200, 515, 16), (130, 260, 17), (257, 190, 33),
          (70, 700, 48), (300, 333, 64), (512, 768, 20)]


def _problem(p, n, r, seed, counts=True):
    """V = Poisson(3 W* H*) / 3 (counts with zeros) or the image-like planted
    V; U(0,1) start."""
    if counts:
        rng = np.random.default_rng(seed)
        Ws = rng.gamma(2.0, 0.5, size=(p, r))
        Hs = rng.exponential(1.0, size=(r, n))
        V = (rng.poisson(3.0 * (Ws @ Hs)) / 3.0).astype(np.float32)
    else:
        V = g.sparse_planted(p, n, r, seed=seed)[0]
    W0, H0 = g.uniform_init(p, n, r, seed=seed + 1)
    return V, W0, H0


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _run(V, W0, H0, iters, **kw):
    from paper_1003_3272_amd import nmf
    Vd, Wd, Hd = (torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (V, W0, H0))
    trace = []
    with nmf.Nmf(Vd, Wd, Hd, loss="poisson", **kw) as ctx:
        trace.append(ctx.objective())
        for _ in range(iters):
            ctx.step(1)
            trace.append(ctx.objective())
    return Wd.cpu().numpy(), Hd.cpu().numpy(), np.array(trace)


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{p}x{n}r{r}" for p, n, r in SHAPES])
def test_poisson_matches_oracle(gpu_lib, shape):
    p, n, r = shape
    V, W0, H0 = _problem(p, n, r, seed=9100 + p)
    W, H, tr = _run(V, W0, H0, 20)
    W10o, H10o, tro = K.run(V, W0, H0, 10)
    _, _, tro20 = K.run(V, W0, H0, 20)
    err = np.abs(tr - tro20) / np.abs(tro20)
    assert np.all(err < 1e-5), (shape, err.max())
    W10, H10, _ = _run(V, W0, H0, 10)
    assert rel(W10, W10o) < 1e-4 and rel(H10, H10o) < 1e-4, (shape, rel(W10, W10o), rel(H10, H10o))


def test_poisson_zero_rows_and_columns(gpu_lib):
    """All-zero rows and columns of V: their factor rows / columns go to zero
    in one iteration (zero numerator) and stay there; no NaN."""
    V, W0, H0 = _problem(96, 200, 12, seed=9200)
    V[5, :] = 0.0
    V[:, 7] = 0.0
    W, H, tr = _run(V, W0, H0, 10)
    Wo, Ho, tro = K.run(V, W0, H0, 10)
    assert np.isfinite(W).all() and np.isfinite(H).all()
    assert np.all(W[5] == 0.0) and np.all(H[:, 7] == 0.0)
    assert rel(W, Wo) < 1e-4 and rel(H, Ho) < 1e-4
    assert np.all(np.abs(tr - tro) <= 1e-5 * np.abs(tro))


def test_poisson_ascent_on_gpu(gpu_lib):
    """L never decreases (the minorization argument of Sec. 2 / 3.1), up to
    float32 rounding, over 100 iterations at every padded-rank class."""
    for p, n, r in ((300, 500, 8), (256, 512, 30), (200, 640, 60)):
        V, W0, H0 = _problem(p, n, r, seed=9300 + r, counts=False)
        _, _, tr = _run(V, W0, H0, 100)
        assert np.all(np.diff(tr) >= -1e-6 * np.abs(tr[1:])), (p, n, r)
        assert tr[-1] > tr[0]


def test_poisson_full_size_two_iterations(gpu_lib):
    """4096 x 16384 image-like V, rank 64 (the headline shape): two
    iterations against the oracle."""
    V, W0, H0 = _problem(4096, 16384, 64, seed=1002, counts=False)
    W, H, tr = _run(V, W0, H0, 2)
    Wo, Ho, tro = K.run(V, W0, H0, 2)
    assert np.all(np.abs(tr - tro) <= 1e-5 * np.abs(tro)), (tr, tro)
    assert rel(W, Wo) < 1e-4 and rel(H, Ho) < 1e-4


def test_poisson_graph_replay_matches_direct_launches(gpu_lib):
    from paper_1003_3272_amd import nmf
    V, W0, H0 = _problem(300, 700, 24, seed=9400)
    out = []
    for use_graph in (True, False):
        Vd, Wd, Hd = (torch.from_numpy(x).cuda() for x in (V, W0, H0))
        with nmf.Nmf(Vd, Wd, Hd, loss="poisson", use_graph=use_graph) as ctx:
            ctx.step(13)
            f = ctx.objective()
        out.append((Wd.cpu(), Hd.cpu(), f))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]


def test_poisson_solve_and_unsupported_calls(gpu_lib):
    """nmf_solve with the relative-change rule on L; the half-step calls and
    the least-squares refit are Euclidean-only."""
    from paper_1003_3272_amd import nmf
    V, W0, H0 = _problem(200, 300, 10, seed=9500)
    Vd, Wd, Hd = (torch.from_numpy(x).cuda() for x in (V, W0, H0))
    with nmf.Nmf(Vd, Wd, Hd, loss="poisson", tol=1e-7, check_every=5) as ctx:
        conv, iters, f, trace = ctx.solve(5000, trace_len=2000)
        assert conv and iters % 5 == 0
        assert all(b >= a - 1e-6 * abs(a) for a, b in zip(trace, trace[1:]))
        for call in (ctx.update_w, ctx.update_h, lambda: ctx.refit_w(1e-3)):
            with pytest.raises(nmf.NmfError) as e:
                call()
            assert e.value.status == nmf.NMF_EUNSUPPORTED
    Wo, Ho, tro = K.run(V, W0, H0, iters)
    assert abs(f - tro[-1]) <= 1e-5 * abs(tro[-1])
