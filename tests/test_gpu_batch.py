"""GPU parity of the batched tier (one persistent launch advances many
problems of uneven p, n and r) against the FP64 oracle, run problem by
problem on the same float32 inputs.

Bars (float32 matrix-core products against float64): per-problem objective
within 1e-5 relative and factors within 1e-4 relative after 10 iterations,
objective within 1e-5 after 40; bit-identical results for identical inputs
and for a step split into several calls."""
import numpy as np
import pytest
import torch

from oracle import nmf_oracle as O
from synth import generators as g

pytestmark = pytest.mark.gpu

# ragged shapes: p and n off the 64-tiles, n % 4 != 0 (aligned copy of V),
# every padded-rank class, r = 1 and r = 64
SHAPES = [
    (37, 129, 1), (64, 128, 4), (100, 300, 5), (200, 515, 16), (130, 260, 17),
    (257, 190, 33), (70, 700, 48), (300, 333, 64), (129, 1000, 20), (65, 64, 64),
    (90, 150, 6),
]


def _host_problems():
    out = []
    for i, (p, n, r) in enumerate(SHAPES):
        if i % 3 == 0:
            V, _, _ = g.uniform_planted(p, n, r, seed=7000 + i)
        else:
            V, _, _ = g.sparse_planted(p, n, r, seed=7000 + i)
        W0, H0 = g.uniform_init(p, n, r, seed=8000 + i)
        out.append((V, W0, H0))
    # last problem: an all-zero row and an all-zero column (guarded ratios)
    V = out[-1][0].copy()
    V[5, :] = 0.0
    V[:, 7] = 0.0
    out[-1] = (V, out[-1][1], out[-1][2])
    return out


def _device(host):
    return [tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in t) for t in host]


@pytest.fixture(scope="module")
def reference():
    host = _host_problems()
    ref = {}
    for i, (V, W0, H0) in enumerate(host):
        W, H, tr10 = O.run(V, W0, H0, 10)
        _, _, tr40 = O.run(V, W, H, 30)
        ref[i] = dict(W10=W, H10=H, f10=tr10[-1], f40=tr40[-1])
    return host, ref


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _check_10(dev, ref, tag):
    for i, (V, W, H) in enumerate(dev):
        r = ref[i]
        assert rel(W.cpu().numpy(), r["W10"]) < 1e-4, (tag, i, SHAPES[i])
        assert rel(H.cpu().numpy(), r["H10"]) < 1e-4, (tag, i, SHAPES[i])


def test_batch_matches_oracle(gpu_lib, reference):
    from paper_1003_3272_amd import nmf
    host, ref = reference
    dev = _device(host)
    with nmf.Batch(dev) as b:
        b.step(10)
        f10 = b.objective()
        _check_10(dev, ref, "default")
        b.step(30)
        f40 = b.objective()
    for i in range(len(SHAPES)):
        fr10, fr40 = ref[i]["f10"], ref[i]["f40"]
        floor = 1e-12 * float(np.sum(np.asarray(host[i][0], np.float64) ** 2))
        assert abs(f10[i] - fr10) <= 1e-5 * fr10 + floor, (i, SHAPES[i], f10[i], fr10)
        assert abs(f40[i] - fr40) <= 1e-5 * fr40 + floor, (i, SHAPES[i], f40[i], fr40)
    for V, W, H in dev:
        assert torch.isfinite(W).all() and torch.isfinite(H).all()
        assert (W >= 0).all() and (H >= 0).all()


@pytest.mark.parametrize("shape_w,shape_h,wg", [(1, 2, 1), (2, 1, 2), (2, 2, 2), (2, 2, 1)])
def test_every_tile_table_matches_oracle(gpu_lib, reference, shape_w, shape_h, wg):
    from paper_1003_3272_amd import nmf
    host, ref = reference
    dev = _device(host)
    with nmf.Batch(dev) as b:
        b.table = [shape_w, shape_h] * 4 + [wg]
        assert b.table == [shape_w, shape_h] * 4 + [wg]
        b.step(10)
        b.check()
    _check_10(dev, ref, (shape_w, shape_h, wg))


def test_deterministic_and_split_steps(gpu_lib, reference):
    from paper_1003_3272_amd import nmf
    host, _ = reference
    runs = []
    for split in ([7], [3, 4], [7], [1, 1, 5]):
        dev = _device(host)
        with nmf.Batch(dev) as b:
            for k in split:
                b.step(k)
            b.check()
        runs.append(dev)
    for other in runs[1:]:
        for (V, W, H), (V2, W2, H2) in zip(runs[0], other):
            assert torch.equal(W, W2) and torch.equal(H, H2)


def test_strided_and_misaligned_inputs(gpu_lib):
    """V given as column slices of a wider matrix: row stride a multiple of 4
    (read in place) and a base 12 bytes off (read from an aligned copy)."""
    from paper_1003_3272_amd import nmf
    Vbig, _, _ = g.sparse_planted(150, 420, 9, seed=7100)
    cases = [(Vbig[:, :397], 9), (Vbig[:, 3:300], 9), (Vbig[:80, 1:], 40)]
    dev, ref = [], []
    big = torch.from_numpy(Vbig).cuda()
    views = [big[:, :397], big[:, 3:300], big[:80, 1:]]
    for k, ((Vh, r), Vd) in enumerate(zip(cases, views)):
        p, n = Vh.shape
        W0, H0 = g.uniform_init(p, n, r, seed=8100 + k)
        W, H, tr = O.run(Vh, W0, H0, 10)
        ref.append((W, H, tr[-1]))
        dev.append((Vd, torch.from_numpy(W0).cuda(), torch.from_numpy(H0).cuda()))
    with nmf.Batch(dev) as b:
        b.step(10)
        f = b.objective()
    for k, ((V, W, H), (Wr, Hr, fr)) in enumerate(zip(dev, ref)):
        assert rel(W.cpu().numpy(), Wr) < 1e-4, k
        assert rel(H.cpu().numpy(), Hr) < 1e-4, k
        assert abs(f[k] - fr) <= 1e-5 * fr, k
    # V was only read
    assert torch.equal(big, torch.from_numpy(Vbig).cuda())


def test_tune_keeps_state_and_load_restarts(gpu_lib, reference):
    from paper_1003_3272_amd import nmf
    host, ref = reference
    dev = _device(host)
    with nmf.Batch(dev) as b:
        b.step(2)
        before = [(W.clone(), H.clone()) for _, W, H in dev]
        f_before = b.objective()
        ms = b.tune(trial_iters=3)
        assert ms > 0
        t = b.table
        assert all(x in (1, 2) for x in t)
        for (_, W, H), (W0, H0) in zip(dev, before):
            assert torch.equal(W, W0) and torch.equal(H, H0)
        assert np.array_equal(b.objective(), f_before)
        # restart from the original start through load()
        for (V, W, H), (Vh, W0, H0) in zip(dev, host):
            W.copy_(torch.from_numpy(W0))
            H.copy_(torch.from_numpy(H0))
        b.load()
        b.step(10)
        b.check()
    _check_10(dev, ref, "after tune + load")


def test_batch_solve_matches_batch_object(gpu_lib, reference):
    import ctypes
    from paper_1003_3272_amd import nmf
    host, _ = reference
    dev1, dev2 = _device(host), _device(host)
    with nmf.Batch(dev1) as b:
        b.step(5)
        f1 = b.objective()
    arr = nmf._problem_list(dev2)
    out = (ctypes.c_double * len(dev2))()
    st = nmf.load().nmf_batch_solve(arr, len(dev2), 5, out, None)
    assert st == nmf.NMF_OK
    assert np.array_equal(np.array(out[:]), f1)
    for (_, W, H), (_, W2, H2) in zip(dev1, dev2):
        assert torch.equal(W, W2) and torch.equal(H, H2)


def test_full_batched_workload(gpu_lib):
    """512 problems, p ~ U{64..1024}, n ~ U{128..4096}, r ~ U{4..64}: the
    objective of every problem does not increase from 50 to 200 iterations
    (float32 slack 1e-6), factors stay finite and nonnegative, and the three
    smallest problems match the oracle after 50 iterations (1e-5)."""
    from paper_1003_3272_amd import nmf
    shapes = g.batch_shapes()
    dev, small = [], sorted(range(len(shapes)), key=lambda b: np.prod(shapes[b]))[:3]
    host_small = {}
    for b, (p, n, r) in enumerate(shapes):
        V, W0, H0 = g.batch_problem(b, p, n, r)
        if b in small:
            host_small[b] = (V, W0, H0)
        dev.append((torch.from_numpy(V).cuda(), torch.from_numpy(W0).cuda(),
                    torch.from_numpy(H0).cuda()))
    with nmf.Batch(dev) as bt:
        bt.step(50)
        f50 = bt.objective()
        bt.step(150)
        f200 = bt.objective()
    assert np.all(np.isfinite(f200))
    assert np.all(f200 <= f50 * (1 + 1e-6)), np.max(f200 / f50)
    for b in small:
        V, W0, H0 = host_small[b]
        _, _, tr = O.run(V, W0, H0, 50)
        assert abs(f50[b] - tr[-1]) <= 1e-5 * tr[-1], (b, shapes[b], f50[b], tr[-1])
    for _, W, H in dev[::37]:
        assert torch.isfinite(W).all() and (W >= 0).all()
        assert torch.isfinite(H).all() and (H >= 0).all()


def test_queue_modes_agree(gpu_lib, reference, monkeypatch):
    """The XCD-local queues (each problem's tiles on one XCD, L1-only
    coherence) and the single global queue (agent-scope release/acquire)
    run the same tile arithmetic in the same reduction order: bit-identical
    factors, both matching the oracle."""
    from paper_1003_3272_amd import nmf
    host, ref = reference
    out = []
    for mode in ("local", "global"):
        if mode == "global":
            monkeypatch.setenv("NMF_BATCH_QUEUES", "1")
        else:
            monkeypatch.delenv("NMF_BATCH_QUEUES", raising=False)
        dev = _device(host)
        with nmf.Batch(dev) as b:
            b.step(10)
            b.check()
        out.append(dev)
    for (_, W, H), (_, W2, H2) in zip(out[0], out[1]):
        assert torch.equal(W, W2) and torch.equal(H, H2)
    _check_10(out[0], ref, "local")
