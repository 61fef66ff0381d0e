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
    # tol = 0 never holds: exactly 5 iterations, as one launch (check_every
    # 5) and as five launches with a check after each (check_every 1)
    for ce in (5, 1):
        dev2 = _device(host)
        arr = nmf._problem_list(dev2)
        out = (ctypes.c_double * len(dev2))()
        it = ctypes.c_int32()
        opts = nmf.options("fp32", "gap", 0.0, ce)
        st = nmf.load().nmf_batch_solve(arr, len(dev2), 5, ctypes.byref(opts), ctypes.byref(it),
                                        out, None)
        assert st == nmf.NMF_ENOTCONVERGED and it.value == 5
        assert np.array_equal(np.array(out[:]), f1)
        for (_, W, H), (_, W2, H2) in zip(dev1, dev2):
            assert torch.equal(W, W2) and torch.equal(H, H2)


def test_batch_solve_stops_at_tolerance(gpu_lib, reference):
    """nmf_batch_solve with the gap rule: it returns at the first check
    where every problem has f / ||V||^2 <= tol (the oracle's gap), and its
    factors are those of the batch object after as many iterations."""
    from paper_1003_3272_amd import nmf
    host, _ = reference
    tol, ce = 2e-2, 10
    dev = _device(host)
    conv, iters, f = nmf.batch_solve(dev, 3000, tol_kind="gap", tol=tol, check_every=ce)
    assert conv and iters % ce == 0 and iters > 0
    nv2 = np.array([float(np.sum(np.asarray(V, np.float64) ** 2)) for V, _, _ in host])
    assert np.all(f / nv2 <= tol)
    dev1 = _device(host)
    with nmf.Batch(dev1) as b:
        b.step(iters - ce)
        f_prev = b.objective()
        b.step(ce)
        f_end = b.objective()
    assert np.array_equal(f_end, f)
    assert np.any(f_prev / nv2 > tol)   # the check before did not pass yet
    for (_, W, H), (_, W2, H2) in zip(dev, dev1):
        assert torch.equal(W, W2) and torch.equal(H, H2)


def test_batch_solve_seeded_start_and_validation(gpu_lib, reference):
    """opt.seed fills every problem's start on the device (problem 0 gets
    nmf_init's draw for the same seed); opt.validate rejects a negative
    entry in any V before any iteration."""
    from paper_1003_3272_amd import nmf
    host, _ = reference
    dev = _device(host)
    conv, iters, f = nmf.batch_solve(dev, 0, seed=1234)
    assert not conv and iters == 0
    V0 = dev[0][0]
    W1, H1 = torch.empty_like(dev[0][1]), torch.empty_like(dev[0][2])
    with nmf.Nmf(V0, W1, H1, seed=1234):
        pass
    assert torch.equal(dev[0][1], W1) and torch.equal(dev[0][2], H1)
    for _, W, H in dev:
        assert (W > 0).all() and (W < 1).all() and (H > 0).all() and (H < 1).all()
    bad = _device(host)
    bad[-1][0][3, 2] = -1.0
    W_before = bad[0][1].clone()
    with pytest.raises(nmf.NmfError) as e:
        nmf.batch_solve(bad, 5, validate=True)
    assert e.value.status == nmf.NMF_EINVAL
    assert torch.equal(bad[0][1], W_before)


def _selected(shapes):
    """Problems of the 512-problem workload checked against the oracle: the
    largest p, the largest n, the most work (p n r), the smallest, and the
    largest problem of every padded-rank class (16, 32, 48, 64)."""
    pick = {max(range(len(shapes)), key=lambda b: shapes[b][0]),
            max(range(len(shapes)), key=lambda b: shapes[b][1]),
            max(range(len(shapes)), key=lambda b: np.prod(shapes[b])),
            min(range(len(shapes)), key=lambda b: np.prod(shapes[b]))}
    for cls in range(4):
        members = [b for b, (p, n, r) in enumerate(shapes) if (r + 15) // 16 - 1 == cls]
        if members:
            pick.add(max(members, key=lambda b: shapes[b][0] * shapes[b][1]))
    return sorted(pick)


def test_full_batched_workload(gpu_lib):
    """512 problems, p ~ U{64..1024}, n ~ U{128..4096}, r ~ U{4..64}.
    Selected problems (largest p, largest n, most work, smallest, the
    largest of each rank class) match the oracle after 10 iterations
    (factors within 1e-4, objective within 1e-5) under the default tile
    table, the table the autotuner picks and a forced alternative table;
    then the objective of every problem does not increase from 50 to 200
    iterations (float32 slack 1e-6) and factors stay finite and
    nonnegative."""
    from paper_1003_3272_amd import nmf
    shapes = g.batch_shapes()
    sel = _selected(shapes)
    dev, starts, host_sel = [], [], {}
    for b, (p, n, r) in enumerate(shapes):
        V, W0, H0 = g.batch_problem(b, p, n, r)
        if b in sel:
            host_sel[b] = (V, W0, H0)
        starts.append((W0, H0))
        dev.append((torch.from_numpy(V).cuda(), torch.from_numpy(W0).cuda(),
                    torch.from_numpy(H0).cuda()))
    ref = {}
    for b in sel:
        V, W0, H0 = host_sel[b]
        W, H, tr = O.run(V, W0, H0, 10)
        ref[b] = (W, H, tr[-1])

    def restart(bt):
        for (_, W, H), (W0, H0) in zip(dev, starts):
            W.copy_(torch.from_numpy(W0))
            H.copy_(torch.from_numpy(H0))
        bt.load()

    def check(bt, tag):
        bt.step(10)
        f10 = bt.objective()
        for b in sel:
            Wo, Ho, fo = ref[b]
            what = (tag, b, shapes[b], bt.table)
            assert rel(dev[b][1].cpu().numpy(), Wo) < 1e-4, what
            assert rel(dev[b][2].cpu().numpy(), Ho) < 1e-4, what
            assert abs(f10[b] - fo) <= 1e-5 * fo, what

    with nmf.Batch(dev) as bt:
        check(bt, "default table")
        restart(bt)
        bt.tune(trial_iters=3)
        tuned = bt.table
        check(bt, "tuned table")
        alt = [2, 2, 2, 2, 2, 2, 2, 2, 1] if tuned != [2, 2, 2, 2, 2, 2, 2, 2, 1] else \
            [1, 2, 1, 2, 1, 2, 1, 2, 2]
        bt.table = alt
        restart(bt)
        check(bt, "alternative table")
        bt.table = tuned
        restart(bt)
        bt.step(50)
        f50 = bt.objective()
        bt.step(150)
        f200 = bt.objective()
    assert np.all(np.isfinite(f200))
    assert np.all(f200 <= f50 * (1 + 1e-6)), np.max(f200 / f50)
    for _, W, H in dev[::37]:
        assert torch.isfinite(W).all() and (W >= 0).all()
        assert torch.isfinite(H).all() and (H >= 0).all()


def test_queue_modes_agree(gpu_lib, reference, monkeypatch):
    """The XCD-local queues (each problem's tiles served by the workgroups
    of one XCD) and the single global queue run the same tile arithmetic in
    the same reduction order: bit-identical factors, both matching the
    oracle.  In both modes every value passed between tiles is read and
    written with device-scope accesses, and a tile's waves drain their
    stores (vmcnt) before the counter that publishes it is advanced."""
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


def test_tile_table_persists(gpu_lib, reference, tmp_path):
    """A tuned table written by save_table and installed by load_table in a
    new batch gives the same results as the tuned batch itself."""
    from paper_1003_3272_amd import nmf
    host, _ = reference
    dev1, dev2 = _device(host), _device(host)
    path = tmp_path / "table.json"
    with nmf.Batch(dev1) as b:
        b.tune(trial_iters=2)
        b.save_table(path)
        b.step(7)
        t1 = b.table
    with nmf.Batch(dev2) as b:
        b.load_table(path)
        assert b.table == t1
        b.step(7)
    for (_, W, H), (_, W2, H2) in zip(dev1, dev2):
        assert torch.equal(W, W2) and torch.equal(H, H2)
