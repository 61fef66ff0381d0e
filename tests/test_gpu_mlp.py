"""GPU parity of the warm-start network against the FP64 network oracle.

The GPU feeds bfloat16 operands to the matrix cores and accumulates in
float32; the oracle's bf16=True path rounds the same operands and
accumulates in float64.  Outputs and gradients then differ only by float32
accumulation (plus rare one-step bf16 rounding differences of an activation
whose float32 and float64 values straddle a rounding boundary)."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as mo
from synth import generators as g

pytestmark = pytest.mark.gpu


def _case(p=300, d=128, r=20, n=700, seed=5):
    params = g.mlp_init(p, d, r, seed)
    rng = np.random.default_rng(seed + 1)
    params[1] = rng.uniform(-0.1, 0.2, size=d).astype(np.float32)
    params[3] = rng.uniform(-0.2, 0.2, size=r).astype(np.float32)
    V = rng.uniform(0, 1, size=(p, n)).astype(np.float32)
    H = rng.exponential(1.0, size=(r, n)).astype(np.float32)
    return params, V, H


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("p,d,r,n", [(300, 128, 20, 700), (1024, 512, 48, 4096), (64, 256, 64, 100)])
def test_forward_matches_oracle(gpu_lib, p, d, r, n):
    from paper_1003_3272_amd import nmf
    params, V, _ = _case(p, d, r, n)
    net = nmf.Mlp(params, max_batch=n)
    H0 = net.predict(torch.from_numpy(V).cuda()).cpu().numpy()
    Y, _ = mo.forward(params, V.T, bf16=True)
    assert rel(H0, Y.T) < 1e-3
    assert np.allclose(H0, Y.T, rtol=5e-3, atol=1e-4)
    net.close()


@pytest.mark.parametrize("p,d,r,n", [(300, 128, 20, 700), (1024, 512, 48, 4096)])
def test_gradients_match_oracle(gpu_lib, p, d, r, n):
    from paper_1003_3272_amd import nmf
    params, V, H = _case(p, d, r, n, seed=7)
    net = nmf.Mlp(params, max_batch=n)
    gpu, loss = net.grads(torch.from_numpy(V).cuda(), torch.from_numpy(H).cuda())
    Y, cache = mo.forward(params, V.T, bf16=True)
    ref = mo.backward(params, cache, Y, H.T, bf16=True)
    assert abs(loss - mo.mse(Y, H.T)) <= 1e-4 * mo.mse(Y, H.T)
    for gg, rr in zip(gpu, ref):
        assert rel(gg.cpu().numpy(), rr) < 5e-3
    # against the exact (float64, unrounded) gradients: the bf16 tier's error
    Y64, cache64 = mo.forward(params, V.T)
    exact = mo.backward(params, cache64, Y64, H.T)
    errs = [rel(gg.cpu().numpy(), ee) for gg, ee in zip(gpu, exact)]
    print("bf16 gradient error vs float64:", ["%.2e" % e for e in errs])
    assert max(errs) < 5e-2


def test_predict_wider_than_batch(gpu_lib):
    """predict on more columns than max_batch runs in chunks: same bits as
    predicting each chunk alone, and oracle parity."""
    from paper_1003_3272_amd import nmf
    params, V, _ = _case(200, 128, 12, 700, seed=13)
    Vd = torch.from_numpy(V).cuda()
    net = nmf.Mlp(params, max_batch=256)
    H0 = net.predict(Vd)
    parts = [net.predict(Vd[:, a:a + 256]) for a in range(0, 700, 256)]
    assert torch.equal(H0, torch.cat(parts, dim=1))
    Y, _ = mo.forward(params, V.T, bf16=True)
    assert rel(H0.cpu().numpy(), Y.T) < 1e-3
    net.close()


def test_column_slice_batches(gpu_lib):
    """A batch given as column slices of wider V and H (row strides ldv, ldh
    larger than n) gives the same loss and gradients, bit for bit, as the
    same columns copied out contiguously, and both match the oracle."""
    from paper_1003_3272_amd import nmf
    params, V, H = _case(300, 128, 20, 900, seed=11)
    Vd, Hd = torch.from_numpy(V).cuda(), torch.from_numpy(H).cuda()
    a, b = 130, 130 + 333
    net = nmf.Mlp(params, max_batch=512)
    g_slice, l_slice = net.grads(Vd[:, a:b], Hd[:, a:b])
    g_copy, l_copy = net.grads(Vd[:, a:b].contiguous(), Hd[:, a:b].contiguous())
    assert l_slice == l_copy
    for x, y in zip(g_slice, g_copy):
        assert torch.equal(x, y)
    Y, cache = mo.forward(params, V[:, a:b].T, bf16=True)
    ref = mo.backward(params, cache, Y, H[:, a:b].T, bf16=True)
    for gg, rr in zip(g_slice, ref):
        assert rel(gg.cpu().numpy(), rr) < 5e-3
    with pytest.raises(ValueError):
        net.grads(Vd[:, a:b], Hd[:, a:b + 1])
    net.close()
    net.close()


def test_adam_step_matches_oracle(gpu_lib):
    from paper_1003_3272_amd import nmf
    params, V, H = _case(256, 128, 16, 512, seed=9)
    net = nmf.Mlp(params, max_batch=512)
    lr = 1e-3
    loss0 = net.train_step(torch.from_numpy(V).cuda(), torch.from_numpy(H).cuda(), lr)
    Y, cache = mo.forward(params, V.T, bf16=True)
    assert abs(loss0 - mo.mse(Y, H.T)) <= 1e-4 * mo.mse(Y, H.T)
    grads = mo.backward(params, cache, Y, H.T, bf16=True)
    zeros = [np.zeros_like(x, dtype=np.float64) for x in params]
    ref, _, _ = mo.adam_step(params, grads, zeros, zeros, 1, lr=lr)
    for got, want, p0 in zip(net.params(), ref, params):
        got = got.cpu().numpy()
        d = np.abs(got - want)
        assert d.max() <= 2.01 * lr                 # a sign flip of a ~0 gradient
        assert np.mean(d < 1e-6) > 0.99
    net.close()


def test_training_reduces_loss(gpu_lib):
    from paper_1003_3272_amd import nmf
    params, V, _ = _case(256, 128, 16, 1024, seed=11)
    teacher = g.mlp_init(256, 128, 16, 99)
    Yt, _ = mo.forward(teacher, V.T)
    Vd = torch.from_numpy(V).cuda()
    Hd = torch.from_numpy(Yt.T.astype(np.float32)).contiguous().cuda()
    net = nmf.Mlp(params, max_batch=1024)
    losses = [net.train_step(Vd, Hd, 3e-3) for _ in range(150)]
    assert losses[-1] < 0.3 * losses[0]
    net.close()


def test_ws_predict_gives_dictionary_and_network_start(gpu_lib):
    """nmf_ws_predict: W0 is the stored W-bar bit for bit and H0 is the
    network's prediction for V, bit-identical to nmf_mlp_predict."""
    from paper_1003_3272_amd import nmf
    params, V, _ = _case(300, 128, 20, 700, seed=11)
    rng = np.random.default_rng(12)
    Wbar = torch.from_numpy(rng.uniform(0.1, 1.0, size=(300, 20)).astype(np.float32)).cuda()
    net = nmf.Mlp(params, max_batch=256)   # 700 columns: three chunks
    Vd = torch.from_numpy(V).cuda()
    with pytest.raises(nmf.NmfError):      # no dictionary stored yet
        net.ws_predict(Vd)
    net.set_dictionary(Wbar)
    W0, H0 = net.ws_predict(Vd)
    torch.cuda.synchronize()
    assert torch.equal(W0, Wbar)
    assert torch.equal(H0, net.predict(Vd))
    Y, _ = mo.forward(params, V.T, bf16=True)
    assert rel(H0.cpu().numpy(), Y.T) < 1e-3
    net.close()


def test_ws_train_equals_its_adam_steps(gpu_lib):
    """nmf_ws_train over one matrix (so the shuffled order is trivial) for
    two epochs with decay 0.5 runs exactly the Adam steps of
    nmf_mlp_train_step over the same minibatches (a ragged last one
    included) with learning rates lr and lr/2: bit-identical weights, and
    the epoch losses are the means of the step losses."""
    from paper_1003_3272_amd import nmf
    params, V, H = _case(300, 128, 20, 700, seed=13)
    Vd, Hd = torch.from_numpy(V).cuda(), torch.from_numpy(H).cuda()
    a = nmf.Mlp(params, max_batch=256)
    b = nmf.Mlp(params, max_batch=256)
    losses = a.train_loop([Vd], [Hd], epochs=2, lr=1e-3, batch=256, decay=0.5, seed=3)
    ref = []
    for lr in (1e-3, 5e-4):
        steps = [b.train_step(Vd[:, c:c + 256], Hd[:, c:c + 256], lr) for c in range(0, 700, 256)]
        ref.append(float(np.mean(steps)))
    for x, y in zip(a.params(), b.params()):
        assert torch.equal(x, y)
    assert np.allclose(losses, ref, rtol=1e-12, atol=0)
    assert losses[1] < losses[0]
    a.close()
    b.close()


def test_ws_train_order_covers_every_matrix(gpu_lib):
    """Several matrices: one epoch of nmf_ws_train equals the Adam steps over
    the matrices in the order of its seeded Fisher-Yates shuffle (splitmix64,
    written out here), and a different seed gives different weights."""
    from paper_1003_3272_amd import nmf
    mats = [_case(128, 128, 8, 256, seed=20 + i)[1:] for i in range(5)]
    params = _case(128, 128, 8, 256, seed=20)[0]
    dev = [(torch.from_numpy(V).cuda(), torch.from_numpy(H).cuda()) for V, H in mats]
    M = (1 << 64) - 1

    def splitmix(state):
        state = (state + 0x9E3779B97F4A7C15) & M
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return state, z ^ (z >> 31)

    order, st = list(range(5)), 99
    for i in range(4, 0, -1):
        st, z = splitmix(st)
        j = z % (i + 1)
        order[i], order[j] = order[j], order[i]
    a = nmf.Mlp(params, max_batch=128)
    b = nmf.Mlp(params, max_batch=128)
    c = nmf.Mlp(params, max_batch=128)
    a.train_loop([v for v, _ in dev], [h for _, h in dev], epochs=1, lr=1e-3, batch=128, seed=99)
    c.train_loop([v for v, _ in dev], [h for _, h in dev], epochs=1, lr=1e-3, batch=128, seed=5)
    for m in order:
        Vd, Hd = dev[m]
        for col in range(0, 256, 128):
            b.train_step(Vd[:, col:col + 128], Hd[:, col:col + 128], 1e-3, want_loss=False)
    for x, y in zip(a.params(), b.params()):
        assert torch.equal(x, y)
    assert not all(torch.equal(x, y) for x, y in zip(a.params(), c.params()))
    for net in (a, b, c):
        net.close()
