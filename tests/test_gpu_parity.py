"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same float32 inputs.

Tolerances (FP32 tier): objective within 1e-5 relative at every iteration of
the first 50, factors within 1e-4 relative (Frobenius) after 10 iterations.
Half-steps are compared elementwise against the oracle's half-step taken from
the GPU's own input state, so each kernel's error is measured on its own.
"""
import numpy as np
import pytest
import torch

from oracle import nmf_oracle as o
from synth import generators as g

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def frob_rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make(gpu_lib, V, W0, H0, **kw):
    from paper_1003_3272_amd import nmf
    Vd, Wd, Hd = dev(V), dev(W0), dev(H0)
    return nmf.Nmf(Vd, Wd, Hd, **kw), Vd, Wd, Hd


# --------------------------------------------------------------- small case
def test_small_uniform_trajectory(gpu_lib):
    """256 x 512, r = 10: f_k within 1e-5 for k <= 50, factors within 1e-4 at
    k = 10, descent at every iteration."""
    V, W0, H0 = g.small_uniform()
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0)
    Wo, Ho, tr = o.run(V, W0, H0, 50)
    fs = [ctx.objective()]
    for k in range(1, 51):
        ctx.step(1)
        fs.append(ctx.objective())
        if k == 10:
            W10, H10, _ = o.run(V, W0, H0, 10)
            assert frob_rel(host(Wd), W10) < 1e-4
            assert frob_rel(host(Hd), H10) < 1e-4
    fs = np.array(fs)
    rel = np.abs(fs - tr) / tr
    assert rel.max() < 1e-5, rel.max()
    assert np.all(np.diff(fs) <= 1e-6 * fs[0])
    ctx.close()


def test_half_steps_elementwise(gpu_lib):
    V, W0, H0 = g.small_uniform()
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0)
    for _ in range(3):
        Win, Hin = host(Wd), host(Hd)
        ctx.update_w()
        Wref = o.update_w(V, Win, Hin)
        assert np.max(np.abs(host(Wd) - Wref) / Wref) < 2e-5
        Win = host(Wd)
        ctx.update_h()
        Href = o.update_h(V, Win, Hin)
        assert np.max(np.abs(host(Hd) - Href) / Href) < 2e-5
    ctx.close()


# -------------------------------------------------- ragged shapes, all ranks
SHAPES = [
    (1000, 3001, 64),   # several tiles + ragged tails on both sides
    (2000, 8000, 64),   # enough tiles for the default (not the narrow) rank-64
    (2000, 8000, 40),   # tiles, 32 x 32 matrix-core shape, ragged tails
    (4099, 1000, 64),   # W update with 4 ranks per thread, p % 4 != 0
    (77, 130, 3),       # smaller than one tile
    (513, 257, 17),     # rank padded 17 -> 32
    (300, 1000, 100),   # rank padded to 128
    (260, 520, 200),    # rank padded to 256
    (1, 5, 1),          # degenerate: one row, rank 1
    (640, 2, 2),        # two columns
    (12, 10, 20),       # rank above both dimensions
    (3, 300, 7),        # rank above p
]


@pytest.mark.parametrize("p,n,r", SHAPES)
def test_ragged_shapes(gpu_lib, p, n, r):
    V, _, _ = g.sparse_planted(p, n, max(1, r // 2), seed=p * 7 + n)
    V = V + np.float32(1e-3)  # keep every row and column nonzero
    W0, H0 = g.uniform_init(p, n, r, seed=p + n + r)
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0)
    iters = 6
    Wo, Ho, tr = o.run(V, W0, H0, iters)
    fs = [ctx.objective()]
    for _ in range(iters):
        ctx.step(1)
        fs.append(ctx.objective())
    # Shapes with n <= r or rank-1 data are factored exactly within an
    # iteration; there f falls to the float32 rounding floor of the residual
    # (a few u^2 ||V||^2, u = 2^-24): the relative test allows 1e-5 of
    # (f + 1e-8 ||V||^2), i.e. an absolute slack of about 28 u^2 ||V||^2.
    nv2 = float(np.sum(V.astype(np.float64) ** 2))
    rel = np.abs(np.array(fs) - tr) / (tr + 1e-8 * nv2)
    assert rel.max() < 1e-5, (rel.max(), fs, tr)
    assert frob_rel(host(Wd), Wo) < 1e-4
    assert frob_rel(host(Hd), Ho) < 1e-4
    ctx.close()


def test_row_stride_not_multiple_of_four(gpu_lib):
    """V as a column slice of a wider matrix (row stride 1003): the library
    reads it through its own aligned copy."""
    p, n, r = 200, 999, 12
    big, _, _ = g.sparse_planted(p, 1003, 6, seed=5)
    big = big + np.float32(1e-3)
    W0, H0 = g.uniform_init(p, n, r, seed=6)
    from paper_1003_3272_amd import nmf
    Bd = dev(big)
    Vd = Bd[:, 2:2 + n]
    assert Vd.stride(0) == 1003
    Wd, Hd = dev(W0), dev(H0)
    ctx = nmf.Nmf(Vd, Wd, Hd)
    ctx.step(5)
    Wo, Ho, tr = o.run(big[:, 2:2 + n], W0, H0, 5)
    f = ctx.objective()
    assert abs(f - tr[-1]) / tr[-1] < 1e-5
    assert frob_rel(host(Wd), Wo) < 1e-4
    ctx.close()


def test_zero_rows_and_columns(gpu_lib):
    """Zero rows/columns of V drive factor entries to zero; the guard keeps
    the 0/0 entries at zero instead of producing NaN."""
    rng = np.random.default_rng(3)
    V = rng.uniform(0, 1, size=(150, 300)).astype(np.float32)
    V[:, [0, 77, 299]] = 0
    V[[5, 149], :] = 0
    W0, H0 = g.uniform_init(150, 300, 8, seed=4)
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0)
    ctx.step(8)
    W, H = host(Wd), host(Hd)
    assert np.all(np.isfinite(W)) and np.all(np.isfinite(H))
    assert np.all(H[:, [0, 77, 299]] == 0) and np.all(W[[5, 149], :] == 0)
    Wo, Ho, tr = o.run(V, W0, H0, 8)
    assert abs(ctx.objective() - tr[-1]) / tr[-1] < 1e-5
    ctx.close()


# ---------------------------------------------------------------- invariants
def test_deterministic_and_resumable(gpu_lib):
    """Two runs give identical bits; 2k iterations equal k, restart, k."""
    V, W0, H0 = g.small_uniform()
    a, _, Wa, Ha = make(gpu_lib, V, W0, H0)
    a.step(20)
    b, _, Wb, Hb = make(gpu_lib, V, W0, H0)
    b.step(20)
    assert torch.equal(Wa, Wb) and torch.equal(Ha, Hb)
    c, Vc, Wc, Hc = make(gpu_lib, V, W0, H0)
    c.step(10)
    c.close()
    from paper_1003_3272_amd import nmf
    d = nmf.Nmf(Vc, Wc, Hc)
    d.step(10)
    assert torch.equal(Wa, Wc) and torch.equal(Ha, Hc)
    for x in (a, b, d):
        x.close()


def test_power_of_two_scaling_exact(gpu_lib):
    """V -> 4V maps W -> 4W and keeps H, bit for bit, on the GPU too."""
    V, W0, H0 = g.small_uniform()
    a, _, Wa, Ha = make(gpu_lib, V, W0, H0)
    b, _, Wb, Hb = make(gpu_lib, 4 * V, W0, H0)
    a.step(7)
    b.step(7)
    assert torch.equal(Wb, 4 * Wa) and torch.equal(Hb, Ha)
    a.close()
    b.close()


def test_objective_matches_oracle_fp64(gpu_lib):
    V, W0, H0 = g.image_like(700, 900, 40, seed=9, init_seed=10)
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0)
    for _ in range(3):
        f = ctx.objective()
        ref = o.objective(V, host(Wd), host(Hd))
        assert abs(f - ref) <= 1e-12 * ref
        ctx.step(5)
    ctx.close()


def test_exact_factorization_fixed_point(gpu_lib):
    rng = np.random.default_rng(12)
    Ws = rng.uniform(0.5, 1, size=(128, 4)).astype(np.float32)
    Hs = rng.uniform(0.5, 1, size=(4, 256)).astype(np.float32)
    V = (Ws.astype(np.float64) @ Hs).astype(np.float32)
    ctx, Vd, Wd, Hd = make(gpu_lib, V, Ws, Hs)
    ctx.step(3)
    assert np.max(np.abs(host(Wd) - Ws) / Ws) < 1e-5
    assert np.max(np.abs(host(Hd) - Hs) / Hs) < 1e-5
    ctx.close()


# -------------------------------------------------------------- options, errors
def test_validate_rejects_negative_and_nan(gpu_lib):
    from paper_1003_3272_amd import nmf
    for bad in (-1.0, float("nan"), float("inf")):
        V = np.ones((64, 64), np.float32)
        V[10, 20] = bad
        W0, H0 = g.uniform_init(64, 64, 4, seed=1)
        with pytest.raises(nmf.NmfError) as e:
            nmf.Nmf(dev(V), dev(W0), dev(H0), validate=True)
        assert e.value.status == nmf.NMF_EINVAL
    V = np.ones((64, 64), np.float32)
    ctx = nmf.Nmf(dev(V), dev(W0), dev(H0), validate=True)
    ctx.close()


def test_seeded_device_initialization(gpu_lib):
    from paper_1003_3272_amd import nmf
    p, n, r = 512, 1024, 16
    V = np.ones((p, n), np.float32)
    outs = []
    for seed in (11, 11, 12):
        Wd = torch.zeros((p, r), device="cuda")
        Hd = torch.zeros((r, n), device="cuda")
        ctx = nmf.Nmf(dev(V), Wd, Hd, seed=seed)
        outs.append((host(Wd), host(Hd)))
        ctx.close()
    W, H = outs[0]
    for x in (W, H):
        assert x.min() > 0 and x.max() < 1
        assert abs(x.mean() - 0.5) < 0.01 and abs(x.var() - 1 / 12) < 0.005
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert not np.array_equal(outs[0][0], outs[2][0])


def test_solve_gap_rule(gpu_lib):
    V, W0, H0 = g.image_like(256, 1024, 8, seed=21, init_seed=22)
    _, _, tr = o.run(V, W0, H0, 200)
    nv2 = float(np.sum(V.astype(np.float64) ** 2))
    tol = float(tr[120] / nv2)
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0, tol_kind="gap", tol=tol, check_every=1)
    conv, it, f, trace = ctx.solve(400, trace_len=401)
    first = int(np.argmax(tr / nv2 <= tol))
    assert conv and abs(it - first) <= 2
    assert f / nv2 <= tol and len(trace) == it + 1
    ctx.close()


def test_solve_rel_change_rule_and_cap(gpu_lib):
    V, W0, H0 = g.small_uniform()
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0, tol=1e-300, check_every=7)
    conv, it, f, trace = ctx.solve(30, trace_len=10)
    assert not conv and it == 30 and len(trace) == 6  # checks at 0,7,14,21,28,30
    ctx.close()
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0, tol=1e-3)
    conv, it, f, trace = ctx.solve(10000, trace_len=10001)
    t = np.array(trace)
    stat = np.abs(np.diff(t)) / (np.abs(t[:-1]) + 1)
    # the rule first holds at the check before the last one: the chunk that
    # was already enqueued behind it ran too, and its objective is f
    first = int(np.argmax(stat < 1e-3))
    assert conv and first == len(stat) - 2 and f == t[-1]
    assert it == len(t) - 1  # check_every = 1
    np.testing.assert_allclose(f, float(np.sum((V.astype(np.float64)
                                                - Wd.cpu().numpy().astype(np.float64)
                                                @ Hd.cpu().numpy().astype(np.float64)) ** 2)),
                               rtol=1e-9)
    ctx.close()


def test_solve_reports_nonfinite(gpu_lib):
    """One entry of V near the float32 maximum (validation off): the float64
    objective of the start is finite, the float32 products overflow within
    the first iterations, and solve returns NMF_ENONFINITE with a non-finite
    f after draining the chunk it had already enqueued."""
    import ctypes
    from paper_1003_3272_amd import nmf
    V, W0, H0 = g.small_uniform()
    V = V.copy()
    V[3, 7] = np.float32(3e38)
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0, check_every=5)
    assert np.isfinite(ctx.objective())
    it, f = ctypes.c_int32(), ctypes.c_double()
    st = nmf.load().nmf_solve(ctx._ctx, 50, ctypes.byref(it), ctypes.byref(f), None, 0)
    assert st == nmf.NMF_ENONFINITE
    # the chunk whose check first sees the overflow, plus the one behind it
    assert 10 <= it.value <= 50 and it.value % 5 == 0 and not np.isfinite(f.value)
    st = nmf.load().nmf_objective(ctx._ctx, ctypes.byref(f))
    assert st == nmf.NMF_ENONFINITE and not np.isfinite(f.value)
    ctx.close()


# ----------------------------------------------------------- full-size case
@pytest.mark.slow
def test_full_size_image_like_one_iteration(gpu_lib):
    """4096 x 16384, r = 64 (the benchmark workload): two iterations against
    the FP64 oracle in full."""
    V, W0, H0 = g.image_like()
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0)
    Wo, Ho, tr = o.run(V, W0, H0, 2)
    fs = [ctx.objective()]
    for _ in range(2):
        ctx.step(1)
        fs.append(ctx.objective())
    assert np.max(np.abs(np.array(fs) - tr) / tr) < 1e-5
    assert frob_rel(host(Wd), Wo) < 1e-4
    assert frob_rel(host(Hd), Ho) < 1e-4
    ctx.close()


# The product tiling depends on the problem size: below 256 workgroups the
# 64-wide tiles, above it the default 128-row / 128-column ones.  The cases
# above are small (64-wide tiles); 2048 x 4096 has 256 workgroups in both
# products with the default tiles, for every padded rank <= 64.
@pytest.mark.parametrize("r", [12, 32, 64])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_default_tiles_mid_size(gpu_lib, r, precision):
    V, W0, H0 = g.image_like(2048, 4096, r, seed=70 + r, init_seed=71 + r)
    if precision == "bf16":
        V = V + np.float32(1e-3)  # no exact zeros in the factors (relative errors)
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0, precision=precision)
    iters = 4
    if precision == "fp32":
        Wo, Ho, tr = o.run(V, W0, H0, iters)
        fs = [ctx.objective()]
        for _ in range(iters):
            ctx.step(1)
            fs.append(ctx.objective())
        assert np.max(np.abs(np.array(fs) - tr) / tr) < 1e-5
        assert frob_rel(host(Wd), Wo) < 1e-4
        assert frob_rel(host(Hd), Ho) < 1e-4
    else:
        for _ in range(iters):
            Win, Hin = host(Wd), host(Hd)
            ctx.update_w()
            err = np.abs(host(Wd) - o.update_w(V, Win, Hin, bf16=True))
            assert np.median(err / host(Wd)) < 1e-5 and np.max(err / host(Wd)) < 2e-3
            Win = host(Wd)
            ctx.update_h()
            err = np.abs(host(Hd) - o.update_h(V, Win, Hin, bf16=True))
            assert np.median(err / host(Hd)) < 1e-5 and np.max(err / host(Hd)) < 2e-3
    ctx.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_tile_override_that_does_not_fit_is_ignored(gpu_lib, monkeypatch, precision):
    """A product tile must divide the padded row counts it copies.  Tile 15
    is 256 rows tall; as the pass-2 tile at padded rank 128 it would read
    past the 128 rows of W^T, so the override is ignored on the host and the
    results equal the default tiling's bit for bit."""
    V, W0, H0 = g.image_like(512, 1024, 100, seed=81, init_seed=82)
    runs = []
    for override in (None, "15"):
        if override:
            monkeypatch.setenv("NMF_DMA2", override)
        else:
            monkeypatch.delenv("NMF_DMA2", raising=False)
        ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0, precision=precision)
        ctx.step(3)
        runs.append((host(Wd), host(Hd), ctx.objective()))
        ctx.close()
    (Wa, Ha, fa), (Wb, Hb, fb) = runs
    assert np.array_equal(Wa, Wb) and np.array_equal(Ha, Hb) and fa == fb


@pytest.mark.slow
@pytest.mark.parametrize("r", [32, 128, 256])
def test_precision_tier_full_size_one_iteration(gpu_lib, r):
    """8192 x 32768 (the precision tier's size) at ranks 32 (split-K passes,
    fused Grams), 128 (separate Gram products, float32 W update, matrix-core
    H update) and 256 (single-tile passes, both updates on the matrix
    cores): one FP32 iteration against the float64 oracle in full."""
    V, W0, H0 = g.precision_tier(r)
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0)
    fs = [ctx.objective()]
    ctx.step(1)
    fs.append(ctx.objective())
    W1, H1 = host(Wd), host(Hd)
    ctx.close()
    del Vd, Wd, Hd
    torch.cuda.empty_cache()
    Wo, Ho, tr = o.run(V, W0, H0, 1)
    assert np.max(np.abs(np.array(fs) - tr) / tr) < 1e-5, (fs, tr)
    assert frob_rel(W1, Wo) < 1e-4
    assert frob_rel(H1, Ho) < 1e-4


# ------------------------------------------------------------------ BF16 tier
# The BF16 tier rounds every product operand (V, W, H and the r x r Grams) to
# bfloat16 (RNE) and accumulates in float32 with float32 master factors.  The
# oracle's bf16=True path rounds the same operands and accumulates in float64,
# so a half-step differs only by accumulation error, except where a float32
# Gram entry and its float64 value round to neighbouring bfloat16 numbers
# (one 2^-8 step in one Gram entry, diluted over r terms of a denominator).
@pytest.mark.parametrize("p,n,r", [(300, 700, 24), (513, 1030, 64), (200, 900, 100),
                                   (160, 300, 230)])
def test_bf16_half_steps_vs_emulated_oracle(gpu_lib, p, n, r):
    V, _, _ = g.sparse_planted(p, n, max(1, r // 2), seed=40 + r)
    V = V + np.float32(1e-3)
    W0, H0 = g.uniform_init(p, n, r, seed=41 + r)
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0, precision="bf16")
    for _ in range(2):
        Win, Hin = host(Wd), host(Hd)
        ctx.update_w()
        Wref = o.update_w(V, Win, Hin, bf16=True)
        err = np.abs(host(Wd) - Wref) / Wref
        assert err.max() < 2e-3 and np.median(err) < 1e-5, (err.max(), np.median(err))
        Win = host(Wd)
        ctx.update_h()
        Href = o.update_h(V, Win, Hin, bf16=True)
        err = np.abs(host(Hd) - Href) / Href
        assert err.max() < 2e-3 and np.median(err) < 1e-5, (err.max(), np.median(err))
    ctx.close()


@pytest.mark.slow
@pytest.mark.parametrize("r", [32, 128, 256])
def test_bf16_half_steps_full_size(gpu_lib, r):
    """8192 x 32768 at ranks 32, 128 and 256, BF16 tier: one W and one H
    half-step against the oracle's bf16-emulated half-steps from the GPU's
    own input state, to the bar of the small cases."""
    V, W0, H0 = g.precision_tier(r)
    V = V + np.float32(1e-3)  # no exact zeros in the factors (relative errors)
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0, precision="bf16")
    Win, Hin = host(Wd), host(Hd)
    ctx.update_w()
    Wg = host(Wd)
    err = np.abs(Wg - o.update_w(V, Win, Hin, bf16=True)) / Wg
    assert err.max() < 2e-3 and np.median(err) < 1e-5, (err.max(), np.median(err))
    ctx.update_h()
    Hg = host(Hd)
    err = np.abs(Hg - o.update_h(V, Wg, Hin, bf16=True)) / Hg
    assert err.max() < 2e-3 and np.median(err) < 1e-5, (err.max(), np.median(err))
    ctx.close()


def test_bf16_objective_close_to_fp64_after_many_iterations(gpu_lib):
    """1024 x 4096 planted rank 32, 300 iterations: the BF16 tier's objective
    is within 1e-2 relative of the FP64 oracle's (and descends)."""
    V, _, _ = g.sparse_planted(1024, 4096, 32, seed=1035)
    W0, H0 = g.uniform_init(1024, 4096, 32, seed=2035)
    ctx, Vd, Wd, Hd = make(gpu_lib, V, W0, H0, precision="bf16")
    fs = [ctx.objective()]
    for _ in range(6):
        ctx.step(50)
        fs.append(ctx.objective())
    _, _, tr = o.run(V, W0, H0, 300)
    rel = abs(fs[-1] - tr[-1]) / tr[-1]
    print(f"bf16 vs fp64 oracle after 300 iterations: rel diff {rel:.3e}")
    assert rel < 1e-2
    assert np.all(np.diff(fs) < 0)
    ctx.close()


def test_graph_replay_matches_direct_launches(gpu_lib):
    """nmf_step replays captured graphs of 16, 8, 4, 2 and 1 iterations (37 =
    16 + 16 + 4 + 1, 5 = 4 + 1, 10 = 8 + 2); every replay, interleaved with
    eager work (objective, half-steps), must give the same bits as direct
    launches."""
    V, W0, H0 = g.image_like(600, 1100, 24, seed=61, init_seed=62)
    a, _, Wa, Ha = make(gpu_lib, V, W0, H0, use_graph=True)
    b, _, Wb, Hb = make(gpu_lib, V, W0, H0, use_graph=False)
    for iters in (37, 1, 16, 5, 10):
        a.step(iters)
        b.step(iters)
        fa, fb = a.objective(), b.objective()
        assert fa == fb
        assert torch.equal(Wa, Wb) and torch.equal(Ha, Hb)
        a.update_w()
        b.update_w()
        assert torch.equal(Wa, Wb)
        a.update_h()
        b.update_h()
        assert torch.equal(Ha, Hb)
    a.close()
    b.close()
