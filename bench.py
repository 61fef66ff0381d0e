#!/usr/bin/env python3
"""Benchmark of the multiplicative-update NMF hot path on one MI355X.

Workload (default): image-like V (4096 x 16384, float32) = W* H* / max with
W* ~ Gamma(2, 0.5)^{4096 x 64} and H* sparse (70% zeros, rest Exp(1)), rank
r = 64, W0, H0 ~ U(0,1).  A step is one full iteration of Algorithm 1 (W
half-step, H half-step, and the two r x r Grams), all on the GPU with V
resident in HBM.  Objective evaluations are not part of a step (fixed-count
iterations, as the paper times its GPU runs); the objective is evaluated
once after the timed region as a sanity check.

Prints one JSON line: iterations/s of the default path (the iterations
replayed from HIP graphs, no profiler), the roofline of the dominant kernel
(its mean duration from HIP events recorded around every stage in a second
window of the same number of iterations, launched directly) and the FP64
CPU oracle timed on a bounded sample of the same workload, on one host core
and on all of them.

Unless --no-ceilings, the rates this GPU sustains (nmf_ceiling: an HBM read
stream and the matrix-core and vector instructions the kernels use) are
measured after the headline's windows, and every pass roofline also states
the time bound they give and the fraction of it the pass reaches.
Then (unless --no-stream-reference) a plain 1.07 GB device copy by torch, as
a practical HBM streaming rate beside the 8000 GB/s peak.
Then (unless --no-rank-sweep) the same shape at ranks 8, 16, 32 and 64 in
both tiers (the HBM-bound regime of the FP32 tier is rank <= 39), and (unless
--no-poisson) the Poisson (KL) update at ranks 64 and 32.
Then (unless --no-precision-tier) the FP32 and BF16 tiers at 8192 x 32768
for ranks 32, 128 and 256, then (unless --no-batch) the batched tier: 512 problems of uneven shape,
200 iterations each in one persistent launch, against a loop of the
single-problem solver.  Then (unless --no-warm-start) the time-to-tolerance
experiment: a stream of
1024 x 4096 matrices sharing a base dictionary (1024 x 48, Gamma(2, 0.5),
perturbed per matrix by LogNormal(0, 0.1)); the warm-start network
(1024 -> 512 -> 48) is trained on solver-converged factors of the first
matrices and the time to an objective gap f / ||V||^2 <= 1e-4 is measured
on held-out matrices for a cold FP32 start and for BF16 + warm start.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NMF iters/sec + time to 1e-4 rel. objective gap: FP32 vs BF16+warm-start"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}
PEAK_F64_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--precision", choices=["fp32", "bf16"], default="fp32")
    ap.add_argument("--p", type=int, default=4096)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--r", type=int, default=64)
    ap.add_argument("--ldv-pad", type=int, default=0,
                    help="extra floats per V row in device memory (row-stride experiment)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-tier run")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the measured rate ceilings (nmf_ceiling)")
    ap.add_argument("--no-stream-reference", action="store_true",
                    help="skip the reference copy that measures a practical HBM rate")
    ap.add_argument("--no-precision-tier", action="store_true",
                    help="skip the 8192 x 32768 FP32 / BF16 rank sweep")
    ap.add_argument("--no-rank-sweep", action="store_true",
                    help="skip the rank sweep {8, 16, 32, 64} at the headline shape")
    ap.add_argument("--sweep-ranks", type=int, nargs="+", default=[8, 16, 32, 64])
    ap.add_argument("--sweep-steps", type=int, default=200)
    ap.add_argument("--no-poisson", action="store_true",
                    help="skip the Poisson (KL) update at the headline shape")
    ap.add_argument("--poisson-ranks", type=int, nargs="+", default=[64, 32])
    ap.add_argument("--no-pet", action="store_true",
                    help="skip the penalized PET reconstruction runs")
    ap.add_argument("--pet-mus", type=float, nargs="+", default=[0.0, 1e-7, 1e-6, 1e-5])
    ap.add_argument("--pet-max-iters", type=int, default=100000)
    ap.add_argument("--pt-iters", type=int, default=200)
    ap.add_argument("--pt-ranks", type=int, nargs="+", default=[32, 128, 256])
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="first copy 256 MiB between two device buffers (a plain copy kernel "
                         "of known size, the reference for hardware byte counters)")
    ap.add_argument("--batch-iters", type=int, default=200)
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the time-to-tolerance experiment")
    ap.add_argument("--ws-train", type=int, default=800, help="training matrices")
    ap.add_argument("--ws-test", type=int, default=64, help="held-out matrices timed")
    ap.add_argument("--ws-epochs", type=int, default=6)
    ap.add_argument("--ws-target-tol", type=float, default=1e-4,
                    help="training targets: each training matrix solved to this gap (the "
                         "solver-converged factors); <= 0 uses --ws-target-iters iterations")
    ap.add_argument("--ws-target-iters", type=int, default=200)
    ap.add_argument("--ws-dict-iters", type=int, default=3000,
                    help="iterations of the joint factorization that gives W-bar")
    ap.add_argument("--ws-dict-precision", choices=["fp32", "bf16"], default="bf16")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="budget of each FP64 oracle baseline leg (0 disables)")
    ap.add_argument("--cpu-gap-seconds", type=float, default=60.0,
                    help="cap of the oracle's time to the 1e-4 gap on one warm-start "
                         "matrix (0 disables)")
    return ap.parse_args()


def host_cpu():
    """Model name and logical core count of this host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "cpu_count": os.cpu_count()}


def _oracle_rate(V64, W0, H0, seconds, max_iters=1000):
    """FP64 oracle iterations per second from (W0, H0), bounded to about
    `seconds` (at least one iteration)."""
    from oracle import nmf_oracle as oracle
    W, H = W0.astype(np.float64), H0.astype(np.float64)
    t0 = time.perf_counter()
    k = 0
    while True:
        W, H = oracle.step(V64, W, H)
        k += 1
        el = time.perf_counter() - t0
        if el >= seconds or k >= max_iters:
            return k, el


def cpu_baseline(V, W0, H0, seconds):
    """The FP64 oracle (numpy BLAS) on the host: iterations/s on all host
    cores (the reported value) and on one core (the paper's CPU baseline ran
    on one core, Sec. 3), each leg bounded to about `seconds`."""
    from threadpoolctl import threadpool_info, threadpool_limits
    V64 = V.astype(np.float64)
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    k_all, el_all = _oracle_rate(V64, W0, H0, seconds)
    with threadpool_limits(1):
        k_one, el_one = _oracle_rate(V64, W0, H0, seconds)
    return {"value": k_all / el_all, "unit": "iters/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{k_all} FP64 iterations (numpy BLAS, {threads} threads) of the same "
                      f"workload from the same start, {el_all:.1f} s",
            "one_core": {"value": k_one / el_one, "unit": "iters/s", "cores": 1,
                         "sample": f"{k_one} FP64 iterations on one thread, {el_one:.1f} s"},
            "host": host_cpu()}


def oracle_time_to_gap(V, m, cap_s, tol=1e-4, check_every=10):
    """The FP64 oracle's wall time to f / ||V||^2 <= tol on one warm-start
    matrix from a U(0,1) start (numpy PCG64, seed 400000 + m), objective
    checked every `check_every` iterations, all host cores; stops at cap_s
    seconds (then reports the gap reached)."""
    from threadpoolctl import threadpool_info

    from oracle import nmf_oracle as oracle
    from synth import generators as gen
    p, n = V.shape
    V64 = V.astype(np.float64)
    W0, H0 = gen.uniform_init(p, n, 48, seed=400000 + m)
    W, H = W0.astype(np.float64), H0.astype(np.float64)
    nv2 = float(np.sum(V64 * V64))
    t0 = time.perf_counter()
    k = 0
    gap = oracle.objective(V64, W, H) / nv2
    while gap > tol and time.perf_counter() - t0 < cap_s:
        for _ in range(check_every):
            W, H = oracle.step(V64, W, H)
        k += check_every
        gap = oracle.objective(V64, W, H) / nv2
    el = time.perf_counter() - t0
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    return {"matrix": m, "seconds": round(el, 2), "iters": k, "gap": gap,
            "converged": bool(gap <= tol), "threads": int(threads), "check_every": check_every,
            "start": "U(0,1) numpy PCG64 seed 400000+m (the GPU cold starts draw on the device)"}


def _gen_matrix(args):
    from threadpoolctl import threadpool_limits

    from synth import generators as gen
    Wb, m = args
    with threadpool_limits(1):
        return gen.warm_start_matrix(Wb, m)[0]


def stream_reference():
    """Practical streaming rate of this GPU's HBM, beside the 8000 GB/s peak:
    the best of 10 device-to-device copies of 1.07 GB by torch (bytes read
    plus written), timed with HIP events.  Context for the roofline
    fractions, not part of any timed region."""
    import torch
    x = torch.rand((8192, 32768), device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(10):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        y.copy_(x)
        e.record()
        e.synchronize()
        best = min(best, s.elapsed_time(e) * 1e-3)
    nbytes = 2 * x.numel() * 4
    del x, y
    torch.cuda.empty_cache()
    return {"copy_GBps": round(nbytes / best / 1e9, 1), "bytes": nbytes,
            "note": "torch device-to-device copy (read + write bytes), best of 10"}


def measured_traffic(stage, p, n, r, precision):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter's reading
    for a copy of known size), for the workload those counters were taken on;
    None for any other workload or once the kernel source has changed."""
    import hashlib
    import re
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "pmc_traffic_k_nt_dma_fp32_4096x16384_r64.md")
    if (p, n, r, precision) != (4096, 16384, 64, "fp32") or not os.path.exists(path):
        return None
    text = open(path).read()
    h = hashlib.sha256()
    for f in ("nmf_kernels.hip", "nmf_device.h"):  # the pass kernels and their device helpers
        h.update(open(os.path.join(here, "paper_1003_3272_amd", "csrc", f), "rb").read())
    sha = re.search(r"kernel_source_sha256: ([0-9a-f]+)", text)
    val = re.search(rf"traffic_bytes_per_launch {stage}: ([0-9]+)", text)
    if not sha or not val or h.hexdigest() != sha.group(1):
        return None
    return int(val.group(1))


def _precision_case(r):
    from synth import generators as gen
    return gen.precision_tier(r)


def timed_steps(ctx, steps):
    """Seconds for `steps` iterations on the default path (iterations
    replayed from the HIP graphs captured beforehand, profiler off),
    synchronized on both sides."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def profiled_steps(ctx, steps):
    """{stage: (total ms, launches)} of `steps` iterations launched directly
    with HIP events recorded around every stage on the context's stream."""
    ctx.profile_start(8 * steps)
    ctx.step(steps)
    return ctx.profile_stop()


# rates measured on this GPU by nmf_ceiling (None until measured_ceilings runs)
CEILINGS = None


def measured_ceilings():
    """What this GPU sustains, beside the published peaks: an HBM read stream
    over a 1 GiB buffer (best of 10 passes in one timed window) and the dense
    throughput of the matrix-core and vector instructions the kernels use.
    Measured after the headline's timed windows, outside any of them."""
    import torch

    from paper_1003_3272_amd import nmf
    global CEILINGS
    buf = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    rate = {k: nmf.ceiling(k, buf, reps=10 if k == "hbm_read" else 5) for k in nmf.CEILING_KINDS}
    del buf
    torch.cuda.empty_cache()
    best_f32 = max(rate["mfma_f32"], rate["mfma_f32_32"])
    best_bf16 = max(rate["mfma_bf16"], rate["mfma_bf16_32"])
    CEILINGS = {
        "hbm_read_GBps": round(rate["hbm_read"] / 1e9, 1),
        # the faster of the 16 x 16 and 32 x 32 shapes of each type
        "mfma_fp32_TFLOPs": round(best_f32 / 1e12, 1),
        "mfma_bf16_TFLOPs": round(best_bf16 / 1e12, 1),
        "mfma_f64_TFLOPs": round(rate["mfma_f64"] / 1e12, 1),
        "fma_f64_TFLOPs": round(rate["fma_f64"] / 1e12, 1),
        "by_shape_TFLOPs": {
            "v_mfma_f32_16x16x4f32": round(rate["mfma_f32"] / 1e12, 1),
            "v_mfma_f32_32x32x2f32": round(rate["mfma_f32_32"] / 1e12, 1),
            "v_mfma_f32_16x16x32_bf16": round(rate["mfma_bf16"] / 1e12, 1),
            "v_mfma_f32_32x32x16_bf16": round(rate["mfma_bf16_32"] / 1e12, 1)},
        "fraction_of_published": {
            "hbm_read": round(rate["hbm_read"] / 1e9 / PEAK_HBM_GBS, 3),
            "mfma_fp32": round(best_f32 / 1e12 / PEAK_TFLOPS["fp32"], 3),
            "mfma_bf16": round(best_bf16 / 1e12 / PEAK_TFLOPS["bf16"], 3),
            "mfma_f64": round(rate["mfma_f64"] / 1e12 / PEAK_F64_TFLOPS, 3),
            "fma_f64": round(rate["fma_f64"] / 1e12 / PEAK_F64_TFLOPS, 3)},
        "how": "nmf_ceiling: a read-only stream of 1020 MiB, and 2048 workgroups of 4 waves "
               "issuing independent chains of one instruction (the float32 and bf16 matrix "
               "shapes 16x16 and 32x32, v_mfma_f64_16x16x4f64, v_fma_f64) with no memory "
               "traffic; each rate timed with HIP events over 5-10 launches"}
    return CEILINGS


def _measured_bound(roof, flops, vbytes, prec, ms):
    """The pass's time bound from the measured ceilings (the slower of its
    flops at the measured matrix-core rate and its V bytes at the measured
    read rate), and the fraction of it the pass reaches."""
    if CEILINGS is None:
        return
    t_mma = flops / (CEILINGS[f"mfma_{prec}_TFLOPs"] * 1e12)
    t_hbm = vbytes / (CEILINGS["hbm_read_GBps"] * 1e9)
    roof["measured_bound"] = "mfma" if t_mma >= t_hbm else "hbm"
    roof["measured_bound_ms"] = round(1e3 * max(t_mma, t_hbm), 4)
    roof["frac_of_measured_bound"] = round(max(t_mma, t_hbm) / (ms * 1e-3), 4)


def pass_roofline(stages, p, n, r, prec):
    """Roofline of the slower V-streaming pass: 2 p n r flops and p n s_V
    bytes of V per launch (s_V = 4 for FP32, 2 for BF16), against whichever
    of the two peaks binds."""
    passes = {k: stages[k][0] / max(1, stages[k][1]) for k in ("gemm_vht", "gemm_wtv")}
    dom = max(passes, key=passes.get)
    ms = passes[dom]
    flops = 2.0 * p * n * r
    vbytes = p * n * (4 if prec == "fp32" else 2)
    peak_t = PEAK_TFLOPS[prec]
    if flops / (peak_t * 1e12) >= vbytes / (PEAK_HBM_GBS * 1e9):
        ach = flops / (ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(ach, 2), "peak": peak_t, "unit": "TFLOP/s"}
    else:
        ach = vbytes / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["kernel"] = dom
    roof["kernel_ms"] = round(ms, 4)
    roof["v_pass_gbs"] = round(vbytes / (ms * 1e-3) / 1e9, 1)
    roof["other_pass_ms"] = round(passes["gemm_wtv" if dom == "gemm_vht" else "gemm_vht"], 4)
    _measured_bound(roof, flops, vbytes, prec, ms)
    return roof


def rank_sweep(Vd, args, log):
    """The headline matrix at factorization ranks 8, 16, 32 and 64, both
    tiers: iterations/s on the default path and the roofline of the slower
    pass (HBM-bound in FP32 below rank 39, in BF16 throughout)."""
    import torch

    from paper_1003_3272_amd import nmf
    from synth import generators as gen
    p, n = Vd.shape
    out = {"workload": f"the headline V ({p}x{n}, planted rank {args.r}), factorization rank r, "
                       f"U(0,1) start seed 2002", "steps": args.sweep_steps, "ranks": {}}
    for r in args.sweep_ranks:
        W0, H0 = gen.uniform_init(p, n, r, seed=2002)
        res = {}
        for prec in ("fp32", "bf16"):
            Wd, Hd = torch.from_numpy(W0).cuda(), torch.from_numpy(H0).cuda()
            with nmf.Nmf(Vd, Wd, Hd, precision=prec) as ctx:
                ctx.prepare_graphs()
                ctx.step(4)
                el = timed_steps(ctx, args.sweep_steps)
                st = profiled_steps(ctx, min(args.sweep_steps, 50))
            res[prec] = {"iters_per_s": round(args.sweep_steps / el, 1),
                         "roofline": pass_roofline(st, p, n, r, prec)}
            del Wd, Hd
        out["ranks"][str(r)] = res
        log(f"rank sweep r={r}: fp32 {res['fp32']['iters_per_s']} it/s "
            f"({res['fp32']['roofline']['bound']} {res['fp32']['roofline']['frac']}), bf16 "
            f"{res['bf16']['iters_per_s']} it/s ({res['bf16']['roofline']['bound']} "
            f"{res['bf16']['roofline']['frac']})")
    return out


def poisson_experiment(Vd, args, log):
    """The Poisson (KL) square-root update on the headline matrix: iterations/s
    on the default path and the roofline of the slower numerator pass.  Each
    pass streams V (or V^T) once and runs 4 p n r flops on the matrix cores
    (the B = W H values it needs, recomputed, and the numerator product)."""
    import torch

    from paper_1003_3272_amd import nmf
    from synth import generators as gen
    p, n = Vd.shape
    out = {"workload": f"the headline V ({p}x{n}), Poisson log-likelihood, factorization rank "
                       f"r, U(0,1) start seed 2002, fp32", "steps": args.sweep_steps, "ranks": {}}
    for r in args.poisson_ranks:
        W0, H0 = gen.uniform_init(p, n, r, seed=2002)
        Wd, Hd = torch.from_numpy(W0).cuda(), torch.from_numpy(H0).cuda()
        with nmf.Nmf(Vd, Wd, Hd, loss="poisson") as ctx:
            L0 = ctx.objective()
            ctx.prepare_graphs()
            ctx.step(4)
            el = timed_steps(ctx, args.sweep_steps)
            st = profiled_steps(ctx, min(args.sweep_steps, 50))
            L1 = ctx.objective()
        passes = {k: st[k][0] / max(1, st[k][1]) for k in ("gemm_vht", "gemm_wtv")}
        dom = max(passes, key=passes.get)
        ms = passes[dom]
        flops = 4.0 * p * n * r
        ach = flops / (ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(ach, 2), "peak": PEAK_TFLOPS["fp32"],
                "unit": "TFLOP/s", "frac": round(ach / PEAK_TFLOPS["fp32"], 4), "kernel": dom,
                "kernel_ms": round(ms, 4), "v_pass_gbs": round(4.0 * p * n / (ms * 1e-3) / 1e9, 1),
                "flops_per_pass": "4 p n r (B = W H recomputed, then the numerator)"}
        _measured_bound(roof, flops, 4.0 * p * n, "fp32", ms)
        out["ranks"][str(r)] = {
            "iters_per_s": round(args.sweep_steps / el, 1), "roofline": roof,
            "stages_ms_per_iter": {k: round(v[0] / max(1, v[1]), 4) for k, v in st.items()
                                   if v[1] > 0},
            "L_start": L0, "L_end": L1}
        log(f"poisson r={r}: {out['ranks'][str(r)]['iters_per_s']} it/s, pass {ms * 1e3:.1f} us "
            f"({roof['frac']} of FP32 MFMA)")
        del Wd, Hd
    return out


def pet_experiment(args, log):
    """Penalized PET reconstruction (Algorithm 2) at the paper's problem size:
    a 64 x 64 image, 2016 lines of flight.  Per iteration: the time of a long
    replayed window (no checks), and, for each roughness constant, the
    solve under the paper's stopping rule (relative change of f below 1e-9,
    checked every iteration, at most --pet-max-iters iterations), plain and
    accelerated by QN(10) (the rule checked every QN iteration).  The
    oracle's float64 iteration is timed on a few iterations for the CPU
    figure."""
    import torch

    from oracle import pet_oracle
    from paper_1003_3272_amd import nmf
    from synth import generators as gen
    E, y, _ = gen.pet_problem()
    d, p = E.shape
    Ed, yd = torch.from_numpy(E).cuda(), torch.from_numpy(y).cuda()
    out = {"workload": f"synthetic PET: {int(np.sqrt(p))}x{int(np.sqrt(p))} phantom, {d} lines "
                       "of flight of a 64-detector ring, Poisson counts of mean 50, start "
                       "lambda = 1, fp32 products, fp64 objective",
           "d": d, "p": p, "nnz_E": int(np.count_nonzero(E)), "mus": {}}
    window = 2000

    def per_iter_us(mu, layout):
        ld = torch.ones(p, dtype=torch.float32, device="cuda")
        with nmf.Pet(Ed, yd, ld, 64, 64, mu, layout=layout) as m:
            m.step(32)                       # graphs captured and warm
            torch.cuda.synchronize()
            t = time.perf_counter()
            m.step(window)
            torch.cuda.synchronize()
            return 1e6 * (time.perf_counter() - t) / window, m.layout

    it_dense, _ = per_iter_us(1e-6, "dense")
    out["dense_layout_us_per_iter"] = round(it_dense, 2)
    for mu in args.pet_mus:
        it_us, out["layout"] = per_iter_us(mu, "auto")
        ld = torch.ones(p, dtype=torch.float32, device="cuda")
        with nmf.Pet(Ed, yd, ld, 64, 64, mu) as m:
            torch.cuda.synchronize()
            t = time.perf_counter()
            conv, iters, f = m.solve(args.pet_max_iters, tol=1e-9, check_every=1)
            el = time.perf_counter() - t
        ld = torch.ones(p, dtype=torch.float32, device="cuda")
        with nmf.Pet(Ed, yd, ld, 64, 64, mu) as m:
            m.solve_qn(4, q=10, tol=0.0)     # QN graph captured and warm
            ld.fill_(1.0)
            torch.cuda.synchronize()
            t = time.perf_counter()
            qconv, qev, qacc, qf, _ = m.solve_qn(min(2 * args.pet_max_iters, 131072), q=10, tol=1e-9,
                                                 check_every=2)
            qel = time.perf_counter() - t
        out["mus"][repr(mu)] = {"us_per_iter": round(it_us, 2), "solve_s": round(el, 4),
                                "iters": iters, "converged": conv, "f": f,
                                "qn10": {"solve_s": round(qel, 4), "evals": qev,
                                         "qn_iters": qev // 2, "accepted": qacc,
                                         "converged": qconv, "f": qf}}
        log(f"pet mu={mu}: {it_us:.1f} us/iter, solve {iters} iters in {el:.3f} s "
            f"({'converged' if conv else 'cap'}), f={f:.10g}; QN(10) {qev // 2} QN iterations "
            f"({qev} maps) in {qel:.3f} s, f={qf:.10g}")
    # one iteration reads the nonzeros of E_s twice (by lines, by pixels) as
    # (float32 value, int32 index) pairs, and gathers lambda and the ratios
    nnz = out["nnz_E"]
    bytes_iter = 2 * 8.0 * nnz
    best = min(v["us_per_iter"] for v in out["mus"].values())
    out["bytes_per_iter"] = bytes_iter
    out["effective_gbs"] = round(bytes_iter / (best * 1e-6) / 1e9, 1)
    out["paper_gpu_s_per_iter"] = "282 s / 100000 iterations (GTX 280, Table 3): context only"
    log(f"pet: {best:.1f} us/iter ({out['layout']}), dense layout {it_dense:.1f} us/iter")
    Es = pet_oracle.scale_columns(E)
    pairs = pet_oracle.neighbour_pairs(64, 64)
    lam = np.ones(p)
    t = time.perf_counter()
    k = 0
    while k < 5 or time.perf_counter() - t < 2.0:
        lam = pet_oracle.step(Es, y, lam, 1e-6, pairs)
        k += 1
    out["oracle_s_per_iter"] = round((time.perf_counter() - t) / k, 5)
    out["oracle_sample"] = f"{k} float64 iterations of the oracle at mu = 1e-6"
    return out


def _fp64_reference():
    """The float64 oracle's 200-iteration trajectory of the precision-tier
    workload, stored by tests/golden/make_precision_tier_fp64.py (None if
    the file is absent)."""
    path = os.path.join(ROOT, "tests", "golden", "precision_tier_fp64.json")
    return json.load(open(path)) if os.path.exists(path) else None


def _sample_positions(rows, cols, count, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, rows, size=count), rng.integers(0, cols, size=count)


def err_vs_fp64(ref, r, f, W, H):
    """Errors of a 200-iteration GPU result against the float64 oracle's:
    objective, Frobenius norms of W and H, and the largest relative error
    over the stored sample of entries of W and H (entries above 1e-6 of the
    sample's largest)."""
    rr = ref["ranks"].get(str(r)) if ref else None
    if rr is None:
        return None
    cnt, seed = ref["sample"]["count"], ref["sample"]["seed"]
    wi, wk = _sample_positions(rr["p"], r, cnt, seed)
    hk, hj = _sample_positions(r, rr["n"], cnt, seed)

    def worst(got, want):
        want = np.asarray(want)
        keep = np.abs(want) > 1e-6 * np.abs(want).max()
        return float(np.max(np.abs(got[keep] - want[keep]) / np.abs(want[keep])))

    f64 = rr["f"]["200"]
    return {"f200_fp64": f64, "f200_rel": abs(f - f64) / f64,
            "normW_rel": abs(float(np.linalg.norm(W)) - rr["norm_W"]["200"]) / rr["norm_W"]["200"],
            "normH_rel": abs(float(np.linalg.norm(H)) - rr["norm_H"]["200"]) / rr["norm_H"]["200"],
            "W_sample_max_rel": worst(W[wi, wk], rr["W200_sample"]),
            "H_sample_max_rel": worst(H[hk, hj], rr["H200_sample"])}


def precision_tier_experiment(args, log):
    """8192 x 32768, planted rank r in {32, 128, 256}: exactly 200
    iterations of each tier from the same start on the default path (their
    time gives iterations/s), the result's error against the float64
    oracle's 200-iteration trajectory, then a profiled window for each
    pass's roofline."""
    import torch

    from paper_1003_3272_amd import nmf

    ref = _fp64_reference()
    out = {"workload": "8192x32768 image-like V (Gamma(2,0.5) x sparse Exp, rescaled), seed "
                       "1003+r, U(0,1) start seed 2003+r", "iterations": args.pt_iters,
           "fp64_reference": "tests/golden/precision_tier_fp64.json (float64 oracle, 200 "
                             "iterations)" if ref else None, "ranks": {}}
    for r in args.pt_ranks:
        t0 = time.perf_counter()
        V, W0, H0 = _precision_case(r)
        t_gen = time.perf_counter() - t0
        Vd = torch.from_numpy(V).cuda()
        del V
        res = {"generate_s": round(t_gen, 1)}
        for prec in ("fp32", "bf16"):
            Wd, Hd = torch.from_numpy(W0).cuda(), torch.from_numpy(H0).cuda()
            with nmf.Nmf(Vd, Wd, Hd, precision=prec) as ctx:
                ctx.prepare_graphs()
                el = timed_steps(ctx, args.pt_iters)
                f = ctx.objective()
                nv2 = ctx.data_norm2()
                W, H = Wd.cpu().numpy(), Hd.cpu().numpy()
                st = profiled_steps(ctx, 20)
            p_, n_ = Vd.shape
            res[prec] = {"iters_per_s": round(args.pt_iters / el, 1),
                         "roofline": pass_roofline(st, p_, n_, r, prec),
                         "objective": f, "gap": f / nv2}
            if args.pt_iters == 200:
                res[prec]["err_vs_fp64"] = err_vs_fp64(ref, r, f, W, H)
            del Wd, Hd, W, H
        res["bf16_rel_objective_vs_fp32"] = abs(res["bf16"]["objective"] - res["fp32"]["objective"]) \
            / res["fp32"]["objective"]
        res["bf16_speedup"] = round(res["bf16"]["iters_per_s"] / res["fp32"]["iters_per_s"], 2)
        out["ranks"][str(r)] = res
        e32 = (res["fp32"].get("err_vs_fp64") or {}).get("f200_rel", float("nan"))
        e16 = (res["bf16"].get("err_vs_fp64") or {}).get("f200_rel", float("nan"))
        log(f"precision tier r={r}: fp32 {res['fp32']['iters_per_s']} it/s (f200 vs fp64 "
            f"{e32:.2e}), bf16 {res['bf16']['iters_per_s']} it/s (f200 vs fp64 {e16:.2e})")
        del Vd
        torch.cuda.empty_cache()
    return out


def _gen_batch_problem(args):
    from threadpoolctl import threadpool_limits

    from synth import generators as gen
    b, (p, n, r) = args
    with threadpool_limits(1):
        return gen.batch_problem(b, p, n, r)


def batched_experiment(args, log):
    """512 problems (p ~ U{64..1024}, n ~ U{128..4096}, r ~ U{4..64}),
    200 iterations each in one persistent launch, after autotuning the tile
    table on the batch; beside it a loop of the single-problem solver over a
    sample of the same problems."""
    import multiprocessing as mp

    import numpy as np
    import torch

    from paper_1003_3272_amd import nmf
    from synth import generators as gen

    shapes = gen.batch_shapes()
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(min(16, mp.cpu_count())) as pool:
        host = pool.map(_gen_batch_problem, list(enumerate(shapes)), chunksize=8)
    t_gen = time.perf_counter() - t0
    dev = [tuple(torch.from_numpy(x).cuda() for x in t) for t in host]
    starts = [(W.clone(), H.clone()) for _, W, H in dev]
    del host
    iters = args.batch_iters
    vbytes = sum(4.0 * p * n for p, n, _ in shapes)
    flops = sum(4.0 * p * n * r for p, n, r in shapes)
    def timed_launch(b):
        """One launch of `iters` iterations from the start (graph already
        captured by a warm-up launch), timed with HIP events."""
        b.step(iters)          # warm-up launch (also captures the graph)
        b.check()
        for (_, W, H), (W0, H0) in zip(dev, starts):
            W.copy_(W0)
            H.copy_(H0)
        b.load()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.step(iters)
        e1.record()
        b.check()
        return e0.elapsed_time(e1)

    with nmf.Batch(dev) as b:
        default_table = b.table
        ms_default = timed_launch(b)
        for (_, W, H), (W0, H0) in zip(dev, starts):
            W.copy_(W0)
            H.copy_(H0)
        b.load()
        ms_tuned = b.tune(trial_iters=5)
        table = b.table
        log(f"batched: default table {default_table} {ms_default / iters:.3f} ms/iteration; "
            f"tuned table {table}, {ms_tuned:.3f} ms/iteration in trials")
        ms = timed_launch(b)
        f = b.objective()
    # the single-problem solver, one problem after another, on a sample
    sample = list(range(0, len(shapes), len(shapes) // 16))[:16]
    t_loop = 0.0
    for k in sample:
        V, _, _ = dev[k]
        W, H = starts[k][0].clone(), starts[k][1].clone()
        with nmf.Nmf(V, W, H) as ctx:
            ctx.step(2)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            ctx.step(iters)
            torch.cuda.synchronize()
            t_loop += time.perf_counter() - ta
    work = lambda ks: sum(shapes[k][0] * shapes[k][1] * shapes[k][2] for k in ks)
    loop_s_est = t_loop * work(range(len(shapes))) / work(sample)
    sec = ms / 1e3
    achieved = 2.0 * vbytes * iters / sec / 1e9
    return {
        "workload": "512 problems, p ~ U{64..1024}, n ~ U{128..4096}, r ~ U{4..64} (seed 4000), "
                    "sparse planted V (seed 100000+b), U(0,1) start (seed 200000+b), fp32",
        "iterations": iters,
        "seconds": round(sec, 4),
        "problem_iters_per_s": round(len(shapes) * iters / sec, 1),
        "effective_GBps": round(achieved, 1),
        "roofline": dict({"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                          "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                          "note": "algorithmic bytes: two float32 reads of every V per iteration"},
                         **({"frac_of_measured_read": round(achieved / CEILINGS["hbm_read_GBps"], 4)}
                            if CEILINGS else {})),
        "tflops": round(flops * iters / sec / 1e12, 2),
        "tile_table": table,
        "default_table": default_table,
        "default_table_seconds": round(ms_default / 1e3, 4),
        "autotuner_gain": round(ms_default / ms, 3),
        "loop_single_solver_s_est": round(loop_s_est, 3),
        "speedup_vs_loop": round(loop_s_est / sec, 2),
        "loop_sample": f"{len(sample)} problems (every 32nd), time scaled by p*n*r",
        "objective_finite": bool(np.all(np.isfinite(f))),
        "generate_s": round(t_gen, 1),
    }


def warm_start_experiment(args, log):
    """Time to a 1e-4 objective gap on held-out matrices: FP32 cold start vs
    BF16 refinement from W-bar and the trained network's H0."""
    import multiprocessing as mp

    import numpy as np
    import torch

    from paper_1003_3272_amd import nmf
    from paper_1003_3272_amd import warmstart as ws
    from synth import generators as gen

    t_all = time.perf_counter()
    Wb = gen.warm_start_base()
    ids = list(range(args.ws_train)) + list(range(800, 800 + args.ws_test))
    with mp.get_context("fork").Pool(min(16, mp.cpu_count())) as pool:
        mats = pool.map(_gen_matrix, [(Wb, m) for m in ids], chunksize=8)
    t_gen = time.perf_counter() - t_all
    Vs = [torch.from_numpy(V).cuda() for V in mats]
    del mats
    train, test = Vs[:args.ws_train], Vs[args.ws_train:]
    t0 = time.perf_counter()
    Wbar = ws.mean_dictionary(train[:16], 48, iters=args.ws_dict_iters,
                              precision=args.ws_dict_precision)
    t_dict = time.perf_counter() - t0
    t0 = time.perf_counter()
    Hs = []
    for a in range(0, len(train), 100):
        if args.ws_target_tol > 0:
            Hs += ws.fit_targets(train[a:a + 100], Wbar, precision="bf16", tol=args.ws_target_tol)
        else:
            Hs += ws.fit_targets(train[a:a + 100], Wbar, iters=args.ws_target_iters,
                                 precision="bf16")
        log(f"targets {min(a + 100, len(train))}/{len(train)} at {time.perf_counter() - t0:.1f} s")
    t_targets = time.perf_counter() - t0
    t0 = time.perf_counter()
    net = ws.make_network(gen.mlp_init(1024, 512, 48, 5001), Hs, max_batch=512)
    net.set_dictionary(Wbar)
    losses = ws.train(net, train, Hs, epochs=args.ws_epochs, lr=1e-3, batch=512, decay=0.8,
                      log=log)
    t_train = time.perf_counter() - t0
    del Hs
    # inference copy sized for a whole test matrix (one pass, no chunks)
    infer = ws.inference_copy(net, max(V.shape[1] for V in test))
    net.close()
    net = infer
    runs = {"fp32_cold": [], "bf16_cold": [], "bf16_wbar": [], "bf16_net": [],
            "bf16_hfit_ls": [], "bf16_net_ls": [], "fp32_cold_qn": [], "bf16_net_ls_qn": []}
    for i, V in enumerate(test):
        m = 800 + i
        runs["fp32_cold"].append(ws.solve_to_gap(V, "cold", precision="fp32", seed=400000 + m,
                                                 Wbar=Wbar))
        runs["bf16_cold"].append(ws.solve_to_gap(V, "cold", precision="bf16", seed=400000 + m,
                                                 Wbar=Wbar))
        runs["bf16_wbar"].append(ws.solve_to_gap(V, "wbar", precision="bf16", Wbar=Wbar))
        runs["bf16_net"].append(ws.solve_to_gap(V, "net", precision="bf16", Wbar=Wbar, net=net))
        runs["bf16_hfit_ls"].append(ws.solve_to_gap(V, "hfit_ls", precision="bf16", Wbar=Wbar))
        runs["bf16_net_ls"].append(ws.solve_to_gap(V, "net_ls", precision="bf16", Wbar=Wbar,
                                                   net=net))
        runs["fp32_cold_qn"].append(ws.solve_to_gap(V, "cold", precision="fp32",
                                                    seed=400000 + m, Wbar=Wbar, qn=4))
        runs["bf16_net_ls_qn"].append(ws.solve_to_gap(V, "net_ls", precision="bf16", Wbar=Wbar,
                                                      net=net, qn=4))
        log(f"test {m}: " + ", ".join(f"{k} {v[-1]['seconds']*1e3:.1f} ms / {v[-1]['iters']} it"
                                      for k, v in runs.items()))
    net.close()
    med = {k: {"ms": round(1e3 * float(np.median([x["seconds"] for x in v])), 2),
               "iters": int(np.median([x["iters"] for x in v])),
               "converged": int(sum(x["converged"] for x in v)),
               "gap_max": float(max(x["gap"] for x in v))} for k, v in runs.items()}
    for k, v in runs.items():
        if v and "qn_accepted" in v[0]:
            med[k]["qn_accepted_median"] = int(np.median([x["qn_accepted"] for x in v]))
    return {
        "workload": "1024x4096 fp32 V_m = W_m H_m / max, W_m = W_base(1024x48, Gamma(2,0.5)) "
                    "* LogNormal(0,0.1), H_m sparse Exp; rank 48; gap f/||V||^2 <= 1e-4, "
                    "objective checked every 10 iterations",
        "train_matrices": args.ws_train, "test_matrices": args.ws_test,
        "targets": (f"H of each training matrix solved from (W-bar, constant H) to gap "
                    f"{args.ws_target_tol:g}, BF16, unit-norm-column gauge"
                    if args.ws_target_tol > 0 else
                    f"H after {args.ws_target_iters} BF16 iterations from (W-bar, constant H)"),
        "network": "1024-512-48 relu/softplus, bf16 products, Adam",
        "median": med,
        "warm_start": "H0 = network(V); W0 = least-squares dictionary for H0, clipped to "
                      "1e-3 max (bf16_net_ls); bf16_net keeps W0 = W-bar; bf16_hfit_ls is the "
                      "same refit without the network (H from 20 H-only updates against W-bar)",
        "speedup_warm_vs_fp32_cold": round(med["fp32_cold"]["ms"] / med["bf16_net_ls"]["ms"], 2),
        "speedup_bf16_net_wbar_vs_fp32_cold": round(med["fp32_cold"]["ms"] / med["bf16_net"]["ms"],
                                                    2),
        "network_gain_vs_wbar": round(med["bf16_wbar"]["ms"] / med["bf16_net"]["ms"], 2),
        "network_gain_vs_hfit_ls": round(med["bf16_hfit_ls"]["ms"] / med["bf16_net_ls"]["ms"], 2),
        "qn": "QN(4) quasi-Newton acceleration (nmf_solve_qn): fp32_cold_qn from the FP32 cold "
              "start, bf16_net_ls_qn from the warm start; iters = map evaluations",
        "speedup_qn_fp32_cold": round(med["fp32_cold"]["ms"] / med["fp32_cold_qn"]["ms"], 2),
        "speedup_qn_warm_vs_fp32_cold": round(med["fp32_cold"]["ms"] / med["bf16_net_ls_qn"]["ms"],
                                              2),
        "train_loss": [round(x, 6) for x in losses],
        "pipeline_seconds": {"generate": round(t_gen, 1), "dictionary": round(t_dict, 1),
                             "targets": round(t_targets, 1), "train": round(t_train, 1),
                             "total": round(time.perf_counter() - t_all, 1)},
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "column-sharded design is described but not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1003_3272_amd import nmf
    from synth import generators as gen

    log = lambda msg: print(msg, file=sys.stderr, flush=True)  # noqa: E731
    p, n, r = args.p, args.n, args.r
    V, _, _ = gen.sparse_planted(p, n, r, seed=1002)
    W0, H0 = gen.uniform_init(p, n, r, seed=2002)
    dev = torch.device("cuda:0")
    if args.ldv_pad > 0:
        Vd = torch.zeros((p, n + args.ldv_pad), dtype=torch.float32, device=dev)[:, :n]
        Vd.copy_(torch.from_numpy(V).to(dev))
    else:
        Vd = torch.from_numpy(V).to(dev)
    Wd = torch.from_numpy(W0).to(dev)
    Hd = torch.from_numpy(H0).to(dev)

    if args.pmc_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = nmf.Nmf(Vd, Wd, Hd, precision=args.precision)
    f0 = ctx.objective()
    ctx.prepare_graphs()          # graph capture stays out of the timed region
    ctx.step(args.warmup)
    # timed region: exactly `steps` iterations on the default path
    elapsed = timed_steps(ctx, args.steps)
    f_end = ctx.objective()
    # second window, same length: per-stage HIP events (direct launches)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    stages = profiled_steps(ctx, args.steps)
    elapsed_prof = time.perf_counter() - tp
    ctx.close()

    iters_per_s = args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    if not args.no_ceilings:
        measured_ceilings()
    roof = pass_roofline(stages, p, n, r, args.precision)
    roof["traffic"] = measured_traffic(roof["kernel"], p, n, r, args.precision)
    roof["timing"] = ("kernel_ms: mean HIP-event duration of the launches of that pass in a "
                      "second window of the same number of iterations, launched directly with "
                      "events around every stage on the library's stream")

    out = {
        "metric": METRIC,
        "value": round(iters_per_s, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16",
        "data": "synthetic",
        "config": {
            "workload": f"image-like V {p}x{n} fp32 (Gamma(2,0.5) x sparse Exp, rescaled "
                        f"to [0,1]), rank {r}, U(0,1) init, {args.precision} products",
            "p": p, "n": n, "r": r, "precision": args.precision,
            "path": "default: iterations replayed from HIP graphs, profiler off",
        },
        "roofline": roof,
        "stages_ms_per_iter": {k: round(v[0] / max(1, v[1]), 4) for k, v in stages.items()
                               if v[1] > 0},
        "profiled_window_ms_per_step": round(1e3 * elapsed_prof / args.steps, 4),
        "objective": {"f0": f0, "f_end": f_end,
                      "gap_end": f_end / float(np.sum(V.astype(np.float64) ** 2))},
    }
    del Wd, Hd
    if not args.no_rank_sweep:
        out["rank_sweep"] = rank_sweep(Vd, args, log)
    if not args.no_poisson:
        out["poisson"] = poisson_experiment(Vd, args, log)
    del Vd
    torch.cuda.empty_cache()
    if not args.no_stream_reference:
        out["hbm_reference"] = stream_reference()
    if CEILINGS is not None:
        out["measured_ceilings"] = CEILINGS
    if not args.no_pet:
        out["pet"] = pet_experiment(args, log)
        torch.cuda.empty_cache()
    if not args.no_precision_tier:
        out["precision_tier"] = precision_tier_experiment(args, log)
        torch.cuda.empty_cache()
    if not args.no_batch:
        out["batched"] = batched_experiment(args, log)
        torch.cuda.empty_cache()
    if not args.no_warm_start:
        out["time_to_gap"] = warm_start_experiment(args, log)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(V, W0, H0, args.cpu_seconds)
        if args.cpu_gap_seconds > 0:
            Wb = gen.warm_start_base()
            Vm = gen.warm_start_matrix(Wb, 800)[0]
            out["cpu_baseline"]["time_to_gap"] = oracle_time_to_gap(Vm, 800, args.cpu_gap_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
