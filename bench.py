"""Throughput of the Block CUR hot path on one MI355X.

One step = one whole decomposition (||A||_F^2, the sketched top-k right
subspace, block scores, sampling, gather, U = C^+ A with one refinement step,
and the residual) with A already resident in HBM.  The default workload is
the large one-GPU share: 65536 x 16384 float32 (rank-100 signal sigma_i =
exp(-i/20), 1e-4 noise), 256 column blocks of 64, k = 100, s = 32, two power
iterations; the range finder's first two iterations run in BF16, its last
pass, the fit and the residual in FP32, the small factorizations in FP64.
`--workload plain-fp32` runs the 8192 x 4096 FP32 workload (256 blocks of
16, k = 50, s = 16).  The test matrix is drawn on the device from the seed.
Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--workload W] [--mode M]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# An FP32 product on the split-BF16 path costs six BF16 MFMA products.
SPLIT_BF16_PRODUCTS = 6


def split_bf16(M, N, K):
    """Whether the library forms an M x N x K FP32 product from the three-term
    BF16 splits of its operands (the rule stated with BCUR_PREC_FP32 in
    include/bcur.h): M, K >= 256, and N >= 256 with at least 8e9
    multiply-adds, or 32 < N <= 128 with at least 1e9."""
    if M < 256 or K < 256:
        return False
    mnk = float(M) * N * K
    return (N >= 256 and mnk >= 8.0e9) or (32 < N <= 128 and mnk >= 1.0e9)


def mfma_roofline(M, N, K, avg_ms, kernel_fp32, kernel_split, **extra):
    """Roofline entry of one FP32 product of 2 M N K FLOP per launch: against
    the FP32 MFMA peak, or on the split-BF16 path against the BF16 MFMA peak
    divided by its six products per FP32 product."""
    flop = 2.0 * M * N * K
    ach = flop / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    if split_bf16(M, N, K):
        peak = PEAK_BF16_MFMA_TFLOPS / SPLIT_BF16_PRODUCTS
        roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": round(peak, 2), "unit": "TFLOP/s",
                "frac": round(ach / peak, 4), "kernel": kernel_split, "mfma_dtype": "bf16",
                "peak_basis": f"BF16 MFMA peak {PEAK_BF16_MFMA_TFLOPS:g} TFLOP/s / {SPLIT_BF16_PRODUCTS} products",
                "bf16_tflops_executed": round(SPLIT_BF16_PRODUCTS * ach, 3)}
    else:
        roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / PEAK_FP32_MFMA_TFLOPS, 4), "kernel": kernel_fp32, "mfma_dtype": "f32"}
    roof.update({"traffic": None, "launches_per_step": 1, "avg_ms": round(avg_ms, 5), "flop_per_launch": flop})
    roof.update(extra)
    return roof


def resid_columns(m, n, c):
    """Columns of A the residual pass covers.  U on C's own columns is the
    identity (C e_k is that column of A: a residual of exactly zero there),
    so where the pass runs on the split-BF16 tile and the shorter pass takes
    fewer rounds of workgroups it covers only the n - c others (the rule
    stated with bcur_decompose in include/bcur.h)."""
    ne = n - c
    ok = ne >= 256 and m >= 256 and c >= 256 and n <= 262144 and float(m) * ne * c >= 8.0e9

    def rounds(cols):   # of 256 workgroups, on 256 x 256 tiles
        return -(-(-(-m // 256) * -(-cols // 256)) // 256)

    return ne if ok and rounds(ne) < rounds(n) else n


def algorithmic_flops(m, n, k, l, q, c):
    """FLOPs the method needs per decomposition (sketch width l, no padding)."""
    rf = (2 * q + 3) * 2.0 * m * n * l              # (q+1) x (A Q, A^T Z) + the Rayleigh-Ritz A Q
    # C^T A, A - C U over the columns outside C; G^-1 H, H - G U, G^-1 F; X^T X
    fit = 2.0 * m * c * n + 2.0 * m * c * resid_columns(m, n, c) + 3 * 2.0 * c * c * n + 2.0 * c ** 3
    return rf, fit


def cpu_baseline(w, budget_s=20.0):
    """The FP64 oracle twin as it stands, on the host cores, on whole
    decompositions of the same workload (bounded by ``budget_s``)."""
    from oracle import bcur_oracle as O
    threads = _cpu_threads()
    done, t0 = 0, time.perf_counter()
    while True:
        O.decompose(w.A, w.offsets, w.k, w.s, w.omega, w.draws, q=w.q)
        done += 1
        el = time.perf_counter() - t0
        if el > budget_s or done >= 3:
            break
    return {"value": done / el, "unit": "decompositions/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{done} whole decomposition(s) of the same {w.m}x{w.n} workload by the FP64 oracle twin "
                      f"(numpy/LAPACK, {el:.1f} s)"}


def serve_bench(args):
    """Continuous batching under Poisson arrivals (the serving workload):
    ``--requests`` distinct requests (2000 by default), each an m x n low-rank
    + noise FP32 matrix with m in [256, 8192], n in [256, 4096], rank 5..50
    (k = rank), block width in {8, 16, 32, 64}, s in [4, 32]; request i has
    its own matrix (drawn on the GPU from seed i), its own test matrix (device
    Philox seed i) and its own draws.  Measures the saturation throughput (all
    requests submitted at once) in plain FP32 and with the BF16 range finder,
    compares them at equal residual accuracy (|err_bf16 - err_fp32| <= 1e-5
    err_fp32 per request), then p50/p99 latency at Poisson arrival rates that
    are fractions of the FP32 saturation throughput."""
    import numpy as np
    import torch

    from paper_1703_06065_amd import Server
    from paper_1703_06065_amd.binding import PREC_BF16, PREC_FP32
    from workloads import gen

    t0 = time.perf_counter()
    specs = [gen.serving_spec(i) for i in range(args.requests)]
    mats = [gen.serving_matrix_device(sp) for sp in specs]
    draws = [gen.draws_u64(sp.s, 7919 + sp.req_id) for sp in specs]
    torch.cuda.synchronize()
    print(f"[serve] {len(specs)} request matrices drawn on the GPU in {time.perf_counter() - t0:.1f} s "
          f"({sum(sp.m * sp.n for sp in specs) * 4 / 2 ** 30:.1f} GiB)", file=sys.stderr, flush=True)

    def run(rate, precision, n_req=None):
        n_req = len(specs) if n_req is None else n_req
        srv = Server(0, hbm_budget=args.budget_gib << 30, max_slots=args.slots)
        rng = np.random.default_rng(12345)
        gaps = rng.exponential(1.0 / rate, size=n_req) if rate > 0 else np.zeros(n_req)
        tickets = []
        next_t = time.perf_counter()
        for i in range(n_req):
            next_t += gaps[i]
            while True:
                now = time.perf_counter()
                if now >= next_t:
                    break
                time.sleep(min(0.0005, next_t - now))
            sp = specs[i]
            tickets.append(srv.submit(mats[i], sp.offsets, sp.k, sp.s, sp.req_id, draws[i], q=2, l=sp.l,
                                      precision=precision))
        errs = np.array([srv.wait(t)["err"] for t in tickets])
        st = srv.stats()
        srv.close()
        print(f"[serve] {n_req} requests at rate {rate:.1f}/s ({'bf16' if precision == PREC_BF16 else 'fp32'}): "
              f"{st['throughput']:.1f}/s p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms", file=sys.stderr,
              flush=True)
        return st, errs

    run(0, PREC_FP32, n_req=min(200, len(specs)))   # warm up every slot
    sat, e32 = run(0, PREC_FP32)
    sat_mixed, e16 = run(0, PREC_BF16)
    gap = np.abs(e16 - e32) / np.maximum(e32, 1e-300)
    equal = gap <= 1e-5
    sweep = []
    for frac in (0.25, 0.5, 0.75, 0.9, 1.0, 1.25):
        st, _ = run(frac * sat["throughput"], PREC_FP32)
        sweep.append({"rate_frac": frac, "offered_per_s": round(frac * sat["throughput"], 2),
                      "throughput": round(st["throughput"], 2), "p50_ms": round(st["p50_ms"], 3),
                      "p99_ms": round(st["p99_ms"], 3), "peak_running": st["peak_running"]})
    makespan_mixed = len(specs) / sat_mixed["throughput"]
    out = {
        "metric": "served block-CUR decompositions/s and p50/p99 latency",
        "value": sat["throughput"], "unit": "decompositions/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32", "data": f"synthetic serving mix: {len(specs)} distinct seeded requests (matrices drawn on "
                                f"the GPU)",
        "config": {"workload": "serving: m 256-8192, n 256-4096, rank 5-50 (k = rank), block 8-64, s 4-32, q = 2",
                   "requests": len(specs), "slots": args.slots, "budget_gib": args.budget_gib},
        "p50_ms": round(sat["p50_ms"], 3), "p99_ms": round(sat["p99_ms"], 3),
        "mixed_vs_fp32": {
            "fp32_per_s": round(sat["throughput"], 2), "bf16_range_finder_per_s": round(sat_mixed["throughput"], 2),
            "ratio": round(sat_mixed["throughput"] / sat["throughput"], 4),
            "requests_at_equal_residual": int(np.sum(equal)),
            "bf16_per_s_counting_equal_residual_only": round(float(np.sum(equal)) / makespan_mixed, 2),
            "max_rel_residual_gap": float(gap.max()), "median_rel_residual_gap": float(np.median(gap))},
        "poisson_sweep": sweep,
    }
    print(json.dumps(out), flush=True)


def alg1_flops(m, n, r, kr, c):
    """FLOPs of Algorithm 1 per decomposition: R R^T and V = R^T U_kr S^-1,
    the Gram matrix of W and W^+, C U (m x c x r) and the residual
    A - (C U) R (m x r x n)."""
    t = min(r, c)
    return (2.0 * r * r * n + 2.0 * n * r * kr + 2.0 * t * t * max(r, c) + 2.0 * c * r * t
            + 2.0 * m * c * r + 2.0 * m * r * n)


def alg1_bench(args):
    """Algorithm 1 (uniform rows, U = W^+) on the same 8192 x 4096 workload:
    r = 128 rows, scores from the top-r right singular vectors of R (the
    listing's choice; --kr picks fewer), s = 16 column blocks."""
    import numpy as np
    import torch

    from paper_1703_06065_amd import Context
    from paper_1703_06065_amd.binding import padded_empty, to_device
    from workloads import gen

    w = gen.plain_fp32(args.seed)
    r = args.rows
    kr = args.kr if args.kr > 0 else r
    draws = gen.draws_u64(r + w.s, args.seed + 1)
    A = to_device(w.A)
    ctx = Context(0)
    Ubuf = padded_empty(w.s * int(np.max(np.diff(w.offsets))), r)
    for _ in range(args.warmup):
        res = ctx.decompose_alg1(A, w.offsets, r, w.s, draws, kr=kr, U_out=Ubuf)
    torch.cuda.synchronize()
    # timed region: only the residual GEMM (stage fit_E) records HIP events
    ctx.timing_enable(("fit_E",))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = ctx.decompose_alg1(A, w.offsets, r, w.s, draws, kr=kr, U_out=Ubuf)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = ctx.timing_read()
    ctx.timing_enable(True)
    nb = min(args.steps, 10)
    for _ in range(nb):
        ctx.decompose_alg1(A, w.offsets, r, w.s, draws, kr=kr, U_out=Ubuf)
    torch.cuda.synchronize()
    breakdown = ctx.timing_read()
    ctx.timing_enable(False)
    el = t1 - t0
    c = int(res["c"])
    # the residual GEMM A - (C U) R: 2 m r n FLOP per launch, one launch per step
    avg_ms = stages["fit_E"][0] / max(stages["fit_E"][1], 1)
    roof = mfma_roofline(w.m, w.n, r, avg_ms, "k_sgemm<128,128,16,2,2> residual epilogue (E = A - (C U) R)",
                         "k_xgemm<256,256> split-BF16, norm-only residual epilogue (E = A - (C U) R)",
                         algorithmic_bytes_per_launch=4.0 * (w.m * r + r * w.n + 2.0 * w.m * w.n))
    out = {
        "metric": "block-CUR decompositions/s (Algorithm 1: uniform rows, U = W^+)",
        "value": args.steps / el,
        "unit": "decompositions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded numpy: rank-50 Haar signal sigma_i = 1/i + 1e-3 Gaussian noise)",
        "config": {"workload": f"plain-fp32 {w.m}x{w.n}, {w.G} column blocks of 16, Algorithm 1 with r={r} "
                               f"uniform rows, kr={kr}, s={w.s}", "m": w.m, "n": w.n, "G": w.G, "r": r, "kr": kr,
                   "s": w.s, "c": c},
        "tflops_total": round(alg1_flops(w.m, w.n, r, kr, c) * args.steps / el / 1e12, 3),
        "stage_ms_per_step": {k: round(v[0] / nb, 5) for k, v in breakdown.items() if v[1]},
        "err": res["err"], "rel_err": res["rel_err"], "rank_w": res["rank_w"], "sweeps": res["sweeps"],
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        from oracle import bcur_oracle as O
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
        except Exception:  # pragma: no cover
            threads = os.cpu_count()
        done, c0 = 0, time.perf_counter()
        while True:
            O.alg1(w.A, w.offsets, r, w.s, None, draws, kr=kr)
            done += 1
            ce = time.perf_counter() - c0
            if ce > 20.0 or done >= 5:
                break
        out["cpu_baseline"] = {"value": done / ce, "unit": "decompositions/s", "cores": int(threads),
                               "kind": "oracle",
                               "sample": f"{done} whole Algorithm 1 decomposition(s) of the same workload by the "
                                         f"FP64 oracle (numpy/LAPACK, {ce:.1f} s)"}
    print(json.dumps(out), flush=True)


def boost_bench(args):
    """Boosting on the 8192 x 4096 workload: one range finder and one set of
    scores, t samplings of s = 16 blocks, each fitted with one refinement
    step; the best trial kept.  One step = one boosted decomposition."""
    import numpy as np
    import torch

    from paper_1703_06065_amd import Context
    from paper_1703_06065_amd.binding import padded_empty, to_device
    from workloads import gen

    w = gen.plain_fp32(args.seed)
    t = args.trials
    draws = gen.draws_u64(t * w.s, args.seed + 2)
    A = to_device(w.A)
    om = torch.from_numpy(w.omega).cuda()
    ctx = Context(0)
    Ubuf = padded_empty(w.s * int(np.max(np.diff(w.offsets))), w.n)
    for _ in range(args.warmup):
        res = ctx.decompose_boost(A, w.offsets, w.k, w.s, om, draws, t, q=w.q, U_out=Ubuf)
    torch.cuda.synchronize()
    # timed region: only the all-trials H = C^T A GEMM (stage fit_H) records HIP events
    ctx.timing_enable(("fit_H",))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = ctx.decompose_boost(A, w.offsets, w.k, w.s, om, draws, t, q=w.q, U_out=Ubuf)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = ctx.timing_read()
    ctx.timing_enable(True)
    nb = min(args.steps, 10)
    for _ in range(nb):
        ctx.decompose_boost(A, w.offsets, w.k, w.s, om, draws, t, q=w.q, U_out=Ubuf)
    torch.cuda.synchronize()
    breakdown = ctx.timing_read()
    ctx.timing_enable(False)
    el = t1 - t0
    # every trial here has c = 256 columns (16 distinct blocks of 16): ctot = t c
    c = int(res["c"])
    ctot = t * c
    avg_ms = stages["fit_H"][0] / max(stages["fit_H"][1], 1)
    roof = mfma_roofline(ctot, w.n, w.m, avg_ms,
                         "k_sgemm<256,128,16,4,2,TA> (H = C^T A over the t trials' concatenated columns)",
                         "k_xgemm<256,256,TA> split-BF16 (H = C^T A over the t trials' concatenated columns)",
                         algorithmic_bytes_per_launch=4.0 * (w.m * ctot + w.m * w.n + ctot * w.n))
    rf_flops, fit_flops = algorithmic_flops(w.m, w.n, w.k, w.l, w.q, c)
    out = {
        "metric": f"block-CUR boosted decompositions/s (t = {t} trials)",
        "value": args.steps / el,
        "unit": "decompositions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded numpy: rank-50 Haar signal sigma_i = 1/i + 1e-3 Gaussian noise)",
        "config": {"workload": f"plain-fp32 {w.m}x{w.n}, {w.G} column blocks of 16, k={w.k}, s={w.s}, q={w.q}, "
                               f"l={w.l}, boosting over t={t} samplings", "m": w.m, "n": w.n, "G": w.G, "k": w.k,
                   "s": w.s, "q": w.q, "l": w.l, "t": t, "c": c, "refine": 1},
        "tflops_total": round((rf_flops + t * fit_flops) * args.steps / el / 1e12, 3),
        "stage_ms_per_step": {k: round(v[0] / nb, 5) for k, v in breakdown.items() if v[1]},
        "errs": [float(e) for e in res["errs"]], "best": res["best"], "err": res["err"],
        "rel_err": res["rel_err"],
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        from oracle import bcur_oracle as O
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
        except Exception:  # pragma: no cover
            threads = os.cpu_count()
        done, c0 = 0, time.perf_counter()
        while True:
            O.boost(w.A, w.offsets, w.k, w.s, w.omega, draws, t, q=w.q)
            done += 1
            ce = time.perf_counter() - c0
            if ce > 20.0 or done >= 3:
                break
        out["cpu_baseline"] = {"value": done / ce, "unit": "decompositions/s", "cores": int(threads),
                               "kind": "oracle",
                               "sample": f"{done} whole boosted decomposition(s) (t = {t}) of the same workload by "
                                         f"the FP64 oracle twin (numpy/LAPACK, {ce:.1f} s)"}
    print(json.dumps(out), flush=True)


def diag_bench(args):
    """The diagnostics of Defs. 3 and 4 on the 8192 x 4096 workload's sketched
    V_k (4096 x 50, 256 blocks of 16) and U_k (8192 x 50).  One step = the
    block stable rank of every block plus the incoherence."""
    import numpy as np
    import torch

    from paper_1703_06065_amd import Context
    from paper_1703_06065_amd.binding import to_device
    from workloads import gen

    w = gen.plain_fp32(args.seed)
    ctx = Context(0)
    Vk, Uk, _ = ctx.range_finder(to_device(w.A), torch.from_numpy(w.omega).cuda(), w.k, q=w.q, want_u=True)
    for _ in range(args.warmup):
        alpha, ratios, steps = ctx.block_stable_rank(Vk, w.offsets, want_steps=True)
        mu = ctx.incoherence(Uk)
    torch.cuda.synchronize()
    ctx.timing_enable(("diag_alpha", "diag_mu"))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        alpha, ratios, steps = ctx.block_stable_rank(Vk, w.offsets, want_steps=True)
        mu = ctx.incoherence(Uk)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = ctx.timing_read()
    ctx.timing_enable(False)
    el = t1 - t0
    # FP64 work of the stable-rank kernel as executed: per block the d x d Gram
    # over the other side, the squaring steps, and the Rayleigh quotient
    widths = np.diff(w.offsets)
    flop = 0.0
    for b, st in zip(widths, steps):
        d, other = min(int(b), w.k), max(int(b), w.k)
        flop += 2.0 * d * d * other + st * (2.0 * d ** 3 + 3.0 * d * d) + 2.0 * d * d
    avg_ms = stages["diag_alpha"][0] / max(stages["diag_alpha"][1], 1)
    ach = flop / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    peak64 = 78.6
    roof = {"bound": "alu", "achieved": round(ach, 4), "peak": peak64, "unit": "TFLOP/s",
            "frac": round(ach / peak64, 5), "traffic": None,
            "kernel": "k_block_stable_rank (one workgroup per block, FP64 vector)", "launches_per_step": 1,
            "avg_ms": round(avg_ms, 5), "flop_per_launch": flop,
            "mu_kernel_ms": round(stages["diag_mu"][0] / max(stages["diag_mu"][1], 1), 5)}
    out = {
        "metric": "block-CUR diagnostics evaluations/s (block stable rank + incoherence)",
        "value": args.steps / el,
        "unit": "evaluations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (the sketched V_k and U_k of the plain-fp32 workload)",
        "config": {"workload": f"sketched V_k {w.n}x{w.k} in {w.G} blocks of 16, U_k {w.m}x{w.k}",
                   "n": w.n, "m": w.m, "k": w.k, "G": w.G},
        "alpha": alpha, "mu": mu, "max_steps": int(np.max(steps)),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        from oracle import bcur_oracle as O
        V64 = Vk.cpu().numpy().astype(np.float64)
        U64 = Uk.cpu().numpy().astype(np.float64)
        done, c0 = 0, time.perf_counter()
        while True:
            O.block_stable_rank(V64, w.offsets)
            O.incoherence(U64)
            done += 1
            ce = time.perf_counter() - c0
            if ce > 10.0 or done >= 50:
                break
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
        except Exception:  # pragma: no cover
            threads = os.cpu_count()
        out["cpu_baseline"] = {"value": done / ce, "unit": "evaluations/s", "cores": int(threads), "kind": "oracle",
                               "sample": f"{done} evaluations of both diagnostics by the FP64 oracle on the same "
                                         f"V_k and U_k ({ce:.1f} s)"}
    print(json.dumps(out), flush=True)


def copy_bench(args):
    """A plain device copy of known size (torch's copy kernel), the yardstick
    for reading the HBM traffic counters: FETCH_SIZE and WRITE_SIZE of this
    launch against its 2 x 1 GiB of algorithmic traffic give the scales that
    turn the counters of the path's kernels into bytes."""
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes,
                      "launches": args.steps}), flush=True)


def scores_bench(args):
    """Block leverage scores (Def. 2) on the stress shape where the pass is
    bandwidth-bound rather than launch-bound: V of 4M x 100 FP32 (1.6 GB) in
    65536 blocks of 64 rows.  One step = one bcur_block_scores call; the
    kernel's own time comes from HIP events on the library's stream."""
    import numpy as np
    import torch

    from paper_1703_06065_amd import Context
    n, k, b = 1 << 22, 100, 64
    g = torch.Generator(device="cuda").manual_seed(args.seed)
    V = torch.randn((n, k), dtype=torch.float32, device="cuda", generator=g)
    off = np.arange(0, n + 1, b, dtype=np.int64)
    ctx = Context(0)
    for _ in range(args.warmup):
        ctx.block_scores(V, off)
    torch.cuda.synchronize()
    ctx.timing_enable(("scores",))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sc = ctx.block_scores(V, off)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = ctx.timing_read()["scores"]
    ctx.timing_enable(False)
    avg_ms = st[0] / max(st[1], 1)
    nbytes = 4.0 * n * k
    ach = nbytes / (avg_ms * 1e-3) / 1e9
    out = {"metric": "block-score passes/s (stress shape)", "value": args.steps / el, "unit": "passes/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32->f64",
           "data": "synthetic (torch.randn V)",
           "config": {"workload": f"block scores: V {n}x{k} FP32, {len(off) - 1} blocks of {b} rows",
                      "n": n, "k": k, "G": len(off) - 1},
           "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None, "kernel": "k_block_scores",
                        "avg_ms": round(avg_ms, 5), "algorithmic_bytes_per_launch": nbytes},
           "sum_of_scores": float(np.sum(sc))}
    print(json.dumps(out), flush=True)


def _cpu_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        return os.cpu_count()


def cpu_baseline_large(w, omega64, budget_fit_cols=(128, 256)):
    """The FP64 oracle as it stands, timed step by step on a bounded sample of
    the large-share workload (a whole oracle decomposition takes minutes):
    ||A||_F^2 on all of A; the twin's range finder with q = 0 on all of A
    (three of the 2q + 3 passes over A, with one QR and the Rayleigh-Ritz
    step), scaled by (2q + 3) / 3; scores and sampling; the least-squares fit
    of two leading column panels of A (lstsq, then the explicit residual),
    extrapolated linearly in the panel width to all n columns (the fit's cost
    is a fixed factorization of C plus a per-column part)."""
    import numpy as np

    from oracle import bcur_oracle as O
    A64 = w.A.astype(np.float64)
    t = {}
    c0 = time.perf_counter()
    O.frob2(A64)
    t["frob2"] = time.perf_counter() - c0
    c0 = time.perf_counter()
    rf = O.range_finder(A64, omega64, 0, w.k)
    t["range_finder_q0"] = time.perf_counter() - c0
    c0 = time.perf_counter()
    sc = O.block_scores(rf["Vk"], w.offsets)
    smp = O.sample_blocks(sc, w.draws[:w.s], w.s)
    C = O.gather_columns(A64, w.offsets, smp["idx"])
    t["scores_sample_gather"] = time.perf_counter() - c0
    fits = []
    for nc in budget_fit_cols:
        c0 = time.perf_counter()
        O.fit_columns(A64[:, :nc], C)
        fits.append(time.perf_counter() - c0)
    n0, n1 = budget_fit_cols
    per_col = max(fits[1] - fits[0], 0.0) / (n1 - n0)
    fit_all = fits[0] + per_col * (w.n - n0)
    total = t["frob2"] + t["range_finder_q0"] * (2 * w.q + 3) / 3.0 + t["scores_sample_gather"] + fit_all
    spent = sum(t.values()) + sum(fits)
    return {"value": 1.0 / total, "unit": "decompositions/s", "cores": int(_cpu_threads()), "kind": "oracle",
            "sample": f"FP64 oracle twin on the same {w.m}x{w.n} input, timed step by step ({spent:.1f} s of CPU "
                      f"time): frob2 {t['frob2']:.2f} s; range finder with q=0 {t['range_finder_q0']:.2f} s, "
                      f"scaled x{(2 * w.q + 3) / 3.0:.3f} to q={w.q}; scores+sampling+gather "
                      f"{t['scores_sample_gather']:.2f} s; lstsq fit of {n0} and {n1} columns "
                      f"{fits[0]:.2f} / {fits[1]:.2f} s, extrapolated to {w.n} columns ({fit_all:.1f} s); "
                      f"estimated {total:.1f} s per decomposition"}


# HBM traffic of the dominant kernels, from rocprofv3 counter runs of
# `bench.py` (FETCH_SIZE and WRITE_SIZE, KiB per dispatch), each scaled by the
# same counter's reading for the plain 1 GiB copy of `bench.py --mode copy`.
# The readings hold for the kernel source whose hash is stored beside them; a
# changed source reports traffic None until the counters are taken again.
# 65536 x 16384 x 2048, rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) on
# `bench.py --steps 1 --warmup 1 --no-cpu-baseline`; the 1 GiB copy reads
# 524300 KiB of FETCH_SIZE (scale 2.0) and 1048576 KiB of WRITE_SIZE (1.0).
TRAFFIC_LARGE = {
    "fit_E": {"src": "3e8df830f82cb630", "fetch_kib": 7348632.0, "fetch_scale": 1.9999, "write_kib": 477.0,
              "write_scale": 1.0},
    "fit_H": {"src": "3e8df830f82cb630", "fetch_kib": 17301575.1, "fetch_scale": 1.9999, "write_kib": 131072.0,
              "write_scale": 1.0},
}
# 8192 x 4096 x 256, the same counters on `bench.py --workload plain-fp32
# --steps 3 --warmup 1 --no-cpu-baseline` (scales from the same copy runs).
TRAFFIC_PLAIN = {
    "fit_E": {"src": "3e8df830f82cb630", "fetch_kib": 90197.5, "fetch_scale": 1.9999, "write_kib": 16.0,
              "write_scale": 1.0},
    "fit_H": {"src": "3e8df830f82cb630", "fetch_kib": 98374.8, "fetch_scale": 1.9999, "write_kib": 65536.0,
              "write_scale": 1.0},
}


def _source_hash():
    import hashlib
    src = os.path.join(ROOT, "paper_1703_06065_amd", "csrc", "k_sgemm.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(table, stage):
    t = table.get(stage)
    if not t or t.get("src") != _source_hash():
        return None
    return round(1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]))


def decompose_bench(args):
    import numpy as np
    import torch

    from paper_1703_06065_amd import Context
    from paper_1703_06065_amd.binding import PREC_BF16, PREC_FP32, padded_empty, to_device
    from workloads import gen

    large = args.workload == "large-share"
    t0 = time.perf_counter()
    w = gen.large_share(args.seed) if large else gen.plain_fp32(args.seed)
    precision = PREC_BF16 if large else PREC_FP32
    print(f"[bench] {w.name} generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    A = to_device(w.A)
    seed = args.seed   # the test matrix is drawn on the device from this seed
    ctx = Context(0)
    cap = w.s * int(np.max(np.diff(w.offsets)))
    Ubuf = padded_empty(cap, w.n)

    def step():
        return ctx.decompose(A, w.offsets, w.k, w.s, seed, w.draws, q=w.q, l=w.l, precision=precision,
                             U_out=Ubuf)

    for _ in range(args.warmup):
        res = step()
    torch.cuda.synchronize()
    # timed region: only the two largest MFMA kernels (the residual GEMM and
    # H = C^T A, one launch each per decomposition) record HIP events
    ctx.timing_enable(("fit_E", "fit_H"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = ctx.timing_read()
    print(f"[bench] timed {args.steps} steps in {t1 - t0:.2f} s", file=sys.stderr, flush=True)
    # per-stage breakdown from a separate, untimed pass (its events slow the host side)
    ctx.timing_enable(True)
    nb = min(args.steps, 10)
    for _ in range(nb):
        step()
    torch.cuda.synchronize()
    breakdown = ctx.timing_read()
    ctx.timing_enable(False)
    el = t1 - t0
    c = int(res["c"])
    rf_flops, fit_flops = algorithmic_flops(w.m, w.n, w.k, w.l, w.q, c)

    # Roofline of the dominant kernel: of the kernels that a throughput
    # roofline bounds, the one with the largest device time per decomposition.
    # At these shapes that is one of the two c-wide products over A, each
    # one launch each per decomposition: the residual ||A - C U||_F^2 (NN,
    # norm-only epilogue, stage fit_E; 2 m c (n - c) FLOP over the columns
    # outside C) or H = C^T A (TN, stage fit_H; 2 m c n), on the split-BF16
    # kernel at these sizes.  The
    # one-workgroup FP64 solvers are latency-bound; their times are in
    # stage_ms_per_step.
    ne = resid_columns(w.m, w.n, c)
    shapes = {"fit_E": (w.m, ne, c), "fit_H": (c, w.n, w.m)}
    abytes = {"fit_E": 4.0 * (w.m * ne + w.m * c + c * ne), "fit_H": 4.0 * (w.m * w.n + w.m * c + c * w.n)}
    names = {"fit_E": ("k_sgemm<128,128,16,2,2> norm-only residual epilogue (||A - C U||_F^2)",
                       "k_xgemm<256,256> split-BF16, norm-only residual epilogue (||A - C U||_F^2)"),
             "fit_H": ("k_sgemm<256,128,16,4,2> TN (H = C^T A)", "k_xgemm<256,256,TA> split-BF16 (H = C^T A)")}
    avg = {st: stages[st][0] / max(stages[st][1], 1) for st in shapes}
    dom = max(avg, key=avg.get)
    table = TRAFFIC_LARGE if large else TRAFFIC_PLAIN
    roof = mfma_roofline(*shapes[dom], avg[dom], *names[dom], stage=dom,
                         algorithmic_bytes_per_launch=abytes[dom],
                         other_stage_avg_ms={st: round(v, 5) for st, v in avg.items() if st != dom})
    roof["traffic"] = traffic_for(table, dom)
    prec = "BF16 range finder (q BF16 power iterations, final FP32 pass), FP32 fit with one refinement step, " \
           "FP64 small factorizations" if large else "FP32 range finder and fit, FP64 small factorizations"
    prec += "; large FP32 products as six BF16 MFMA products of exact three-term BF16 splits, FP32 accumulation"
    out = {
        "metric": "block-CUR decompositions/s",
        "value": args.steps / el,
        "unit": "decompositions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": ("synthetic (seeded numpy: rank-100 Haar signal sigma_i = exp(-i/20) + 1e-4 Gaussian noise)" if large
                 else "synthetic (seeded numpy: rank-50 Haar signal sigma_i = 1/i + 1e-3 Gaussian noise)"),
        "config": {"workload": f"{w.name}: {w.G} column blocks of {int(w.offsets[1])}, k={w.k}, s={w.s}, q={w.q}, "
                               f"l={w.l}; {prec}",
                   "m": w.m, "n": w.n, "G": w.G, "k": w.k, "s": w.s, "q": w.q, "l": w.l, "c": c, "refine": 1,
                   "precision": "bf16-range-finder" if large else "fp32", "test_matrix": f"Philox seed {seed}"},
        "tflops_total": round((rf_flops + fit_flops) * args.steps / el / 1e12, 3),
        "stage_ms_per_step": {k: round(v[0] / nb, 5) for k, v in breakdown.items() if v[1]},
        "err": res["err"], "rel_err": res["rel_err"], "rr_sweeps": res["rr_sweeps"],
        "roofline": roof,
    }
    del A
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        from oracle import bcur_oracle as O
        om64 = O.rademacher_omega(w.n, w.l, seed)
        if large:
            out["cpu_baseline"] = cpu_baseline_large(w, om64)
        else:
            out["cpu_baseline"] = cpu_baseline(dataclasses_replace_omega(w, om64))
    print(json.dumps(out), flush=True)


def dataclasses_replace_omega(w, omega):
    import dataclasses
    return dataclasses.replace(w, omega=omega)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", choices=["decompose", "serve", "alg1", "boost", "diag", "copy", "scores"],
                    default="decompose")
    ap.add_argument("--workload", choices=["large-share", "plain-fp32"], default="large-share",
                    help="decompose mode: 65536 x 16384 (BF16 range finder) or 8192 x 4096 (FP32)")
    ap.add_argument("--trials", type=int, default=3, help="boosting: t = ln(1/delta) trials (3 for delta = 0.05)")
    ap.add_argument("--rows", type=int, default=128, help="Algorithm 1: rows drawn (r)")
    ap.add_argument("--kr", type=int, default=0,
                    help="Algorithm 1: right singular vectors of R behind the scores (0: r, as in the listing)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gib", type=int, default=16)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    {"serve": serve_bench, "alg1": alg1_bench, "boost": boost_bench, "diag": diag_bench, "copy": copy_bench,
     "scores": scores_bench, "decompose": decompose_bench}[args.mode](args)


if __name__ == "__main__":
    main()
