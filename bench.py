#!/usr/bin/env python3
"""Benchmark of the rerandomization hot path on one MI355X.

Metric: balance-checked draws per second at n = d = 1000 (BF16 hi+lo MFMA form, with the
plain FP32 form run on the same workload and its accepted set compared).  One step is one
pass of the whole path over one synthetic problem: rr_prepare (whitening), rr_draw_balance
(generate, contract, accept, key-only output) and rr_rand_test (201-point null grid).

Workload (default): n = 1000, n1 = 500, d = 1000 iid N(0, 1) covariates, ridge 1e-2,
1e8 Philox draws, q = 1.2e-5 (1200 accepted).  Inputs are resident in HBM before timing.
Other workloads: --workload batched_512 (512 uneven pools in one graph launch) and
--workload highdim_n256_d768 (d > n under the standardise-only metric, the Gram form against
the W X~ forms).

Prints one JSON line.  --gpus above 1 exits with an error: this path runs on one GPU.
--alone {split,fp32,i8,gram} replaces the benchmark with three rr_balance_keys calls on 2^20 keys
of the workload's pool (generation, then contraction, on one stream), for kernel traces of
each kernel on its own.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "balance-checked draws/sec at n=d=1000: BF16-split MFMA vs FP32, same accept set"
METRIC_GRAM = ("balance-checked draws/sec at n=256, d=768 (standardise-only metric): Gram form vs W X~ "
               "forms, same accept set")
PEAK_BF16_TFLOPS = 2500.0      # MI355X dense BF16 MFMA
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 (matrix / vector)
PEAK_INT8_TOPS = 5000.0        # MI355X dense int8 MFMA


CONTRACT_SRC = os.path.join(ROOT, "paper_2501_07642_amd", "csrc", "rr_contract.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "contract_traffic_stream_n1000_d1000.md")


def measured_traffic(draws_per_launch):
    """HBM bytes per contraction launch from the committed PMC summary, or None when the
    summary is missing, was taken on a different contraction source, or on launches of another
    length than this run's full chunks (the autotuner picks the chunk per box)."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip()] = v.strip().strip("`")
    src = hashlib.sha256(open(CONTRACT_SRC, "rb").read()).hexdigest()
    if fields.get("contract_source_sha256") != src:
        return None
    try:
        if int(fields["draws_per_launch"]) != int(draws_per_launch):
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(X, w, sample, sample_1t):
    """The oracle, as it stands, on the first `sample` draws of the workload with the host's
    BLAS threads, and on the first `sample_1t` draws with one thread."""
    import numpy as np
    from oracle import accept, pipeline
    from threadpoolctl import threadpool_info, threadpool_limits

    def run(count):
        keys = np.arange(count, dtype=np.uint64)
        t0 = time.perf_counter()
        M = pipeline.balance_of_keys(X, w["n1"], w["ridge_rel"], w["seed"], keys,
                                     metric=w.get("metric", "mahalanobis"))
        accept.accept_quantile(keys, M, accept.quantile_count(w["q"], count))
        return count / (time.perf_counter() - t0), time.perf_counter() - t0

    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    rate, dt = run(sample)
    with threadpool_limits(1):
        rate1, dt1 = run(sample_1t)
    return {"value": rate, "unit": "draws/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {sample} draw keys of the workload: Philox draws, n1-of-n selection, "
                      f"FP64 textbook M, q-quantile acceptance over the sample ({dt:.1f} s; BLAS on {threads} "
                      f"threads, the oracle's NumPy element-wise steps on one)",
            "cpu_model": cpu_model(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "one_thread": {"value": rate1, "unit": "draws/s", "cores": 1,
                           "sample": f"first {sample_1t} draw keys ({dt1:.1f} s)"}}


def run_batched(args, rr, inputs, np, torch):
    """Batched pools: one graph launch over all pools vs one rr_draw_balance call per pool."""
    w = inputs.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    N, q = w["num_draws"], w["q"]
    if args.draws:
        N = args.draws
    t0 = time.perf_counter()
    Ps, seeds = [], []
    for p in range(w["num_problems"]):
        X, n1, seed = inputs.batched_problem(p, args.workload)
        Ps.append(rr.rr_prepare(torch.from_numpy(X).to(dev), n1, w["ridge_rel"]))
        seeds.append(seed)
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0
    shapes = inputs.batched_shapes(w["num_problems"], w["shape_seed"])
    flops = sum(4.0 * n * d for n, _, d in shapes) * N
    for _ in range(args.warmup):
        rr.rr_draw_balance_batched(Ps, seeds, 0, N, rr.MODE_QUANTILE, q, rr.PREC_SPLIT_BF16)
    torch.cuda.synchronize()
    graph_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = rr.rr_draw_balance_batched(Ps, seeds, 0, N, rr.MODE_QUANTILE, q, rr.PREC_SPLIT_BF16)
        graph_ms += rr.rr_last_timing()["contract_ms"]
    torch.cuda.synchronize()
    ms_per_step = 1000.0 * (time.perf_counter() - t0) / args.steps
    kernels = rr.rr_last_timing()["launches"]
    band_total = rr.rr_last_timing()["band"]
    i8 = None
    if not args.no_i8:
        rr.rr_draw_balance_batched(Ps, seeds, 0, N, rr.MODE_QUANTILE, q, rr.PREC_FIXED_I8)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            out8 = rr.rr_draw_balance_batched(Ps, seeds, 0, N, rr.MODE_QUANTILE, q, rr.PREC_FIXED_I8)
        torch.cuda.synchronize()
        ms8 = 1000.0 * (time.perf_counter() - t1) / args.steps
        same8 = all(bool(torch.equal(out8[i][0], out[i][0])) for i in range(len(Ps)))
        i8 = {"draws_per_s": w["num_problems"] * N / (ms8 / 1000.0), "ms_per_step": ms8,
              "graph_gpu_ms": rr.rr_last_timing()["contract_ms"], "same_accept_sets": same8,
              "speedup_vs_split": ms_per_step / ms8}
    # per-pool launch sequences, one pass
    t1 = time.perf_counter()
    same = True
    for i, P in enumerate(Ps):
        keys, M, _ = rr.rr_draw_balance(P, seeds[i], 0, N, rr.MODE_QUANTILE, q, rr.PREC_SPLIT_BF16)
        if i % 64 == 0:
            same = same and bool(torch.equal(keys, out[i][0])) and bool(torch.equal(M, out[i][1]))
    torch.cuda.synchronize()
    loop_ms = 1000.0 * (time.perf_counter() - t1)
    total = w["num_problems"] * N
    value = total / (ms_per_step / 1000.0)
    achieved = flops / (graph_ms / args.steps / 1000.0) / 1e12
    print(json.dumps({
        "metric": "batched pools: balance-checked draws/s (512 pools, n~U[50,2000], d~U[10,500])",
        "value": value, "unit": "draws/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": args.workload, "num_problems": w["num_problems"], "num_draws": N, "q": q,
                   "step": "rr_draw_balance_batched (one graph launch)"},
        "graph_gpu_ms_per_step": graph_ms / args.steps, "graph_kernels": kernels, "guard_band_total": band_total,
        "mfma_tflops_over_graph": achieved, "frac_bf16_peak_over_graph": achieved / PEAK_BF16_TFLOPS,
        "per_pool_calls": {"ms": loop_ms, "draws_per_s": total / (loop_ms / 1000.0),
                           "batched_speedup": loop_ms / ms_per_step, "same_results_sampled": same},
        "prepare_s_all_pools": prep_s, "i8_form": i8,
        "tuner_batched_classes": [e for e in rr.rr_tune_report()["rr_tune"] if e["batched"] == 1]}), flush=True)


def run_alone(args, rr, torch, w, Xd):
    """Generation and contraction without overlap: rr_balance_keys runs them one after the
    other on one stream (no FP64 values), so a kernel trace shows each kernel's time alone."""
    prec = {"split": rr.PREC_SPLIT_BF16, "fp32": rr.PREC_FP32, "i8": rr.PREC_FIXED_I8,
            "gram": rr.PREC_GRAM_BF16}[args.alone]
    metric_id = rr.METRIC_DIAGONAL if w.get("metric") == "diagonal" else rr.METRIC_MAHALANOBIS
    P = rr.rr_prepare(Xd, w["n1"], w["ridge_rel"], metric=metric_id)
    keys = torch.arange(1 << 20, dtype=torch.int64, device="cuda:0")
    for it in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rr.rr_balance_keys(P, w["seed"], keys, prec, want_m64=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(json.dumps({"alone": args.alone, "workload": args.workload, "keys": 1 << 20, "iteration": it,
                          "wall_ms": 1000.0 * dt}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="stream_n1000_d1000")
    ap.add_argument("--draws", type=int, default=None, help="override the draw count (not the benchmark)")
    ap.add_argument("--cpu-sample", type=int, default=200000)
    ap.add_argument("--cpu-sample-1t", type=int, default=20000, help="draws of the one-thread oracle run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-i8", action="store_true", help="skip the fixed-point int8 comparison leg")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (PMC byte-counter scale)")
    ap.add_argument("--alone", choices=["split", "fp32", "i8", "gram"], default=None,
                    help="instead of the benchmark: generation and contraction one after the other "
                         "(rr_balance_keys on 2^20 keys of the workload's pool, 3 times), for kernel traces")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this hot path runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding of the path is not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2501_07642_amd as rr
    from paper_2501_07642_amd import inputs

    if args.calibrate_copy_mb:
        src = torch.ones(args.calibrate_copy_mb << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = dict(inputs.WORKLOADS[args.workload])
    if w["kind"] == "batched":
        return run_batched(args, rr, inputs, np, torch)
    if args.draws:
        w["num_draws"] = args.draws
    n, n1, d, N, q = w["n"], w["n1"], w["d"], w["num_draws"], w["q"]
    dev = torch.device("cuda:0")
    X = inputs.workload_X(args.workload)
    Xd = torch.from_numpy(X).to(dev)
    taus = w["taus"]
    if args.alone:
        return run_alone(args, rr, torch, w, Xd)

    gram = w["precision"] == "gram_bf16"
    main_prec = rr.PREC_GRAM_BF16 if gram else rr.PREC_SPLIT_BF16
    metric_id = rr.METRIC_DIAGONAL if w.get("metric") == "diagonal" else rr.METRIC_MAHALANOBIS

    def step(Yd, obs, prec=main_prec):
        P = rr.rr_prepare(Xd, n1, w["ridge_rel"], metric=metric_id)
        keys, M, flags = rr.rr_draw_balance(P, w["seed"], w["key_begin"], N, rr.MODE_QUANTILE, q, prec)
        t = rr.rr_last_timing()
        counts = None
        if Yd is not None:
            counts, _ = rr.rr_rand_test(P, w["seed"], keys, obs, Yd, taus)
        return P, keys, t, counts

    # first pass builds the outcome vector from an accepted assignment (product output)
    P, keys, _, _ = step(None, 0)
    obs = inputs.obs_pick(len(keys), w["obs_seed"])
    bits = rr.rr_regenerate(P, w["seed"], keys[obs:obs + 1]).cpu().numpy().view(np.uint32)
    wo = ((bits[0][np.arange(n) // 32] >> (np.arange(n) % 32)) & 1).astype(np.float64)
    Yd = torch.from_numpy(inputs.outcomes(X, wo, w["tau"], w["noise_sd"], w["y_seed"])).to(dev)
    del P
    for _ in range(args.warmup):
        step(Yd, obs)
    torch.cuda.synchronize()
    contract_ms = 0.0
    gen_ms = 0.0
    launches = 0
    band = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P, keys_s, t, counts = step(Yd, obs)
        contract_ms += t["contract_ms"]
        gen_ms += t["gen_ms"]
        launches += t["launches"]
        band = t["band"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    value = N / (ms_per_step / 1000.0)
    keys_split = keys_s.cpu().numpy()
    # error of the FP32 balance values against FP64 on the accepted draws (outside the timed
    # region): both device paths on the same keys, with the rigorous bound of each draw
    m32, err32, m64 = rr.rr_balance_keys(P, w["seed"], keys_s, main_prec)
    m32n, errn, m64n = (x.cpu().numpy().astype(np.float64) for x in (m32, err32, m64))
    m_err = {"draws": int(len(m64n)), "max_rel_err": float(np.max(np.abs(m32n - m64n) / m64n)),
             "max_err_over_bound": float(np.max(np.abs(m32n - m64n) / errn)),
             "median_bound_rel": float(np.median(errn / m64n))} if len(m64n) else None

    # Algorithmic work of one balance check (the method, not the dense form): the treated sum
    # G = sum_{i in T} X~_i is n1 d additions, and ||G||^2 is d multiply-adds.  The dense form
    # issues the hi and lo products of W X~ over all n units (the Gram form: W K, K n x n).
    alg_flops_per_draw = float(n1 * d + 2 * d)
    issued_per_draw = 4.0 * n * (n if gram else d)
    launches_per_step = launches / args.steps
    avg_launch_ms = contract_ms / max(launches, 1)
    # full chunk length of this run's launches (a power of two; the last chunk of a pool is short)
    full_chunk = 1 << int(round(math.log2(N / max(launches_per_step, 1))))
    achieved = alg_flops_per_draw * N * args.steps / (contract_ms / 1000.0) / 1e12
    issued = issued_per_draw * N * args.steps / (contract_ms / 1000.0) / 1e12
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None if gram else measured_traffic(full_chunk),
                "kernel": ("contract_kernel<Gram BF16> (W K on 32x32x16 BF16 MFMA + w^T (W K) + prefilter)" if gram else
                           "contract_kernel<split BF16> (W X~ on 32x32x16 BF16 MFMA + reduce + prefilter)"),
                "avg_launch_ms": avg_launch_ms, "launches_per_step": launches_per_step,
                "draws_per_launch": N / max(launches_per_step, 1), "full_chunk_draws": full_chunk,
                "algorithmic_flops_per_draw": alg_flops_per_draw,
                "issued_mfma_flops_per_draw": issued_per_draw, "issued_mfma_tflops": issued,
                "issued_mfma_frac": issued / PEAK_BF16_TFLOPS,
                "gen_kernel_ms_per_step": gen_ms / args.steps}

    split = None
    if gram:
        # the same step with the W X~ split form
        step(Yd, obs, rr.PREC_SPLIT_BF16)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            _, keys_w, t, _ = step(Yd, obs, rr.PREC_SPLIT_BF16)
        torch.cuda.synchronize()
        msw = 1000.0 * (time.perf_counter() - t1) / args.steps
        split = {"draws_per_s": N / (msw / 1000.0), "ms_per_step": msw,
                 "same_accept_set": bool(np.array_equal(keys_w.cpu().numpy(), keys_split)),
                 "gram_speedup": msw / ms_per_step}

    fp32 = None
    if not args.no_fp32 and not gram:
        P = rr.rr_prepare(Xd, n1, w["ridge_rel"])
        # untimed first call of the FP32 bucket: the autotuner probes its candidates there
        rr.rr_draw_balance(P, w["seed"], w["key_begin"], min(N, 1 << 23), rr.MODE_QUANTILE, q, rr.PREC_FP32)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        keys32, _, _ = rr.rr_draw_balance(P, w["seed"], w["key_begin"], N, rr.MODE_QUANTILE, q, rr.PREC_FP32)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        t = rr.rr_last_timing()
        same = bool(np.array_equal(keys32.cpu().numpy(), keys_split))
        a32 = 2.0 * n * d * N / (t["contract_ms"] / 1000.0) / 1e12
        fp32 = {"draws_per_s": N / dt, "contract_kernel_ms": t["contract_ms"], "same_accept_set": same,
                "mfma_tflops": a32, "frac_fp32_peak": a32 / PEAK_FP32_TFLOPS,
                "split_speedup": (N / dt) and value / (N / dt)}

    i8 = None
    if not args.no_i8:
        # the same step with the fixed-point int8 operand form (exact int32 accumulation)
        step(Yd, obs, rr.PREC_FIXED_I8)
        torch.cuda.synchronize()
        c8 = g8 = 0.0
        t1 = time.perf_counter()
        for _ in range(args.steps):
            _, keys8, t, _ = step(Yd, obs, rr.PREC_FIXED_I8)
            c8 += t["contract_ms"]
            g8 += t["gen_ms"]
        torch.cuda.synchronize()
        ms8 = 1000.0 * (time.perf_counter() - t1) / args.steps
        a8 = issued_per_draw * N * args.steps / (c8 / 1000.0) / 1e12
        g8_alg = alg_flops_per_draw * N * args.steps / (c8 / 1000.0) / 1e12
        i8 = {"draws_per_s": N / (ms8 / 1000.0), "ms_per_step": ms8, "contract_kernel_ms_per_step": c8 / args.steps,
              "gen_kernel_ms_per_step": g8 / args.steps,
              "same_accept_set": bool(np.array_equal(keys8.cpu().numpy(), keys_split)),
              "algorithmic_tops": g8_alg, "algorithmic_frac_int8_peak": g8_alg / PEAK_INT8_TOPS,
              "issued_mfma_tops": a8, "issued_frac_int8_peak": a8 / PEAK_INT8_TOPS, "guard_band": t["band"],
              "speedup_vs_split": ms_per_step / ms8,
              "kernel": "contract_kernel<fixed I8> (x = s (128 hi + lo), 32x32x32 int8 MFMA, exact int32)",
              "algorithmic_ops_per_draw": alg_flops_per_draw, "issued_ops_per_draw": issued_per_draw}

    base = None
    if not args.no_cpu_baseline:
        base = cpu_baseline(X, w, args.cpu_sample, args.cpu_sample_1t)

    out = {
        "metric": METRIC_GRAM if gram else METRIC, "value": value, "unit": "draws/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "n1": n1, "d": d, "num_draws": N, "q": q,
                   "accepted": int(len(keys_split)), "ridge_rel": w["ridge_rel"], "precision": w["precision"],
                   "metric": w.get("metric", "mahalanobis"),
                   "step": "rr_prepare + rr_draw_balance + rr_rand_test(201 nulls)"},
        "roofline": roofline, "cpu_baseline": base, "fp32_form": fp32, "i8_form": i8, "split_form": split,
        "contract_kernel_ms_per_step": contract_ms / args.steps, "guard_band": band, "m32_vs_fp64": m_err,
        "rand_test_counts_min": int(counts.min().item()) if counts is not None else None,
        "tuner": [e for e in rr.rr_tune_report()["rr_tune"] if e["batched"] == 0],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
