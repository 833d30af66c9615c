#!/usr/bin/env python3
"""Writes a golden fixture: the oracle's accepted draws of a large Monte Carlo pool.

The pools of the streaming workloads (up to 1e8 draws at n = d = 1000) take the oracle an
hour or more on a host's cores, too long for a test, so their accepted sets are computed
once here and stored under tests/golden/.  This script calls only the oracle (and the seeded
input generator, which holds no method arithmetic): every stored key and M comes from
``oracle.pipeline.balance_of_keys`` followed by ``oracle.accept`` -- the oracle's
``draw_balance`` over the whole key range, evaluated in slabs of draws (batching does not
change any result: each draw's M depends only on its key).

Usage:
    python tests/golden/make_pool_fixture.py WORKLOAD --scratch DIR [--procs P] [--slab S]

Per-slab M arrays go to DIR (reused when present, so an interrupted run resumes); the fixture
is written to tests/golden/pool_<WORKLOAD>.json.  For the batched workload the fixture holds
the accepted sets of a sample of its pools (--pools, chosen by a fixed seed together with the
pools of the smallest and largest n and d and a pool with d >= n - 1), one process per pool.
"""

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import accept, pipeline  # noqa: E402
from paper_2501_07642_amd import inputs  # noqa: E402


def _slab(job):
    name, start, stop, path = job
    if os.path.exists(path):
        return start, 0.0
    from threadpoolctl import threadpool_limits
    w = inputs.WORKLOADS[name]
    X = inputs.workload_X(name)
    keys = np.arange(w["key_begin"] + start, w["key_begin"] + stop, dtype=np.uint64)
    t0 = time.perf_counter()
    with threadpool_limits(1):
        M = pipeline.balance_of_keys(X, w["n1"], w["ridge_rel"], w["seed"], keys,
                                     metric=w.get("metric", "mahalanobis"))
    np.save(path + ".tmp.npy", M)
    os.replace(path + ".tmp.npy", path)
    return start, time.perf_counter() - t0


def _batched_pool(job):
    name, p = job
    from threadpoolctl import threadpool_limits
    w = inputs.WORKLOADS[name]
    X, n1, seed = inputs.batched_problem(p, name)
    N = w["num_draws"]
    keys = np.arange(w["key_begin"], w["key_begin"] + N, dtype=np.uint64)
    t0 = time.perf_counter()
    with threadpool_limits(1):
        M = pipeline.balance_of_keys(X, n1, w["ridge_rel"], seed, keys)
    k = accept.quantile_count(w["q"], N)
    acc = accept.accept_quantile(keys, M, k)
    Macc = M[(acc - np.uint64(w["key_begin"])).astype(np.int64)]
    return dict(pool=p, n=int(X.shape[0]), n1=int(n1), d=int(X.shape[1]), seed=int(seed), k=k,
                keys=[int(x) for x in acc], M=[float(x) for x in Macc]), time.perf_counter() - t0


def batched_main(args):
    w = inputs.WORKLOADS[args.workload]
    shapes = inputs.batched_shapes(w["num_problems"], w["shape_seed"])
    rng = np.random.default_rng(2501)
    pick = set(rng.choice(w["num_problems"], size=max(args.pools - 5, 0), replace=False).tolist())
    ns = [s[0] for s in shapes]
    ds = [s[2] for s in shapes]
    pick |= {int(np.argmin(ns)), int(np.argmax(ns)), int(np.argmin(ds)), int(np.argmax(ds))}
    degenerate = [p for p, (n, _, d) in enumerate(shapes) if d >= n - 1]
    if degenerate:
        pick.add(degenerate[0])
    pools = sorted(pick)
    t0 = time.perf_counter()
    out_pools, busy = [], 0.0
    with mp.get_context("fork").Pool(args.procs) as pool:
        for i, (rec, dt) in enumerate(pool.imap_unordered(_batched_pool, [(args.workload, p) for p in pools])):
            out_pools.append(rec)
            busy += dt
            print(f"{i + 1}/{len(pools)} pools, {time.perf_counter() - t0:.0f} s", flush=True)
    out_pools.sort(key=lambda r: r["pool"])
    out = {
        "cite": "accepted draws of Monte Carlo pools: key-only storage (section 2.1), acceptance at "
                "probability q as the k = ceil(q N) smallest M (section 2.2), M on the chi^2_d scale; "
                "several experiments batched (section 2.1)",
        "written_by": "tests/golden/make_pool_fixture.py (oracle only)",
        "command": f"python tests/golden/make_pool_fixture.py {args.workload} --scratch DIR --procs {args.procs} "
                   f"--pools {args.pools}",
        "workload": args.workload, "num_problems": w["num_problems"], "num_draws": w["num_draws"],
        "key_begin": w["key_begin"], "q": w["q"], "ridge_rel": w["ridge_rel"],
        "oracle_seconds": busy, "pools": out_pools,
    }
    path = os.path.join(ROOT, "tests", "golden", f"pool_{args.workload}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print(f"wrote {path}: {len(out_pools)} pools, {busy:.0f} s of oracle time", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--scratch", required=True, help="directory for per-slab M arrays")
    ap.add_argument("--procs", type=int, default=max(1, (os.cpu_count() or 2) - 2))
    ap.add_argument("--slab", type=int, default=200_000)
    ap.add_argument("--pools", type=int, default=32, help="batched workload: pools in the fixture")
    args = ap.parse_args()
    w = inputs.WORKLOADS[args.workload]
    if w["kind"] == "batched":
        return batched_main(args)
    if w["kind"] != "mc" or w["mode"] != "quantile":
        raise SystemExit("only Monte Carlo pools with q-quantile acceptance")
    N = w["num_draws"]
    os.makedirs(args.scratch, exist_ok=True)
    jobs = [(args.workload, s, min(s + args.slab, N), os.path.join(args.scratch, f"M_{s:012d}.npy"))
            for s in range(0, N, args.slab)]
    t0 = time.perf_counter()
    busy = 0.0
    with mp.get_context("fork").Pool(args.procs) as pool:
        for i, (start, dt) in enumerate(pool.imap_unordered(_slab, jobs)):
            busy += dt
            if (i + 1) % 10 == 0 or i + 1 == len(jobs):
                print(f"{i + 1}/{len(jobs)} slabs, {time.perf_counter() - t0:.0f} s", flush=True)
    M = np.concatenate([np.load(j[3]) for j in jobs])
    keys = np.arange(w["key_begin"], w["key_begin"] + N, dtype=np.uint64)
    k = accept.quantile_count(w["q"], N)
    acc = accept.accept_quantile(keys, M, k)
    Macc = M[(acc - np.uint64(w["key_begin"])).astype(np.int64)]
    t = float(np.sort(M)[k - 1])
    out = {
        "cite": "accepted draws of a Monte Carlo pool: key-only storage (section 2.1), acceptance at "
                "probability q as the k = ceil(q N) smallest M (section 2.2), M on the chi^2_d scale",
        "written_by": "tests/golden/make_pool_fixture.py (oracle only)",
        "command": f"python tests/golden/make_pool_fixture.py {args.workload} --scratch DIR "
                   f"--procs {args.procs} --slab {args.slab}",
        "workload": args.workload, "n": w["n"], "n1": w["n1"], "d": w["d"], "seed": w["seed"],
        "key_begin": w["key_begin"], "num_draws": N, "q": w["q"], "k": k, "ridge_rel": w["ridge_rel"],
        "metric": w.get("metric", "mahalanobis"), "kth_M": t,
        "near_kth": int(np.sum(np.abs(M - t) <= accept.EPS_TIE * t)),
        "oracle_seconds": busy, "oracle_processes": args.procs,
        "keys": [int(x) for x in acc], "M": [float(x) for x in Macc],
    }
    path = os.path.join(ROOT, "tests", "golden", f"pool_{args.workload}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print(f"wrote {path}: {len(acc)} keys, k-th M {t!r}, {busy:.0f} s of oracle time", flush=True)


if __name__ == "__main__":
    main()
