#!/usr/bin/env python3
"""Benchmark of the per-GPU relational hot path on one MI355X.

Step = one fused star query over HBM-resident synthetic tables of the measured
shape (build 1.5M rows {key, segment}, probe 60M rows {fk, date, price}):
filter segment == 1 and date < 1200, join fk = key, GROUP BY key SUM(price),
i.e. dimension filter + hash build + one fused probe/aggregate pass over the
fact columns + group compaction.  value = probe rows per second.

Beside the headline line it reports, measured outside the timed region:
  roofline      : the fused probe kernel's algorithmic bytes / its mean HIP-event
                  duration against the 8 TB/s HBM peak (+ counter traffic when
                  a committed counter profile matches the current kernel source)
  cpu_baseline  : the CPU oracle (single thread) on a bounded sample
  partition     : hash partition of the probe table, fanout 2 / 8 / 64
  chain         : the two-join chain query (fact 120M, Zipf s = 0 and 1)
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROBE_ROW_BYTES = 16   # fk int32 + date int32 + price int64
BUILD_ROW_BYTES = 8    # key int32 + segment int32
GROUP_OUT_BYTES = 16   # key int64 + sum int64


def source_hash():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2512_02862_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def counter_traffic(kernel, workload):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it is current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel + "|" + workload)
    except ValueError:
        return None
    if not rec or rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def to_dev(d):
    import torch
    return {k: torch.from_numpy(v).cuda() for k, v in d.items()}


def timed_loop(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--build-rows", type=int, default=1_500_000)
    ap.add_argument("--probe-rows", type=int, default=60_000_000)
    ap.add_argument("--max-load", type=float, default=0.5)
    ap.add_argument("--no-extras", action="store_true", help="skip the partition and chain measurements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=30_000_000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the shuffle stops at the "
              "partitioned per-destination buffers); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    from paper_2512_02862_amd import pyst

    def log(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    nb, npr = args.build_rows, args.probe_rows
    log("generating star tables: build %d, probe %d" % (nb, npr))
    b_host, p_host = gen.star_tables(nb, npr, workload=1)
    b = to_dev(b_host)
    p = to_dev(p_host)
    fact = [p["fk"], p["date"], p["price"]]
    ctx = pyst.Ctx(0, 8 << 30)
    plan = pyst.star_plan(b, max_load=args.max_load)
    out_cap = nb
    keys = torch.empty(out_cap, dtype=torch.int64, device="cuda")

    def step():
        pyst.query(ctx, plan, fact, out_cap=out_cap)

    log("warmup %d, timed %d steps" % (args.warmup, args.steps))
    for _ in range(args.warmup):
        step()
    ctx.check()
    ctx.timing(True)
    elapsed = timed_loop(step, args.steps, 0)
    ctx.timing(False)
    fact_ms, launches = ctx.kernel_time("fact_pass")
    ctx.check()
    k, s, ng = pyst.query(ctx, plan, fact, out_cap=out_cap)
    ctx.check()
    n_groups = int(ng.item())
    del keys

    ms_per_step = elapsed / args.steps * 1e3
    rows_per_s = args.steps * npr / elapsed
    fact_mean_s = fact_ms / max(launches, 1) / 1e3
    fact_bytes = npr * PROBE_ROW_BYTES
    achieved = fact_bytes / fact_mean_s / 1e9
    query_bytes = npr * PROBE_ROW_BYTES + nb * BUILD_ROW_BYTES + n_groups * GROUP_OUT_BYTES
    workload = "star_b%d_p%d" % (nb, npr)
    traffic = counter_traffic("k_fact_pass", workload)

    result = {
        "metric": "probe rows/s and % HBM peak for filter+join+agg; batched p50/p99 latency",
        "value": rows_per_s,
        "unit": "probe rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic (seeded splitmix64 tables of the measured shape; no dataset)",
        "config": {
            "workload": "star query, build %d rows {key, segment}, probe %d rows {fk, date, price}: "
                        "segment == 1, date < 1200, join fk = key, GROUP BY key SUM(price)" % (nb, npr),
            "build_rows": nb, "probe_rows": npr, "max_load": args.max_load, "groups": n_groups,
            "parallelism": "single GPU",
        },
        "query_hbm": {"algorithmic_bytes": query_bytes, "gbs": query_bytes / (ms_per_step / 1e3) / 1e9,
                      "frac_of_peak": query_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS},
        "roofline": {
            "kernel": "k_fact_pass (fused filter + probe + SUM)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": fact_bytes, "mean_launch_us": fact_mean_s * 1e6,
            "launches": launches,
        },
    }

    if not args.no_extras:
        result["partition"] = bench_partition(ctx, pyst, p, npr, log)
        del b, p, fact
        torch.cuda.empty_cache()
        result["chain"] = bench_chain(ctx, pyst, gen, log)

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(b_host, p_host, args.cpu_sample_rows, log)

    ctx.close()
    print(json.dumps(result), flush=True)


def bench_partition(ctx, pyst, p, npr, log):
    import torch
    out = {}
    for fanout in (2, 8, 64):
        log("partition fanout %d" % fanout)

        def step():
            pyst.partition(ctx, p["fk"], [p["date"], p["price"]], fanout)

        for _ in range(2):
            step()
        ctx.check()
        ctx.timing(True)
        el = timed_loop(step, 10, 0)
        ctx.timing(False)
        sc_ms, sc_n = ctx.kernel_time("part_scatter")
        ctx.kernel_time("partition")
        ctx.check()
        alg = npr * 32  # read 16 B + write 16 B per row
        ms = el / 10 * 1e3
        out["F%d" % fanout] = {"ms": ms, "rows_per_s": npr / (ms / 1e3), "gbs": alg / (ms / 1e3) / 1e9,
                              "frac_of_peak": alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                              "scatter_kernel_us": sc_ms / max(sc_n, 1) * 1e3}
        torch.cuda.empty_cache()
    return out


def bench_chain(ctx, pyst, gen, log):
    import torch
    na, nbd, nf = 3_000_000, 300_000, 120_000_000
    out = {}
    a_h, b_h = gen.chain_dims(na, nbd)
    a, b = to_dev(a_h), to_dev(b_h)
    for zs in (0.0, 1.0):
        log("chain query, fact %d, zipf s=%g" % (nf, zs))
        f_h = gen.chain_fact(nf, na, nbd, zs)
        f = to_dev(f_h)
        del f_h
        fact = [f[c] for c in ("a_fk", "b_fk", "date", "price", "discount")]
        plan = pyst.chain_plan(a, b)
        cap = 16_000_000

        def step():
            pyst.query(ctx, plan, fact, out_cap=cap)

        step()
        ctx.check()
        ctx.timing(True)
        el = timed_loop(step, 5, 0)
        ctx.timing(False)
        fms, fn = ctx.kernel_time("fact_pass")
        k, s, ng = pyst.query(ctx, plan, fact, out_cap=cap)
        ctx.check()
        groups = int(ng.item())
        alg = nf * 24 + na * 8 + nbd * 8 + groups * 16
        ms = el / 5 * 1e3
        out["s%g" % zs] = {"ms": ms, "fact_rows_per_s": nf / (ms / 1e3), "groups": groups,
                           "algorithmic_bytes": alg, "gbs": alg / (ms / 1e3) / 1e9,
                           "frac_of_peak": alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                           "fact_pass_us": fms / max(fn, 1) * 1e3}
        del f, fact, k, s
        torch.cuda.empty_cache()
    return out


def cpu_baseline(b_host, p_host, sample_rows, log):
    import oracle
    sample_rows = min(sample_rows, len(p_host["fk"]))
    sample = {c: v[:sample_rows] for c, v in p_host.items()}
    log("cpu oracle on %d probe rows" % sample_rows)
    t0 = time.perf_counter()
    oracle.star_query(b_host, sample)
    dt = time.perf_counter() - t0
    return {"value": sample_rows / dt, "unit": "probe rows/s", "cores": 1, "kind": "oracle",
            "sample": "full build table (%d rows), first %d probe rows; %.1f s single-threaded"
                      % (len(b_host["key"]), sample_rows, dt)}


if __name__ == "__main__":
    main()
