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
  cpu_baseline  : the CPU oracle (single thread) on a bounded sample, and the
                  threaded CPU baseline over every usable host core
  partition     : hash partition of the probe table, fanout 2 / 8 / 64
  chain         : the two-join chain query (fact 120M, Zipf s = 0 and 1)
  groupby       : GROUP BY orderkey SUM(quantity) over 60M lineitem-like rows
                  (about 14.7M groups), radix-partitioned path vs HBM hash table
  join          : the materializing join of the join microbenchmark at one GPU's
                  share (build 60M / probe 160M, hit ratio 0.5, k = 1, 4, 8
                  8-byte columns a side)
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


KERNEL_SOURCES = {  # the files that define each profiled kernel (name patterns as rocprofv3 prints them)
    "k_fast_fact": ["fast.hip", "pyst_internal.h", "table.h", "query.h"],
    "k_fast_fact<2, 8, 2": ["fast.hip", "pyst_internal.h", "table.h", "query.h"],
    "k_join_probe": ["ops.hip", "pyst_internal.h", "table.h"],
    "k_join_build": ["ops.hip", "pyst_internal.h", "table.h"],
    "k_gather_rows<4": ["ops.hip", "pyst_internal.h"],
    "k_gather<": ["ops.hip", "pyst_internal.h"],
}
CHAIN_WORKLOAD = "chain_a3000000_b300000_f120000000"  # fact-pass counters averaged over s = 0 and 1
JOIN_WORKLOAD = "join_b60000000_p160000000_k4"  # counters of the k = 4 materializing join


def source_hash(kernel="k_fast_fact"):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2512_02862_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _db_rows(db, sql):
    import sqlite3
    return list(sqlite3.connect(db).execute(sql))


def summarize(args):
    """Turn rocprofv3 result databases into the text summaries and traffic.json kept in profiles/.

    --summarize trace DB OUT.txt CMD...          kernel-trace statistics (top kernels)
    --summarize pmc FETCH_DB WRITE_DB COPY_FETCH_DB COPY_WRITE_DB KERNEL WORKLOAD CMD...
        per-dispatch FETCH_SIZE / WRITE_SIZE of KERNEL, scaled by the same counters of a plain
        1 GiB copy (bench.py --calibrate-copy), into profiles/traffic.json and a text summary.
    """
    kind, rest = args[0], args[1:]
    prof = os.path.join(ROOT, "profiles")
    if kind == "trace":
        db, out, cmd = rest[0], rest[1], " ".join(rest[2:])
        rows = _db_rows(db, "select name, total_calls, total_duration, average, percentage from top_kernels")
        with open(os.path.join(prof, out), "w") as fh:
            fh.write("# rocprofv3 --kernel-trace --stats\n# command: %s\n" % cmd)
            fh.write("%-90s %6s %14s %12s %7s\n" % ("kernel", "calls", "total_us", "avg_us", "pct"))
            for r in rows:
                fh.write("%-90s %6d %14.1f %12.2f %7.2f\n" % (r[0][:90], r[1], r[2], r[3], r[4]))
        return
    fdb, wdb, cfdb, cwdb, kernel, workload = rest[:6]
    cmd = " ".join(rest[6:])

    def avg(db, counter, like):
        r = _db_rows(db, "select avg(value), count(*) from counters_collection where counter_name='%s' "
                         "and kernel_name like '%%%s%%'" % (counter, like))
        return r[0]

    fetch, nf = avg(fdb, "FETCH_SIZE", kernel)
    write, nw = avg(wdb, "WRITE_SIZE", kernel)
    copy_bytes = 1 << 30
    cfetch, _ = avg(cfdb, "FETCH_SIZE", "copyBuffer")
    cwrite, _ = avg(cwdb, "WRITE_SIZE", "copyBuffer")
    ffac, wfac = copy_bytes / 1024 / cfetch, copy_bytes / 1024 / cwrite
    traffic = fetch * ffac * 1024 + write * wfac * 1024
    path = os.path.join(prof, "traffic.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    rec[kernel + "|" + workload] = {
        "bytes_per_launch": traffic, "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write,
        "fetch_scale": ffac, "write_scale": wfac, "dispatches": [nf, nw], "source_hash": source_hash(kernel),
        "command": cmd}
    json.dump(rec, open(path, "w"), indent=1, sort_keys=True)
    fname = "".join(ch if ch.isalnum() else "_" for ch in kernel).strip("_")
    fname = "_".join(x for x in fname.split("_") if x)  # k_fast_fact<2, 8, 2 -> k_fast_fact_2_8_2
    with open(os.path.join(prof, "%s_%s_traffic.txt" % (fname, workload)), "w") as fh:
        fh.write("# HBM traffic of %s on %s from rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE\n" % (kernel, workload))
        fh.write("# command: %s\n" % cmd)
        fh.write("FETCH_SIZE KiB/dispatch %.1f (x%.3f from a 1 GiB copy reading %.1f KiB)\n" % (fetch, ffac, cfetch))
        fh.write("WRITE_SIZE KiB/dispatch %.1f (x%.3f from a 1 GiB copy writing %.1f KiB)\n" % (write, wfac, cwrite))
        fh.write("HBM bytes per launch %.4g\n" % traffic)


def counter_traffic(kernel, workload):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it is current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel + "|" + workload)
    except ValueError:
        return None
    if not rec or rec.get("source_hash") != source_hash(kernel):
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
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize":
        summarize(sys.argv[2:])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--build-rows", type=int, default=1_500_000)
    ap.add_argument("--probe-rows", type=int, default=60_000_000)
    ap.add_argument("--max-load", type=float, default=0.5)
    ap.add_argument("--no-extras", action="store_true", help="skip every measurement beside the headline")
    ap.add_argument("--extras", default="partition,chain,groupby,join,stream,batch,serve",
                    help="comma-separated extra measurements to run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=30_000_000)
    ap.add_argument("--stream-rows", type=int, default=240_000_000, help="chain fact rows streamed from pinned host")
    ap.add_argument("--join-k", default="1,4,8", help="8-byte columns a side of the join microbenchmark")
    ap.add_argument("--batch-fragments", type=int, default=512)
    ap.add_argument("--batch-max-rows", type=float, default=2e7, help="largest fragment probe size")
    ap.add_argument("--serve-rows", type=int, default=512_000_000, help="pinned host fact rows of the server")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 4, "launches": 5}))
        return
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
    ctx = pyst.Ctx(0, 16 << 30)
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
    traffic = counter_traffic("k_fast_fact", workload)

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
            "kernel": "k_fast_fact (fused filter + probe + SUM)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": fact_bytes, "mean_launch_us": fact_mean_s * 1e6,
            "launches": launches,
        },
    }

    extras = [] if args.no_extras else args.extras.split(",")
    def extra(name, fn, *a):
        # an extra that fails is recorded with its error; the headline line is still printed
        if name not in extras:
            return
        try:
            result[name] = fn(*a)
        except Exception as e:  # noqa: BLE001
            log("extra %s failed: %r" % (name, e))
            result[name] = {"error": repr(e)}
        torch.cuda.empty_cache()

    extra("partition", bench_partition, ctx, pyst, p, npr, log)
    del b, p, fact
    torch.cuda.empty_cache()
    extra("chain", bench_chain, ctx, pyst, gen, log)
    extra("groupby", bench_groupby, ctx, pyst, gen, log)
    extra("join", bench_join, ctx, pyst, gen, log, 60_000_000, 160_000_000, [int(x) for x in args.join_k.split(",")])
    extra("stream", bench_stream, ctx, pyst, gen, log, args.stream_rows)
    extra("batch", bench_batch, ctx, pyst, gen, log, args.batch_fragments, args.batch_max_rows)
    extra("serve", bench_serve, pyst, gen, log, args.serve_rows, args.serve_requests)

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
    # HBM bytes per launch of the chain's fact pass from committed counters (null
    # when the kernel's source has changed since they were taken)
    out["fact_pass_traffic"] = counter_traffic("k_fast_fact<2, 8, 2", CHAIN_WORKLOAD)
    out["fact_pass_algorithmic_bytes"] = nf * 24
    return out


def bench_groupby(ctx, pyst, gen, log, n=60_000_000, n_orders=15_000_000):
    """GROUP BY orderkey SUM(quantity), groups far beyond the caches: both group-by paths."""
    import torch
    li = gen.q18_lineitem(n, n_orders)
    k, v = torch.from_numpy(li["orderkey"]).cuda(), torch.from_numpy(li["quantity"]).cuda()
    del li
    out = {"rows": n, "key_range": n_orders}
    for path, hash_only in (("radix", False), ("hash", True)):
        log("group-by %d rows, path %s" % (n, path))
        ctx.groupby_hash_only(hash_only)

        def step():
            return pyst.groupby_sum(ctx, k, v, max_groups=n_orders)

        r = step()
        ctx.check()
        groups = int(r[2].item())
        del r
        ctx.timing(True)
        el = timed_loop(step, 5, 0)
        ctx.timing(False)
        g_ms, g_n = ctx.kernel_time("groupby_" + path)
        ctx.check()
        ms = el / 5 * 1e3
        alg = n * 8 + groups * 16  # key and value read once, each group written once
        out[path] = {"ms": ms, "rows_per_s": n / (ms / 1e3), "groups": groups, "algorithmic_bytes": alg,
                     "gbs": alg / (ms / 1e3) / 1e9, "frac_of_peak": alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "region_us": g_ms / max(g_n, 1) * 1e3}
    ctx.groupby_hash_only(False)
    out["radix_speedup"] = out["hash"]["ms"] / out["radix"]["ms"]
    return out


def bench_join(ctx, pyst, gen, log, nb=60_000_000, npr=160_000_000, ks=(1, 4, 8)):
    """Build + probe + materialize of k 8-byte columns per side (one pyst_join_materialize call)."""
    import torch
    out = {"build_rows": nb, "probe_rows": npr, "hit_ratio": 0.5}
    for k in ks:
        log("join microbenchmark: build %d, probe %d, k = %d" % (nb, npr, k))
        b_h, p_h = gen.join_tables(nb, npr, k)
        bk, pk = torch.from_numpy(b_h["key"]).cuda(), torch.from_numpy(p_h["key"]).cuda()
        bc = [torch.from_numpy(b_h["c%d" % c]).cuda() for c in range(k)]
        pc = [torch.from_numpy(p_h["c%d" % c]).cuda() for c in range(k)]
        del b_h, p_h

        def step():
            return pyst.join_materialize(ctx, bk, bc, pk, pc)

        r = step()
        ctx.check()
        m = int(r[3].item())
        del r
        ctx.timing(True)
        el = timed_loop(step, 5, 0)
        ctx.timing(False)
        b_ms, b_n = ctx.kernel_time("join_build")
        p_ms, p_n = ctx.kernel_time("join_probe")
        g_ms, g_n = ctx.kernel_time("gather")
        r_ms, r_n = ctx.kernel_time("gather_rows")
        k_ms, k_n = ctx.kernel_time("pack_rows")
        ctx.check()
        ms = el / 5 * 1e3
        cap = 1 << (int(nb / 0.5)).bit_length()
        # algorithmic bytes: keys read once, one table slot written per build row and
        # read per probe row, the table cleared, (probe row, build row) pairs written
        # and read back, k values read and written per match and side
        gather_bytes = m * (4 + 16 * k)  # per gather launch
        alg = nb * (4 + 8) + cap * 8 + npr * (4 + 8) + m * 8 + 2 * gather_bytes
        g_us = g_ms / max(g_n, 1) * 1e3
        out["k%d" % k] = {
            "ms": ms, "matches": m, "probe_rows_per_s": npr / (ms / 1e3), "output_tuples_per_s": m / (ms / 1e3),
            "algorithmic_bytes": alg, "gbs": alg / (ms / 1e3) / 1e9,
            "frac_of_peak": alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
            "build_us": b_ms / max(b_n, 1) * 1e3, "probe_us": p_ms / max(p_n, 1) * 1e3,
            # column gathers: the probe side (and the build side at k = 1); packed-row
            # gathers: the build side at k > 1, after packing its columns row-major
            "gather_us": g_us, "gather_gbs": gather_bytes / (g_us / 1e6) / 1e9 if g_us > 0 else None,
            "gather_rows_us": r_ms / r_n * 1e3 if r_n else None, "pack_rows_us": k_ms / k_n * 1e3 if k_n else None}
        del bk, pk, bc, pc
        torch.cuda.empty_cache()
    # HBM bytes per launch from committed counters of the k = 4 run (null once the kernels changed)
    out["k4_counter_traffic"] = {"k_join_probe": counter_traffic("k_join_probe", JOIN_WORKLOAD),
                                 "k_gather_rows": counter_traffic("k_gather_rows<4", JOIN_WORKLOAD),
                                 "k_gather": counter_traffic("k_gather<", JOIN_WORKLOAD)}
    return out


def pinned_empty(n, dtype):
    import torch
    return torch.empty(n, dtype=dtype, pin_memory=True)


def chain_fact_pinned(gen, n, na, nb, zs):
    """Chain fact columns generated straight into pinned host tensors."""
    import torch
    cols = {"a_fk": torch.int32, "b_fk": torch.int32, "date": torch.int32, "price": torch.int64,
            "discount": torch.int32}
    t = {c: pinned_empty(n, d) for c, d in cols.items()}
    gen.chain_fact(n, na, nb, zs, out={c: v.numpy() for c, v in t.items()})
    return [t[c] for c in ("a_fk", "b_fk", "date", "price", "discount")]


def h2d_peak(host_t, log):
    """Plain pinned host-to-device copy rate of a large buffer (GB/s)."""
    import torch
    d = torch.empty(host_t.numel(), dtype=host_t.dtype, device="cuda")
    d.copy_(host_t, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        d.copy_(host_t, non_blocking=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    gbs = host_t.numel() * host_t.element_size() / dt / 1e9
    log("pinned H2D copy: %.1f GB/s" % gbs)
    return gbs


def bench_stream(ctx, pyst, gen, log, nrows):
    """Chain query over a pinned host fact table streamed in 64M-row chunks, double-buffered."""
    import torch
    na, nbd = 3_000_000, 300_000
    a_h, b_h = gen.chain_dims(na, nbd)
    a, b = to_dev(a_h), to_dev(b_h)
    log("stream: generating %d pinned fact rows" % nrows)
    host = chain_fact_pinned(gen, nrows, na, nbd, 0.0)
    peak = h2d_peak(host[3], log)
    plan = pyst.chain_plan(a, b, max_groups=min(nrows // 8, 150_000_000))
    chunk = 64_000_000
    out = {}
    for nbuf in (2, 3):
        ctx.timing(True)
        t0 = time.perf_counter()
        k, s, ng = pyst.query_streamed(ctx, plan, host, chunk_rows=chunk, nbuf=nbuf, out_cap=plan.max_groups)
        ctx.check()
        dt = time.perf_counter() - t0
        ctx.timing(False)
        copy_ms, copies = ctx.kernel_time("h2d_chunk")
        fact_ms, _ = ctx.kernel_time("fact_pass")
        gbs = nrows * 24 / dt / 1e9
        out["nbuf%d" % nbuf] = {"seconds": dt, "fact_rows_per_s": nrows / dt, "h2d_gbs": gbs,
                                "frac_of_pinned_h2d": gbs / peak, "copy_busy_ms": copy_ms,
                                "compute_busy_ms": fact_ms, "chunks": copies, "groups": int(ng.item())}
        del k, s
    # the same columns bit-packed on the host: the link carries the packed bytes
    log("stream: packing %d rows" % nrows)
    t0 = time.perf_counter()
    packed = [(*pyst.pack(t), nrows, t.dtype) for t in host]
    pack_s = time.perf_counter() - t0
    packed_bytes = sum(bl.numel() * 8 + w.numel() * 4 for bl, w, _, _ in packed)
    for nbuf in (2, 3):
        ctx.timing(True)
        t0 = time.perf_counter()
        k, s, ng = pyst.query_streamed_packed(ctx, plan, packed, chunk_rows=chunk, nbuf=nbuf,
                                              out_cap=plan.max_groups)
        ctx.check()
        dt = time.perf_counter() - t0
        ctx.timing(False)
        copy_ms, copies = ctx.kernel_time("h2d_chunk")
        unpack_ms, unpacks = ctx.kernel_time("unpack")
        fact_ms, _ = ctx.kernel_time("fact_pass")
        out["packed_nbuf%d" % nbuf] = {
            "seconds": dt, "fact_rows_per_s": nrows / dt, "link_gbs": packed_bytes / dt / 1e9,
            "frac_of_pinned_h2d": packed_bytes / dt / 1e9 / peak, "copy_busy_ms": copy_ms,
            "unpack_busy_ms": unpack_ms, "compute_busy_ms": fact_ms, "groups": int(ng.item()),
            "speedup_vs_raw": out["nbuf%d" % nbuf]["seconds"] / dt}
        del k, s
    out["packed"] = {"bytes": packed_bytes, "bytes_per_row": packed_bytes / nrows,
                     "ratio": nrows * 24 / packed_bytes, "host_encode_s": pack_s}
    out.update({"rows": nrows, "chunk_rows": chunk, "pinned_h2d_peak_gbs": peak,
                "workload": "chain query, fact %d rows (24 B/row) in pinned host memory" % nrows})
    del host, packed
    return out


def bench_batch(ctx, pyst, gen, log, nfrag, max_rows):
    """512 star fragments in one batch vs one at a time (each read back, as a sizing caller must)."""
    import torch
    sizes, builds = gen.fragment_sizes(nfrag, hi=max_rows)
    log("batch: generating %d fragments, %d probe rows" % (nfrag, int(sizes.sum())))
    frags = []
    for f, (p, b) in enumerate(zip(sizes, builds)):
        bt, pt = gen.star_tables(max(int(b), 1), int(p), workload=3, fragment=f)
        bd = to_dev(bt)
        frags.append((pyst.star_plan(bd), [torch.from_numpy(pt[c]).cuda() for c in ("fk", "date", "price")]))
    batch = pyst.Batch(ctx, frags)
    best, best_ms = batch.autotune(reps=2)
    log("autotune best %s: %.3f ms" % (best, best_ms))
    batch.run(best)
    ctx.check()
    el = timed_loop(lambda: batch.run(best), 5, 0)
    batched_s = el / 5
    # the same batch captured once as a HIP graph and replayed
    graph = batch.graph(best)
    graph.launch()
    ctx.check()
    graph_s = timed_loop(graph.launch, 5, 0) / 5
    graph.close()

    def one_at_a_time():
        for plan, fact in frags:
            k, s, ng = pyst.query(ctx, plan, fact)
            int(ng.item())

    one_at_a_time()
    t0 = time.perf_counter()
    one_at_a_time()
    seq_s = time.perf_counter() - t0
    # results of the two executions agree fragment by fragment
    res = batch.results()
    mismatches = 0
    for (k, s), (plan, fact) in zip(res, frags):
        r = pyst.query(ctx, plan, fact)
        m = int(r[2].item())
        if m != k.numel() or not torch.equal(torch.sort(k).values, torch.sort(r[0][:m]).values):
            mismatches += 1
    total_rows = int(sizes.sum())
    return {"fragments": nfrag, "probe_rows": total_rows, "tuning": {"fanout": best[0], "block": best[1],
            "max_load": best[2]}, "batched_ms": batched_s * 1e3, "sequential_ms": seq_s * 1e3,
            "batched_fragments_per_s": nfrag / batched_s, "sequential_fragments_per_s": nfrag / seq_s,
            "speedup": seq_s / batched_s, "graph_ms": graph_s * 1e3, "graph_speedup": seq_s / graph_s,
            "batched_probe_rows_per_s": total_rows / batched_s,
            "batched_gbs": total_rows * 16 / batched_s / 1e9, "result_mismatches": mismatches}


def bench_serve(pyst, gen, log, nrows, nreq):
    """Poisson stream of star/chain requests over a pinned host fact table: continuous batching
    (shared scan, up to 8 active) vs one-at-a-time FIFO on the same trace."""
    import threading

    import numpy as np
    import torch
    na, nbd = 3_000_000, 300_000
    a_h, b_h = gen.chain_dims(na, nbd)
    a, b = to_dev(a_h), to_dev(b_h)
    log("serve: generating %d pinned fact rows" % nrows)
    host = chain_fact_pinned(gen, nrows, na, nbd, 0.0)
    rows = np.minimum(gen.loguniform_i64(nreq, 1e6, nrows, gen.seed(4, 7, 0)), nrows)
    kinds = ["star" if i % 2 == 0 else "chain" for i in range(nreq)]

    def plan_for(kind, r):
        if kind == "star":
            return pyst.fact_star_plan(b), nbd
        g = int(min(max(r // 8, 1024), 150_000_000))
        return pyst.chain_plan(a, b, max_groups=g), g

    def run(max_active, arrivals, packed=None):
        srv = pyst.Server(None if packed else host, budget=48 << 30, max_active=max_active, nbuf=2,
                          chunk_rows=16_000_000, packed=packed)
        # warm the resident dimension tables outside the trace
        for kind in ("star", "chain"):
            p, c = plan_for(kind, 1_000_000)
            srv.wait(srv.submit(p, 1_000_000, c))
        t_start = time.perf_counter()
        tickets = [None] * nreq

        def producer():
            for i in range(nreq):
                delay = t_start + arrivals[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                p, c = plan_for(kinds[i], int(rows[i]))
                tickets[i] = srv.submit(p, int(rows[i]), c)

        th = threading.Thread(target=producer)
        th.start()
        lat = []
        for i in range(nreq):
            while tickets[i] is None:
                time.sleep(0.0005)
            lat.append(srv.wait(tickets[i])[2])
        th.join()
        makespan = time.perf_counter() - t_start
        st = srv.stats()
        srv.check()
        srv.close()
        lat = np.array(lat)
        return {"p50_ms": float(np.percentile(lat, 50, method="nearest")),
                "p99_ms": float(np.percentile(lat, 99, method="nearest")),
                "mean_ms": float(lat.mean()), "makespan_s": makespan,
                "requests_per_s": nreq / makespan, "rows_per_s": float(rows.sum()) / makespan,
                "chunks_copied": st["chunks_copied"], "h2d_gb": st["bytes_copied"] / 1e9,
                "max_active_seen": st["max_active_seen"], "admission_waits": st["admission_waits"]}

    # service rate of one-at-a-time execution, from a back-to-back burst
    burst = run(1, np.zeros(nreq))
    lam = 0.9 * burst["requests_per_s"]
    arrivals = gen.poisson_arrivals(nreq, lam, gen.seed(4, 8, 0))
    log("serve: Poisson rate %.2f req/s (0.9 x one-at-a-time capacity)" % lam)
    fifo = run(1, arrivals)
    cont = run(8, arrivals)
    # the same trace served from bit-packed host columns (decoded on the device per chunk)
    log("serve: packing %d rows" % nrows)
    packed = [(*pyst.pack(t), nrows, t.dtype) for t in host]
    cont_packed = run(8, arrivals, packed)
    packed_bytes = sum(bl.numel() * 8 + w.numel() * 4 for bl, w, _, _ in packed)
    del host, packed
    return {"fact_rows": nrows, "requests": nreq, "arrival_rate_per_s": lam, "one_at_a_time": fifo,
            "continuous_batching": cont, "continuous_batching_packed": cont_packed,
            "packed_bytes_per_row": packed_bytes / nrows, "burst_one_at_a_time": burst,
            "workload": "50/50 star and chain requests, scan sizes log-uniform in [1e6, %d]" % nrows}


def host_cpu_info():
    """Cores this process may run on, the machine's count and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"affinity_cores": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count(), "model": model}


def cpu_baseline(b_host, p_host, sample_rows, log):
    """The oracle on one core over a bounded sample, and the threaded CPU
    baseline (the same algorithm over every core this process may use) on the
    whole probe table, checked equal to the oracle on the sample first."""
    import numpy as np

    import oracle
    info = host_cpu_info()
    sample_rows = min(sample_rows, len(p_host["fk"]))
    sample = {c: v[:sample_rows] for c, v in p_host.items()}
    log("cpu oracle on %d probe rows" % sample_rows)
    t0 = time.perf_counter()
    ok, osum = oracle.star_query(b_host, sample)
    dt = time.perf_counter() - t0
    out = {"value": sample_rows / dt, "unit": "probe rows/s", "cores": 1, "kind": "oracle",
           "sample": "full build table (%d rows), first %d probe rows; %.1f s single-threaded"
                     % (len(b_host["key"]), sample_rows, dt),
           "host": info}
    threads = info["affinity_cores"]
    tk, ts, used = oracle.star_query_threaded(b_host, sample, threads=threads)
    equal = bool(np.array_equal(tk, ok) and np.array_equal(ts, osum))
    n = len(p_host["fk"])
    log("threaded cpu baseline on %d probe rows, %d threads" % (n, threads))
    t0 = time.perf_counter()
    oracle.star_query_threaded(b_host, p_host, threads=threads)
    dtm = time.perf_counter() - t0
    out["threaded"] = {"value": n / dtm, "unit": "probe rows/s", "cores": used, "kind": "threaded baseline",
                       "equal_to_oracle_on_sample": equal,
                       "sample": "full build table, all %d probe rows; %.2f s on %d threads" % (n, dtm, used)}
    return out


if __name__ == "__main__":
    main()
