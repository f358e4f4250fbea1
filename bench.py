#!/usr/bin/env python3
"""Benchmark of the MBEA search on one MI355X.

A step is one full pass of the hot path over the benchmark graph already resident in HBM:
CSR validation, candidate ranking and the persistent depth-first search, through the C-ABI
call mbe_count.  The graph is the Chung-Lu power-law bipartite workload (|U| = 100k,
|V| = 50k, 1M edges, exponent 2.1 on both sides, seeded).  Prints one JSON line.

The power-law line also carries, as extra keys, the batched form on the 4,096-graph batch
workload ("batched": graphs/s of one batched call against one call per graph) and the serving
form on a Poisson request stream ("served": p50/p99 latency and graphs/s), unless --no-batch /
--no-serve.  --workload batch and --workload serve print those forms as lines of their own.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
                  [--workload power-law|er-small|skewed-sample|batch|serve|call-overhead] [--batch-n N]
                  [--serve-n N --rate R --slots S] [--no-batch] [--no-serve]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _hw_queues() -> str:
    """Hardware queues for this process (GPU_MAX_HW_QUEUES, read when the GPU is first used).
    A search runs one persistent kernel per mask-width class, concurrently on streams of their
    own, and each needs a queue of its own: HIP gives a process 4 by default, and streams
    beyond that share queues, so two class launches then run one after the other (measured on
    the power-law step: 38.9 ms with 4 queues, 35.5 ms with 8).  So at least 8, unless
    --hw-queues says otherwise.  Hardware counters are read per dispatch and count whatever
    runs meanwhile, so counter runs want one queue (launches one at a time): the traffic
    children take 1, and so does a run given --hw-queues 1."""
    if "--traffic-child" in sys.argv:
        return "1"
    for i, a in enumerate(sys.argv[:-1]):
        if a == "--hw-queues":
            return sys.argv[i + 1]
    try:
        cur = int(os.environ.get("GPU_MAX_HW_QUEUES", "0"))
    except ValueError:
        cur = 0
    return str(max(cur, 8))


os.environ["GPU_MAX_HW_QUEUES"] = _hw_queues()

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
BOX_THREADS = 16       # host threads of one GPU's share of the box


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_workload(name):
    import graphgen as gg
    if name == "power-law":
        g = gg.config2()
        desc = {"workload": "chung-lu power-law bipartite", "n_u": g.n_u, "n_v": g.n_v, "edges": g.n_edges,
                "gamma": 2.1, "weight_cap": "floor(sqrt(E/10))", "seed": 20240107}
        return g, desc, None
    if name == "er-small":
        g = gg.config1()
        return g, {"workload": "erdos-renyi bipartite", "n_u": 200, "n_v": 300, "p": 0.05, "edges": g.n_edges,
                   "seed": 20240106}, None
    if name == "skewed-sample":
        g = gg.config3()
        return g, {"workload": "skewed dense chung-lu + 50 planted bicliques, 64 top-level candidates",
                   "n_u": g.n_u, "n_v": g.n_v, "edges": g.n_edges, "gamma": 1.9, "seed": 20240108}, (2000, 2064)
    raise SystemExit(f"unknown workload {name}")


def _counter_rows(out_dir, counter):
    """(kernel name, value) of every dispatch row of counter in rocprofv3's CSV output."""
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(out_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") == counter:
                    rows.append((r.get("Kernel_Name", ""), float(r.get("Counter_Value", 0.0))))
    return rows


def measure_traffic(args):
    """HBM bytes of one step's search launches, measured: this script runs twice as a child
    under rocprofv3 --pmc (FETCH_SIZE, then WRITE_SIZE), each child making one plain 1 GiB
    device copy and one production step, with one hardware queue so that the class launches
    run one at a time and each dispatch's counters are its own.  Each counter is scaled by
    what it reads for the copy (1 GiB read and 1 GiB written).  Runs before this process
    touches the GPU; returns None when the profiler is missing or its output is incomplete."""
    import shutil
    import subprocess
    import tempfile
    prof = shutil.which("rocprofv3") or "/opt/rocm/bin/rocprofv3"
    if not os.path.exists(prof):
        return None
    got = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        d = tempfile.mkdtemp(prefix="mbe_pmc_", dir="/tmp")
        cmd = ["timeout", "-s", "KILL", "150", prof, "--pmc", ctr, "--output-format", "csv", "-d", d, "-o", "run",
               "--", sys.executable, os.path.abspath(__file__), "--traffic-child", "--copy-mib", "1024",
               "--workload", args.workload]
        log("traffic:", ctr)
        r = subprocess.run(cmd, cwd="/tmp", env=dict(os.environ, TMPDIR="/tmp"), capture_output=True, text=True)
        rows = _counter_rows(d, ctr)
        shutil.rmtree(d, ignore_errors=True)
        copy = sum(v for k, v in rows if "copyBuffer" in k)
        search = [v for k, v in rows if "search_kernel" in k]
        if r.returncode not in (0, 139) or copy <= 0 or not search:
            log(f"traffic: {ctr} not measured (rc {r.returncode}, {len(rows)} rows)")
            return None
        # counters are in KiB; the copy moves 1 GiB each way
        scale = float(1 << 30) / (copy * 1024.0)
        got[ctr] = {"kib": sum(search), "scale": scale, "bytes": sum(search) * 1024.0 * scale,
                    "launches": len(search)}
    return {"bytes": got["FETCH_SIZE"]["bytes"] + got["WRITE_SIZE"]["bytes"], "counters": got}


def traffic_child(args):
    """One plain 1 GiB device copy, then one production step (no diagnostics run)."""
    import numpy as np
    import torch
    import graphgen as gg
    import paper_2401_05039_amd as mbe
    mbe.load()
    g, desc, rng_range = make_workload(args.workload)
    dev = torch.device("cuda:0")
    dg = gg.BiGraph(g.n_u, g.n_v, *[torch.from_numpy(np.asarray(a)).to(dev) for a in
                                    (g.u_off, g.u_adj, g.v_off, g.v_adj)])
    n = args.copy_mib << 20
    src = torch.ones(n, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    lo, hi = rng_range if rng_range else (0, 0)
    mbe.mbe_count(dg, mbe.Options(root_lo=lo, root_hi=hi))
    torch.cuda.synchronize()


def cpu_baseline(g, rng_range, threads, frac=0.2, chunks=64):
    """The oracle (serial MBEA, split by top-level rank over host threads) on a bounded
    sample of the same graph: evenly spaced chunks of top-level candidates."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.build(force=False)
    n = oracle.num_roots(g)
    lo0, hi0 = rng_range if rng_range else (0, n)
    span = hi0 - lo0
    if rng_range is not None:
        frac, chunks = 1.0, min(16, span)
    per = max(1, int(span * frac / chunks))
    starts = np.linspace(lo0, hi0 - per, chunks).astype(np.int64)
    t0 = time.time()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda s: oracle.mbea(g, rank_lo=int(s), rank_hi=int(s) + per), starts))
    dt = time.time() - t0
    cnt = sum(p["count"] for p in parts)
    return {"value": cnt / dt, "unit": "bicliques/s", "cores": threads, "kind": "oracle",
            "sample": f"{chunks} evenly spaced chunks of {per} top-level candidates ({chunks * per} of {n}), "
                      f"{cnt} bicliques in {dt:.2f} s wall on {threads} threads"}


def load_study(mbe, dg, rng, steal_ks=(1, 2, 3)):
    """Per-workgroup load of the search (the per-block time distribution and the work-sharing
    ablation of the paper's evaluation, section IV): one tally run per steal depth k with a load
    record per workgroup.  A workgroup is busy from its start to its end minus the time it
    spent finding work; the launch span runs from the first start to the last end."""
    import numpy as np
    lo, hi = rng if rng else (0, 0)
    out = {}
    for k in steal_ks:
        res, rec = mbe.mbe_count_loads(dg, mbe.Options(steal_k=k, root_lo=lo, root_hi=hi))
        start, end, wait = rec[:, 1].astype(np.float64), rec[:, 2].astype(np.float64), rec[:, 3].astype(np.float64)
        span = end.max() - start.min()
        busy = end - start - wait
        frac = busy / span
        out[f"k{k}"] = {
            "search_ms": res["kernel_ms"],
            "workgroups": int(len(rec)),
            "busy_frac": {q: float(np.percentile(frac, p)) for q, p in
                          (("min", 0), ("p10", 10), ("p50", 50), ("p90", 90), ("max", 100))},
            "idle_share": float(1.0 - busy.sum() / (len(rec) * span)),
            "busy_max_over_median": float(busy.max() / max(np.median(busy), 1.0)),
            "shared_chunks": res["shared_chunks"],
            "count": res["count"],
        }
        log(f"load study k={k}: {res['kernel_ms']:.1f} ms, idle share {out[f'k{k}']['idle_share']:.3f}")
    return out


def steal_ablation(mbe, dg, rng, steps=3):
    """Search time per step under steal depth k = 1, 2, 3 (same answers)."""
    lo, hi = rng if rng else (0, 0)
    out = {}
    for k in (1, 2, 3):
        opt = mbe.Options(steal_k=k, root_lo=lo, root_hi=hi)
        mbe.mbe_count(dg, opt)
        ks = [mbe.mbe_count(dg, opt)["kernel_ms"] for _ in range(steps)]
        out[f"k{k}_ms"] = sum(ks) / len(ks)
    return out


def prune_study(mbe, dg, rng, plain, steps=3):
    """The tree and search time under the pruning of section II-C (same answers): iMBEA's
    candidate pruning (prune = 1) and the pivot rule (prune = 2), both run by the generic-width
    search, beside the plain tree of the fixed-width classes (plain: its diagnostics result)."""
    lo, hi = rng if rng else (0, 0)
    out = {"plain": {"nodes": plain["nodes"], "nonmaximal": plain["nonmaximal"], "max_depth": plain["max_depth"]}}
    for name, mode in (("imbea", 1), ("pivot", 2)):
        d = mbe.mbe_count(dg, mbe.Options(prune=mode, diagnostics=1, root_lo=lo, root_hi=hi))
        assert (d["count"], d["hash"]) == (plain["count"], plain["hash"]), name
        opt = mbe.Options(prune=mode, root_lo=lo, root_hi=hi)
        mbe.mbe_count(dg, opt)
        ks = [mbe.mbe_count(dg, opt)["kernel_ms"] for _ in range(steps)]
        out[name] = {"nodes": d["nodes"], "nonmaximal": d["nonmaximal"], "max_depth": d["max_depth"],
                     "search_ms": sum(ks) / len(ks)}
    return out


def generate(fn, items, workers=BOX_THREADS):
    """[fn(x) for x in items], on a pool of forked worker processes when more than one host
    thread is available (the graphs are seeded per item, so the result is the same).  Called
    before this process touches the GPU."""
    items = list(items)
    workers = min(workers, os.cpu_count() or 1, len(items))
    if workers <= 1:
        return [fn(x) for x in items]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(fn, items, chunksize=max(1, len(items) // (8 * workers)))


def batch_inputs(n):
    import graphgen as gg
    t0 = time.time()
    gs = generate(gg.config4_graph, range(n))
    log(f"generated {len(gs)} batch graphs, {sum(g.n_edges for g in gs)} edges, in {time.time() - t0:.1f} s")
    return gs


def serve_inputs(n, rate, big_max_u):
    import graphgen as gg
    t0 = time.time()
    arr = gg.config5_arrivals(n, rate, big_max_u=big_max_u)
    reqs = list(zip([t for t, _ in arr], generate(gg.config5_build, [sp for _, sp in arr])))
    log(f"generated {len(reqs)} requests ({sum(1 for _, g in reqs if g.n_u >= 20000)} large), "
        f"{sum(g.n_edges for _, g in reqs)} edges, in {time.time() - t0:.1f} s")
    return reqs


def batch_form(mbe, gs, tune_every, batch_calls=1, plain_defaults=False, waves=0, grid=0):
    """Batched form against the plain form on the graphs gs.  The launch setting is picked by
    the autotuner (mbe_tune_batch) on every tune_every-th graph and then used by both forms;
    with plain_defaults the plain form also runs under the library's defaults and the faster
    of the two is its time.  Both forms take host graphs, so both include the upload and the
    preparation.  Per-graph count and hash must agree between the forms."""
    base = mbe.Options(wg_waves=waves, grid=grid)
    t0 = time.perf_counter()
    sample = gs[::tune_every]
    opt, tuned_ms = mbe.mbe_tune_batch(sample, base)
    t_tune = time.perf_counter() - t0
    log(f"tuned on {len(sample)} graphs in {t_tune:.1f} s: wg_waves={opt.wg_waves} steal_k={opt.steal_k} "
        f"({tuned_ms:.0f} ms per sample batch)")
    mbe.mbe_count_batch(gs[:64], opt)
    for g in gs[:8]:
        mbe.mbe_count(g, opt)
    t0 = time.perf_counter()
    plain = [mbe.mbe_count(g, opt) for g in gs]
    t_plain_tuned = time.perf_counter() - t0
    t_plain, t_plain_def = t_plain_tuned, None
    if plain_defaults:
        t0 = time.perf_counter()
        plain_def = [mbe.mbe_count(g, base) for g in gs]
        t_plain_def = time.perf_counter() - t0
        if t_plain_def < t_plain:
            t_plain, plain = t_plain_def, plain_def
    log(f"plain: {t_plain_tuned:.3f} s tuned setting" +
        (f", {t_plain_def:.3f} s defaults" if t_plain_def is not None else ""))
    times, attempts = [], []
    for _ in range(max(1, batch_calls)):
        t0 = time.perf_counter()
        res = mbe.mbe_count_batch(gs, opt)
        times.append(time.perf_counter() - t0)
        attempts.append(max(r["attempts"] for r in res) if res else 1)
    t_batch = min(times)
    log(f"batched: {', '.join(f'{t:.3f}' for t in times)} s")
    for i, (a, b) in enumerate(zip(plain, res)):
        assert (a["count"], a["hash"]) == (b["count"], b["hash"]), i
    total = sum(r["count"] for r in res)
    # share of the plain time spent on the graphs that need >= 10% of a second alone
    heavy = sorted((r["kernel_ms"] for r in plain), reverse=True)
    return {
        "graphs": len(gs), "edges": sum(g.n_edges for g in gs), "bicliques": total,
        "batched_s": t_batch, "batched_calls": len(times), "batched_attempts": attempts,
        "plain_s": t_plain, "plain_s_tuned_setting": t_plain_tuned, "plain_s_defaults": t_plain_def,
        "batched_graphs_per_s": len(gs) / t_batch, "plain_graphs_per_s": len(gs) / t_plain,
        "batched_over_plain": t_plain / t_batch,
        "bicliques_per_s_batched": total / t_batch,
        "plain_kernel_ms_heaviest_graphs": sum(k for k in heavy if k >= 100.0),
        "plain_heaviest_graphs": sum(1 for k in heavy if k >= 100.0),
        "tuned": {"wg_waves": opt.wg_waves, "steal_k": opt.steal_k, "tune_s": t_tune, "sample_graphs": len(sample)},
    }


def serve_form(mbe, reqs, slots, saturated=True):
    """Serving form: the requests are submitted at their Poisson arrival times to a
    continuous-batching server (admission by device footprint, one slot reserved for small
    requests); latency is submission to completion.  Then the same requests are submitted all
    at once (the server's capacity) and run one mbe_count call at a time (the plain form),
    and every result must be the same in the mix, saturated and alone."""
    import threading
    import numpy as np
    lat = [0.0] * len(reqs)
    res = [None] * len(reqs)
    sat = None
    with mbe.Server(slots=slots) as sv:
        for tk in [sv.submit(g) for _, g in reqs[:8]]:  # warm the slots' workspaces
            sv.wait(tk)
        tickets = [None] * len(reqs)
        start = time.perf_counter()

        def feed():
            for i, (t, g) in enumerate(reqs):
                delay = start + t - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tickets[i] = sv.submit(g)

        th = threading.Thread(target=feed)
        th.start()
        th.join()
        for i in range(len(reqs)):
            res[i], lat[i] = sv.wait(tickets[i])
        span = time.perf_counter() - start
        log(f"poisson run: {span:.1f} s")
        if saturated:
            t0 = time.perf_counter()
            tks = [sv.submit(g) for _, g in reqs]
            sat = [sv.wait(tk)[0] for tk in tks]
            t_sat = time.perf_counter() - t0
            log(f"saturated run: {t_sat:.1f} s")
    t0 = time.perf_counter()
    plain = [mbe.mbe_count(g) for _, g in reqs]
    t_plain = time.perf_counter() - t0
    log(f"plain run: {t_plain:.1f} s")
    for i in range(len(reqs)):
        assert (res[i]["count"], res[i]["hash"]) == (plain[i]["count"], plain[i]["hash"]), i
        if sat is not None:
            assert (sat[i]["count"], sat[i]["hash"]) == (plain[i]["count"], plain[i]["hash"]), i
    lat_a = np.array(lat)
    small = np.array([g.n_u < 20000 for _, g in reqs])
    n_big = int((~small).sum())
    return {
        "requests": len(reqs), "large_requests": n_big, "slots": slots,
        "edges": sum(g.n_edges for _, g in reqs), "bicliques": sum(r["count"] for r in res),
        "span_s": span, "graphs_per_s": len(reqs) / span,
        "p50_ms": float(np.percentile(lat_a, 50)),
        "p99_ms": float(np.percentile(lat_a, 99)),
        "p50_ms_small": float(np.percentile(lat_a[small], 50)),
        "p99_ms_small": float(np.percentile(lat_a[small], 99)),
        "p50_ms_large": float(np.percentile(lat_a[~small], 50)) if n_big else None,
        "saturated_graphs_per_s": len(reqs) / t_sat if sat is not None else None,
        "plain_graphs_per_s": len(reqs) / t_plain,
        "served_over_plain": t_plain / t_sat if sat is not None else None,
    }


def call_overhead(mbe, dev, calls):
    """Wall time of one mbe_count call on tiny graphs, from device-resident CSR arrays and from
    host arrays, against the search time the call reports: what a call costs beyond its
    search (launches, copies, the waits on the preparation's statistics).  K_{4,4} has one
    maximal biclique and a four-node tree (the call's fixed cost); crown(9) has 510 and a
    tree nine levels deep (a small request's dependent steps)."""
    import numpy as np
    import torch
    import graphgen as gg
    out = {"calls": calls}
    for name, g in (("k44", gg.complete(4, 4)), ("crown9", gg.crown(9))):
        dg = gg.BiGraph(g.n_u, g.n_v, *[torch.from_numpy(np.asarray(a)).to(dev) for a in
                                        (g.u_off, g.u_adj, g.v_off, g.v_adj)])
        for key, gr in (("device_csr", dg), ("host_csr", g)):
            for _ in range(10):
                mbe.mbe_count(gr)
            torch.cuda.synchronize()
            ks = []
            t0 = time.perf_counter()
            for _ in range(calls):
                ks.append(mbe.mbe_count(gr)["kernel_ms"])
            dt = time.perf_counter() - t0
            out[f"{name}_{key}_ms_per_call"] = dt * 1000.0 / calls
            out[f"{name}_{key}_search_ms"] = sum(ks) / len(ks)
    return out


def bench_call_overhead(args, mbe, dev):
    r = call_overhead(mbe, dev, max(1, args.steps))
    out = {
        "metric": "wall ms per mbe_count call on a tiny graph",
        "value": r["k44_device_csr_ms_per_call"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": r["calls"],
        "warmup": 10,
        "ms_per_step": r["k44_device_csr_ms_per_call"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "K_{4,4} (one maximal biclique) and crown(9) (9 x 9 vertices, 72 edges, 510 "
                               "maximal bicliques)"},
        **r,
    }
    print(json.dumps(out), flush=True)


def bench_batch(args, mbe, gs):
    r = batch_form(mbe, gs, tune_every=8, batch_calls=args.steps, plain_defaults=True,
                   waves=args.waves, grid=args.grid)
    out = {
        "metric": "graphs/s batched vs plain",
        "value": r["batched_graphs_per_s"],
        "unit": "graphs/s",
        "n_gpus": 1,
        "steps": r["batched_calls"],
        "warmup": 1,
        "ms_per_step": r["batched_s"] * 1000.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"batch of {len(gs)} ER / Chung-Lu bipartite graphs, sides log-uniform [50, 2000], "
                               f"density U[0.01, 0.1]", "graphs": len(gs), "edges": r["edges"],
                   "bicliques": r["bicliques"], "tuned": r["tuned"]},
        **{k: r[k] for k in ("plain_graphs_per_s", "plain_s_tuned_setting", "plain_s_defaults",
                             "batched_over_plain", "plain_kernel_ms_heaviest_graphs", "plain_heaviest_graphs",
                             "bicliques_per_s_batched", "batched_attempts")},
    }
    print(json.dumps(out), flush=True)


def bench_serve(args, mbe, reqs):
    r = serve_form(mbe, reqs, args.slots)
    out = {
        "metric": "served graphs/s; p50/p99 solve latency",
        "value": r["graphs_per_s"],
        "unit": "graphs/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": r["span_s"] * 1000.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"Poisson stream of {len(reqs)} requests at {args.rate}/s, 90% batch-style graphs, "
                               f"10% Chung-Lu |U| up to {args.big_max_u}", "slots": args.slots,
                   "large_requests": r["large_requests"], "edges": r["edges"], "bicliques": r["bicliques"]},
        **{k: r[k] for k in ("p50_ms", "p99_ms", "p50_ms_small", "p99_ms_small", "p50_ms_large",
                             "saturated_graphs_per_s", "plain_graphs_per_s", "served_over_plain")},
        "offered_rate": args.rate,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="power-law")
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a reference "
                         "kernel of known traffic for scaling hardware byte counters)")
    ap.add_argument("--batch-n", type=int, default=4096)
    ap.add_argument("--serve-n", type=int, default=200)
    ap.add_argument("--rate", type=float, default=2.5)
    ap.add_argument("--slots", type=int, default=2)
    ap.add_argument("--big-max-u", type=int, default=200_000)
    ap.add_argument("--no-traffic", action="store_true",
                    help="skip the two rocprofv3 counter runs that measure the step's HBM traffic")
    ap.add_argument("--traffic-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-load-study", action="store_true",
                    help="skip the per-workgroup load study (k = 1, 2, 3) on the skewed sample")
    ap.add_argument("--no-batch", action="store_true",
                    help="power-law line: skip the batched-form figures (--batch-n graphs)")
    ap.add_argument("--no-serve", action="store_true",
                    help="power-law line: skip the serving-form figures (--line-serve-n requests at --line-rate)")
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="GPU_MAX_HW_QUEUES for this run (default: at least 8; 1 serialises the class "
                         "launches, for hardware-counter runs)")
    ap.add_argument("--line-serve-n", type=int, default=100)
    ap.add_argument("--line-rate", type=float, default=4.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the search runs on one GPU (sharding across GPUs is a design only); --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.traffic_child:
        return traffic_child(args)
    traffic = None
    if args.workload in ("power-law", "skewed-sample", "er-small") and not args.no_traffic:
        # (before this process initialises the GPU: the profiled children are started from here)
        traffic = measure_traffic(args)
    # the batched and served inputs are generated here too, on forked workers, before the GPU
    # is touched
    gs = reqs = None
    if args.workload == "batch" or (args.workload == "power-law" and not args.no_batch):
        gs = batch_inputs(args.batch_n)
    if args.workload == "serve":
        reqs = serve_inputs(args.serve_n, args.rate, args.big_max_u)
    elif args.workload == "power-law" and not args.no_serve:
        reqs = serve_inputs(args.line_serve_n, args.line_rate, args.big_max_u)

    import numpy as np
    import torch
    import paper_2401_05039_amd as mbe

    if not torch.cuda.is_available():
        raise SystemExit("no HIP device")
    mbe.load()
    if args.workload == "batch":
        return bench_batch(args, mbe, gs)
    if args.workload == "serve":
        return bench_serve(args, mbe, reqs)
    if args.workload == "call-overhead":
        return bench_call_overhead(args, mbe, torch.device("cuda:0"))
    g, desc, rng_range = make_workload(args.workload)
    log("graph", desc)
    dev = torch.device("cuda:0")
    import graphgen as gg
    dg = gg.BiGraph(g.n_u, g.n_v, *[torch.from_numpy(np.asarray(a)).to(dev) for a in
                                    (g.u_off, g.u_adj, g.v_off, g.v_adj)])
    if args.copy_mib > 0:
        n = args.copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {n} bytes")
        del src, dst
    lo, hi = rng_range if rng_range else (0, 0)
    base = dict(wg_waves=args.waves, grid=args.grid, root_lo=lo, root_hi=hi)

    # one untimed run with diagnostics gives the method's tree (nodes, algorithmic bytes) and the
    # time split over search phases; one untimed run of the production search with its
    # design-byte tally gives the bytes its loads and stores request (deterministic)
    diag = mbe.mbe_count(dg, mbe.Options(diagnostics=1, **base))
    tally = mbe.mbe_count(dg, mbe.Options(diagnostics=2, **base))
    assert (tally["count"], tally["hash"]) == (diag["count"], diag["hash"])
    ph = diag["phase_cycles"]
    ph_tot = max(1, sum(ph.values()))
    phase_share = {k: round(v / ph_tot, 4) for k, v in ph.items()}
    log("diagnostics", {k: diag[k] for k in ("count", "hash", "nodes", "nonmaximal", "bytes_alg", "max_depth",
                                             "kernel_ms")})
    opt = mbe.Options(**base)
    for _ in range(args.warmup):
        mbe.mbe_count(dg, opt)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = mbe.mbe_count(dg, opt)
        kms.append(r["kernel_ms"])
        assert r["count"] == diag["count"] and r["hash"] == diag["hash"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1000.0 / args.steps
    value = diag["count"] * args.steps / dt
    kavg = sum(kms) / len(kms)
    achieved = tally["bytes_design"] / (kavg / 1000.0) / 1e9
    out = {
        "metric": "maximal bicliques/s",
        "value": value,
        "unit": "bicliques/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": dict(desc, count=diag["count"], hash=hex(diag["hash"]), search_nodes=diag["nodes"]),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic["bytes"] if traffic else None,
                     "traffic_gbs": traffic["bytes"] / (kavg / 1000.0) / 1e9 if traffic else None,
                     "traffic_frac": traffic["bytes"] / (kavg / 1000.0) / 1e9 / HBM_PEAK_GBS if traffic else None,
                     "traffic_counters": traffic["counters"] if traffic else None,
                     "kernel": "search_kernel (all mask-width launches of one step)",
                     "kernel_ms": kavg, "bytes_design": tally["bytes_design"]},
        # the paper's reverse-scanning method would move bytes_alg for the same tree; this
        # design never performs those scans, so the rate is an effective one, not traffic
        "paper_method_rate": {"bytes_alg": diag["bytes_alg"], "gbs": diag["bytes_alg"] / (kavg / 1000.0) / 1e9},
        "search_ms_median": sorted(kms)[len(kms) // 2],
        "phase_share": phase_share,
    }
    # end to end from host arrays: validation on the host, the upload of the CSR (PCIe), the
    # preparation, the search and the result (the line's value starts from device arrays)
    mbe.mbe_count(g, opt)
    e2e = []
    for _ in range(3):
        t1 = time.perf_counter()
        r = mbe.mbe_count(g, opt)
        e2e.append((time.perf_counter() - t1) * 1000.0)
        assert (r["count"], r["hash"]) == (diag["count"], diag["hash"])
    out["host_csr_end_to_end_ms"] = sorted(e2e)[1]
    out["steal_ablation"] = steal_ablation(mbe, dg, rng_range)
    log("prune study")
    out["prune_study"] = prune_study(mbe, dg, rng_range, diag)
    if not args.no_load_study:
        # the load study on the skewed graph's sample of 64 top-level candidates (deep,
        # unbalanced subtrees)
        if args.workload == "skewed-sample":
            sg, srng = dg, rng_range
        else:
            g3 = gg.config3()
            sg = gg.BiGraph(g3.n_u, g3.n_v, *[torch.from_numpy(np.asarray(a)).to(dev) for a in
                                              (g3.u_off, g3.u_adj, g3.v_off, g3.v_adj)])
            srng = (2000, 2064)
        out["load_study"] = dict(workload="skewed dense chung-lu 20k x 5k + 50 planted, top-level ranks [2000, 2064)",
                                 **load_study(mbe, sg, srng))
    if rng_range is not None:
        # one top-level candidate of the skewed graph holds ~0.8M bicliques: the oracle needs
        # minutes for the smallest sample, so no bounded baseline exists for this workload
        out["cpu_baseline"] = {"value": None, "unit": "bicliques/s", "cores": 0, "kind": "oracle",
                               "sample": "skipped: a single top-level candidate takes the oracle minutes"}
    elif not args.no_cpu_baseline:
        threads = min(BOX_THREADS, os.cpu_count() or 1)
        log("cpu baseline on", threads, "threads")
        out["cpu_baseline"] = cpu_baseline(g, rng_range, threads)
        # the same oracle on one core, on a smaller sample (about half the parallel leg's work)
        log("cpu baseline on 1 thread")
        out["cpu_baseline_serial"] = cpu_baseline(g, rng_range, 1, frac=0.1, chunks=32)
    if gs is not None:
        # the batched form on the batch workload's own graphs: tuner on every 32nd graph, one
        # batched call against one mbe_count call per graph (the faster of the tuned setting
        # and the defaults)
        del dg
        torch.cuda.empty_cache()
        log("batched form")
        out["batched"] = dict(workload=f"{len(gs)} ER / Chung-Lu bipartite graphs, sides log-uniform [50, 2000], "
                                       "density U[0.01, 0.1]", **batch_form(mbe, gs, tune_every=32, plain_defaults=True))
        del gs
    out["call_overhead"] = call_overhead(mbe, dev, 200)
    if reqs is not None:
        log("serving form")
        out["served"] = dict(workload=f"Poisson stream of {len(reqs)} requests at {args.line_rate}/s, 90% batch-style "
                                      f"graphs, 10% Chung-Lu |U| in [20k, {args.big_max_u}]",
                             offered_rate=args.line_rate, **serve_form(mbe, reqs, args.slots))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
