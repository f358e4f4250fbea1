"""Write tests/golden/workloads.json: oracle results for the seeded workloads.

Every value here comes from the CPU oracle (oracle/, serial MBEA split by top-level rank over
host threads) on graphs from graphgen; nothing is taken from the HIP library.  Run from the
repository root:  python tests/golden/make_golden.py [--skip-big]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workloads.json")
KEYS = ("count", "hash", "out_ints", "nodes", "nonmaximal", "bytes_alg", "bytes_rs", "max_depth", "side")


def pick(r):
    return {k: int(r[k]) for k in KEYS}


def main():
    skip_big = "--skip-big" in sys.argv
    old = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            old = json.load(f)
    res = dict(old)
    t = time.time()
    g1 = gg.config1()
    res["config1"] = dict(pick(oracle.mbea(g1)), graph=g1.name, edges=g1.n_edges)
    print("config1", res["config1"], "%.1fs" % (time.time() - t), flush=True)
    if not skip_big:
        t = time.time()
        g2 = gg.config2()
        r2 = oracle.mbea_parallel(g2, threads=os.cpu_count())
        res["config2"] = dict(pick(r2), graph=g2.name, edges=g2.n_edges,
                              oracle_seconds=round(time.time() - t, 1), oracle_threads=r2["threads"])
        print("config2", res["config2"], flush=True)
        t = time.time()
        g3 = gg.config3()
        n3 = oracle.num_roots(g3)
        ranks = [0, n3 // 4, n3 // 2, (3 * n3) // 4, n3 - 1]
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(len(ranks)) as ex:
            parts = list(ex.map(lambda r: oracle.mbea(g3, rank_lo=r, rank_hi=r + 1), ranks))
        res["config3_samples"] = {"graph": g3.name, "edges": g3.n_edges, "roots": n3,
                                  "samples": [dict(pick(p), rank_lo=r, rank_hi=r + 1) for r, p in zip(ranks, parts)],
                                  "oracle_seconds": round(time.time() - t, 1)}
        print("config3 samples", res["config3_samples"], flush=True)
        t = time.time()
        # every mask class of the skewed graph (degrees 208-256: W = 4, 257-512: W = 8,
        # 513-585: W = 16), and the whole W = 16 class as one rank range
        class_ranges = [(r, r + 1) for r in (0, 100, 222, 223, 500, 3000, 4000, 4500, 4800, 4900, 4967,
                                              4968, 4980, 4999)] + [(4968, n3)]
        with ThreadPoolExecutor(os.cpu_count()) as ex:
            parts = list(ex.map(lambda lh: oracle.mbea(g3, rank_lo=lh[0], rank_hi=lh[1]), class_ranges))
        res["config3_classes"] = {"graph": g3.name, "edges": g3.n_edges, "roots": n3,
                                  "samples": [dict(pick(p), rank_lo=lo, rank_hi=hi)
                                              for (lo, hi), p in zip(class_ranges, parts)],
                                  "oracle_seconds": round(time.time() - t, 1)}
        print("config3 classes", round(time.time() - t, 1), "s", flush=True)
        t = time.time()
        # the smallest Chung-Lu request of the serving stream (200 requests at 2.5/s)
        reqs = gg.config5_requests(200, 2.5)
        k5 = 191
        g5 = reqs[k5][1]
        r5 = oracle.mbea_parallel(g5, threads=os.cpu_count())
        res["config5_request"] = dict(pick(r5), request=k5, graph=g5.name, edges=g5.n_edges,
                                      oracle_seconds=round(time.time() - t, 1))
        print("config5 request", res["config5_request"], flush=True)
    # a fixed subset of the batch (graphs of mask classes W = 1, 2 and 4 whose oracle runs take
    # seconds; the batch also holds graphs with 1e8 bicliques)
    t = time.time()
    c4 = {1: [1, 2, 3, 5, 7, 12, 14, 23], 2: [6, 8, 9, 13, 16, 22, 29, 47, 64, 106],
          4: [0, 11, 30, 56, 65, 162, 195, 220, 248, 258, 306, 352]}
    idx = sorted(i for v in c4.values() for i in v)
    from concurrent.futures import ThreadPoolExecutor as TPE
    with TPE(os.cpu_count()) as ex:
        parts = list(ex.map(lambda i: oracle.mbea(gg.config4_graph(i)), idx))
    res["config4_subset"] = {"graphs": [dict(pick(p), index=i, name=gg.config4_graph(i).name)
                                        for i, p in zip(idx, parts)],
                             "classes": {str(w): v for w, v in c4.items()},
                             "oracle_seconds": round(time.time() - t, 1)}
    print("config4 subset", round(time.time() - t, 1), "s", flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
