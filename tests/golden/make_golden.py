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
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
