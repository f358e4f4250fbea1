"""SHA-256 fingerprints of the seeded workload inputs, so that a change to a generator (or to
the numpy it runs on) shows up as a changed input rather than as changed results."""
from __future__ import annotations

import hashlib
import os
from typing import Dict

import numpy as np

import graphgen as gg


def digest(g) -> str:
    """SHA-256 of (n_u, n_v) and the four CSR arrays as little-endian int32."""
    h = hashlib.sha256()
    h.update(np.asarray([g.n_u, g.n_v], dtype="<i8").tobytes())
    for a in (g.u_off, g.u_adj, g.v_off, g.v_adj):
        h.update(np.ascontiguousarray(a, dtype="<i4").tobytes())
    return h.hexdigest()


def _batch_digest(i: int) -> str:
    return digest(gg.config4_graph(i))


def _request_digest(spec) -> str:
    return digest(gg.config5_build(spec))


def _map(fn, items, workers):
    items = list(items)
    workers = max(1, min(workers, os.cpu_count() or 1, len(items)))
    if workers == 1:
        return [fn(x) for x in items]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(fn, items, chunksize=max(1, len(items) // (8 * workers)))


def combined(digests) -> str:
    h = hashlib.sha256()
    for d in digests:
        h.update(bytes.fromhex(d))
    return h.hexdigest()


def manifest(workers: int = 8, batch_n: int = 4096, serve_n: int = 200, rate: float = 2.5) -> Dict[str, str]:
    """Digests of the ER, power-law and skewed workloads, and combined digests of the batch
    workload's graphs and of the serving stream's request graphs (with their arrival times)."""
    out = {
        "config1": digest(gg.config1()),
        "config2": digest(gg.config2()),
        "config3": digest(gg.config3()),
    }
    out[f"config4_graphs_0_{batch_n}"] = combined(_map(_batch_digest, range(batch_n), workers))
    arr = gg.config5_arrivals(serve_n, rate)
    times = hashlib.sha256(np.asarray([t for t, _ in arr], dtype="<f8").tobytes()).hexdigest()
    out[f"config5_requests_{serve_n}_at_{rate}"] = combined([times] + _map(_request_digest, [s for _, s in arr], workers))
    return out
