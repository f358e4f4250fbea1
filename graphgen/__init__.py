"""Seeded synthetic bipartite graphs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and builds CSR arrays.  It holds none of the
enumeration's arithmetic (no neighbourhood intersections, no hashing of bicliques), so
both the HIP path and the CPU oracle can consume its output without sharing code.

Random numbers come from a counter-based SplitMix64 stream (Steele, Lea and Flood,
OOPSLA 2014): value i of stream s under seed k is the SplitMix64 output function applied
to ``base(k, s) + (i + 1) * 0x9E3779B97F4A7C15``.  Every generator is a pure function of
its arguments, so a seed names a graph for good, independent of the numpy version.

Graph model vocabulary follows the paper's background section: a bipartite graph
G = (U u V, E) with E a subset of U x V; N(v) is the neighbour set of v.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterable, List, Sequence, Tuple

import numpy as np

__all__ = [
    "BiGraph", "stream_u64", "stream_uniform", "from_edges", "erdos_renyi_pairs",
    "erdos_renyi_m", "chung_lu", "planted_bicliques", "union",
    "config1", "config2", "config3", "config4_graph", "config4_batch", "config5_requests",
    "config5_arrivals", "config5_build",
    "complete", "perfect_matching", "crown", "chain", "private_neighbours", "complete_minus_edge", "edgeless",
    "disjoint_union", "transpose", "relabel", "random_small",
]

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_BASE_SEED = 20240105


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _base(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
        s = _mix(s + _GAMMA)
        s = _mix(s ^ np.uint64((stream * 0xD1342543DE82EF95) & 0xFFFFFFFFFFFFFFFF))
    return s[0]


def stream_u64(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """n values of the counter-based SplitMix64 stream (seed, stream), from index start."""
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(_base(seed, stream) + idx * _GAMMA)


def stream_uniform(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """n doubles uniform in [0, 1): the top 53 bits of the stream."""
    return (stream_u64(seed, stream, n, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclasses.dataclass
class BiGraph:
    """A bipartite graph as two sorted CSR arrays that are exact transposes.

    u_off[n_u+1], u_adj[E]: row u lists N(u) in V, strictly ascending.
    v_off[n_v+1], v_adj[E]: row v lists N(v) in U, strictly ascending.
    """
    n_u: int
    n_v: int
    u_off: np.ndarray
    u_adj: np.ndarray
    v_off: np.ndarray
    v_adj: np.ndarray
    name: str = ""

    @property
    def n_edges(self) -> int:
        return int(self.u_adj.shape[0])

    def edges(self) -> Tuple[np.ndarray, np.ndarray]:
        us = np.repeat(np.arange(self.n_u, dtype=np.int32), np.diff(self.u_off))
        return us, self.u_adj.copy()

    def row_u(self, u: int) -> np.ndarray:
        return self.u_adj[self.u_off[u]:self.u_off[u + 1]]

    def row_v(self, v: int) -> np.ndarray:
        return self.v_adj[self.v_off[v]:self.v_off[v + 1]]

    def nbytes(self) -> int:
        return 4 * (self.n_u + self.n_v + 2 + 2 * self.n_edges)


def _csr(n_rows: int, rows: np.ndarray, cols: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    order = np.lexsort((cols, rows))
    r = rows[order]
    c = cols[order].astype(np.int32)
    counts = np.bincount(r, minlength=n_rows) if r.size else np.zeros(n_rows, dtype=np.int64)
    off = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    if off[-1] > np.iinfo(np.int32).max:
        raise ValueError("edge count exceeds int32")
    return off.astype(np.int32), c


def from_edges(n_u: int, n_v: int, us: Iterable[int], vs: Iterable[int], name: str = "",
               dedupe: bool = False) -> BiGraph:
    """Build both CSR sides from an edge list (u in U, v in V)."""
    us = np.asarray(us, dtype=np.int64).ravel()
    vs = np.asarray(vs, dtype=np.int64).ravel()
    if us.shape != vs.shape:
        raise ValueError("edge arrays differ in length")
    if us.size:
        if us.min() < 0 or us.max() >= n_u or vs.min() < 0 or vs.max() >= n_v:
            raise ValueError("vertex id out of range")
    key = us * max(n_v, 1) + vs
    uniq = np.unique(key)
    if uniq.size != key.size and not dedupe:
        raise ValueError("duplicate edges")
    us = (uniq // max(n_v, 1)).astype(np.int64)
    vs = (uniq % max(n_v, 1)).astype(np.int64)
    u_off, u_adj = _csr(n_u, us, vs)
    v_off, v_adj = _csr(n_v, vs, us)
    return BiGraph(n_u, n_v, u_off, u_adj, v_off, v_adj, name)


def union(*graphs: BiGraph, name: str = "") -> BiGraph:
    """Edge union of graphs on the same vertex sets."""
    n_u, n_v = graphs[0].n_u, graphs[0].n_v
    us, vs = [], []
    for g in graphs:
        assert g.n_u == n_u and g.n_v == n_v
        a, b = g.edges()
        us.append(a)
        vs.append(b)
    return from_edges(n_u, n_v, np.concatenate(us), np.concatenate(vs), name=name, dedupe=True)


# ----------------------------------------------------------------------------- random models

def erdos_renyi_pairs(n_u: int, n_v: int, p: float, seed: int, name: str = "") -> BiGraph:
    """Each of the n_u * n_v pairs is an edge independently with probability p."""
    r = stream_uniform(seed, 1, n_u * n_v)
    idx = np.nonzero(r < p)[0]
    return from_edges(n_u, n_v, idx // n_v, idx % n_v, name=name)


def _distinct_pairs(draw, m: int, n_v: int, seed: int) -> np.ndarray:
    """Draw pair keys u*n_v+v with draw(stream, count) until m distinct keys exist.

    Duplicates are dropped; the stream continues where it stopped, so the result only
    depends on the seed.  Order of first appearance decides which draws are kept."""
    keys = np.zeros(0, dtype=np.int64)
    pos = 0
    batch = max(1024, int(m * 1.05) + 16)
    rounds = 0
    while keys.size < m:
        new = draw(pos, batch)
        pos += batch
        allk = np.concatenate([keys, new])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        keys = allk[first]
        rounds += 1
        if rounds > 200:
            raise RuntimeError("could not draw enough distinct edges")
        batch = max(1024, int((m - keys.size) * 1.3) + 16)
    return keys[:m]


def erdos_renyi_m(n_u: int, n_v: int, m: int, seed: int, name: str = "") -> BiGraph:
    """Exactly m distinct edges, each pair equally likely."""
    total = n_u * n_v
    m = min(m, total)
    if m * 2 > total:
        # dense: rank all pairs by a random key and keep the m smallest
        key = stream_u64(seed, 2, total)
        idx = np.argsort(key, kind="stable")[:m]
        return from_edges(n_u, n_v, idx // n_v, idx % n_v, name=name)

    def draw(pos, cnt):
        r = stream_u64(seed, 3, cnt, pos)
        return (r % np.uint64(total)).astype(np.int64)

    keys = _distinct_pairs(draw, m, n_v, seed)
    return from_edges(n_u, n_v, keys // n_v, keys % n_v, name=name)


def _capped_weights(n: int, gamma: float, total: float, cap: float) -> np.ndarray:
    """Power-law weights w_i ~ i^(-1/(gamma-1)), scaled to sum `total`, water-filled at `cap`."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    w *= total / w.sum()
    capped = np.zeros(n, dtype=bool)
    for _ in range(100):
        over = w > cap
        if not over.any():
            break
        capped |= over
        w[capped] = cap
        free = ~capped
        rest = total - cap * capped.sum()
        if rest <= 0 or not free.any():
            break
        w[free] *= rest / w[free].sum()
    return w


def _inverse_cdf_sampler(w: np.ndarray):
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    def sample(u: np.ndarray) -> np.ndarray:
        return np.minimum(np.searchsorted(cdf, u, side="right"), w.size - 1)
    return sample


def _permutation(n: int, seed: int, stream: int) -> np.ndarray:
    return np.argsort(stream_u64(seed, stream, n), kind="stable").astype(np.int64)


def chung_lu(n_u: int, n_v: int, m: int, gamma_u: float, gamma_v: float, seed: int,
             cap_u: float | None = None, cap_v: float | None = None, shuffle: bool = True,
             name: str = "") -> BiGraph:
    """Chung-Lu bipartite graph by ball dropping: each draw picks u with probability
    proportional to w^U and v proportional to w^V; duplicates are dropped and draws
    continue until exactly m distinct edges exist.  Weights are power laws with the
    given exponents, water-filled at a cap.  The default cap is floor(sqrt(m / 10)), so
    that no pair has edge probability w_u w_v / m above 0.1: with the admissibility cap
    floor(sqrt(m)) the top vertices of both sides form an almost complete block, whose
    maximal bicliques are too many to enumerate."""
    m = min(m, n_u * n_v)
    cap = float(math.isqrt(max(m // 10, 1)))
    cu = min(cap if cap_u is None else cap_u, n_v)
    cv = min(cap if cap_v is None else cap_v, n_u)
    wu = _capped_weights(n_u, gamma_u, m, cu)
    wv = _capped_weights(n_v, gamma_v, m, cv)
    su, sv = _inverse_cdf_sampler(wu), _inverse_cdf_sampler(wv)

    def draw(pos, cnt):
        a = su(stream_uniform(seed, 4, cnt, pos))
        b = sv(stream_uniform(seed, 5, cnt, pos))
        return a.astype(np.int64) * n_v + b.astype(np.int64)

    keys = _distinct_pairs(draw, m, n_v, seed)
    us, vs = keys // n_v, keys % n_v
    if shuffle:
        us = _permutation(n_u, seed, 6)[us]
        vs = _permutation(n_v, seed, 7)[vs]
    return from_edges(n_u, n_v, us, vs, name=name)


def planted_bicliques(n_u: int, n_v: int, count: int, lo: int, hi: int, seed: int) -> BiGraph:
    """`count` complete K_{a,b}, a and b uniform in [lo, hi], on uniformly random vertex
    sets (no repeated vertex inside one block)."""
    us, vs = [], []
    sizes = stream_u64(seed, 8, 2 * count)
    for k in range(count):
        a = lo + int(sizes[2 * k] % np.uint64(hi - lo + 1))
        b = lo + int(sizes[2 * k + 1] % np.uint64(hi - lo + 1))
        pu = np.argsort(stream_u64(seed, 100 + 2 * k, n_u), kind="stable")[:a]
        pv = np.argsort(stream_u64(seed, 101 + 2 * k, n_v), kind="stable")[:b]
        us.append(np.repeat(pu, b))
        vs.append(np.tile(pv, a))
    return from_edges(n_u, n_v, np.concatenate(us), np.concatenate(vs), dedupe=True)


# ----------------------------------------------------------------------------- the five workloads

def config1(seed: int = _BASE_SEED + 1) -> BiGraph:
    """Erdos-Renyi bipartite |U|=200, |V|=300, edge probability 0.05 (about 3k edges)."""
    return erdos_renyi_pairs(200, 300, 0.05, seed, name="er-200x300-p0.05")


def config2(seed: int = _BASE_SEED + 2, scale: float = 1.0) -> BiGraph:
    """Chung-Lu power law |U|=100k, |V|=50k, 1M edges, exponent 2.1 on both sides."""
    n_u, n_v, m = int(100_000 * scale), int(50_000 * scale), int(1_000_000 * scale)
    return chung_lu(n_u, n_v, m, 2.1, 2.1, seed, name=f"chunglu-{n_u}x{n_v}-m{m}-g2.1")


def config3(seed: int = _BASE_SEED + 3, scale: float = 1.0) -> BiGraph:
    """Skewed dense |U|=20k, |V|=5k, about 2M edges: Chung-Lu background (exponent 1.9,
    cap floor(sqrt(2M / 10)) = 447) united with 50 planted K_{a,b}, a, b uniform in [10, 40]."""
    n_u, n_v, m = int(20_000 * scale), int(5_000 * scale), int(2_000_000 * scale)
    planted = planted_bicliques(n_u, n_v, 50, 10, 40, seed)
    cap = float(math.isqrt(m // 10))
    # the background is sized so that background u planted has about m edges
    bg = chung_lu(n_u, n_v, m - planted.n_edges, 1.9, 1.9, seed, cap_u=cap, cap_v=cap)
    g = union(bg, planted, name=f"skewed-{n_u}x{n_v}-m{m}-g1.9-planted50")
    return g


def config4_graph(i: int, base_seed: int = _BASE_SEED) -> BiGraph:
    """Graph i of the batched workload: |U|, |V| log-uniform in [50, 2000], density
    uniform in [0.01, 0.1], Erdos-Renyi or Chung-Lu (exponent 2.1) with probability 1/2,
    E = round(density * |U| * |V|)."""
    seed = base_seed * 10_000 + i
    r = stream_uniform(seed, 9, 4)
    n_u = int(round(math.exp(math.log(50) + r[0] * (math.log(2000) - math.log(50)))))
    n_v = int(round(math.exp(math.log(50) + r[1] * (math.log(2000) - math.log(50)))))
    dens = 0.01 + 0.09 * r[2]
    m = max(1, int(round(dens * n_u * n_v)))
    if r[3] < 0.5:
        return erdos_renyi_m(n_u, n_v, m, seed, name=f"b{i}-er-{n_u}x{n_v}-m{m}")
    return chung_lu(n_u, n_v, m, 2.1, 2.1, seed, name=f"b{i}-cl-{n_u}x{n_v}-m{m}")


def config4_batch(n: int = 4096, base_seed: int = _BASE_SEED) -> List[BiGraph]:
    return [config4_graph(i, base_seed) for i in range(n)]


def config5_arrivals(n: int, rate: float, seed: int = _BASE_SEED + 5,
                     big_frac: float = 0.1, big_max_u: int = 200_000,
                     big_min_u: int = 20_000) -> List[Tuple[float, tuple]]:
    """Arrival times and graph specifications of the serving workload (see config5_requests);
    config5_build turns a specification into its graph, so that the graphs can be generated
    in parallel."""
    r = stream_uniform(seed, 10, 3 * n)
    t = 0.0
    out = []
    for k in range(n):
        t += -math.log(1.0 - r[3 * k]) / rate
        if r[3 * k + 1] < big_frac:
            lu = math.log(big_min_u) + r[3 * k + 2] * (math.log(big_max_u) - math.log(big_min_u))
            n_u = int(round(math.exp(lu)))
            out.append((t, ("big", k, n_u, seed)))
        else:
            out.append((t, ("small", k, 0, seed)))
    return out


def config5_build(spec: tuple) -> BiGraph:
    kind, k, n_u, seed = spec
    if kind == "big":
        n_v = n_u // 2
        m = min(5_000_000, 25 * n_u)
        return chung_lu(n_u, n_v, m, 2.1, 2.1, seed * 1000 + k, name=f"req{k}-cl-{n_u}x{n_v}")
    return config4_graph(k, base_seed=seed)


def config5_requests(n: int, rate: float, seed: int = _BASE_SEED + 5,
                     big_frac: float = 0.1, big_max_u: int = 200_000,
                     big_min_u: int = 20_000) -> List[Tuple[float, BiGraph]]:
    """Serving workload: Poisson arrivals at `rate` requests/s; each request is a batched-
    workload graph with probability 1 - big_frac, else a Chung-Lu graph (exponent 2.1)
    with |U| log-uniform in [big_min_u, big_max_u], |V| = |U|/2, E = min(5e6, 25 |U|).
    Returns (arrival time in seconds, graph) pairs in arrival order."""
    return [(t, config5_build(spec)) for t, spec in
            config5_arrivals(n, rate, seed, big_frac, big_max_u, big_min_u)]


def wide_hubs(n_u: int, n_v: int, hub_degrees: Sequence[int], p: float, seed: int, name: str = "") -> BiGraph:
    """Top-level candidates of any degree: hubs u_0 .. u_{h-1} of U whose neighbourhoods are
    random subsets of V of the given sizes, plus an Erdos-Renyi background on the other
    vertices of U (each pair an edge with probability p).  With |U| < |V| the candidates are
    U, so a hub's neighbour set is as wide as its degree."""
    h = len(hub_degrees)
    us, vs = [], []
    for j, d in enumerate(hub_degrees):
        perm = np.argsort(stream_u64(seed, 10 + j, n_v), kind="stable")
        sel = np.sort(perm[:d])
        us.append(np.full(d, j, dtype=np.int64))
        vs.append(sel.astype(np.int64))
    r = stream_uniform(seed, 9, (n_u - h) * n_v)
    idx = np.nonzero(r < p)[0]
    us.append(idx // n_v + h)
    vs.append(idx % n_v)
    return from_edges(n_u, n_v, np.concatenate(us), np.concatenate(vs),
                      name=name or f"hubs{n_u}x{n_v}s{seed}")


# ----------------------------------------------------------------------------- closed-form families

def hub_lists(n: int) -> BiGraph:
    """A hub u0 adjacent to n candidates v_0..v_{n-1} of degree 1 and to x = v_n, which is
    also adjacent to u1; z = v_{n+1} is adjacent to u1 and u2.  |U| = n + 3 > |V| = n + 2, so
    V holds the candidates, and the top-level list of x has n earlier-ranked entries.  Its
    maximal bicliques are ({u0}, {v_0..v_n}), ({u1}, {x, z}), ({u0, u1}, {x}) and
    ({u1, u2}, {z})."""
    us = [0] * (n + 1) + [1, 1, 2]
    vs = list(range(n + 1)) + [n, n + 1, n + 1]
    return from_edges(n + 3, n + 2, us, vs, name=f"hub{n}")


def hub_lists_bicliques(n: int) -> List[Tuple[Tuple[int, ...], Tuple[int, ...]]]:
    """The four maximal bicliques of hub_lists(n), in canonical order."""
    return sorted([((0,), tuple(range(n + 1))), ((1,), (n, n + 1)), ((0, 1), (n,)), ((1, 2), (n + 1,))])


def complete(m: int, n: int) -> BiGraph:
    us = np.repeat(np.arange(m), n)
    vs = np.tile(np.arange(n), m)
    return from_edges(m, n, us, vs, name=f"K{m},{n}")


def perfect_matching(n: int) -> BiGraph:
    return from_edges(n, n, np.arange(n), np.arange(n), name=f"matching{n}")


def crown(n: int) -> BiGraph:
    """K_{n,n} minus a perfect matching."""
    us = np.repeat(np.arange(n), n)
    vs = np.tile(np.arange(n), n)
    keep = us != vs
    return from_edges(n, n, us[keep], vs[keep], name=f"crown{n}")


def private_neighbours(m: int, n: int) -> BiGraph:
    """K_{m,n} (U = u_0 .. u_{m-1}, V = w_0 .. w_{n-1}) plus one private neighbour p_i of each
    u_i (V id n + i)."""
    us, vs = [], []
    for i in range(m):
        us.extend([i] * (n + 1))
        vs.extend(list(range(n)) + [n + i])
    return from_edges(m, n + m, us, vs, name=f"private{m}x{n}")


def chain(n: int) -> BiGraph:
    """Half graph: N(u_i) = {v_0 .. v_i}."""
    us, vs = [], []
    for i in range(n):
        us.extend([i] * (i + 1))
        vs.extend(range(i + 1))
    return from_edges(n, n, us, vs, name=f"chain{n}")


def complete_minus_edge(m: int, n: int, u: int = 0, v: int = 0) -> BiGraph:
    us = np.repeat(np.arange(m), n)
    vs = np.tile(np.arange(n), m)
    keep = ~((us == u) & (vs == v))
    return from_edges(m, n, us[keep], vs[keep], name=f"K{m},{n}-e")


def edgeless(m: int, n: int) -> BiGraph:
    return from_edges(m, n, [], [], name=f"empty{m},{n}")


def disjoint_union(a: BiGraph, b: BiGraph) -> BiGraph:
    ua, va = a.edges()
    ub, vb = b.edges()
    return from_edges(a.n_u + b.n_u, a.n_v + b.n_v, np.concatenate([ua, ub + a.n_u]),
                      np.concatenate([va, vb + a.n_v]), name=f"({a.name})+({b.name})")


def transpose(g: BiGraph) -> BiGraph:
    return BiGraph(g.n_v, g.n_u, g.v_off.copy(), g.v_adj.copy(), g.u_off.copy(), g.u_adj.copy(),
                   name=f"T({g.name})")


def relabel(g: BiGraph, perm_u: Sequence[int], perm_v: Sequence[int]) -> BiGraph:
    """New id of u is perm_u[u], of v is perm_v[v]."""
    us, vs = g.edges()
    pu = np.asarray(perm_u, dtype=np.int64)
    pv = np.asarray(perm_v, dtype=np.int64)
    return from_edges(g.n_u, g.n_v, pu[us], pv[vs], name=f"relabel({g.name})")


def random_small(n_u: int, n_v: int, p: float, seed: int) -> BiGraph:
    return erdos_renyi_pairs(n_u, n_v, p, seed, name=f"er{n_u}x{n_v}p{p:.2f}s{seed}")
