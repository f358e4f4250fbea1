"""Pins of the CPU oracle against things other than itself (no GPU needed).

* the definition of a maximal biclique written out (brute force over subsets, section II-A);
* the closure route: A-sides are the non-empty intersections of neighbour rows;
* closed forms of graph families whose maximal bicliques are known by hand;
* invariants: transpose, relabelling, choice of candidate side, splitting the top level;
* the SplitMix64 output function against its published first outputs.
"""
import itertools
import json
import os

import numpy as np
import pytest

import graphgen as gg

MASK = (1 << 64) - 1
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_mix_matches_published_splitmix64(orc):
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if l.startswith("0x")]
    k = 0x9E3779B97F4A7C15
    for i, want in enumerate(vals, start=1):
        assert orc.mix64((i * k) & MASK) == want


def test_hash_properties(orc):
    # independent of the order of vertices inside a side
    assert orc.hash_pair([3, 1, 2], [9, 4]) == orc.hash_pair([1, 2, 3], [4, 9])
    # orientation matters: the U-side and V-side terms differ
    assert orc.hash_pair([1], [2]) != orc.hash_pair([2], [1])
    # different bicliques give different terms (no trivial collisions)
    seen = {orc.hash_pair([a], [b]) for a in range(20) for b in range(20)}
    assert len(seen) == 400


def _rand_graph(seed):
    rng = np.random.default_rng(seed)
    nu = int(rng.integers(1, 13))
    nv = int(rng.integers(1, 15))
    p = float(rng.random())
    return gg.random_small(nu, nv, p, seed)


@pytest.mark.parametrize("chunk", range(8))
def test_mbea_equals_brute_force(orc, chunk):
    for seed in range(chunk * 60, chunk * 60 + 60):
        g = _rand_graph(seed)
        a = orc.mbea(g, want_list=True)
        b = orc.brute(g)
        assert a["list"] == b["list"], (seed, g.name)
        assert a["count"] == b["count"] and a["hash"] == b["hash"] and a["out_ints"] == b["out_ints"]
        assert a["nodes"] == a["count"] + a["nonmaximal"]


def test_mbea_equals_closure_on_workload1(orc):
    g = gg.config1()
    a = orc.mbea(g, want_list=True)
    c = orc.closure(g)
    assert a["list"] == c["list"]
    assert a["hash"] == c["hash"] and a["count"] == c["count"] == len(c["list"])


@pytest.mark.parametrize("seed", range(6))
def test_mbea_equals_closure_medium(orc, seed):
    g = gg.random_small(40 + seed * 7, 30 + seed * 5, 0.15, 1000 + seed)
    a = orc.mbea(g, want_list=True)
    c = orc.closure(g)
    assert a["list"] == c["list"]


# ----------------------------------------------------------------------------- closed forms

def _formula_check(orc, g, expected):
    r = orc.mbea(g, want_list=True)
    exp = sorted((tuple(sorted(a)), tuple(sorted(b))) for a, b in expected)
    assert r["list"] == exp
    assert r["count"] == len(exp)
    h = 0
    for a, b in exp:
        h = (h + orc.hash_pair(a, b)) & MASK
    assert r["hash"] == h
    return r


@pytest.mark.parametrize("m,n", [(1, 1), (1, 5), (4, 3), (7, 7), (30, 50)])
def test_complete_has_one(orc, m, n):
    _formula_check(orc, gg.complete(m, n), [(range(m), range(n))])


@pytest.mark.parametrize("n", [1, 2, 5, 40])
def test_matching_has_n(orc, n):
    _formula_check(orc, gg.perfect_matching(n), [([i], [i]) for i in range(n)])


@pytest.mark.parametrize("n", [2, 3, 5, 8, 12])
def test_crown_has_2n_minus_2(orc, n):
    exp = []
    for k in range(1, n):
        for a in itertools.combinations(range(n), k):
            exp.append((a, [j for j in range(n) if j not in a]))
    r = _formula_check(orc, gg.crown(n), exp)
    assert r["count"] == 2 ** n - 2


@pytest.mark.parametrize("n", [1, 4, 25])
def test_chain_has_n(orc, n):
    _formula_check(orc, gg.chain(n), [(range(i, n), range(i + 1)) for i in range(n)])


@pytest.mark.parametrize("m,n", [(2, 2), (3, 5), (9, 4)])
def test_complete_minus_edge_has_two(orc, m, n):
    _formula_check(orc, gg.complete_minus_edge(m, n), [(range(1, m), range(n)), (range(m), range(1, n))])


def test_edgeless_has_none(orc):
    r = orc.mbea(gg.edgeless(5, 7))
    assert r["count"] == 0 and r["hash"] == 0 and r["nodes"] == 0


def test_disjoint_union_adds(orc):
    a, b = gg.crown(5), gg.chain(6)
    u = gg.disjoint_union(a, b)
    ra, rb, ru = orc.mbea(a), orc.mbea(b), orc.mbea(u)
    assert ru["count"] == ra["count"] + rb["count"]
    ex = [(x, y) for x, y in orc.mbea(a, want_list=True)["list"]]
    ex += [(tuple(i + a.n_u for i in x), tuple(j + a.n_v for j in y)) for x, y in orc.mbea(b, want_list=True)["list"]]
    assert orc.mbea(u, want_list=True)["list"] == sorted(ex)


# ----------------------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", range(5))
def test_transpose_invariance(orc, seed):
    g = gg.random_small(35, 25, 0.2, 500 + seed)
    a = orc.mbea(g, want_list=True)["list"]
    t = orc.mbea(gg.transpose(g), want_list=True)["list"]
    assert sorted((b, a_) for a_, b in a) == t


@pytest.mark.parametrize("seed", range(5))
def test_relabel_invariance(orc, seed):
    g = gg.random_small(30, 30, 0.2, 600 + seed)
    rng = np.random.default_rng(seed)
    pu, pv = rng.permutation(g.n_u), rng.permutation(g.n_v)
    a = orc.mbea(g, want_list=True)["list"]
    r = orc.mbea(gg.relabel(g, pu, pv), want_list=True)["list"]
    assert sorted((tuple(sorted(pu[list(x)])), tuple(sorted(pv[list(y)]))) for x, y in a) == r


@pytest.mark.parametrize("seed", range(5))
def test_candidate_side_invariance(orc, seed):
    g = gg.random_small(28, 33, 0.18, 700 + seed)
    a = orc.mbea(g, side=1, want_list=True)
    b = orc.mbea(g, side=2, want_list=True)
    assert a["list"] == b["list"] and a["hash"] == b["hash"]


def test_top_level_split_adds_up(orc):
    g = gg.config1()
    whole = orc.mbea(g)
    n = orc.num_roots(g)
    cuts = [0, 3, 50, 51, n // 2, n - 1, n]
    parts = [orc.mbea(g, rank_lo=cuts[i], rank_hi=cuts[i + 1]) for i in range(len(cuts) - 1)]
    for k in ("count", "nodes", "nonmaximal", "bytes_alg", "out_ints"):
        assert sum(p[k] for p in parts) == whole[k]
    assert sum(p["hash"] for p in parts) & MASK == whole["hash"]
    assert max(p["max_depth"] for p in parts) == whole["max_depth"]
    par = orc.mbea_parallel(g, threads=4)
    assert par["count"] == whole["count"] and par["hash"] == whole["hash"]


def test_golden_workload1_reproduces(orc):
    gold = json.load(open(os.path.join(GOLDEN, "workloads.json")))["config1"]
    r = orc.mbea(gg.config1())
    for k in ("count", "hash", "nodes", "nonmaximal", "bytes_alg", "max_depth"):
        assert r[k] == gold[k], k


def test_degree_zero_vertices_are_skipped(orc):
    # an isolated vertex on either side changes nothing (reading: no empty-sided pairs)
    g = gg.complete(3, 4)
    us, vs = g.edges()
    h = gg.from_edges(5, 6, us, vs)
    assert orc.mbea(h, want_list=True)["list"] == orc.mbea(g, want_list=True)["list"]
    assert orc.brute(h)["list"] == orc.mbea(h, want_list=True)["list"]


def test_hub_lists_closed_form(orc):
    """hub_lists(n): the closure (definition) and the MBEA oracle give the four bicliques."""
    for n in (1, 3, 6, 20):
        g = gg.hub_lists(n)
        want = gg.hub_lists_bicliques(n)
        assert orc.closure(g)["list"] == want
        r = orc.mbea(g, want_list=True)
        assert r["list"] == want and r["count"] == 4
