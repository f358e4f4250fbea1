"""Pins of the oracle's pivot variant: MBEA with the pivot pruning of section II-C.  In every
list below the top level the candidate p of the largest count (the first such) is taken
first, and the candidates whose neighbourhoods within R lie inside p's are covered: never
taken at that node, candidates for p's node, Q entries for the nodes after them.

* The answer: equal to the definition (brute force) on small random graphs, and to the plain
  search on medium ones (count, hash, records).
* The tree: node counts, depths and byte tallies derived by hand for two small graphs and a
  family (the derivations are in the docstrings); the plain tree wherever no candidate covers
  another; nodes = bicliques + non-maximal nodes.
* Rank ranges: the top-level list keeps its order, so ranges add up to the whole run.
"""
import numpy as np
import pytest

import graphgen as gg

TALLY = ("count", "hash", "out_ints", "nodes", "nonmaximal", "bytes_alg", "bytes_rs")


def private_neighbours(m, n):
    return gg.private_neighbours(m, n)


@pytest.mark.parametrize("chunk", range(4))
def test_pivot_equals_brute_force(orc, chunk):
    rng = np.random.default_rng(900 + chunk)
    for k in range(50):
        nu, nv = int(rng.integers(1, 13)), int(rng.integers(1, 30))
        g = gg.random_small(nu, nv, float(rng.uniform(0.1, 0.9)), 9000 + 100 * chunk + k)
        b = orc.brute(g)
        r = orc.pivot(g, want_list=True)
        assert (r["count"], r["hash"], r["out_ints"]) == (b["count"], b["hash"], b["out_ints"]), g.name
        assert r["list"] == b["list"], g.name
        assert r["nodes"] - r["nonmaximal"] == r["count"]


@pytest.mark.parametrize("seed", range(6))
def test_pivot_same_answer_as_plain(orc, seed):
    rng = np.random.default_rng(seed)
    nu, nv = int(rng.integers(20, 70)), int(rng.integers(20, 90))
    g = gg.random_small(nu, nv, float(rng.uniform(0.05, 0.4)), 9500 + seed)
    us, vs = g.edges()
    # rows copied and rows cut down to subsets: candidates that cover others
    eu, ev = [], []
    for j in range(min(nu, 12)):
        row = g.row_u(j)
        keep = row if j % 2 == 0 else row[: max(1, len(row) // 2)]
        eu += [nu + j] * len(keep)
        ev += list(keep)
    h = gg.from_edges(nu + min(nu, 12), nv, np.concatenate([us, eu]).astype(np.int64),
                      np.concatenate([vs, ev]).astype(np.int64))
    for gr in (g, h, gg.transpose(h)):
        p = orc.mbea(gr, want_list=True)
        r = orc.pivot(gr, want_list=True)
        assert (r["count"], r["hash"], r["out_ints"], r["list"]) == (p["count"], p["hash"], p["out_ints"], p["list"])
        assert r["nodes"] - r["nonmaximal"] == r["count"]


def test_hand_worked_example_deeper_tree(orc):
    """U = {x, y, z}, V = {0, .., 6}; N(x) = {0, 1, 2}, N(y) = {0, 1, 3, 4}, N(z) = {0, 5, 6}.
    Degrees: x 3, y 4, z 3; 0: 3, 1: 2, the others 1.  Top level (deg, id): x, z, y.

    x: R' = {0, 1, 2}; z meets it in {0} (1), y in {0, 1} (2): the list [z, y].
      Plain: z (R'' = {0}; y joins: ({x, z, y}, {0})), then y (R'' = {0, 1}; z in Q meets it
      in one vertex: ({x, y}, {0, 1})).
      Pivot: p = y covers z ({0} inside {0, 1}): the list [y, z*].  y (R'' = {0, 1}; z meets
      it in one vertex: P' = [z]), below it z (R''' = {0}: ({x, y, z}, {0}), depth 3); z* is
      passed over.
    z: R' = {0, 5, 6}, Q = {x} meets it in {0}: maximal; y meets it in {0}: the list [y]; y
      (R'' = {0}) is not maximal (x holds 0).
    y: R' = {0, 1, 3, 4}, Q = {x, z}: maximal, no list.
    Both trees: 6 nodes, 1 non-maximal, 5 bicliques; depth 2 plain, 3 pivot.

    Bytes, 4 [(2 + deg x) + min(rs, fw) + |P| + |Q| + |R'| + |P'| + |Q'|] per node (P: the
    entries after the candidate, Q: the node's Q and the entries before it):
      x: rs = 5 + 4 + 3 = 12, fw = 5 + 6 = 11; 5 + 2 + 0 + 3 + 2 + 0 = 12 -> 92;
      plain z: rs = 5, fw = 6; 5 + 1 + 0 + 1 = 7 -> 48;  plain y: rs = 9, fw = 5 (z);
      6 + 0 + 1 + 2 + 0 + 1 = 10 -> 60;
      pivot y: rs = 9, fw = 5 (z*); 6 + 1 + 0 + 2 + 1 = 10 -> 60;  pivot z (depth 3): rs = 5,
      fw = 0; 5 + 1 = 6 -> 24;
      z (top): rs = 11, fw = 6 + 5 = 11; 5 + 1 + 1 + 3 + 1 + 1 = 12 -> 92;  y below z: rs = 5,
      fw = 5 (x); not maximal, 6 + 0 + 1 + 1 = 8 -> 52;
      y (top): rs = 5 + 4 + 3 + 3 = 15, fw = 5 + 5 = 10; 6 + 0 + 2 + 4 + 0 + 2 = 14 -> 96.
    Plain 92 + 48 + 60 + 92 + 52 + 96 = 440; pivot 92 + 60 + 24 + 92 + 52 + 96 = 416."""
    g = gg.from_edges(3, 7, [0, 0, 0, 1, 1, 1, 1, 2, 2, 2], [0, 1, 2, 0, 1, 3, 4, 0, 5, 6])
    p = orc.mbea(g)
    r = orc.pivot(g)
    assert (p["nodes"], p["nonmaximal"], p["count"], p["max_depth"], p["bytes_alg"]) == (6, 1, 5, 2, 440)
    assert (r["nodes"], r["nonmaximal"], r["count"], r["max_depth"], r["bytes_alg"]) == (6, 1, 5, 3, 416)
    assert r["hash"] == p["hash"]


def test_hand_worked_example_covered_entries_in_q(orc):
    """U = {x, a, b, c}, V = {0, .., 6}; N(x) = {0, 1, 2}, N(a) = {0, 3, 4}, N(b) = {0, 1, 5},
    N(c) = {1, 2, 6}.  All candidates have degree 3 (top level x, a, b, c); degrees of V: 0 and
    1: 3, 2: 2, the others 1.

    x: R' = {0, 1, 2}: a meets it in {0}, b in {0, 1}, c in {1, 2}: the list [a, b, c].
      Pivot: p = b (the first of count 2) covers a but not c: [b, a*, c].  b (R'' = {0, 1},
      P' = [a, c]) with below it a ({x, b, a} x {0}) and c ({x, b, c} x {1}, a in Q); a* is
      passed over; c (R'' = {1, 2}, Q = {b, a*}: b meets it, a does not) gives {x, c} x {1, 2}.
      Plain: a (b joins: {x, a, b} x {0}); b (Q = {a}; P' = [c], below it c: {x, b, c} x {1});
      c (Q = {a, b}).
    a, b, c at the top level: maximal; a's list [b] and b's list [c] are not maximal below them
    (x holds 0, resp. 1); c has no list.  Both: 10 nodes, 2 non-maximal, 8 bicliques, depth 3.

    Bytes (as in the first example):
      x 112 (rs 14, fw 15; 5 + 3 + 3 + 3 = 14);
      pivot b 84 (rs 10, fw 10; 5 + 2 + 2 + 2 = 11), a 48, c 48 (depth 3), c 76 (rs 9, fw 10:
      b and a* in Q; 5 + 0 + 2 + 2 + 0 + 1 = 10);
      plain a 52 (rs 5, fw 10; 5 + 2 + 1 = 8), b 84 (rs 10, fw 5 + 5; 5 + 1 + 1 + 2 + 1 + 1 = 11),
      c 48 (depth 3), c 76;
      a (top) 96, b below a 48, b (top) 108, c below b 52, c (top) 100.
    Plain 776, pivot 772.  Were the covered a* not a Q entry for c, c's node would count
    |Q| = 1 and fw = 5: 56 instead of 76."""
    g = gg.from_edges(4, 7, [0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3], [0, 1, 2, 0, 3, 4, 0, 1, 5, 1, 2, 6])
    p = orc.mbea(g)
    r = orc.pivot(g)
    assert (p["nodes"], p["nonmaximal"], p["count"], p["max_depth"], p["bytes_alg"]) == (10, 2, 8, 3, 776)
    assert (r["nodes"], r["nonmaximal"], r["count"], r["max_depth"], r["bytes_alg"]) == (10, 2, 8, 3, 772)
    assert r["hash"] == p["hash"]


@pytest.mark.parametrize("m,n", [(2, 3), (4, 3), (6, 5), (9, 2)])
def test_private_neighbour_family(orc, m, n):
    """K_{m,n} plus a private neighbour p_i of each u_i.  Every u_i has degree n + 1, so the
    top level is u_0 .. u_{m-1}, each maximal ({u_i} x W + p_i).  Below u_k the list holds
    u_{k+1} .. u_{m-1}, all meeting R' = W + p_k in W (twins).
      Plain: below u_0 the first is maximal (U x W, the rest join) and the other m - 2 are
      not (the first is in Q); below u_k (k >= 1) all m - 1 - k are not maximal (u_0 in Q'
      holds W).  Nodes m + m(m - 1)/2, non-maximal m(m - 1)/2 - 1.
      Pivot: the first covers the rest, so one node per list: below u_0 maximal, below u_k
      (1 <= k <= m - 2) not.  Nodes 2m - 1, non-maximal m - 2.
    Both: m + 1 bicliques, depth 2."""
    g = private_neighbours(m, n)
    p = orc.mbea(g)
    r = orc.pivot(g)
    assert (p["nodes"], p["nonmaximal"], p["count"], p["max_depth"]) == (m + m * (m - 1) // 2, m * (m - 1) // 2 - 1,
                                                                        m + 1, 2)
    assert (r["nodes"], r["nonmaximal"], r["count"], r["max_depth"]) == (2 * m - 1, m - 2, m + 1, 2)
    assert r["hash"] == p["hash"]


@pytest.mark.parametrize("n", [3, 6, 9])
def test_no_cover_keeps_the_plain_tree(orc, n):
    """Crown: below u_i the list entries meet R' = V - {v_i} in V - {v_i, v_j}, all of one
    count, none inside another: the pivot is the first entry and covers nothing, so the tree,
    bytes included, is the plain one.  Matching, chain and K_{m,n} have no lists below the top
    level."""
    for g in (gg.crown(n), gg.perfect_matching(n), gg.chain(n), gg.complete(n, n + 2)):
        p = orc.mbea(g)
        r = orc.pivot(g)
        for k in TALLY + ("max_depth",):
            assert r[k] == p[k], (g.name, k)


@pytest.mark.parametrize("seed", range(3))
def test_rank_ranges_add_up(orc, seed):
    g = gg.random_small(40, 55, 0.25, 9900 + seed)
    whole = orc.pivot(g)
    n = orc.num_roots(g)
    cuts = [0, n // 3, n // 2, n - 2, n]
    parts = [orc.pivot(g, rank_lo=a, rank_hi=b) for a, b in zip(cuts[:-1], cuts[1:])]
    for k in TALLY:
        assert sum(p[k] for p in parts) % (1 << 64) == whole[k] % (1 << 64), k
    assert max(p["max_depth"] for p in parts) == whole["max_depth"]
