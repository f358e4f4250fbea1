"""Pins of the oracle's iMBEA variant: MBEA with the candidate pruning of section II-C (a
candidate that joins L' during x's maximal expansion and has no neighbour in R outside R'
leaves P and joins Q with x).

* The answer: equal to the definition (brute force) on small random graphs, and to the plain
  search on medium ones (count, hash, records).
* The tree: never larger than the plain search's (nodes, non-maximal nodes, depth), and node
  counts derived by hand for families whose trees can be followed on paper (the derivations
  are in the docstrings); the plain search's tallies for them are pinned by hand in
  test_oracle_pins.py.
* Rank ranges: the tallies of disjoint top-level ranges add up to the whole run's.
"""
import numpy as np
import pytest

import graphgen as gg

TALLY = ("count", "hash", "out_ints", "nodes", "nonmaximal", "bytes_alg", "bytes_rs")


@pytest.mark.parametrize("chunk", range(4))
def test_imbea_equals_brute_force(orc, chunk):
    rng = np.random.default_rng(700 + chunk)
    for k in range(50):
        nu, nv = int(rng.integers(1, 13)), int(rng.integers(1, 30))
        g = gg.random_small(nu, nv, float(rng.uniform(0.1, 0.9)), 7000 + 100 * chunk + k)
        b = orc.brute(g)
        r = orc.imbea(g, want_list=True)
        assert (r["count"], r["hash"], r["out_ints"]) == (b["count"], b["hash"], b["out_ints"]), g.name
        assert r["list"] == b["list"], g.name


@pytest.mark.parametrize("seed", range(6))
def test_imbea_same_answer_smaller_tree(orc, seed):
    rng = np.random.default_rng(seed)
    nu, nv = int(rng.integers(20, 70)), int(rng.integers(20, 90))
    g = gg.random_small(nu, nv, float(rng.uniform(0.05, 0.4)), 7500 + seed)
    # duplicate some candidates' rows so that twins (equal neighbourhoods) occur
    us, vs = g.edges()
    extra_u, extra_v = [], []
    for j in range(0, min(nu, 12)):
        row = g.row_u(j)
        extra_u += [nu + j] * len(row)
        extra_v += list(row)
    h = gg.from_edges(nu + min(nu, 12), nv, np.concatenate([us, extra_u]).astype(np.int64),
                      np.concatenate([vs, extra_v]).astype(np.int64))
    for gr in (g, h, gg.transpose(h)):
        p = orc.mbea(gr, want_list=True)
        r = orc.imbea(gr, want_list=True)
        assert (r["count"], r["hash"], r["list"]) == (p["count"], p["hash"], p["list"])
        assert r["nodes"] <= p["nodes"] and r["nonmaximal"] <= p["nonmaximal"]
        assert r["max_depth"] <= p["max_depth"]
        assert r["nodes"] - r["nonmaximal"] == r["count"]
    # the twins leave P: the duplicated graph's tree is strictly smaller
    assert orc.imbea(h)["nodes"] < orc.mbea(h)["nodes"]


def test_hand_worked_example(orc):
    """U = {u0, u1, u2}, V = {v0, v1, v2}; N(u0) = N(u1) = {v0, v1}, N(u2) = {v1, v2}.  The
    candidates are U (a tie), taken u0, u1, u2 (degree 2 each, ties by id).

    Plain: u0 is maximal ({u0, u1} x {v0, v1}; u1 joins L', u2 meets R' in v1 and forms P'),
    its child node u2 is maximal ({u0, u1, u2} x {v1}); u1 is not maximal (u0 in Q holds
    {v0, v1}); u2 is maximal ({u2} x {v1, v2}).  4 nodes, 1 non-maximal, 3 bicliques.
    iMBEA: u1 joins L' at u0 and has no neighbour in R outside R' = {v0, v1}, so it leaves P
    with u0 and is never taken: 3 nodes, none non-maximal, the same 3 bicliques.

    Bytes, 4 [(2 + deg x) + min(rs, fw) + |P| + |Q| + |R'| + |P'| + |Q'|] per node with the P
    and Q of that moment (degrees: u 2, 2, 2; v0 2, v1 3, v2 1):
      u0 (top): rs = 4 + 5 = 9, fw = 4 + 4 = 8; |P| = 2, |Q| = 0, |R'| = 2, |P'| = 1 -> 68;
      u2 below u0: R'' = {v1}, rs = 5, fw = 0; |R''| = 1 -> 20;
      plain u1: rs = 9, fw = 4 (u2) + 4 (u0) = 8; |P| = 1, |Q| = 1, |R'| = 2, not maximal -> 64;
      u2 (top), Q = {u0, u1}: rs = 5 + 3 = 8, fw = 8; |Q| = 2, |R'| = 2, |Q'| = 2 -> 72.
    Plain 68 + 20 + 64 + 72 = 224; iMBEA 68 + 20 + 72 = 160."""
    g = gg.from_edges(3, 3, [0, 0, 1, 1, 2, 2], [0, 1, 0, 1, 1, 2])
    p = orc.mbea(g)
    r = orc.imbea(g)
    assert (p["nodes"], p["nonmaximal"], p["count"], p["bytes_alg"], p["max_depth"]) == (4, 1, 3, 224, 2)
    assert (r["nodes"], r["nonmaximal"], r["count"], r["bytes_alg"], r["max_depth"]) == (3, 0, 3, 160, 2)
    assert r["hash"] == p["hash"]


@pytest.mark.parametrize("m,n", [(1, 1), (3, 4), (7, 2), (12, 30)])
def test_complete_one_node(orc, m, n):
    """K_{m,n}: the first candidate is maximal with R' = the whole other side, and every other
    candidate joins L' with no neighbour outside R': all of them leave P.  One node, maximal;
    the plain search takes every candidate (min(m, n) nodes, all but the first non-maximal)."""
    r = orc.imbea(gg.complete(m, n))
    assert (r["nodes"], r["nonmaximal"], r["max_depth"], r["count"]) == (1, 0, 1, 1)
    assert orc.mbea(gg.complete(m, n))["nodes"] == min(m, n)


@pytest.mark.parametrize("blocks", [[(2, 3)], [(2, 3), (4, 1), (3, 3)], [(5, 6), (1, 1), (2, 9), (7, 4)]])
def test_disjoint_complete_blocks(orc, blocks):
    """A disjoint union of complete blocks K_{a,b}: in each block the first candidate taken is
    maximal (no candidate of another block meets its neighbourhood) and the rest of its
    block leaves P with it; nothing meets R' outside the block, so no node has children.  One
    maximal node per block."""
    g = gg.complete(*blocks[0])
    for a, b in blocks[1:]:
        g = gg.disjoint_union(g, gg.complete(a, b))
    r = orc.imbea(g)
    assert (r["nodes"], r["nonmaximal"], r["max_depth"], r["count"]) == (len(blocks), 0, 1, len(blocks))


@pytest.mark.parametrize("n", [3, 6, 9])
def test_twin_free_families_keep_the_plain_tree(orc, n):
    """Perfect matching, crown and chain: no candidate that joins some L' has its neighbourhood
    within R equal to R' (matching: no joiners; crown: a joiner would need its missing
    partner inside the node's L, which never holds; chain: every joiner has neighbours outside
    R' = N(x) at the top level), so nothing leaves P and the tree is the plain one."""
    for g in (gg.perfect_matching(n), gg.crown(n), gg.chain(n)):
        p = orc.mbea(g)
        r = orc.imbea(g)
        for k in TALLY + ("max_depth",):
            assert r[k] == p[k], (g.name, k)


@pytest.mark.parametrize("seed", range(3))
def test_rank_ranges_add_up(orc, seed):
    g = gg.random_small(40, 55, 0.25, 7900 + seed)
    us, vs = g.edges()
    # copies u40 .. u49 of the rows of u0 .. u9: twins that the range cuts separate
    cu, cv = [], []
    for j in range(10):
        row = g.row_u(j)
        cu += [40 + j] * len(row)
        cv += list(row)
    h = gg.from_edges(50, 55, np.concatenate([us, cu]).astype(np.int64), np.concatenate([vs, cv]).astype(np.int64))
    whole = orc.imbea(h)
    n = orc.num_roots(h)
    cuts = [0, n // 3, n // 2, n - 2, n]
    parts = [orc.imbea(h, rank_lo=a, rank_hi=b) for a, b in zip(cuts[:-1], cuts[1:])]
    for k in TALLY:
        assert sum(p[k] for p in parts) % (1 << 64) == whole[k] % (1 << 64), k
    assert max(p["max_depth"] for p in parts) == whole["max_depth"]
