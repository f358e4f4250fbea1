"""Pins of the oracle's hash and of its search-tree tallies against things outside the oracle.

* The hash.  hash_contract.py writes the hash out in plain Python integers.  Its mix is
  checked here against the published first outputs of SplitMix64, and the oracle's per-vertex
  terms are checked against the same published outputs (hu(a) is output 2a+1 of the
  generator started from state 0, hv(b) output 2b+2).  The oracle's h(A, B) must then equal
  the plain-integer one on fixed bicliques, and its total H must equal the plain-integer sum
  over the brute-force (definition) list.
* The tree.  Node, non-maximal-node, depth and byte tallies derived by hand for graph
  families whose MBEA trees can be followed on paper (complete, matching, chain, crown), with
  the candidate order of reading r5 (ascending count, ties in the parent's order; the top
  level by degree, ties by id).  The derivations are in the docstrings.
"""
import os

import numpy as np
import pytest

import graphgen as gg
import hash_contract as hc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _published():
    return [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if l.startswith("0x")]


def test_plain_mix_matches_published_outputs():
    vals = _published()
    assert len(vals) >= 5
    for k, want in enumerate(vals, start=1):
        assert hc.mix(k * hc.K) == want


def test_oracle_vertex_terms_are_published_outputs(orc):
    vals = _published()
    # output k of SplitMix64 from state 0 is mix(k K): hu(a) = output 2a+1, hv(b) = output 2b+2
    for k, want in enumerate(vals, start=1):
        if k % 2 == 1:
            assert orc.hash_u((k - 1) // 2) == want
        else:
            assert orc.hash_v((k - 2) // 2) == want


def _fixed_bicliques():
    """24 fixed (A, B) pairs: singletons, both sides long, large ids, one side much longer."""
    out = [([0], [0]), ([1], [0]), ([0], [1]), ([5], [7]), ([7], [5]), ([0, 1], [0]), ([0], [0, 1]),
           ([2, 3, 4], [9, 11]), ([100000], [49999]), ([2 ** 31 - 1], [0]), ([0], [2 ** 31 - 1])]
    rng = np.random.default_rng(12345)
    for k in range(13):
        na, nb = int(rng.integers(1, 40)), int(rng.integers(1, 300))
        a = sorted(set(rng.integers(0, 10 ** 6, na).tolist()))
        b = sorted(set(rng.integers(0, 10 ** 6, nb).tolist()))
        out.append((a, b))
    return out


def test_oracle_pair_hash_equals_plain_integers(orc):
    pairs = _fixed_bicliques()
    assert len(pairs) >= 20
    seen = set()
    for a, b in pairs:
        want = hc.h(a, b)
        assert orc.hash_pair(a, b) == want, (a[:3], b[:3])
        seen.add(want)
    assert len(seen) == len(pairs)


@pytest.mark.parametrize("seed", range(40))
def test_oracle_total_hash_is_the_plain_sum_over_the_definition(orc, seed):
    rng = np.random.default_rng(seed)
    g = gg.random_small(int(rng.integers(1, 14)), int(rng.integers(1, 16)), float(rng.uniform(0.1, 0.8)), 7000 + seed)
    b = orc.brute(g)  # the definition's list; its own hash is not used
    r = orc.mbea(g)
    assert r["count"] == len(b["list"])
    assert r["hash"] == hc.total(b["list"])


# ----------------------------------------------------------------------------- tree tallies

def _tallies(orc, g):
    r = orc.mbea(g)
    return r["count"], r["nodes"], r["nonmaximal"], r["max_depth"], r["bytes_alg"]


@pytest.mark.parametrize("m,n", [(1, 1), (1, 6), (6, 1), (3, 3), (4, 9), (9, 4), (12, 30)])
def test_complete_tree(orc, m, n):
    """K_{m,n}: the c = |C| candidates (C the smaller side, U on a tie; o = |O|) all have
    degree o, so they are taken by id.  The first has R' = O, every other candidate has count
    o = |R'| and joins L', and Q is empty: one maximal node, no child.  Each later candidate
    finds the first in Q with count o: non-maximal.  So c nodes, c - 1 non-maximal, depth 1.
    Bytes per node: 4 [2 + o + |P| + |Q| + |R'| + min(sum_{R'} (2 + c), sum_{P u Q} (2 + o))]
    with |P| + |Q| = c - 1 and |R'| = o, the same for every node."""
    c, o = (m, n) if m <= n else (n, m)
    per = 4 * (2 + o + (c - 1) + o + min(o * (2 + c), (c - 1) * (2 + o)))
    assert _tallies(orc, gg.complete(m, n)) == (1, c, c - 1, 1, c * per)


@pytest.mark.parametrize("n", [1, 2, 7, 40])
def test_matching_tree(orc, n):
    """Perfect matching: candidate u_i has R' = {v_i}, which no other candidate meets: every
    node is maximal with an empty child.  n nodes, none non-maximal, depth 1.  Bytes per node:
    4 [2 + 1 + (n - 1) + 1 + min(3, 3 (n - 1))]."""
    per = 4 * (2 + 1 + (n - 1) + 1 + min(3, 3 * (n - 1)))
    assert _tallies(orc, gg.perfect_matching(n)) == (n, n, 0, 1, n * per)


@pytest.mark.parametrize("n", [1, 2, 5, 25])
def test_chain_tree(orc, n):
    """Chain: N(u_i) = {v_0 .. v_i}, so deg u_i = i + 1 and deg v_j = n - j; candidates are
    taken u_0, u_1, ...  For u_i, R' = {v_0 .. v_i}; each earlier u_k (in Q) has count
    k + 1 < i + 1, so the node is maximal and Q' holds all i of them; each later candidate has
    count i + 1 and joins L'.  n nodes, all maximal, depth 1.  Bytes of node i:
    4 [2 + (i+1) + (n-1-i) + i + (i+1) + i + min(sum_{j<=i} (2 + n - j), sum_{k != i} (k + 3))]."""
    tot = 0
    for i in range(n):
        rs = sum(2 + n - j for j in range(i + 1))
        fw = sum(k + 3 for k in range(n) if k != i)
        tot += 4 * (2 + (i + 1) + (n - 1 - i) + i + (i + 1) + i + min(rs, fw))
    assert _tallies(orc, gg.chain(n)) == (n, n, 0, 1, tot)


@pytest.mark.parametrize("n", [2, 3, 6, 10])
def test_crown_tree(orc, n):
    """Crown: N(u_i) = V minus v_i.  At a node whose L is a set S of k vertices, R = V minus
    {v_s : s in S} and every other candidate or Q entry u_j misses exactly v_j of R.  Taking
    x gives |R'| = |R| - 1, and every other entry then has count |R| - 2 < |R'|: no Q entry
    holds R' (every node is maximal) and nobody joins L' (|L'| = depth).  The nodes are in
    one-to-one correspondence with the 2^n - 2 bicliques, and the deepest has |L'| = n - 1."""
    c, nodes, nonmax, depth, _ = _tallies(orc, gg.crown(n))
    assert (c, nodes, nonmax, depth) == (2 ** n - 2, 2 ** n - 2, 0, n - 1)
