"""The oracle's pins catch plausible mistakes.  Each test plants one mistake in a copy of the
oracle's C source (on the CPU), builds it, and runs the pins on the copy alone:

* the definition: count and canonical list against brute force over subsets (the brute-force
  route of the unmodified source, whose hash is not used);
* the hash: the copy's total against the plain-integer hash of the definition's list, and its
  h(A, B) against the plain-integer one on fixed bicliques (tests/hash_contract.py, whose mix
  is pinned to the published SplitMix64 outputs);
* the tree: node, non-maximal, depth and byte tallies of the hand-derived closed forms.

A mutant must fail at least one of them.  The plain search's mutants are planted outside the
variants' code, and each variant's mutants inside its own; a variant's pins are its
definition list (brute force) and its hand-derived trees (tests/test_oracle_imbea.py,
tests/test_oracle_pivot.py)."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import graphgen as gg
import hash_contract as hc

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "mbe_oracle.c")

MUTANTS = {
    "no_maximality_check": ("if (c == nRp) { maximal = 0; break; }", "if (0) { maximal = 0; break; }"),
    "no_expansion": ("if (c == nRp) Lp[nLp++] = v;", "if (0) Lp[nLp++] = v;"),
    "child_keeps_zero_counts": ("else if (c > 0) { Pp[nPp].key = c;", "else if (c >= 0) { Pp[nPp].key = c;"),
    "q_drops_partial": ("else if (c > 0) Qp[nQp++] = Q[i];", "else if (c > 1) Qp[nQp++] = Q[i];"),
    "x_not_moved_to_q": ("Q[nQ++] = x;", "(void)x;"),
    "intersect_off_by_one": ("while (i < nr && j < nn) {", "while (i < nr && j < nn - 1) {"),
    "hv_equals_hu": ("static uint64_t orc_hv(int32_t b) { return orc_mix(ORC_K * (2ULL * (uint64_t)b + 2ULL)); }",
                     "static uint64_t orc_hv(int32_t b) { return orc_hu(b); }"),
    "outer_mix_dropped": ("return orc_mix(sa + orc_mix(sb + ORC_K));", "return sa + orc_mix(sb + ORC_K);"),
    "inner_mix_dropped": ("return orc_mix(sa + orc_mix(sb + ORC_K));", "return orc_mix(sa + sb + ORC_K);"),
    "sides_swapped_in_hash": ("res->hash += orc_hash_pair(a, na, b, nb);", "res->hash += orc_hash_pair(b, nb, a, na);"),
    "node_counted_twice": ("g->res->nodes += 1;", "g->res->nodes += 2;"),
    "nonmaximal_not_counted": ("g->res->nonmaximal += 1;", "(void)0;"),
    "depth_starts_at_zero": ("Q, nQ, 1,", "Q, nQ, 0,"),
    "bytes_reverse_scan_only": ("g->res->bytes_alg += 4 * (base + (rs < fw ? rs : fw));",
                                "g->res->bytes_alg += 4 * (base + rs);"),
}


IMBEA_MUTANTS = {
    "imbea_moved_ones_still_taken": ("if (gone[ip]) continue;", "(void)gone;"),
    "imbea_every_joiner_moved": ("if (meet_count(R, nR, g->c_adj + g->c_off[v], (int32_t)deg_c(g, v)) == nRp) Cs[nC++] = i;",
                                 "Cs[nC++] = i;"),
    "imbea_tested_against_r_prime": ("if (meet_count(R, nR, g->c_adj", "if (meet_count(Rp, nRp, g->c_adj"),
    "imbea_moved_not_put_in_q": ("Q[nQ++] = P[Cs[k]].v;", "(void)0;"),
    "imbea_silent_prefix_counted": ("if (!silent) {\n            g->res->nodes += 1;", "{\n            g->res->nodes += 1;"),
}

PIVOT_MUTANTS = {
    "pivot_containment_reversed": ("in[i] = meet_count(Np, nNp, nv, dv) == meet_count(R, nR, nv, dv);",
                                   "in[i] = meet_count(Np, nNp, nv, dv) == nNp;"),
    "pivot_first_entry_not_largest": ("if (P0[i].key > P0[ip].key) ip = i;", "if (0) ip = i;"),
    "pivot_last_of_largest": ("if (P0[i].key > P0[ip].key) ip = i;", "if (P0[i].key >= P0[ip].key) ip = i;"),
    "pivot_covered_still_taken": ("if (covered[ip]) { Q[nQ++] = x; continue; }", "if (0) { Q[nQ++] = x; continue; }"),
    "pivot_covered_not_in_q": ("if (covered[ip]) { Q[nQ++] = x; continue; }", "if (covered[ip]) { continue; }"),
    "pivot_at_top_level": ("if (depth == 1 || nP < 2) {", "if (nP < 2) {"),
}

# each variant's code: (start marker, end marker) spans of the source
_SPANS = {
    "imbea": [("/* |R n N(v)| for ascending R and N(v)", "/*\n * Algorithm 1 with a pivot rule"),
              ("/*\n * As orc_mbea, with iMBEA's candidate pruning", "/*\n * As orc_mbea, with the pivot rule")],
    "pivot": [("/*\n * Algorithm 1 with a pivot rule", "/* Candidate side: 1 = U, 2 = V"),
              ("/*\n * As orc_mbea, with the pivot rule", "/* Number of top-level candidates")],
}


def _split(src):
    """(text outside the variants' code with placeholders, {variant: its pieces})."""
    pieces = {}
    for name, spans in _SPANS.items():
        for a, b in spans:
            i, j = src.index(a), src.index(b)
            pieces.setdefault(name, []).append(src[i:j])
            src = src[:i] + f"@@{name}{len(pieces[name]) - 1}@@" + src[j:]
    return src, pieces


def _join(outside, pieces):
    for name, ps in pieces.items():
        for k, p in enumerate(ps):
            outside = outside.replace(f"@@{name}{k}@@", p)
    return outside


def _plant(src, old, new, inside=None):
    """The source with old replaced by new, inside one variant's code (inside = its name) or
    outside every variant's; old must occur there exactly once."""
    outside, pieces = _split(src)
    if inside:
        assert sum(p.count(old) for p in pieces[inside]) == 1, old
        pieces[inside] = [p.replace(old, new) for p in pieces[inside]]
    else:
        assert outside.count(old) == 1, old
        outside = outside.replace(old, new)
    return _join(outside, pieces)


def _build(src_text):
    d = tempfile.mkdtemp(prefix="orc_mut_")
    c = os.path.join(d, "m.c")
    so = os.path.join(d, "m.so")
    open(c, "w").write(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", so, c])
    return so


class _Copy:
    """ctypes view of a built copy of the oracle source."""

    def __init__(self, orc, so):
        self.orc = orc
        lib = ctypes.CDLL(so)
        p32 = ctypes.POINTER(ctypes.c_int32)
        lib.orc_mbea.argtypes = [ctypes.c_int32, ctypes.c_int32, p32, p32, p32, p32, ctypes.c_int, ctypes.c_int64,
                                 ctypes.c_int64, p32, ctypes.c_int64, ctypes.POINTER(orc.OrcResult)]
        lib.orc_imbea.argtypes = lib.orc_mbea.argtypes
        lib.orc_pivot.argtypes = lib.orc_mbea.argtypes
        lib.orc_hash_pair.argtypes = [p32, ctypes.c_int64, p32, ctypes.c_int64]
        lib.orc_hash_pair.restype = ctypes.c_uint64
        self.lib, self.p32 = lib, p32

    def mbea(self, g, fn="orc_mbea", lo=0, hi=-1):
        arrs = [np.ascontiguousarray(x, dtype=np.int32) for x in (g.u_off, g.u_adj, g.v_off, g.v_adj)]
        buf = np.zeros(1 << 16, dtype=np.int32)
        res = self.orc.OrcResult()
        getattr(self.lib, fn)(g.n_u, g.n_v, *[a.ctypes.data_as(self.p32) for a in arrs], 0, lo, hi,
                              buf.ctypes.data_as(self.p32), buf.size, ctypes.byref(res))
        lst = self.orc.canonical(self.orc.split_records(buf, res.written)) if res.written >= 0 else None
        return res, lst

    def hash_pair(self, a, b):
        aa, bb = np.ascontiguousarray(a, dtype=np.int32), np.ascontiguousarray(b, dtype=np.int32)
        return int(self.lib.orc_hash_pair(aa.ctypes.data_as(self.p32), aa.size, bb.ctypes.data_as(self.p32), bb.size))


def _closed_forms():
    """(graph, count, nodes, nonmaximal, max_depth) from the hand derivations in
    test_oracle_pins.py."""
    out = []
    for m, n in ((4, 9), (9, 4), (3, 3)):
        c = min(m, n)
        out.append((gg.complete(m, n), 1, c, c - 1, 1))
    out.append((gg.perfect_matching(7), 7, 7, 0, 1))
    out.append((gg.chain(6), 6, 6, 0, 1))
    out.append((gg.crown(6), 62, 62, 0, 5))
    return out


def _pins_fail(orc, cp):
    """Name of the first pin the copy fails, or None."""
    for g, cnt, nodes, nonmax, depth in _closed_forms():
        res, _ = cp.mbea(g)
        if (res.count, res.nodes, res.nonmaximal, res.max_depth) != (cnt, nodes, nonmax, depth):
            return "closed-form tree " + g.name
    # hand-derived bytes: perfect matching 4 n (n + 3 + min(3, 3 (n - 1))); K_{4,9} (c = 4,
    # o = 9) 4 c (2 + o + (c - 1) + o + min(o (2 + c), (c - 1)(2 + o)))
    res, _ = cp.mbea(gg.perfect_matching(7))
    if res.bytes_alg != 4 * 7 * (7 + 3 + 3):
        return "closed-form bytes (matching)"
    res, _ = cp.mbea(gg.complete(4, 9))
    if res.bytes_alg != 4 * 4 * (2 + 9 + 3 + 9 + min(9 * 6, 3 * 11)):
        return "closed-form bytes (complete)"
    for a, b in [([0], [0]), ([3, 1], [2]), ([5], [7, 8, 9]), ([100], [99])]:
        if cp.hash_pair(a, b) != hc.h(a, b):
            return "plain-integer pair hash"
    graphs = [gg.crown(6), gg.chain(7), gg.complete_minus_edge(4, 5)]
    graphs += [gg.random_small(10, 12, 0.4, s) for s in range(30)]
    for g in graphs:
        b = orc.brute(g)
        res, lst = cp.mbea(g)
        if res.count != len(b["list"]) or lst != b["list"]:
            return "definition " + g.name
        if res.hash != hc.total(b["list"]):
            return "plain-integer total hash " + g.name
    return None


def _imbea_pins_fail(orc, cp):
    """Name of the first iMBEA pin the copy fails, or None (tests/test_oracle_imbea.py)."""
    hand = gg.from_edges(3, 3, [0, 0, 1, 1, 2, 2], [0, 1, 0, 1, 1, 2])
    res, _ = cp.mbea(hand, "orc_imbea")
    if (res.nodes, res.nonmaximal, res.count, res.bytes_alg, res.max_depth) != (3, 0, 3, 160, 2):
        return "hand-worked tree"
    for m, n in ((4, 9), (3, 3)):
        res, _ = cp.mbea(gg.complete(m, n), "orc_imbea")
        if (res.nodes, res.nonmaximal, res.count) != (1, 0, 1):
            return "complete"
    blocks = gg.disjoint_union(gg.disjoint_union(gg.complete(2, 3), gg.complete(4, 1)), gg.complete(3, 3))
    res, _ = cp.mbea(blocks, "orc_imbea")
    if (res.nodes, res.nonmaximal, res.count) != (3, 0, 3):
        return "complete blocks"
    # ranges: the prefix before rank_lo runs silently
    res, _ = cp.mbea(gg.complete(4, 9), "orc_imbea", 1, -1)
    if (res.nodes, res.count) != (0, 0):
        return "silent prefix"
    graphs = [gg.chain(7), gg.complete_minus_edge(4, 5)] + [gg.random_small(10, 12, 0.4, s) for s in range(30)]
    for g in graphs:
        b = orc.brute(g)
        res, lst = cp.mbea(g, "orc_imbea")
        if res.count != len(b["list"]) or lst != b["list"] or res.hash != hc.total(b["list"]):
            return "definition " + g.name
    return None


def _pivot_pins_fail(orc, cp):
    """Name of the first pivot pin the copy fails, or None (tests/test_oracle_pivot.py)."""
    g1 = gg.from_edges(3, 7, [0, 0, 0, 1, 1, 1, 1, 2, 2, 2], [0, 1, 2, 0, 1, 3, 4, 0, 5, 6])
    res, _ = cp.mbea(g1, "orc_pivot")
    if (res.nodes, res.nonmaximal, res.count, res.max_depth, res.bytes_alg) != (6, 1, 5, 3, 416):
        return "hand-worked tree (deeper)"
    g2 = gg.from_edges(4, 7, [0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3], [0, 1, 2, 0, 3, 4, 0, 1, 5, 1, 2, 6])
    res, _ = cp.mbea(g2, "orc_pivot")
    if (res.nodes, res.nonmaximal, res.count, res.max_depth, res.bytes_alg) != (10, 2, 8, 3, 772):
        return "hand-worked tree (covered entries in Q)"
    us, vs = [], []
    for i in range(5):
        us += [i] * 4
        vs += [0, 1, 2, 3 + i]
    res, _ = cp.mbea(gg.from_edges(5, 8, us, vs), "orc_pivot")
    if (res.nodes, res.nonmaximal, res.count, res.max_depth) != (9, 3, 6, 2):
        return "private-neighbour family"
    graphs = [gg.crown(6), gg.chain(7), gg.complete_minus_edge(4, 5)] + [gg.random_small(10, 12, 0.4, s) for s in range(30)]
    for g in graphs:
        b = orc.brute(g)
        res, lst = cp.mbea(g, "orc_pivot")
        if res.count != len(b["list"]) or lst != b["list"] or res.hash != hc.total(b["list"]):
            return "definition " + g.name
    return None


def test_unmodified_source_passes_every_pin(orc):
    cp = _Copy(orc, _build(open(SRC).read()))
    assert _pins_fail(orc, cp) is None
    assert _imbea_pins_fail(orc, cp) is None
    assert _pivot_pins_fail(orc, cp) is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(orc, name):
    old, new = MUTANTS[name]
    cp = _Copy(orc, _build(_plant(open(SRC).read(), old, new)))
    assert _pins_fail(orc, cp) is not None, f"mutant {name} passed every pin"


@pytest.mark.parametrize("name", sorted(IMBEA_MUTANTS))
def test_imbea_pins_catch_mutant(orc, name):
    old, new = IMBEA_MUTANTS[name]
    cp = _Copy(orc, _build(_plant(open(SRC).read(), old, new, inside="imbea")))
    assert _imbea_pins_fail(orc, cp) is not None, f"mutant {name} passed every pin"


@pytest.mark.parametrize("name", sorted(PIVOT_MUTANTS))
def test_pivot_pins_catch_mutant(orc, name):
    old, new = PIVOT_MUTANTS[name]
    cp = _Copy(orc, _build(_plant(open(SRC).read(), old, new, inside="pivot")))
    assert _pivot_pins_fail(orc, cp) is not None, f"mutant {name} passed every pin"
