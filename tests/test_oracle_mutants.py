"""The oracle's pins catch plausible mistakes.  Each test plants one mistake in a copy of the
oracle's C source (on the CPU), builds it, and runs the pins on the copy alone:

* the definition: count and canonical list against brute force over subsets (the brute-force
  route of the unmodified source, whose hash is not used);
* the hash: the copy's total against the plain-integer hash of the definition's list, and its
  h(A, B) against the plain-integer one on fixed bicliques (tests/hash_contract.py, whose mix
  is pinned to the published SplitMix64 outputs);
* the tree: node, non-maximal, depth and byte tallies of the hand-derived closed forms.

A mutant must fail at least one of them.  The plain search's mutants are planted outside the
iMBEA variant's code, and the variant's mutants inside it; the variant's pins are its
definition list (brute force) and its hand-derived trees (tests/test_oracle_imbea.py)."""
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

# the iMBEA variant's code: from its count-only merge to the plain entry's side rule, and its
# entry point
_IMBEA_SPANS = [("/* |R n N(v)| for ascending R and N(v)", "/* Candidate side: 1 = U, 2 = V"),
                ("/*\n * As orc_mbea, with iMBEA's candidate pruning", "/* Number of top-level candidates")]


def _split(src):
    """(text outside the iMBEA code with placeholders, the iMBEA pieces)."""
    pieces = []
    for a, b in _IMBEA_SPANS:
        i, j = src.index(a), src.index(b)
        pieces.append(src[i:j])
        src = src[:i] + f"@@IMBEA{len(pieces) - 1}@@" + src[j:]
    return src, pieces


def _join(outside, pieces):
    for k, p in enumerate(pieces):
        outside = outside.replace(f"@@IMBEA{k}@@", p)
    return outside


def _plant(src, old, new, inside):
    outside, pieces = _split(src)
    if inside:
        assert sum(p.count(old) for p in pieces) == 1, old
        pieces = [p.replace(old, new) for p in pieces]
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


def test_unmodified_source_passes_every_pin(orc):
    cp = _Copy(orc, _build(open(SRC).read()))
    assert _pins_fail(orc, cp) is None
    assert _imbea_pins_fail(orc, cp) is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(orc, name):
    old, new = MUTANTS[name]
    cp = _Copy(orc, _build(_plant(open(SRC).read(), old, new, inside=False)))
    assert _pins_fail(orc, cp) is not None, f"mutant {name} passed every pin"


@pytest.mark.parametrize("name", sorted(IMBEA_MUTANTS))
def test_imbea_pins_catch_mutant(orc, name):
    old, new = IMBEA_MUTANTS[name]
    cp = _Copy(orc, _build(_plant(open(SRC).read(), old, new, inside=True)))
    assert _imbea_pins_fail(orc, cp) is not None, f"mutant {name} passed every pin"
