"""CPU oracle for maximal biclique enumeration -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The product library never calls it and shares no code with it.

Routes to the set of maximal bicliques (paper, section II-A):
  * ``brute``   -- the definition written out over all subsets A of U (tiny graphs);
  * ``closure`` -- the definition through common-neighbour sets: every A = N(B) for a
                   non-empty B is an intersection of neighbour rows N(b), so the A-sides of
                   the maximal bicliques are exactly the non-empty members of the closure of
                   {N(b) : b in V} under pairwise intersection (pure Python, small graphs);
  * ``mbea``    -- Algorithm 1 (section II-B) serially in C, with the reverse-scanning count
                   of section III-E and the ascending common-neighbour candidate order.

All three return the same canonical record list; ``mbea`` also returns the count, the
order-independent 64-bit hash and the tree diagnostics.  Two variants of ``mbea`` prune the
tree (section II-C) with the same answer and their own tallies: ``imbea`` (candidates with the
pivot's neighbourhood within R leave P with it) and ``pivot`` (one pivot per list below the top
level, taken first, covering the candidates whose neighbourhoods within R it contains).  The C part is compiled by
``oracle.build()`` (gcc) into ``oracle/liborc_mbe.so``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mbe_oracle.c")
# MBE_ORACLE_SANITIZE=1: a copy built with AddressSanitizer and UndefinedBehaviorSanitizer
# (the process must preload gcc's libasan and libubsan; tests/test_oracle_sanitized.py does)
_SANITIZE = os.environ.get("MBE_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liborc_mbe_san.so" if _SANITIZE else "liborc_mbe.so")
_lib = None
_lock = threading.Lock()

MASK64 = (1 << 64) - 1


class OrcResult(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_uint64), ("hash", ctypes.c_uint64), ("out_ints", ctypes.c_uint64),
        ("nodes", ctypes.c_uint64), ("nonmaximal", ctypes.c_uint64),
        ("bytes_alg", ctypes.c_uint64), ("bytes_rs", ctypes.c_uint64),
        ("max_depth", ctypes.c_uint32), ("side", ctypes.c_uint32), ("written", ctypes.c_int64),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle's C source with gcc into a shared library next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=all"] if _SANITIZE else ["-O2"]
        subprocess.check_call(["gcc", *flags, "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            p32 = ctypes.POINTER(ctypes.c_int32)
            lib.orc_mbea.argtypes = [ctypes.c_int32, ctypes.c_int32, p32, p32, p32, p32, ctypes.c_int,
                                     ctypes.c_int64, ctypes.c_int64, p32, ctypes.c_int64,
                                     ctypes.POINTER(OrcResult)]
            lib.orc_mbea.restype = ctypes.c_int
            lib.orc_imbea.argtypes = lib.orc_mbea.argtypes
            lib.orc_imbea.restype = ctypes.c_int
            lib.orc_pivot.argtypes = lib.orc_mbea.argtypes
            lib.orc_pivot.restype = ctypes.c_int
            lib.orc_brute.argtypes = [ctypes.c_int32, ctypes.c_int32, p32, p32, p32, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int64)]
            lib.orc_brute.restype = ctypes.c_int64
            lib.orc_num_roots.argtypes = [ctypes.c_int32, ctypes.c_int32, p32, p32, ctypes.c_int]
            lib.orc_num_roots.restype = ctypes.c_int64
            lib.orc_hash_pair.argtypes = [p32, ctypes.c_int64, p32, ctypes.c_int64]
            lib.orc_hash_pair.restype = ctypes.c_uint64
            lib.orc_mix64.argtypes = [ctypes.c_uint64]
            lib.orc_mix64.restype = ctypes.c_uint64
            lib.orc_hash_u.argtypes = [ctypes.c_int32]
            lib.orc_hash_u.restype = ctypes.c_uint64
            lib.orc_hash_v.argtypes = [ctypes.c_int32]
            lib.orc_hash_v.restype = ctypes.c_uint64
            _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _arrays(g):
    return tuple(np.ascontiguousarray(x, dtype=np.int32) for x in (g.u_off, g.u_adj, g.v_off, g.v_adj))


def mix64(z: int) -> int:
    """SplitMix64 output function, as the oracle computes it."""
    return int(_load().orc_mix64(ctypes.c_uint64(z & MASK64)))


def hash_u(a: int) -> int:
    """hu(a), the term of vertex a of U in a biclique's hash."""
    return int(_load().orc_hash_u(int(a)))


def hash_v(b: int) -> int:
    """hv(b), the term of vertex b of V in a biclique's hash."""
    return int(_load().orc_hash_v(int(b)))


def hash_pair(a: Sequence[int], b: Sequence[int]) -> int:
    """h(A, B) of one biclique, A in U and B in V."""
    aa = np.ascontiguousarray(a, dtype=np.int32)
    bb = np.ascontiguousarray(b, dtype=np.int32)
    return int(_load().orc_hash_pair(_p32(aa), aa.size, _p32(bb), bb.size))


def num_roots(g, side: int = 0) -> int:
    u_off, _, v_off, _ = _arrays(g)
    return int(_load().orc_num_roots(g.n_u, g.n_v, _p32(u_off), _p32(v_off), side))


def split_records(buf: np.ndarray, n_ints: int) -> List[Tuple[Tuple[int, ...], Tuple[int, ...]]]:
    """Decode [|A|, |B|, A..., B...] records into (A, B) tuples."""
    out = []
    i = 0
    flat = buf[:n_ints].tolist()
    while i < n_ints:
        na, nb = flat[i], flat[i + 1]
        a = tuple(flat[i + 2:i + 2 + na])
        b = tuple(flat[i + 2 + na:i + 2 + na + nb])
        out.append((a, b))
        i += 2 + na + nb
    return out


def canonical(records) -> List[Tuple[Tuple[int, ...], Tuple[int, ...]]]:
    """Records with each side ascending, ordered by A lexicographically."""
    return sorted((tuple(sorted(a)), tuple(sorted(b))) for a, b in records)


def flatten(records) -> np.ndarray:
    out: List[int] = []
    for a, b in records:
        out.append(len(a))
        out.append(len(b))
        out.extend(a)
        out.extend(b)
    return np.asarray(out, dtype=np.int32)


def mbea(g, side: int = 0, rank_lo: int = 0, rank_hi: int = -1, want_list: bool = False,
         list_cap: int = 1 << 26) -> Dict:
    """Serial MBEA (Algorithm 1) over the graph, or over top-level ranks [rank_lo, rank_hi).

    Returns a dict with count, hash, out_ints, nodes, nonmaximal, bytes_alg, bytes_rs,
    max_depth, side and (when want_list) the canonical record list."""
    lib = _load()
    u_off, u_adj, v_off, v_adj = _arrays(g)
    res = OrcResult()
    buf = np.zeros(list_cap if want_list else 1, dtype=np.int32)
    rc = lib.orc_mbea(g.n_u, g.n_v, _p32(u_off), _p32(u_adj), _p32(v_off), _p32(v_adj), side,
                      rank_lo, rank_hi, _p32(buf) if want_list else None, buf.size, ctypes.byref(res))
    if rc != 0:
        raise RuntimeError("oracle mbea failed")
    out = {k: getattr(res, k) for k, _ in OrcResult._fields_}
    if want_list:
        if res.written < 0:
            raise RuntimeError("oracle record buffer too small")
        out["list"] = canonical(split_records(buf, res.written))
    return out


def imbea(g, side: int = 0, rank_lo: int = 0, rank_hi: int = -1, want_list: bool = False,
          list_cap: int = 1 << 26) -> Dict:
    """MBEA with iMBEA's candidate pruning (the C set of section II-C): the same answer as
    mbea, its own tree tallies.  Fields as mbea's."""
    lib = _load()
    u_off, u_adj, v_off, v_adj = _arrays(g)
    res = OrcResult()
    buf = np.zeros(list_cap if want_list else 1, dtype=np.int32)
    rc = lib.orc_imbea(g.n_u, g.n_v, _p32(u_off), _p32(u_adj), _p32(v_off), _p32(v_adj), side,
                       rank_lo, rank_hi, _p32(buf) if want_list else None, buf.size, ctypes.byref(res))
    if rc != 0:
        raise RuntimeError("oracle imbea failed")
    out = {k: getattr(res, k) for k, _ in OrcResult._fields_}
    if want_list:
        if res.written < 0:
            raise RuntimeError("oracle record buffer too small")
        out["list"] = canonical(split_records(buf, res.written))
    return out


def pivot(g, side: int = 0, rank_lo: int = 0, rank_hi: int = -1, want_list: bool = False,
          list_cap: int = 1 << 26) -> Dict:
    """MBEA with the pivot rule (the pivot pruning of section II-C, one pivot per list below
    the top level covering the candidates whose neighbourhoods within R it contains): the same
    answer as mbea, its own tree tallies.  Fields as mbea's."""
    lib = _load()
    u_off, u_adj, v_off, v_adj = _arrays(g)
    res = OrcResult()
    buf = np.zeros(list_cap if want_list else 1, dtype=np.int32)
    rc = lib.orc_pivot(g.n_u, g.n_v, _p32(u_off), _p32(u_adj), _p32(v_off), _p32(v_adj), side,
                       rank_lo, rank_hi, _p32(buf) if want_list else None, buf.size, ctypes.byref(res))
    if rc != 0:
        raise RuntimeError("oracle pivot failed")
    out = {k: getattr(res, k) for k, _ in OrcResult._fields_}
    if want_list:
        if res.written < 0:
            raise RuntimeError("oracle record buffer too small")
        out["list"] = canonical(split_records(buf, res.written))
    return out


def mbea_parallel(g, side: int = 0, threads: int = 0, chunks: int = 0) -> Dict:
    """The same serial MBEA split by top-level rank ranges over host threads.  Count, hash
    and byte tallies are sums and max_depth a maximum, so the split result is exact."""
    n = num_roots(g, side)
    threads = threads or os.cpu_count() or 1
    chunks = chunks or max(1, min(n, threads * 16))
    # ranks are ascending in degree, so cut the range into interleaved chunks of equal size
    bounds = np.linspace(0, n, chunks + 1).astype(np.int64)
    parts = []
    with ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(mbea, g, side, int(bounds[i]), int(bounds[i + 1])) for i in range(chunks)
                if bounds[i] < bounds[i + 1]]
        parts = [f.result() for f in futs]
    tot = {"count": 0, "hash": 0, "out_ints": 0, "nodes": 0, "nonmaximal": 0, "bytes_alg": 0,
           "bytes_rs": 0, "max_depth": 0, "side": 0}
    for p in parts:
        for k in ("count", "out_ints", "nodes", "nonmaximal", "bytes_alg", "bytes_rs"):
            tot[k] += p[k]
        tot["hash"] = (tot["hash"] + p["hash"]) & MASK64
        tot["max_depth"] = max(tot["max_depth"], p["max_depth"])
        tot["side"] = p["side"]
    tot["threads"] = threads
    return tot


def brute(g) -> Dict:
    """The definition over all subsets A of U (|U| <= 24, |V| <= 64)."""
    lib = _load()
    u_off, u_adj, _, _ = _arrays(g)
    h = ctypes.c_uint64(0)
    ints = ctypes.c_int64(0)
    n = lib.orc_brute(g.n_u, g.n_v, _p32(u_off), _p32(u_adj), None, 0, ctypes.byref(h), ctypes.byref(ints))
    if n < 0:
        raise ValueError("graph too large for brute force")
    buf = np.zeros(max(1, ints.value), dtype=np.int32)
    n2 = lib.orc_brute(g.n_u, g.n_v, _p32(u_off), _p32(u_adj), _p32(buf), buf.size, None, None)
    assert n2 == n
    recs = split_records(buf, ints.value)
    return {"count": int(n), "hash": int(h.value), "out_ints": int(ints.value), "list": canonical(recs)}


def closure(g) -> Dict:
    """Maximal bicliques through the intersection closure of the neighbour rows N(b), b in V.

    A set A of U is the U-side of a maximal biclique exactly when A = N(B) for a non-empty B
    in V and A is non-empty; N(B) is the intersection of the rows N(b), so these sets are the
    non-empty members of the closure of {N(b)} under intersection.  The V-side is N(A).
    Sets are Python integers used as bitmasks.  Meant for graphs with a few thousand
    maximal bicliques at most."""
    rows_v = []
    for b in range(g.n_v):
        m = 0
        for a in g.v_adj[g.v_off[b]:g.v_off[b + 1]].tolist():
            m |= 1 << a
        rows_v.append(m)
    fam = set()
    for b in range(g.n_v):
        nb = rows_v[b]
        new = {nb}
        for f in fam:
            new.add(f & nb)
        fam |= new
    fam.discard(0)
    rows_u = []
    for a in range(g.n_u):
        m = 0
        for b in g.u_adj[g.u_off[a]:g.u_off[a + 1]].tolist():
            m |= 1 << b
        rows_u.append(m)
    recs = []
    for amask in fam:
        a = [i for i in range(g.n_u) if amask >> i & 1]
        bmask = (1 << g.n_v) - 1
        for i in a:
            bmask &= rows_u[i]
        b = [j for j in range(g.n_v) if bmask >> j & 1]
        recs.append((tuple(a), tuple(b)))
    recs = canonical(recs)
    h = 0
    for a, b in recs:
        h = (h + hash_pair(a, b)) & MASK64
    return {"count": len(recs), "hash": h, "out_ints": sum(2 + len(a) + len(b) for a, b in recs), "list": recs}
