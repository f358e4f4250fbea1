"""The oracle's pins catch plausible mistakes: each test plants one mistake in a copy of
the oracle's C source (on the CPU), builds it, and checks that brute force or a closed form
tells it apart from the definition."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import graphgen as gg

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "mbe_oracle.c")

MUTANTS = {
    "no_maximality_check": ("if (c == nRp) { maximal = 0; break; }", "if (0) { maximal = 0; break; }"),
    "no_expansion": ("if (c == nRp) Lp[nLp++] = v;", "if (0) Lp[nLp++] = v;"),
    "child_keeps_zero_counts": ("else if (c > 0) { Pp[nPp].key = c;", "else if (c >= 0) { Pp[nPp].key = c;"),
    "q_drops_partial": ("else if (c > 0) Qp[nQp++] = Q[i];", "else if (c > 1) Qp[nQp++] = Q[i];"),
    "x_not_moved_to_q": ("Q[nQ++] = x;", "(void)x;"),
    "intersect_off_by_one": ("while (i < nr && j < nn) {", "while (i < nr && j < nn - 1) {"),
}


def _build(src_text):
    d = tempfile.mkdtemp(prefix="orc_mut_")
    c = os.path.join(d, "m.c")
    so = os.path.join(d, "m.so")
    open(c, "w").write(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", so, c])
    return so


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(orc, name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    so = _build(src.replace(old, new))
    lib = ctypes.CDLL(so)
    p32 = ctypes.POINTER(ctypes.c_int32)
    lib.orc_mbea.argtypes = [ctypes.c_int32, ctypes.c_int32, p32, p32, p32, p32, ctypes.c_int, ctypes.c_int64,
                             ctypes.c_int64, p32, ctypes.c_int64, ctypes.POINTER(orc.OrcResult)]

    def run(g):
        arrs = [np.ascontiguousarray(x, dtype=np.int32) for x in (g.u_off, g.u_adj, g.v_off, g.v_adj)]
        res = orc.OrcResult()
        lib.orc_mbea(g.n_u, g.n_v, *[a.ctypes.data_as(p32) for a in arrs], 0, 0, -1, None, 0, ctypes.byref(res))
        return res.count, res.hash

    graphs = [gg.crown(6), gg.chain(7), gg.complete_minus_edge(4, 5)]
    graphs += [gg.random_small(10, 12, 0.4, s) for s in range(30)]
    caught = False
    for g in graphs:
        b = orc.brute(g)
        if run(g) != (b["count"], b["hash"]):
            caught = True
            break
    assert caught, f"mutant {name} passed every pin"
