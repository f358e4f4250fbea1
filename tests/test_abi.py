"""The C-ABI library on the CPU: it loads, exports every entry point include/mbe.h declares,
and rejects bad arguments and malformed host graphs before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mbe.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*\**\s*(mbe_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2401_05039_amd as m
    return m, m.load()


def test_every_declared_symbol_is_exported(lib):
    _, so = lib
    names = _declared()
    assert {"mbe_count", "mbe_enumerate", "mbe_strerror", "mbe_version"} <= set(names)
    for n in names:
        assert hasattr(so, n), n


def test_strerror_and_version(lib):
    m, _ = lib
    assert m.mbe_strerror(0) == "ok"
    for code in range(-9, 0):
        assert m.mbe_strerror(code) and m.mbe_strerror(code) != "unknown error"
    assert m.mbe_strerror(-99) == "unknown error"
    assert re.match(r"^\d+\.\d+\.\d+$", m.mbe_version())


def test_null_arguments(lib):
    _, so = lib
    res = ctypes.c_void_p(None)
    assert so.mbe_count(None, None, None) == -1
    g, keep = __import__("paper_2401_05039_amd")._marshal_graph(gg.complete(2, 2))
    assert so.mbe_count(ctypes.byref(g), None, None) == -1


def _bad(g, **kw):
    import paper_2401_05039_amd as m
    with pytest.raises(m.MbeError) as e:
        m.mbe_count(g, m.Options(**kw))
    return e.value.code


def _mk(n_u, n_v, u_off, u_adj, v_off, v_adj):
    return gg.BiGraph(n_u, n_v, np.array(u_off, np.int32), np.array(u_adj, np.int32),
                      np.array(v_off, np.int32), np.array(v_adj, np.int32))


def test_invalid_graphs_rejected_on_host():
    good = gg.complete(2, 3)
    # unsorted row
    assert _bad(_mk(2, 3, [0, 3, 6], [0, 2, 1, 0, 1, 2], good.v_off, good.v_adj)) == -2
    # duplicate in a row
    assert _bad(_mk(2, 3, [0, 3, 6], [0, 1, 1, 0, 1, 2], good.v_off, good.v_adj)) == -2
    # id out of range
    assert _bad(_mk(2, 3, [0, 3, 6], [0, 1, 3, 0, 1, 2], good.v_off, good.v_adj)) == -2
    # offsets not ending at n_edges
    assert _bad(_mk(2, 3, [0, 3, 5], [0, 1, 2, 0, 1, 2], good.v_off, good.v_adj)) == -2
    # not transposes: drop (1, 2) from the V side only
    assert _bad(_mk(2, 3, good.u_off, good.u_adj, [0, 2, 4, 5], [0, 1, 0, 1, 0])) == -2


def test_host_validation_transpose_rules():
    """The host check accepts exactly the CSR pairs whose V side is the transpose of the U side
    with sorted rows: a V row with its entries out of order, an entry moved to another V row
    (the counts of the sides still agree), or V offsets that decrease are refused; valid
    random graphs pass the check (the call then needs a device, so on a machine without one it
    fails later, with MBE_ERR_DEVICE, not MBE_ERR_INVALID_GRAPH)."""
    import paper_2401_05039_amd as m
    good = gg.complete(2, 3)  # N(u0) = N(u1) = {0, 1, 2}; V rows [0, 1] each
    # V row 0 holds its entries in the wrong order
    assert _bad(_mk(2, 3, good.u_off, good.u_adj, [0, 2, 4, 6], [1, 0, 0, 1, 0, 1])) == -2
    # u0-v2 missing from V row 2, u1 listed twice: same count, not the transpose
    assert _bad(_mk(2, 3, good.u_off, good.u_adj, [0, 2, 4, 6], [0, 1, 0, 1, 1, 1])) == -2
    # an entry moved from V row 2 to V row 0 (offsets adjusted)
    assert _bad(_mk(2, 3, good.u_off, good.u_adj, [0, 3, 5, 6], [0, 1, 1, 0, 1, 1])) == -2
    # V offsets that decrease
    assert _bad(_mk(2, 3, good.u_off, good.u_adj, [0, 4, 2, 6], [0, 1, 0, 1, 0, 1])) == -2
    for s in range(20):
        g = gg.random_small(9, 13, 0.4, 300 + s)
        if g.n_edges == 0:
            continue
        try:
            m.mbe_count(g)
        except m.MbeError as e:
            assert e.code != -2, g.name


def test_bad_options_rejected():
    g = gg.complete(2, 2)
    assert _bad(g, side=3) == -1
    assert _bad(g, wg_waves=9) == -1
    assert _bad(g, steal_k=4) == -1
    assert _bad(g, steal_k=-1) == -1


def test_tuner_rejects_bad_input_before_device_work():
    import paper_2401_05039_amd as m
    with pytest.raises(m.MbeError) as e:
        m.mbe_tune_batch([])
    assert e.value.code == -1
    good = gg.complete(2, 3)
    bad = _mk(2, 3, [0, 3, 6], [0, 2, 1, 0, 1, 2], good.v_off, good.v_adj)
    with pytest.raises(m.MbeError) as e:
        m.mbe_tune_batch([good, bad])
    assert e.value.code == -2


def test_empty_graphs_need_no_device():
    import paper_2401_05039_amd as m
    for g in (gg.edgeless(4, 5), gg.edgeless(0, 3), gg.edgeless(3, 0)):
        r = m.mbe_count(g)
        assert r["count"] == 0 and r["hash"] == 0


def test_workspace_size_needs_no_device_for_trivial_input(lib):
    import paper_2401_05039_amd as m
    _, so = lib
    g, keep = m._marshal_graph(gg.complete(2, 2))
    assert so.mbe_workspace_size(ctypes.byref(g), None, None) == -1
    for e in (gg.edgeless(4, 5), gg.edgeless(0, 3)):
        assert m.mbe_workspace_size(e) == 0
    with pytest.raises(m.MbeError) as err:
        m.mbe_workspace_size(gg.complete(2, 2), m.Options(steal_k=9))
    assert err.value.code == -1


def test_batch_rejects_bad_input_before_device_work():
    import paper_2401_05039_amd as m
    good = gg.complete(2, 3)
    bad = _mk(2, 3, [0, 3, 6], [0, 2, 1, 0, 1, 2], good.v_off, good.v_adj)
    with pytest.raises(m.MbeError) as e:
        m.mbe_count_batch([good, bad, good])
    assert e.value.code == -2
    with pytest.raises(m.MbeError) as e:
        m.mbe_count_batch([good], m.Options(wg_waves=99))
    assert e.value.code == -1
    assert m.mbe_count_batch([]) == []
    r = m.mbe_count_batch([gg.edgeless(3, 3), gg.edgeless(0, 2)])
    assert all(x["count"] == 0 and x["hash"] == 0 for x in r)


def test_server_rejects_bad_options():
    import paper_2401_05039_amd as m
    with pytest.raises(m.MbeError) as e:
        m.Server(slots=99)
    assert e.value.code == -1


def test_server_rejects_bad_deadlines(lib):
    import paper_2401_05039_amd as m
    _, so = lib
    for bad in (-1.0, float("nan")):
        with pytest.raises(m.MbeError) as e:
            m.Server(request_timeout_ms=bad)
        assert e.value.code == -1
    g, keep = m._marshal_graph(gg.complete(2, 2))
    t = ctypes.c_uint64()
    assert so.mbe_server_submit_timeout(None, ctypes.byref(g), ctypes.c_double(1.0), ctypes.byref(t)) == -1
    assert so.mbe_server_cancel(None, ctypes.c_uint64(1)) == -1


def test_workspace_arguments_checked_before_device_work():
    import paper_2401_05039_amd as m
    g = gg.complete(2, 3)
    for kw in (dict(workspace=0, workspace_bytes=1 << 20), dict(workspace=4096, workspace_bytes=0)):
        with pytest.raises(m.MbeError) as e:
            m.mbe_count(g, m.Options(**kw))
        assert e.value.code == -1
    ws = dict(workspace=1 << 20, workspace_bytes=1 << 20)  # (never touched: refused first)
    for call in (lambda: m.mbe_count_batch([g], m.Options(**ws)),
                 lambda: m.mbe_enumerate(g, m.Options(**ws), cap_ints=64),
                 lambda: m.mbe_count_noalloc(g, m.Options(**ws)),
                 lambda: m.mbe_workspace_size(g, m.Options(**ws)),
                 lambda: m.Server(opt=m.Options(**ws))):
        with pytest.raises(m.MbeError) as e:
            call()
        assert e.value.code == -1


def test_batch_totals_past_int32_refused_before_device_work():
    # the same host arrays repeated until the packed edge count passes 2^31 - 1: refused with
    # MBE_ERR_INVALID_ARG by the 64-bit size check, before any packing or device work
    import paper_2401_05039_amd as m
    g = gg.erdos_renyi_m(1000, 1000, 1_000_000, 5)
    n = (2**31) // g.n_edges + 1
    with pytest.raises(m.MbeError) as e:
        m.mbe_count_batch([g] * n, m.Options(no_validate=True))
    assert e.value.code == -1
    # ids past int32 too: many copies of a wide, sparse graph
    h = gg.from_edges(2_000_000, 1_000_000, [0], [0])
    with pytest.raises(m.MbeError) as e:
        m.mbe_count_batch([h] * 2200, m.Options(no_validate=True))
    assert e.value.code == -1
