"""mbe_count_noalloc (the entry point for callers that cannot allocate device memory) against
mbe_count through the C-ABI: same count, hash, out_ints and tree diagnostics, on consecutive
calls whose second input is smaller (the fixed scratch keeps the first call's contents), for
host and device graphs, and a clean MBE_ERR_SCRATCH_LIMIT for a graph that does not fit."""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu

KEYS = ("count", "hash", "out_ints", "nodes", "nonmaximal", "bytes_alg", "max_depth", "side")


def _same(a, b):
    assert {k: a[k] for k in KEYS} == {k: b[k] for k in KEYS}


def _pairs():
    # (larger, smaller) inputs of each pair, run back to back
    return [
        (gg.config1(), gg.random_small(40, 30, 0.2, 7)),
        (gg.crown(12), gg.complete(3, 5)),
        (gg.chung_lu(3000, 2000, 30000, 2.1, 2.1, 11), gg.erdos_renyi_pairs(60, 50, 0.1, 12)),
    ]


@pytest.mark.parametrize("diag", [False, True])
def test_noalloc_equals_count_twice(mbe, diag):
    for big, small in _pairs():
        opt = mbe.Options(diagnostics=diag)
        for g in (big, small):
            want = mbe.mbe_count(g, opt)
            got = mbe.mbe_count_noalloc(g, opt)
            _same(got, want)


def test_noalloc_device_graphs_and_options(mbe):
    import torch
    for g in (gg.config1(), gg.crown(9)):
        dg = gg.BiGraph(g.n_u, g.n_v, *[torch.from_numpy(np.asarray(a)).cuda()
                                        for a in (g.u_off, g.u_adj, g.v_off, g.v_adj)])
        for opt in (mbe.Options(diagnostics=True), mbe.Options(wg_waves=4, steal_k=3, diagnostics=True),
                    mbe.Options(side=2, steal_k=1), mbe.Options(root_lo=5, root_hi=60)):
            _same(mbe.mbe_count_noalloc(dg, opt), mbe.mbe_count(g, opt))
    torch.cuda.synchronize()


def test_noalloc_scratch_limit_then_recovers(mbe):
    # 2M candidates of degree 1 on one hub: the local universe of every candidate is the whole
    # candidate side, far beyond what one arena slot of the scratch can hold
    n = 2_000_000
    u_off = np.arange(n + 1, dtype=np.int32)
    u_adj = np.zeros(n, dtype=np.int32)
    v_off = np.array([0, n], dtype=np.int32)
    v_adj = np.arange(n, dtype=np.int32)
    g = gg.BiGraph(n, 1, u_off, u_adj, v_off, v_adj)
    with pytest.raises(mbe.MbeError) as e:
        mbe.mbe_count_noalloc(g, mbe.Options(side=1, no_validate=True))
    assert e.value.code == mbe.MBE_ERR_SCRATCH_LIMIT
    small = gg.config1()
    _same(mbe.mbe_count_noalloc(small, mbe.Options(diagnostics=True)),
          mbe.mbe_count(small, mbe.Options(diagnostics=True)))


def test_noalloc_wide_top_level_candidates(mbe):
    # candidates of degree above 1024 go to the wide search, whose arena also comes from the
    # scratch
    g = gg.wide_hubs(200, 5000, [1100 + 300 * k for k in range(12)], 0.002, 4)
    for opt in (mbe.Options(diagnostics=True), mbe.Options(steal_k=3)):
        _same(mbe.mbe_count_noalloc(g, opt), mbe.mbe_count(g, opt))
    small = gg.crown(7)
    _same(mbe.mbe_count_noalloc(small, mbe.Options(diagnostics=True)),
          mbe.mbe_count(small, mbe.Options(diagnostics=True)))
