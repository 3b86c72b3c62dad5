"""Launch tuning is result-neutral: every bucket layout, grid cap and hash size gives bit-identical labels, objective and
per-pass trace (plain calls and fused batches), and the autotuner only picks among such settings."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

TUNINGS = [
    dict(bucket_max=[0, 0, 0, 0, 0, 0, 0]),              # every row with an edge through the hub chunks
    dict(bucket_max=[1, 2, 3, 4, 5, 6, 7], grid_cap=64),   # tiny buckets, few workgroups
    dict(bucket_max=[4, 8, 16, 32, 64, 512, 2048], grid_cap=4096),
    dict(bucket_max=[0, 8, 8, 32, 32, 1024, 1024], grid_cap=65536),
    dict(bucket_max=[4, 4, 4, 4, 128, 128, 128]),         # no 8/16/32-lane groups, no workgroup hashes
    dict(bucket_max=[4, 8, 16, 32, 128, 1024, 8192]),     # rows 4097-8192 on the 16384-slot workgroups
    dict(hash_shift=1),                                   # LDS hashes at twice the capacity
    dict(bucket_max=[4, 8, 16, 32, 128, 1024, 8192], hash_shift=2),  # 4 times, capped at every table
]

CASES = [
    ("hubs", lambda: U.hub_graph(), O.PLOUVAIN, (1, 1, True), O.VW_WEIGHTED_DEGREE),
    ("hubs-leiden", lambda: U.hub_graph(n=12000, hub_deg=(9000, 6000, 1500), seed=4), O.PLEIDEN_PLUS,
     (1, 20, False), O.VW_UNIT),
    ("lattice", lambda: gg.lattice(48, 48, seed=7), O.PLEIDEN, (1, 20, False), O.VW_UNIT),
    ("rmat12", lambda: gg.rmat(12, seed=11), O.PLOUVAIN, (1, 1, True), O.VW_WEIGHTED_DEGREE),
    ("sbm", lambda: gg.config1_sbm(), O.LOUVAIN, (1, 1, True), O.VW_WEIGHTED_DEGREE),
]


def _with_tuning(t, fn):
    import paper_2608_01503_amd as L
    ctx = U.ctx()
    old = ctx.get_tuning()
    ctx.set_tuning(L.lcc_default_tuning(**t))
    try:
        return fn()
    finally:
        ctx.set_tuning(old)


@pytest.mark.parametrize("name,make,variant,lam,mode", CASES, ids=[c[0] for c in CASES])
def test_every_tuning_gives_the_same_result(name, make, variant, lam, mode):
    g = make()
    ref_lab, ref = U.run_gpu(g, variant, lam, mode)
    orc = U.run_oracle(g, variant, lam, mode)
    assert np.array_equal(ref_lab, orc.labels) and ref.N == orc.N
    for t in TUNINGS:
        lab, res = _with_tuning(t, lambda: U.run_gpu(g, variant, lam, mode))
        assert np.array_equal(lab, ref_lab), (name, t)
        assert (res.N, res.levels, res.flags, res.num_clusters) == (ref.N, ref.levels, ref.flags, ref.num_clusters)
        assert np.array_equal(res.trace, ref.trace), (name, t)


def test_fused_batch_under_tunings():
    import torch
    import paper_2608_01503_amd as L
    graphs = [gg.random_gnp(300 + 97 * k, 0.03, 70 + k, w_max=5) for k in range(12)]
    graphs.append(U.hub_graph(n=12000, hub_deg=(9000, 3000, 1500), seed=12))
    dev = [U.device_graph(g, O.VW_WEIGHTED_DEGREE) for g in graphs]
    lams = [(1, 1, True)] * len(graphs)
    var = [L.LCC_PLOUVAIN] * len(graphs)
    ref_lab, ref = U.ctx().cluster_batch(dev, lams, var)
    ref_lab = [x.cpu().numpy() for x in ref_lab]
    for t in TUNINGS:
        labs, res = _with_tuning(t, lambda: U.ctx().cluster_batch(dev, lams, var))
        torch.cuda.synchronize()
        for i in range(len(graphs)):
            assert np.array_equal(labs[i].cpu().numpy(), ref_lab[i]), (i, t)
            assert res[i].N == ref[i].N and res[i].levels == ref[i].levels


def test_set_tuning_rejects_out_of_range_settings():
    import paper_2608_01503_amd as L
    ctx = U.ctx()
    before = L.tuning_dict(ctx.get_tuning())
    bad = [dict(bucket_max=[5, 8, 16, 32, 128, 1024, 4096]),     # above a bucket's capacity
           dict(bucket_max=[4, 8, 16, 32, 128, 1024, 8193]),
           dict(bucket_max=[4, 8, 6, 32, 128, 1024, 4096]),      # decreasing
           dict(bucket_max=[-1, 8, 16, 32, 128, 1024, 4096]),
           dict(grid_cap=32), dict(grid_cap=70000), dict(hash_shift=-1), dict(hash_shift=3)]
    for t in bad:
        with pytest.raises(L.LccError) as e:
            ctx.set_tuning(L.lcc_default_tuning(**t))
        assert e.value.status == -1
        assert L.tuning_dict(ctx.get_tuning()) == before


def test_autotune_keeps_a_valid_tuning_and_results():
    import paper_2608_01503_amd as L
    ctx = L.Context(0)
    g = U.hub_graph(n=12000, hub_deg=(7000, 5000, 2000), seed=21)
    graph = U.device_graph(g, O.VW_WEIGHTED_DEGREE)
    before, bres = ctx.cluster(graph, (1, 1, True), L.LCC_PLOUVAIN)
    best, ms = ctx.autotune([graph], [(1, 1, True)], [L.LCC_PLOUVAIN], trials=1)
    assert ms > 0
    t = L.tuning_dict(best)
    assert t == L.tuning_dict(ctx.get_tuning())
    caps = [4, 8, 16, 32, 128, 1024, 8192]
    assert all(0 <= b <= c for b, c in zip(t["bucket_max"], caps)) and 64 <= t["grid_cap"] <= 65536
    assert 0 <= t["hash_shift"] <= 2
    after, ares = ctx.cluster(graph, (1, 1, True), L.LCC_PLOUVAIN)
    assert np.array_equal(before.cpu().numpy(), after.cpu().numpy()) and ares.N == bres.N
    # a batch of graphs
    graphs = [U.device_graph(gg.random_gnp(500 + 50 * k, 0.02, 90 + k, w_max=3), O.VW_WEIGHTED_DEGREE)
              for k in range(8)]
    best2, ms2 = ctx.autotune(graphs, [(1, 1, True)] * 8, [L.LCC_PLOUVAIN] * 8, trials=1)
    assert ms2 > 0 and L.tuning_dict(best2) == L.tuning_dict(ctx.get_tuning())
    ctx.close()
