"""GPU parity of the fused batched form: many graphs clustered together as one union graph must give, graph by
graph, exactly the oracle's result (labels, exact objective, cluster and level counts, flags)."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

MOD = ((1, 1, True), O.VW_WEIGHTED_DEGREE)
CPM20 = ((1, 20, False), O.VW_UNIT)
CPM3 = ((1, 3, False), O.VW_UNIT)


def _batch(items, opts_kw=None, offsets32=()):
    """items: (graph, variant, lam, vw_mode, vw).  Runs one fused call and checks every graph."""
    import torch
    import paper_2608_01503_amd as L
    graphs = [U.device_graph(g, m, vw, offsets32=(i in offsets32)) for i, (g, v, lam, m, vw) in enumerate(items)]
    opts = L.lcc_default_options(**(opts_kw or {}))
    labs, ress = U.ctx().cluster_batch(graphs, [it[2] for it in items], [it[1] for it in items], opts=opts)
    torch.cuda.synchronize()
    for i, ((g, v, lam, m, vw), lab, res) in enumerate(zip(items, labs, ress)):
        ref = U.run_oracle(g, v, lam, m, vw, opts_kw)
        assert ref.status == 0
        got = lab.cpu().numpy()
        assert np.array_equal(got, ref.labels), f"graph {i}: labels differ ({(got != ref.labels).sum()} of {g.n})"
        assert res.N == ref.N and res.obj_den == ref.q, f"graph {i}"
        assert res.num_clusters == ref.num_clusters and res.levels == ref.levels and res.flags == ref.flags, i
    return ress


def test_fused_mixed_graphs_and_objectives():
    rng = np.random.default_rng(3)
    items = [
        (gg.config1_sbm(), O.PLOUVAIN, *MOD, None),
        (gg.random_gnp(1500, 0.004, 101, w_max=7), O.LOUVAIN, *MOD, None),
        (gg.random_gnp(5000, 0.001, 102, w_max=100), O.PLOUVAIN, *CPM20, None),
        (U.hub_graph(), O.PLOUVAIN, *MOD, None),
        (gg.Graph(n=0, off=np.zeros(1, np.int64), idx=np.zeros(0, np.int32), w=np.zeros(0, np.int32)),
         O.PLOUVAIN, *CPM20, None),
        (gg.rmat(12, 16, seed=21), O.PLOUVAIN, *CPM3, None),
        (gg.from_pairs(2, [(0, 1)]), O.PLOUVAIN, *MOD, None),
        (gg.Graph(n=5, off=np.zeros(6, np.int64), idx=np.zeros(0, np.int32), w=np.zeros(0, np.int32)),
         O.LOUVAIN, *CPM20, None),
        (gg.lattice(40, 30, 0.1, 100, 3), O.PLOUVAIN, *CPM20, None),
    ]
    g9 = gg.random_gnp(800, 0.01, 5, w_max=9)
    items.append((g9, O.PLOUVAIN, (1, 400, False), O.VW_GIVEN, rng.integers(0, 20, size=g9.n)))
    _batch(items, offsets32=(0, 6))


def test_fused_many_small_graphs():
    rng = np.random.default_rng(11)
    items = []
    for k in range(120):
        n = int(np.exp(rng.uniform(np.log(30), np.log(3000))))
        p = min(0.5, 8.0 / n)
        g = gg.random_gnp(n, p, 1000 + k, w_max=int(rng.integers(1, 50)))
        obj = [MOD, CPM20, CPM3][k % 3]
        items.append((g, O.PLOUVAIN if k % 4 else O.LOUVAIN, *obj, None))
    _batch(items)


def test_fused_options_and_repeat():
    items = [(gg.rmat(11, 16, seed=30 + k), O.PLOUVAIN, *MOD, None) for k in range(5)]
    for kw in [dict(pass_limit=12, phases=((3, 4, 8), (1, 4, 12))), dict(eps=(0, 1)), dict(pass_limit=1),
               dict(max_levels=2)]:
        _batch(items, opts_kw=kw)
    a = _batch(items)
    b = _batch(items)
    assert [r.N for r in a] == [r.N for r in b]


def test_fused_errors_match_single():
    import paper_2608_01503_amd as L
    good = gg.random_gnp(300, 0.02, 7, w_max=3)
    asym = gg.Graph(n=3, off=np.array([0, 1, 2, 3], np.int64), idx=np.array([1, 2, 0], np.int32),
                    w=np.array([1, 1, 1], np.int32))
    graphs = [U.device_graph(good, O.VW_WEIGHTED_DEGREE), U.device_graph(asym, O.VW_WEIGHTED_DEGREE)]
    with pytest.raises(L.LccError) as e:
        U.ctx().cluster_batch(graphs, [(1, 1, True)] * 2, [O.PLOUVAIN] * 2)
    assert e.value.status == -2  # not symmetric
    graphs = [U.device_graph(good, O.VW_WEIGHTED_DEGREE)] * 2
    with pytest.raises(L.LccError) as e:
        U.ctx().cluster_batch(graphs, [(1, 1, True), (3, 2, False)], [O.PLOUVAIN] * 2)
    assert e.value.status == -6  # lambda outside [0, 1]
    # a good batch still runs on the same context afterwards
    _batch([(good, O.PLOUVAIN, *MOD, None), (good, O.LOUVAIN, *CPM20, None)])


def test_knn_generator_device_matches_host():
    import torch
    for n, K, g in [(2000, 7, 3), (6000, 33, 11)]:
        ref = gg.knn_graph(n, K, 5, g)
        off, idx, w = gg.knn_graph_torch(n, K, 5, g, torch.device("cuda:0"))
        assert np.array_equal(off.cpu().numpy(), ref.off)
        assert np.array_equal(idx.cpu().numpy(), ref.idx)
        assert np.array_equal(w.cpu().numpy(), ref.w)


def test_fused_knn_batch_full_size_sample():
    """48 graphs of the batched kNN workload at their full sizes (500..50,000 vertices) in one fused call:
    every graph equals its own plain call, and every third graph (the largest included) equals the oracle."""
    import torch
    import paper_2608_01503_amd as L
    dev = torch.device("cuda:0")
    spec = gg.knn_batch_spec(48, 5)
    keep, graphs = [], []
    for g, (n, K) in enumerate(spec):
        t = gg.knn_graph_torch(n, K, 5, g, dev)
        keep.append(t)
        graphs.append(L.make_graph(*t, None, L.LCC_VW_WEIGHTED_DEGREE))
    opts = L.lcc_default_options()
    labs, ress = U.ctx().cluster_batch(graphs, [(1, 1, True)] * len(graphs), [L.LCC_PLOUVAIN] * len(graphs), opts=opts)
    torch.cuda.synchronize()
    for i, gr in enumerate(graphs):
        lab, res = U.ctx().cluster(gr, (1, 1, True), L.LCC_PLOUVAIN, opts)
        torch.cuda.synchronize()
        assert torch.equal(lab, labs[i]) and res.N == ress[i].N and res.levels == ress[i].levels, i
    big = max(range(len(graphs)), key=lambda i: graphs[i].n)
    for i in sorted({big} | set(range(0, len(graphs), 3))):
        off, idx, w = keep[i]
        g = gg.Graph(n=graphs[i].n, off=off.cpu().numpy(), idx=idx.cpu().numpy(), w=w.cpu().numpy())
        ref = O.cluster(g, O.PLOUVAIN, lam=(1, 1, True), vw_mode=O.VW_WEIGHTED_DEGREE)
        assert np.array_equal(labs[i].cpu().numpy(), ref.labels) and ress[i].N == ref.N, i


def test_fused_batch_with_ablation_options():
    items = [(gg.rmat(11, 16, seed=50 + k), O.PLOUVAIN, *MOD, None) for k in range(3)] + \
            [(gg.random_gnp(900, 0.006, 60, w_max=5), O.LOUVAIN, *CPM20, None)]
    for sym in (1, 2):
        _batch(items, opts_kw=dict(phases=((0, 1, 6),), symmetry=sym))


def _empty(n):
    return gg.Graph(n=n, off=np.zeros(n + 1, np.int64), idx=np.zeros(0, np.int32), w=np.zeros(0, np.int32))


def test_fused_pleiden_mixed_graphs():
    """pLeiden and pLeiden+ graphs in one fused call: alternate local moves (Sec. V-A) on some graphs and not on
    others at the same level, refinements that make no progress (those graphs repeat their level while the
    others go on; a two-vertex graph stops with the no-progress flag), empty graphs, hubs and per-graph
    lambdas and vertex weights."""
    rng = np.random.default_rng(5)
    items = [
        (gg.random_gnp(400, 0.01, 100, w_max=3), O.PLEIDEN, *CPM20, None),
        (gg.random_gnp(400, 0.01, 102, w_max=3), O.PLEIDEN_PLUS, *CPM20, None),
        (gg.rmat(11, seed=40), O.PLEIDEN, (1, 10, False), O.VW_UNIT, None),
        (gg.lattice(40, 40, seed=52), O.PLEIDEN_PLUS, *CPM20, None),
        (gg.config1_sbm(), O.PLEIDEN_PLUS, *MOD, None),
        (gg.knn_graph(800, 8, 5, 2), O.PLEIDEN, *MOD, None),
        (gg.from_pairs(2, [(0, 1)]), O.PLEIDEN, *CPM20, None),
        (_empty(0), O.PLEIDEN, *CPM20, None),
        (_empty(5), O.PLEIDEN_PLUS, *CPM20, None),
        (U.hub_graph(n=12000, hub_deg=(9000, 6000, 1500), seed=4), O.PLEIDEN_PLUS, *CPM20, None),
        (gg.rmat(12, 16, seed=21), O.PLEIDEN, *CPM3, None),
    ]
    g9 = gg.random_gnp(800, 0.01, 5, w_max=9)
    items.append((g9, O.PLEIDEN, (1, 400, False), O.VW_GIVEN, rng.integers(0, 20, size=g9.n)))
    ress = _batch(items, offsets32=(0, 6))
    assert ress[6].flags & 2  # the two-vertex graph: no progress in three refinements


def test_fused_pleiden_many_small_graphs_and_options():
    rng = np.random.default_rng(17)
    items = []
    for k in range(96):
        n = int(np.exp(rng.uniform(np.log(20), np.log(2500))))
        g = gg.random_gnp(n, min(0.5, 6.0 / n), 2000 + k, w_max=int(rng.integers(1, 30)))
        obj = [MOD, CPM20, CPM3][k % 3]
        items.append((g, O.PLEIDEN_PLUS if k % 2 else O.PLEIDEN, *obj, None))
    _batch(items)
    for kw in [dict(max_levels=3), dict(seed=7), dict(pass_limit=2, phases=((1, 2, 2),))]:
        _batch(items[:40], opts_kw=kw)


def test_mixed_families_run_one_by_one():
    """A batch with both families is not fused; the results are still every graph's own."""
    items = [(gg.random_gnp(300, 0.02, 70, w_max=3), O.PLOUVAIN, *MOD, None),
             (gg.random_gnp(300, 0.02, 71, w_max=3), O.PLEIDEN, *CPM20, None)]
    _batch(items)
