"""lcc_cluster_noalloc (the entry point that allocates nothing) against lcc_cluster, through the C-ABI: the same
labels, exact objective, level count, flags and per-pass trace, on two calls in a row with the second input
smaller than the first, without a single call of the context's allocator; and a graph beyond the scratch size is
refused before any device work."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _counting_context():
    import torch
    import paper_2608_01503_amd as L
    calls = []

    def alloc(nbytes):
        calls.append(int(nbytes))
        return torch.cuda.caching_allocator_alloc(int(nbytes), 0)

    def free(p):
        torch.cuda.caching_allocator_delete(p)

    return L.Context(0, allocator=(alloc, free)), calls


def test_noalloc_equals_cluster_and_allocates_nothing():
    import torch
    import paper_2608_01503_amd as L
    ctx, calls = _counting_context()
    cases = [  # the larger input first: the second call reuses the array with a smaller layout
        (gg.rmat(14, 16, seed=3), L.LCC_PLEIDEN, (1, 20, False), L.LCC_VW_UNIT),
        (gg.config1_sbm(), L.LCC_PLOUVAIN, (1, 1, True), L.LCC_VW_WEIGHTED_DEGREE),
        (gg.lattice(60, 50, 0.1, 100, 3), L.LCC_PLEIDEN_PLUS, (1, 20, False), L.LCC_VW_UNIT),
    ]
    for g, variant, lam, mode in cases:
        assert L.lcc_workspace_bytes(g.n, int(g.off[-1]), variant) <= L.LCC_NOALLOC_SCRATCH_BYTES
        graph = U.device_graph(g, mode)
        out = torch.full((g.n,), -1, dtype=torch.int32, device="cuda:0")
        torch.cuda.synchronize()
        before = len(calls)
        lab_a, res_a = ctx.cluster(graph, lam, variant, labels_out=out, trace_capacity=1 << 14, noalloc=True)
        torch.cuda.synchronize()
        assert len(calls) == before, "lcc_cluster_noalloc called the context's allocator"
        got = lab_a.cpu().numpy()
        lab_b, res_b = ctx.cluster(graph, lam, variant, trace_capacity=1 << 14)
        torch.cuda.synchronize()
        assert np.array_equal(got, lab_b.cpu().numpy())
        assert (res_a.N, res_a.obj_den, res_a.num_clusters, res_a.levels, res_a.flags) == \
            (res_b.N, res_b.obj_den, res_b.num_clusters, res_b.levels, res_b.flags)
        assert np.array_equal(res_a.trace, res_b.trace)
        ref = U.run_oracle(g, variant, lam, mode)
        assert np.array_equal(got, ref.labels) and res_a.N == ref.N
    # once more after the plain calls grew the context's own workspace: still no allocation, same result
    g, variant, lam, mode = cases[1]
    graph = U.device_graph(g, mode)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()
    before = len(calls)
    lab, res = ctx.cluster(graph, lam, variant, labels_out=out, noalloc=True)
    torch.cuda.synchronize()
    assert len(calls) == before
    assert np.array_equal(lab.cpu().numpy(), O.cluster(g, O.PLOUVAIN).labels)
    ctx.close()


def test_noalloc_refuses_graphs_beyond_the_scratch():
    import torch
    import paper_2608_01503_amd as L
    ctx, calls = _counting_context()
    n = 1 << 16
    while L.lcc_workspace_bytes(n, 0, L.LCC_PLOUVAIN) <= L.LCC_NOALLOC_SCRATCH_BYTES:
        n *= 2
    off = torch.zeros(n + 1, dtype=torch.int64, device="cuda:0")  # a valid graph without edges
    idx = torch.zeros(1, dtype=torch.int32, device="cuda:0")[:0]
    graph = L.make_graph(off, idx, None, None, L.LCC_VW_UNIT)
    out = torch.empty(n, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()
    with pytest.raises(L.LccError) as e:
        ctx.cluster(graph, (1, 20, False), L.LCC_PLOUVAIN, labels_out=out, noalloc=True)
    assert e.value.status == -1 and "no-allocation scratch" in str(e.value)
    assert not calls
    # the entry point still works afterwards
    g = gg.config1_sbm()
    lab, res = ctx.cluster(U.device_graph(g, L.LCC_VW_WEIGHTED_DEGREE), (1, 1, True), L.LCC_PLOUVAIN,
                           labels_out=torch.empty(g.n, dtype=torch.int32, device="cuda:0"), noalloc=True)
    assert np.array_equal(lab.cpu().numpy(), O.cluster(g, O.PLOUVAIN).labels)
    ctx.close()
