"""Device memory comes only from the caller's allocator: a refused allocation is reported as LCC_ERR_OOM,
leaves the context usable (also after a failed workspace growth), and everything is returned by
lcc_destroy."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


class BudgetAllocator:
    """torch's caching allocator behind a byte budget; counts what is outstanding."""

    def __init__(self, budget):
        self.budget = budget
        self.live = {}

    @property
    def used(self):
        return sum(self.live.values())

    def alloc(self, nbytes):
        import torch
        if self.used + nbytes > self.budget:
            return None
        p = torch.cuda.caching_allocator_alloc(nbytes, 0)
        self.live[p] = nbytes
        return p

    def free(self, p):
        import torch
        self.live.pop(p)
        torch.cuda.caching_allocator_delete(p)


def test_refused_allocations_report_oom_and_the_context_recovers():
    import paper_2608_01503_amd as L
    small = gg.random_gnp(600, 0.02, 31, w_max=3)
    big = gg.rmat(13, seed=5)
    lam = (1, 1, True)
    ref_small = O.cluster(small, O.PLOUVAIN, lam=lam, vw_mode=O.VW_WEIGHTED_DEGREE)
    ref_big = O.cluster(big, O.PLOUVAIN, lam=lam, vw_mode=O.VW_WEIGHTED_DEGREE)
    gs = U.device_graph(small, O.VW_WEIGHTED_DEGREE)
    gb = U.device_graph(big, O.VW_WEIGHTED_DEGREE)
    a = BudgetAllocator(1 << 10)
    ctx = L.Context(0, allocator=(a.alloc, a.free))
    with pytest.raises(L.LccError) as e:  # not even the workspace fits
        ctx.cluster(gs, lam, L.LCC_PLOUVAIN)
    assert e.value.status == -8
    a.budget = 1 << 34
    lab, res = ctx.cluster(gs, lam, L.LCC_PLOUVAIN)
    assert np.array_equal(lab.cpu().numpy(), ref_small.labels) and res.N == ref_small.N
    # the workspace must grow for the larger graph and cannot: the old one is gone, the sizes must be too
    a.budget = a.used + (1 << 16)
    with pytest.raises(L.LccError) as e:
        ctx.cluster(gb, lam, L.LCC_PLOUVAIN)
    assert e.value.status == -8
    a.budget = 1 << 34
    lab, res = ctx.cluster(gs, lam, L.LCC_PLOUVAIN)
    assert np.array_equal(lab.cpu().numpy(), ref_small.labels) and res.N == ref_small.N
    lab, res = ctx.cluster(gb, lam, L.LCC_PLOUVAIN)
    assert np.array_equal(lab.cpu().numpy(), ref_big.labels) and res.N == ref_big.N
    ctx.close()
    assert a.live == {}
