"""The continuous-batching server: every request's result equals the same request run alone (a plain call),
whatever else is in flight, including fused groups of small Louvain requests and invalid requests."""
from __future__ import annotations

import threading
import time

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _drain(srv, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t, n in tickets.items():
            if t in out:
                continue
            try:
                r = srv.poll(t, n)
            except Exception as e:  # the request's own status
                out[t] = e
                continue
            if r is not None:
                out[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.001)
    return out


def _small_pool():
    pool = gg.serve_pool(sbm_blocks=(2, 60), rmat_scales=(9, 13), knn_n=(300, 3000), n_sbm=6, n_knn=6)
    graphs = [gg.serve_graph(s) for s in pool]
    fam = {"sbm": [], "rmat": [], "knn": []}
    for s, g in zip(pool, graphs):
        fam[s[0]].append(g)
    return fam


def test_server_mix_equals_alone():
    import paper_2608_01503_amd as L
    fam = _small_pool()
    reqs = gg.serve_requests(90, {k: len(v) for k, v in fam.items()})
    ctx = L.Context(0, allocator="hip")
    srv = L.Server(ctx, 32 << 30)
    tickets, meta = {}, {}
    for f, e, o, v in reqs:  # submitted back to back: many requests are queued together and fused
        g = fam[f][e]
        lam, mode = gg.SERVE_OBJECTIVES[o]
        t = srv.submit(U.host_graph(g, mode), lam, v)
        tickets[t] = g.n
        meta[t] = (g, lam, mode, v)
    done = _drain(srv, tickets)
    srv.close()
    for k, (t, r) in enumerate(done.items()):
        g, lam, mode, v = meta[t]
        assert not isinstance(r, Exception), r
        lab, res = r
        alone, ares = U.run_gpu(g, v, lam, mode, trace=False)
        assert np.array_equal(lab, alone) and res.N == ares.N and res.levels == ares.levels, (k, g.name)
        if k % 15 == 0:  # and a sample against the oracle
            ref = O.cluster(g, v, lam=lam, vw_mode=mode)
            assert np.array_equal(lab, ref.labels) and res.N == ref.N
    ctx.close()


def test_server_invalid_request_in_fused_group():
    import paper_2608_01503_amd as L
    good = [gg.random_gnp(400 + 50 * k, 0.02, 40 + k, w_max=4) for k in range(6)]
    asym = gg.Graph(n=3, off=np.array([0, 1, 2, 3], np.int64), idx=np.array([1, 2, 0], np.int32),
                    w=np.array([1, 1, 1], np.int32))
    ctx = L.Context(0, allocator="hip")
    srv = L.Server(ctx, 8 << 30)
    tickets, meta = {}, {}
    for g in good[:3] + [asym] + good[3:]:
        t = srv.submit(U.host_graph(g, O.VW_WEIGHTED_DEGREE), (1, 1, True), L.LCC_PLOUVAIN)
        tickets[t] = g.n
        meta[t] = g
    done = _drain(srv, tickets)
    srv.close()
    for t, r in done.items():
        g = meta[t]
        if g is asym:
            assert isinstance(r, L.LccError) and r.status == -2
        else:
            assert not isinstance(r, Exception), r
            ref = O.cluster(g, O.PLOUVAIN, lam=(1, 1, True), vw_mode=O.VW_WEIGHTED_DEGREE)
            assert np.array_equal(r[0], ref.labels) and r[1].N == ref.N
    with pytest.raises(L.LccError):
        srv2 = L.Server(ctx, 1 << 10)  # a budget below any footprint refuses the job
        try:
            srv2.submit(U.host_graph(good[0], O.VW_WEIGHTED_DEGREE), (1, 1, True), L.LCC_PLOUVAIN)
        finally:
            srv2.close()
    ctx.close()


class CountingAllocator:
    """torch's caching allocator, counting what is outstanding and its peak (called from the slot threads)."""

    def __init__(self):
        self.live = {}
        self.peak = 0
        self.lock = threading.Lock()

    def alloc(self, nbytes):
        import torch
        p = torch.cuda.caching_allocator_alloc(nbytes, 0)
        with self.lock:
            self.live[p] = nbytes
            self.peak = max(self.peak, sum(self.live.values()))
        return p

    def free(self, p):
        import torch
        with self.lock:
            self.live.pop(p)
        torch.cuda.caching_allocator_delete(p)


def _footprint(g, variant):
    import ctypes
    import paper_2608_01503_amd as L
    fp = ctypes.c_size_t(0)
    assert L.load().lcc_workspace_bytes(g.n, g.nnz, variant, ctypes.byref(fp)) == 0
    return fp.value


def test_server_holds_device_memory_within_the_budget():
    """Large and small jobs of both families mixed under a budget of about two large footprints: every byte the
    slots hold, idle ones included, is counted, so the allocator never has more outstanding than the budget, and every
    result equals the same request run alone."""
    import paper_2608_01503_amd as L
    large = [gg.rmat(14, seed=30 + k) for k in range(3)] + [gg.lattice(150, 150, seed=k) for k in range(2)]
    small = [gg.random_gnp(300 + 40 * k, 0.02, 50 + k, w_max=3) for k in range(24)]
    budget = 2 * max(_footprint(g, L.LCC_PLOUVAIN) for g in large) + (8 << 20)
    a = CountingAllocator()
    ctx = L.Context(0, allocator=(a.alloc, a.free))
    srv = L.Server(ctx, budget)
    tickets, meta = {}, {}
    jobs = [(g, L.LCC_PLOUVAIN) for g in large] + [(g, L.LCC_LOUVAIN) for g in small]
    jobs += [(large[0], L.LCC_PLEIDEN), (large[3], L.LCC_PLEIDEN_PLUS)]
    jobs += [(g, L.LCC_PLEIDEN if k % 2 else L.LCC_PLEIDEN_PLUS) for k, g in enumerate(small[:12])]  # fused groups
    order = np.random.default_rng(1).permutation(len(jobs))
    for i in order:
        g, v = jobs[i]
        t = srv.submit(U.host_graph(g, O.VW_WEIGHTED_DEGREE), (1, 1, True), v)
        tickets[t] = g.n
        meta[t] = (g, v)
    done = _drain(srv, tickets)
    srv.close()
    assert a.peak <= budget, (a.peak, budget)
    assert not a.live  # every slot context returned its memory when the server closed
    for t, r in done.items():
        g, v = meta[t]
        assert not isinstance(r, Exception), r
        alone, ares = U.run_gpu(g, v, (1, 1, True), O.VW_WEIGHTED_DEGREE, trace=False)
        assert np.array_equal(r[0], alone) and r[1].N == ares.N, (g.name, v)
    ctx.close()


def test_server_refuses_a_job_that_outgrows_the_budget_alone():
    """A budget equal to a job's footprint estimate while the job needs more (Louvain+ keeps every coarse level,
    and a slow coarsening keeps more than two input-sized levels): the job is refused the memory, rerun alone,
    refused again and reported as LCC_ERR_OOM; the server then runs the next job normally."""
    import paper_2608_01503_amd as L
    # an 80 x 80 unit-weight grid under CPM 2/3: each level merges few vertices, 13 levels of similar size
    cands = [(gg.lattice(80, 80, 0.0, 1, seed=2), (2, 3, False)), (gg.lattice(80, 80, 0.0, 1, seed=2), (3, 4, False))]
    a = CountingAllocator()
    pick = None
    for g, lam in cands:
        probe = L.Context(0, allocator=(a.alloc, a.free))
        a.peak = 0
        probe.cluster(U.host_graph(g, O.VW_UNIT), lam, L.LCC_PLOUVAIN)
        probe.close()
        if a.peak > _footprint(g, L.LCC_PLOUVAIN):
            pick = (g, lam)
            break
    if pick is None:
        pytest.skip("every candidate's coarse levels fit the footprint estimate")
    g, lam = pick
    ctx = L.Context(0, allocator=(a.alloc, a.free))
    srv = L.Server(ctx, _footprint(g, L.LCC_PLOUVAIN))
    t = srv.submit(U.host_graph(g, O.VW_UNIT), lam, L.LCC_PLOUVAIN)
    done = _drain(srv, {t: g.n})
    assert isinstance(done[t], L.LccError) and done[t].status == -8
    small = gg.random_gnp(200, 0.03, 9)
    t2 = srv.submit(U.host_graph(small, O.VW_WEIGHTED_DEGREE), (1, 1, True), L.LCC_PLOUVAIN)
    r = _drain(srv, {t2: small.n})[t2]
    ref = O.cluster(small, O.PLOUVAIN, lam=(1, 1, True), vw_mode=O.VW_WEIGHTED_DEGREE)
    assert not isinstance(r, Exception) and np.array_equal(r[0], ref.labels)
    srv.close()
    ctx.close()
