"""The continuous-batching server: every request's result equals the same request run alone (a plain call),
whatever else is in flight, including fused groups of small Louvain requests and invalid requests."""
from __future__ import annotations

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
