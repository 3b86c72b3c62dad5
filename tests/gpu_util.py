"""Helpers for the GPU parity tests: run the HIP library and the oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np

import graphgen as gg
import oracle as O

_CTX = None


def ctx():
    global _CTX
    import paper_2608_01503_amd as L
    if _CTX is None:
        _CTX = L.Context(0)
    return _CTX


def device_graph(g, vw_mode, vw=None, offsets32=False, with_w=True):
    import torch
    import paper_2608_01503_amd as L
    dev = torch.device("cuda:0")
    off = torch.from_numpy(g.off.astype(np.int32) if offsets32 else g.off).to(dev)
    idx = torch.from_numpy(np.ascontiguousarray(g.idx)).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(g.w)).to(dev) if with_w else None
    vwt = torch.from_numpy(np.asarray(vw, dtype=np.int64)).to(dev) if vw is not None else None
    return L.make_graph(off, idx, w, vwt, vw_mode)


def host_graph(g, vw_mode, vw=None):
    import paper_2608_01503_amd as L
    vwa = np.ascontiguousarray(vw, dtype=np.int64) if vw is not None else None
    return L.make_graph(np.ascontiguousarray(g.off), np.ascontiguousarray(g.idx), np.ascontiguousarray(g.w), vwa,
                        vw_mode)


def run_gpu(g, variant, lam, vw_mode, vw=None, opts_kw=None, host=False, offsets32=False, trace=True, init=None,
            constraint=None):
    import torch
    import paper_2608_01503_amd as L
    graph = host_graph(g, vw_mode, vw) if host else device_graph(g, vw_mode, vw, offsets32)
    opts = L.lcc_default_options(**(opts_kw or {}))

    def arr(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.int32)
        return a if host else torch.from_numpy(a).cuda()
    labels, res = ctx().cluster(graph, lam, variant, opts, trace_capacity=1 << 14 if trace else 0,
                                init=arr(init), constraint=arr(constraint))
    torch.cuda.synchronize()
    lab = labels if isinstance(labels, np.ndarray) else labels.cpu().numpy()
    return lab, res


def run_oracle(g, variant, lam, vw_mode, vw=None, opts_kw=None, init=None, constraint=None):
    kw = dict(opts_kw or {})
    kw.pop("validate", None)
    o = O.make_opts(**kw) if kw else None
    return O.cluster(g, variant, lam=lam, vw_mode=vw_mode, vw=vw, opts=o, init=init, constraint=constraint)


def fp64_report(g, labels, lam, vw_mode, vw=None):
    """Eq. 1 and the Newman-Girvan modularity recomputed in FP64 from the labels alone (no integer score form):
    lambdaCC = I - lambda (sum_c W_c^2 - sum_v w(v)^2) with I the internal ordered edge weight, and
    Q = sum_c [I_c / W - gamma (W_c / W)^2].  Returns (lambdaCC, its scale, Q or None, Q's scale); a scale is
    the sum of the magnitudes of the terms, the yardstick of the rounding error near zero."""
    w = g.w.astype(np.float64) if g.w is not None else np.ones(len(g.idx))
    src = np.repeat(np.arange(g.n), np.diff(g.off))
    if vw_mode == O.VW_WEIGHTED_DEGREE:
        vwf = np.bincount(src, weights=w, minlength=g.n)
    elif vw_mode == O.VW_UNIT:
        vwf = np.ones(g.n)
    else:
        vwf = np.asarray(vw, dtype=np.float64)
    lab = np.asarray(labels, dtype=np.int64)
    same = lab[src] == lab[g.idx]
    I = float(w[same].sum())
    Wc = np.bincount(lab, weights=vwf, minlength=int(lab.max()) + 1 if g.n else 1)
    W = float(vwf.sum())
    lamf = lam[0] / (lam[1] * (W if lam[2] else 1.0))
    sW2, sw2 = float((Wc * Wc).sum()), float((vwf * vwf).sum())
    obj = I - lamf * (sW2 - sw2)
    scale = I + lamf * (sW2 + sw2)
    Q = Qs = None
    if vw_mode == O.VW_WEIGHTED_DEGREE and lam[2] and W > 0:
        gamma = lam[0] / lam[1]
        Q = I / W - gamma * sW2 / (W * W)
        Qs = I / W + gamma * sW2 / (W * W)
    return obj, scale, Q, Qs


def assert_fp64_report(g, labels, res, lam, vw_mode, vw=None, rel=1e-12):
    """The FP64 fields of a result agree with the independent FP64 recompute to `rel` (relative to the scale)."""
    obj, scale, Q, Qs = fp64_report(g, labels, lam, vw_mode, vw)
    assert abs(res.objective - obj) <= rel * max(scale, 1e-300), (res.objective, obj, scale)
    if Q is None:
        assert np.isnan(res.modularity)
    else:
        assert abs(res.modularity - Q) <= rel * Qs, (res.modularity, Q)


def assert_parity(g, variant, lam, vw_mode, vw=None, opts_kw=None, **kw):
    ref = run_oracle(g, variant, lam, vw_mode, vw, opts_kw, init=kw.get("init"), constraint=kw.get("constraint"))
    lab, res = run_gpu(g, variant, lam, vw_mode, vw, opts_kw, **kw)
    assert ref.status == 0
    assert np.array_equal(lab, ref.labels), f"labels differ ({(lab != ref.labels).sum()} of {g.n})"
    assert res.N == ref.N and res.obj_den == ref.q
    assert_fp64_report(g, lab, res, lam, vw_mode, vw)
    assert res.num_clusters == ref.num_clusters and res.levels == ref.levels and res.flags == ref.flags
    if res.trace is not None:
        assert res.trace.shape == ref.trace.shape, (res.trace.shape, ref.trace.shape)
        bad = np.nonzero((res.trace != ref.trace).any(axis=1))[0]
        assert len(bad) == 0, f"trace differs at records {bad[:5]}: gpu {res.trace[bad[:3]]} oracle {ref.trace[bad[:3]]}"
    return ref, res


def hub_graph(n=20000, hubs=(0, 1, 2), hub_deg=(9000, 6000, 3000), extra_p=0.0004, seed=9, w_max=5):
    """Random sparse graph plus a few hubs of given degrees (exercises every degree bucket)."""
    rng = np.random.default_rng(seed)
    pairs = []
    for h, d in zip(hubs, hub_deg):
        nb = rng.choice(np.arange(len(hubs), n), size=d, replace=False)
        pairs.append(np.stack([np.full(d, h), nb], axis=1))
    m = int(extra_p * n * n / 2)
    a = rng.integers(0, n, size=m)
    b = rng.integers(0, n, size=m)
    pairs.append(np.stack([a, b], axis=1))
    # some mid-degree vertices (buckets 4-6)
    for k, d in enumerate((100, 300, 900, 1500, 2500)):
        v = 10 + k
        nb = rng.choice(np.arange(20, n), size=d, replace=False)
        pairs.append(np.stack([np.full(d, v), nb], axis=1))
    P = np.concatenate(pairs)
    wts = rng.integers(1, w_max + 1, size=len(P))
    return gg.from_pairs(n, P, wts, name="hubs")
