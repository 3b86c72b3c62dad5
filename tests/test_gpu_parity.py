"""GPU parity: the HIP library (through the C-ABI) against the CPU oracle, bit for bit.

Labels, the exact objective numerator, cluster and level counts, flags and the per-pass / per-level trace
(candidates, kept moves, objective after every pass) must all be identical.  Inputs are seeded and
synthetic; sizes span several tiles of every kernel and every degree bucket (sub-wave groups, wavefront,
workgroup, hub chunks)."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

VARIANTS = [O.LOUVAIN, O.PLOUVAIN, O.PLEIDEN, O.PLEIDEN_PLUS]
MOD = ((1, 1, True), O.VW_WEIGHTED_DEGREE)
CPM20 = ((1, 20, False), O.VW_UNIT)
CPM3 = ((1, 3, False), O.VW_UNIT)
LP = ((0, 1, False), O.VW_UNIT)


@pytest.mark.parametrize("variant", VARIANTS)
def test_sbm_2000_all_variants(variant):
    g = gg.config1_sbm()
    U.assert_parity(g, variant, *MOD, offsets32=True)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("obj", [MOD, CPM20, CPM3, LP], ids=["mod", "cpm20", "cpm3", "lp"])
def test_random_graphs(variant, obj):
    for k, (n, p, wmax) in enumerate([(300, 0.02, 1), (1500, 0.004, 7), (5000, 0.001, 100)]):
        g = gg.random_gnp(n, p, 100 + k, w_max=wmax)
        U.assert_parity(g, variant, *obj)


@pytest.mark.parametrize("variant", VARIANTS)
def test_hubs_every_bucket(variant):
    g = U.hub_graph()
    d = np.diff(g.off)
    # hub chunks (above 8192), the 16384- and 8192-slot workgroup tables, the 2048-slot one
    assert d.max() > 8192 and ((d > 4096) & (d <= 8192)).any() and ((d > 1024) & (d <= 4096)).any()
    assert ((d > 128) & (d <= 1024)).any()
    U.assert_parity(g, variant, *MOD)
    U.assert_parity(g, variant, *CPM20)


@pytest.mark.parametrize("variant", VARIANTS)
def test_rmat_scale14(variant):
    g = gg.rmat(14, 16, seed=7)
    U.assert_parity(g, variant, *MOD)


@pytest.mark.parametrize("variant", [O.PLEIDEN, O.PLOUVAIN])
def test_lattice_cpm(variant):
    g = gg.lattice(96, 80, 0.1, 100, 3)
    U.assert_parity(g, variant, *CPM20)


def test_given_vertex_weights_and_options():
    g = gg.random_gnp(800, 0.01, 5, w_max=9)
    vw = np.random.default_rng(1).integers(0, 20, size=g.n)
    U.assert_parity(g, O.PLOUVAIN, (1, 400, False), O.VW_GIVEN, vw=vw)
    U.assert_parity(g, O.PLEIDEN, (1, 400, False), O.VW_GIVEN, vw=vw)
    # other temperature schedules, tie windows, pass limits and seeds
    for kw in [dict(pass_limit=12, phases=((3, 4, 8), (1, 4, 12))), dict(phases=((0, 1, 6),)),
               dict(eps=(0, 1)), dict(eps=(1, 2)), dict(pass_limit=1), dict(seed=12345)]:
        U.assert_parity(g, O.PLOUVAIN, *MOD, opts_kw=kw)
        U.assert_parity(g, O.PLEIDEN, *CPM20, opts_kw=kw)


def test_host_memory_and_32bit_offsets():
    g = gg.random_gnp(2500, 0.003, 17, w_max=4)
    U.assert_parity(g, O.PLOUVAIN, *MOD, host=True)
    U.assert_parity(g, O.PLEIDEN, *CPM20, offsets32=True)


def test_edge_cases():
    # isolated vertices only (CPM: everything stays a singleton)
    g = gg.Graph(n=7, off=np.zeros(8, np.int64), idx=np.zeros(0, np.int32), w=np.zeros(0, np.int32))
    for v in VARIANTS:
        U.assert_parity(g, v, *CPM20)
    # one edge, and a path
    U.assert_parity(gg.from_pairs(2, [(0, 1)]), O.PLOUVAIN, *MOD)
    U.assert_parity(gg.from_pairs(6, [(i, i + 1) for i in range(5)]), O.PLEIDEN, *MOD)
    # two cliques joined by one edge
    pairs = [(i, j) for i in range(6) for j in range(i + 1, 6)] + [(6 + i, 6 + j) for i in range(6) for j in range(i + 1, 6)]
    g2 = gg.from_pairs(12, pairs + [(5, 6)])
    for v in VARIANTS:
        ref, res = U.assert_parity(g2, v, *MOD)
        assert res.num_clusters == 2
    # star with more leaves than a hub chunk
    g3 = gg.from_pairs(9001, [(0, i) for i in range(1, 9001)])
    for v in VARIANTS:
        U.assert_parity(g3, v, *MOD)
        U.assert_parity(g3, v, *CPM3)


def test_empty_graph():
    import paper_2608_01503_amd as L
    g = gg.Graph(n=0, off=np.zeros(1, np.int64), idx=np.zeros(0, np.int32), w=np.zeros(0, np.int32))
    lab, res = U.run_gpu(g, O.PLOUVAIN, *CPM20)
    assert len(lab) == 0 and res.num_clusters == 0


def _status_gpu(g, lam, vw_mode, vw=None):
    import paper_2608_01503_amd as L
    try:
        U.run_gpu(g, O.PLOUVAIN, lam, vw_mode, vw)
        return 0
    except L.LccError as e:
        return e.status


def test_error_statuses_match_oracle():
    def G(n, off, idx, w):
        return gg.Graph(n=n, off=np.array(off, np.int64), idx=np.array(idx, np.int32), w=np.array(w, np.int32))
    cases = [
        (G(2, [0, 1, 2], [0, 0], [1, 1]), MOD),                   # self-loop
        (G(3, [0, 2, 3, 4], [2, 1, 0, 0], [1, 1, 1, 1]), MOD),    # unsorted
        (G(3, [0, 1, 2, 3], [1, 2, 0], [1, 1, 1]), MOD),          # not symmetric
        (G(2, [0, 1, 2], [1, 0], [2, 3]), MOD),                   # asymmetric weight
        (G(2, [0, 1, 2], [1, 0], [0, 0]), MOD),                   # weight 0
        (G(2, [0, 1, 2], [1, 5], [1, 1]), MOD),                   # index out of range
        (G(3, [0, 1, 3, 4], [1, 0, 2, 1], [1, 1, 2, 2]), ((3, 2, False), O.VW_UNIT)),   # lambda > 1
        (G(3, [0, 1, 3, 4], [1, 0, 2, 1], [1, 1, 2, 2]), ((1, 0, False), O.VW_UNIT)),   # zero denominator
        (G(3, [0, 1, 3, 4], [1, 0, 2, 1], [2 ** 31 - 1] * 4), MOD),       # total edge weight >= 2^32
        (G(3, [0, 0, 0, 0], [], []), MOD),                        # modularity with no edges: W = 0
        (G(4, [0, 1, 2, 3, 4], [2, 3, 1, 0], [1, 1, 1, 1]), MOD), # as many upper as lower entries, no reverses
        (G(2, [0, 1, 2], [1, 0], [759250125] * 2), MOD),         # q W_E + p W^2 = 8 x^2 just above 2^62
        (G(2, [0, 1, 2], [1, 0], [2 ** 30] * 2), MOD),           # (the bound before it was raised)
    ]
    for g, (lam, mode) in cases:
        ref = O.cluster(g, O.PLOUVAIN, lam=lam, vw_mode=mode)
        assert ref.status != 0
        assert _status_gpu(g, lam, mode) == ref.status, (g, lam)


@pytest.mark.parametrize("where", ["hub", "wave", "group"])
def test_symmetry_check_is_exact(where):
    """One entry's weight changed (or one reverse entry moved to another neighbour) in a hub row, a mid-degree
    row or a short row: the device check compares every entry with its reverse, so each is NOT_SYMMETRIC, as
    in the oracle; the unmodified graph passes."""
    g = U.hub_graph(n=12000, hub_deg=(9000, 2000, 700), seed=12)  # row 0 in the hub chunks
    deg = np.diff(g.off)
    v = {"hub": 0, "wave": int(np.nonzero((deg > 32) & (deg <= 128))[0][0]),
         "group": int(np.nonzero((deg > 1) & (deg <= 4))[0][0])}[where]
    assert _status_gpu(g, *MOD) == 0
    w = g.w.copy()
    w[g.off[v] + 1] += 1
    bad = gg.Graph(n=g.n, off=g.off, idx=g.idx, w=w)
    assert O.cluster(bad, O.PLOUVAIN, lam=MOD[0], vw_mode=MOD[1]).status == -2
    assert _status_gpu(bad, *MOD) == -2
    # the last entry of row v moved to a larger id whose row has no entry for v (the row stays ascending)
    idx = g.idx.copy()
    j = g.off[v + 1] - 1
    cand = [u for u in range(idx[j] + 1, g.n) if u != v]
    if cand:
        idx[j] = cand[0]
        bad2 = gg.Graph(n=g.n, off=g.off, idx=idx, w=g.w)
        assert O.cluster(bad2, O.PLOUVAIN, lam=MOD[0], vw_mode=MOD[1]).status == -2
        assert _status_gpu(bad2, *MOD) == -2


def test_symmetry_check_by_transposition():
    """Graphs above 2^23 entries are checked by transposing (stable sort by target, then an entry-by-entry
    comparison with the CSR) instead of searching: one weight changed on one side, one entry moved to another
    neighbour, or one reverse entry of a hub edge missing are each NOT_SYMMETRIC, as in the oracle, and the
    unmodified graph passes."""
    g = gg.rmat(19, seed=3)
    assert g.nnz > 2 ** 23
    assert _status_gpu(g, *MOD) == 0
    deg = np.diff(g.off)
    hub = int(np.argmax(deg))
    mid = int(np.nonzero((deg > 32) & (deg <= 128))[0][7])
    w = g.w.copy()
    w[g.off[mid] + 3] += 1
    bad = gg.Graph(n=g.n, off=g.off, idx=g.idx, w=w)
    assert O.setup(bad)[0] == -2 and _status_gpu(bad, *MOD) == -2
    # the last entry of the hub's row moved to a larger id whose row has no entry for the hub
    idx = g.idx.copy()
    j = g.off[hub + 1] - 1
    u = next(x for x in range(int(idx[j]) + 1, g.n)
             if x != hub and hub not in g.idx[g.off[x]:g.off[x + 1]])
    idx[j] = u
    bad2 = gg.Graph(n=g.n, off=g.off, idx=idx, w=g.w)
    assert O.setup(bad2)[0] == -2 and _status_gpu(bad2, *MOD) == -2
    # the check transposes the entries towards higher ids and matches them with the entries towards lower ids:
    # a lower entry's weight changed, a lower entry moved to another lower id, and the last lower entry of a row
    # moved to a higher id (one lower entry fewer than upper ones) are each NOT_SYMMETRIC as well
    rows = np.repeat(np.arange(g.n), deg)
    lo = np.bincount(rows[g.idx < rows], minlength=g.n)

    def gap_after(j, x0):  # the smallest id in (x0, idx[j + 1]) whose row lacks the row of j
        r = int(rows[j])
        return next((x for x in range(x0 + 1, int(g.idx[j + 1])) if x != r and r not in g.idx[g.off[x]:g.off[x + 1]]),
                    None)

    cand = np.nonzero((lo >= 3) & (deg - lo >= 2) & (deg <= 64))[0]
    r = next(int(x) for x in cand if gap_after(g.off[x], int(g.idx[g.off[x]])) is not None
             and gap_after(g.off[x] + lo[x] - 1, int(x)) is not None)
    w = g.w.copy()
    w[g.off[r]] += 1
    assert _status_gpu(gg.Graph(n=g.n, off=g.off, idx=g.idx, w=w), *MOD) == -2
    idx = g.idx.copy()
    idx[g.off[r]] = gap_after(g.off[r], int(g.idx[g.off[r]]))
    bad3 = gg.Graph(n=g.n, off=g.off, idx=idx, w=g.w)
    assert O.setup(bad3)[0] == -2 and _status_gpu(bad3, *MOD) == -2
    idx = g.idx.copy()
    jl = g.off[r] + lo[r] - 1
    idx[jl] = gap_after(jl, r)
    bad4 = gg.Graph(n=g.n, off=g.off, idx=idx, w=g.w)
    assert O.setup(bad4)[0] == -2 and _status_gpu(bad4, *MOD) == -2


HEAVY = [("rmat12", lambda: gg.rmat(12, seed=11), O.PLOUVAIN),
         ("hubs", lambda: U.hub_graph(n=12000, hub_deg=(9000, 6000, 1500), seed=4), O.PLEIDEN_PLUS),
         ("lattice", lambda: gg.lattice(40, 40, seed=7), O.PLEIDEN),
         ("sbm", lambda: gg.sbm(8, 120, 0.2, 0.01, seed=3), O.LOUVAIN)]


@pytest.mark.parametrize("name,make,variant", HEAVY, ids=[h[0] for h in HEAVY])
def test_modularity_with_weight_total_above_2_30(name, make, variant):
    """Weight totals between 2^30 and the 2^62 bound (W about 1.45e9): scores, deltas, gains and objective
    numerators then run up to about 2^62, where only 128-bit tests and modulo-2^64 sums stay exact."""
    g = gg.reweight(make(), 1_450_000_000, seed=17)
    W = int(g.w.astype(np.int64).sum())
    assert 2 ** 30 < W and W * W + W * W < 2 ** 62
    U.assert_parity(g, variant, *MOD)


def test_largest_admitted_pair():
    g = gg.Graph(n=2, off=np.array([0, 1, 2], np.int64), idx=np.array([1, 0], np.int32),
                 w=np.array([759250124] * 2, np.int32))
    ref, res = U.assert_parity(g, O.PLOUVAIN, *MOD)
    assert res.N == 2 * 759250124 ** 2


def test_deterministic_repeat():
    g = gg.rmat(13, 16, seed=11)
    a, ra = U.run_gpu(g, O.PLEIDEN, *MOD)
    b, rb = U.run_gpu(g, O.PLEIDEN, *MOD)
    assert np.array_equal(a, b) and ra.N == rb.N


def test_objective_entry_point():
    import paper_2608_01503_amd as L
    g = gg.random_gnp(3000, 0.002, 23, w_max=3)
    rng = np.random.default_rng(2)
    C = rng.integers(0, 50, size=g.n).astype(np.int32)
    st, vw, p, q = O.setup(g)
    want = O.objective(g, vw, p, q, C)
    import torch
    res = U.ctx().objective(U.device_graph(g, O.VW_WEIGHTED_DEGREE), torch.from_numpy(C).cuda(), (1, 1, True))
    assert res.N == want and res.obj_den == q
    # the host evaluation (lcc_objective) and the device one (lcc_objective_device) agree field by field
    hg = L.make_graph(g.off, g.idx, g.w, None, L.LCC_VW_WEIGHTED_DEGREE)
    h = L.lcc_objective(hg, C, (1, 1, True))
    assert (h.N, h.obj_den, h.num_clusters, h.levels, h.flags) == (res.N, res.obj_den, res.num_clusters, res.levels,
                                                                   res.flags)
    assert h.objective == res.objective and h.modularity == res.modularity


def test_batch_equals_single():
    import torch
    import paper_2608_01503_amd as L
    gs = [gg.random_gnp(200 + 150 * k, 0.02, 300 + k, w_max=5) for k in range(6)]
    lams = [(1, 1, True), (1, 20, False)] * 3
    modes = [O.VW_WEIGHTED_DEGREE, O.VW_UNIT] * 3
    variants = [O.PLOUVAIN, O.PLEIDEN, O.LOUVAIN, O.PLEIDEN_PLUS, O.PLOUVAIN, O.PLEIDEN]
    graphs = [U.device_graph(g, m) for g, m in zip(gs, modes)]
    labs, ress = U.ctx().cluster_batch(graphs, lams, variants)
    torch.cuda.synchronize()
    for g, lam, m, v, lab, res in zip(gs, lams, modes, variants, labs, ress):
        ref = O.cluster(g, v, lam=lam, vw_mode=m)
        assert np.array_equal(lab.cpu().numpy(), ref.labels) and res.N == ref.N


def test_pleiden_cpm_large_alternate_moves():
    """R-MAT scale 16 with CPM 1/10: about 30 levels run the alternate local move, with up to ~7,500 movers
    (the per-cluster prefix flows span several sort tiles)."""
    g = gg.rmat(16, 16, seed=8)
    ref, res = U.assert_parity(g, O.PLEIDEN, (1, 10, False), O.VW_UNIT)
    k = [int(r[4]) for r in ref.trace if r[0] == 3]
    assert len(k) > 10 and max(k) > 4096


@pytest.mark.parametrize("variant", [O.PLEIDEN, O.PLEIDEN_PLUS])
def test_iterated_pleiden_from_initial_clustering(variant):
    """pLeiden fed its own previous output (Alg. 5's C_in), three iterations, each against the oracle."""
    for g, obj in [(gg.config1_sbm(), MOD), (gg.rmat(13, 16, seed=12), CPM20), (U.hub_graph(), MOD)]:
        prev = U.run_oracle(g, variant, *obj).labels
        for _ in range(3):
            ref, res = U.assert_parity(g, variant, *obj, init=prev)
            prev = ref.labels


def test_louvain_initial_and_constraint_clusterings():
    rng = np.random.default_rng(4)
    for g, obj in [(gg.config1_sbm(), MOD), (gg.rmat(14, 16, seed=13), MOD), (gg.lattice(60, 50, 0.1, 100, 3), CPM20),
                   (U.hub_graph(), CPM3)]:
        first = U.run_oracle(g, O.PLOUVAIN, *obj)
        # the Louvain+ iteration of Sec. IV-D: the previous result as the constraint
        U.assert_parity(g, O.PLOUVAIN, *obj, constraint=first.labels)
        U.assert_parity(g, O.LOUVAIN, *obj, constraint=rng.integers(0, 9, size=g.n))
        # the older iteration: the previous result as the level-0 start
        U.assert_parity(g, O.PLOUVAIN, *obj, init=first.labels)
    g = gg.random_gnp(2500, 0.003, 17, w_max=4)
    first = U.run_oracle(g, O.PLOUVAIN, *MOD)
    U.assert_parity(g, O.PLOUVAIN, *MOD, host=True, constraint=first.labels)
    U.assert_parity(g, O.PLEIDEN, *MOD, host=True, init=first.labels)


def test_iteration_input_errors():
    import paper_2608_01503_amd as L
    g = gg.random_gnp(300, 0.02, 7, w_max=3)
    z = np.zeros(g.n, dtype=np.int32)
    for kw, variant in [(dict(constraint=z), O.PLEIDEN), (dict(constraint=z, init=z), O.PLOUVAIN),
                        (dict(init=np.full(g.n, g.n, dtype=np.int32)), O.PLEIDEN)]:
        assert U.run_oracle(g, variant, *MOD, **kw).status == -1
        with pytest.raises(L.LccError) as e:
            U.run_gpu(g, variant, *MOD, **kw)
        assert e.value.status == -1


@pytest.mark.parametrize("sym", [1, 2], ids=["none", "mlh"])
def test_symmetry_breaking_ablations(sym):
    """Table 2's ablations: no symmetry breaking, or the minimum label heuristic in odd passes; phi = 0."""
    kw = dict(phases=((0, 1, 6),), symmetry=sym)
    for g, obj in [(gg.config1_sbm(), MOD), (gg.rmat(13, 16, seed=5), MOD), (U.hub_graph(), CPM20),
                   (gg.lattice(50, 40, 0.1, 100, 3), CPM20)]:
        for v in (O.PLOUVAIN, O.PLEIDEN):
            U.assert_parity(g, v, *obj, opts_kw=kw)


@pytest.mark.parametrize("base", [2 ** 32 - 7, 2 ** 32 - 4, 2 ** 32 - 2])
def test_tag_wraparound(monkeypatch, base):
    """Free-id marks and single-pass scans tag their words instead of clearing them; when the 32-bit tags run
    out the arrays are cleared and numbering restarts.  Starting the sequence just before its end makes every
    call cross the wrap-around (at each offset of the three tags a pass takes, including a mark tag of 2^32 - 1);
    results must not change."""
    import paper_2608_01503_amd as L
    monkeypatch.setenv("LCC_TAG_BASE", str(base))
    ctx = L.Context(0)  # a fresh context: the variable is read when its workspace is allocated
    for g, v, lam, mode in [(U.hub_graph(n=12000, hub_deg=(9000, 6000, 1500), seed=8), L.LCC_PLEIDEN_PLUS,
                             (1, 20, False), L.LCC_VW_UNIT),
                            (gg.random_gnp(3000, 0.004, 77, w_max=4), L.LCC_PLOUVAIN, (1, 1, True),
                             L.LCC_VW_WEIGHTED_DEGREE)]:
        ref = U.run_oracle(g, v, lam, mode)
        lab, res = ctx.cluster(U.device_graph(g, mode), lam, v, trace_capacity=1 << 14)
        assert np.array_equal(lab.cpu().numpy(), ref.labels) and res.N == ref.N
        assert np.array_equal(res.trace, ref.trace)
    ctx.close()


@pytest.mark.parametrize("variant,lam,mode", [(O.PLOUVAIN, (1, 1, True), O.VW_WEIGHTED_DEGREE),
                                              (O.PLEIDEN, (1, 50, False), O.VW_UNIT)])
def test_dense_cross_rows(variant, lam, mode):
    """Few coarse rows with tens of thousands of cross entries each: the contraction's per-row sort takes its
    long-row path with many tiles per row and a single radix pass (fewer than 257 coarse vertices)."""
    g = gg.sbm(20, 500, 0.1, 0.01, seed=23)
    U.assert_parity(g, variant, lam, mode)
