"""Pins for the CPU oracle: each test checks it against something other than itself -- a published
test vector, the set-based definitions of Sec. II in exact rationals (tests/defs.py), a textbook or
library routine (Newman-Girvan modularity, scipy sparse P^T A P), brute force over all partitions or
over every LeidenR run on tiny graphs, closed-form special cases and invariants.

CPU only (no GPU marker)."""
from __future__ import annotations

import random
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import graphgen as gg
import oracle as O
from tests import defs

GOLDEN = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def tiny_graphs(count, n_lo=4, n_hi=9, seed=0, w_max=5):
    rng = random.Random(seed)
    for k in range(count):
        n = rng.randint(n_lo, n_hi)
        p = rng.choice([0.3, 0.5, 0.8])
        yield gg.random_gnp(n, p, seed * 1000 + k, w_max=w_max)


def lam_choices(g, vw):
    W = int(np.sum(vw))
    out = [(0, 1, False), (1, 1, True), (1, 20, False), (1, 3, False)]
    if W > 0:
        out.append((3, 2, True))
    return out


def resolved(g, mode=O.VW_WEIGHTED_DEGREE, lam=(1, 1, True), vw=None):
    st, vwr, p, q = O.setup(g, mode, lam, vw)
    assert st == 0, O.STATUS[st]
    return vwr, p, q


# ------------------------------------------------------------------------------------------------
# hash functions: published test vectors
# ------------------------------------------------------------------------------------------------

def test_splitmix64_test_vector():
    # splitmix64 seeded with 1234567: first two outputs of the published reference generator
    assert O.fmix64((1234567 + GOLDEN) & M64) == 6457827717110365317
    assert O.fmix64((1234567 + 2 * GOLDEN) & M64) == 3203168211198807973


def test_fmix32_is_a_bijection_on_a_block():
    vals = {O.fmix32(x) for x in range(1 << 14)}
    assert len(vals) == 1 << 14
    assert O.fmix32(0) == 0  # the finaliser fixes zero: only xor-shifts and odd multiplications


# ------------------------------------------------------------------------------------------------
# setup: validation and lambda
# ------------------------------------------------------------------------------------------------

def _g(n, off, idx, w):
    return gg.Graph(n=n, off=np.array(off, np.int64), idx=np.array(idx, np.int32), w=np.array(w, np.int32))


def test_setup_rejects_invalid_graphs():
    ok = _g(3, [0, 1, 3, 4], [1, 0, 2, 1], [1, 1, 2, 2])
    assert O.setup(ok)[0] == 0
    assert O.setup(_g(2, [0, 1, 2], [0, 0], [1, 1]))[0] == -3                      # self-loop
    assert O.setup(_g(3, [0, 2, 3, 4], [2, 1, 0, 0], [1, 1, 1, 1]))[0] == -4      # unsorted row
    assert O.setup(_g(3, [0, 1, 2, 3], [1, 2, 0], [1, 1, 1]))[0] == -2            # not symmetric
    assert O.setup(_g(2, [0, 1, 2], [1, 0], [2, 3]))[0] == -2                     # asymmetric weight
    assert O.setup(_g(2, [0, 1, 2], [1, 0], [0, 0]))[0] == -5                     # weight <= 0
    assert O.setup(_g(2, [0, 1, 2], [1, 5], [1, 1]))[0] == -1                     # index out of range
    assert O.setup(ok, O.VW_UNIT, (3, 2, False))[0] == -6                          # lambda > 1
    assert O.setup(ok, O.VW_UNIT, (1, 0, False))[0] == -6                          # zero denominator
    big = _g(3, [0, 1, 3, 4], [1, 0, 2, 1], [2 ** 31 - 1] * 4)
    assert O.setup(big)[0] == -7                                                   # total weight >= 2^32
    vbig = np.array([2 ** 31, 1, 1], np.int64)
    assert O.setup(ok, O.VW_GIVEN, (1, 20, False), vbig)[0] == -7                  # vertex weight >= 2^31
    assert O.setup(ok, O.VW_GIVEN, (1, 20, False), -vbig)[0] == -5                 # negative vertex weight


def test_setup_exactness_bound_is_2_62():
    """Two vertices joined by one edge of weight x under modularity: W_E = W = 2x and lambda = 1/(2x), so
    q W_E + p W^2 = 8 x^2, which stays below 2^62 exactly up to x = floor(sqrt(2^59 - 1))."""
    x_max = int(np.floor(np.sqrt(2.0 ** 59)))
    while 8 * (x_max + 1) ** 2 < 2 ** 62:
        x_max += 1
    while 8 * x_max ** 2 >= 2 ** 62:
        x_max -= 1
    assert x_max == 759250124
    for x, want in ((x_max, 0), (x_max + 1, -7), (2 ** 30, -7)):
        g = _g(2, [0, 1, 2], [1, 0], [x, x])
        st, vw, p, q = O.setup(g)
        assert st == want, (x, st)
        if st == 0:
            assert (p, q) == (1, 2 * x) and q * 2 * x + p * (2 * x) ** 2 == 8 * x * x < 2 ** 62
            r = O.cluster(g, O.PLOUVAIN)
            # joining the pair: internal weight 2x, (sum W_c^2 - sum w^2) = 2 x^2 -> N = 2x * 2x - 2x^2
            assert r.status == 0 and defs.same_partition(r.labels, [0, 0]) and r.N == 2 * x * x


def test_heavy_weights_above_2_30_stay_exact():
    """Modularity with a weight total between 2^30 and the 2^62 bound (about 1.5e9): the oracle's objective
    matches Eq. 1 in exact rationals and the textbook modularity, and the two heavy cliques are found."""
    g = gg.reweight(defs_two_cliques(6), 1_450_000_000, seed=5)
    vw, p, q = resolved(g)
    W = int(vw.sum())
    assert 2 ** 30 < W <= 1_450_000_000 and q * W + p * W * W < 2 ** 62
    D = defs.Dense(g, vw)
    rng = random.Random(3)
    for _ in range(20):
        C = [rng.randrange(4) for _ in range(g.n)]
        assert Fraction(O.objective(g, vw, p, q, C), q) == D.lambdacc(C, Fraction(p, q))
    for variant in VARIANTS:
        r = O.cluster(g, variant)
        assert r.status == 0
        assert Fraction(r.N, r.q) == D.lambdacc(list(r.labels), Fraction(p, q))
        Q = (r.N - p * int(np.sum(vw.astype(object) ** 2))) / (q * W)
        assert abs(Q - defs.textbook_modularity(g, r.labels)) < 1e-12
        assert defs.same_partition(r.labels, [0] * 6 + [1] * 6)


def test_setup_lambda_reduced():
    g = defs_two_cliques(4)
    st, vw, p, q = O.setup(g, O.VW_WEIGHTED_DEGREE, (1, 1, True))
    W = int(vw.sum())
    assert st == 0 and Fraction(p, q) == Fraction(1, W) and vw.tolist() == list(np.diff(g.off))
    st, vw, p, q = O.setup(g, O.VW_UNIT, (2, 40, False))
    assert (p, q) == (1, 20) and vw.tolist() == [1] * g.n
    st, vw, p, q = O.setup(g, O.VW_UNIT, (0, 7, False))
    assert (p, q) == (0, 1)


def defs_two_cliques(k, bridge_w=1):
    pairs = [(i, j) for i in range(k) for j in range(i + 1, k)]
    pairs += [(k + i, k + j) for i in range(k) for j in range(i + 1, k)]
    pairs.append((k - 1, k))
    w = [1] * (len(pairs) - 1) + [bridge_w]
    return gg.from_pairs(2 * k, pairs, w)


# ------------------------------------------------------------------------------------------------
# objective (Eq. 1)
# ------------------------------------------------------------------------------------------------

def test_objective_matches_eq1_pairwise_sum():
    rng = random.Random(7)
    cases = 0
    for g in tiny_graphs(25, seed=1):
        for mode in (O.VW_WEIGHTED_DEGREE, O.VW_UNIT):
            for lam in [(0, 1, False), (1, 1, True), (1, 20, False), (2, 3, False)]:
                st, vw, p, q = O.setup(g, mode, lam)
                if st != 0:
                    continue
                D = defs.Dense(g, vw)
                for _ in range(3):
                    C = [rng.randrange(g.n) for _ in range(g.n)]
                    N = O.objective(g, vw, p, q, C)
                    assert Fraction(N, q) == D.lambdacc(C, Fraction(p, q))
                    cases += 1
    assert cases > 100


def test_modularity_matches_textbook():
    rng = np.random.default_rng(3)
    for g in list(tiny_graphs(10, 6, 12, seed=2)) + [gg.config1_sbm()]:
        vw, p, q = resolved(g)
        if vw.sum() == 0:
            continue
        for _ in range(3):
            C = rng.integers(0, max(2, g.n // 5), size=g.n).astype(np.int32)
            N = O.objective(g, vw, p, q, C)
            W = int(vw.sum())
            Q = (N - p * int(np.sum(vw.astype(object) ** 2))) / (q * W)
            assert abs(Q - defs.textbook_modularity(g, C)) < 1e-12


# ------------------------------------------------------------------------------------------------
# one local-move pass (Alg. 2 + Alg. 3)
# ------------------------------------------------------------------------------------------------

def _expected_destination(D, C, v, lam):
    """Destination from the definitions: argmax of w'(v, X) over adjacent clusters X != C[v], lowest id
    on ties; EMPTY when v's own contribution and the best are both negative."""
    cl = defs.clusters_of(C)
    cur = D.wprime([v], cl[int(C[v])], lam)
    best, bval = None, None
    for c in sorted(cl):
        if c == int(C[v]) or not any(D.A[v][u] for u in cl[c]):
            continue
        val = D.wprime([v], cl[c], lam)
        if best is None or val > bval:
            best, bval = c, val
    if cur < 0 and (best is None or bval < 0):
        return O.EMPTY, Fraction(0), cur
    if best is None:
        return O.NONE, None, cur
    return best, bval, cur


def test_lm_pass_destination_and_candidates_bruteforce():
    rng = random.Random(11)
    checked = 0
    for g in tiny_graphs(30, seed=3):
        for mode in (O.VW_WEIGHTED_DEGREE, O.VW_UNIT):
            for lam in [(1, 1, True), (1, 20, False), (1, 2, False), (0, 1, False)]:
                st, vw, p, q = O.setup(g, mode, lam)
                if st != 0:
                    continue
                D = defs.Dense(g, vw)
                L = Fraction(p, q)
                C = [rng.randrange(g.n) for _ in range(g.n)]
                for phi in [(3, 4), (1, 4), (0, 1)]:
                    r = O.lm_pass(g, vw, p, q, C, phi=phi)
                    for v in range(g.n):
                        dst, sd, cur = _expected_destination(D, C, v, L)
                        if dst == O.NONE:
                            assert not r["cand"][v]
                            continue
                        assert int(r["D"][v]) == dst, (v, dst, r["D"][v])
                        assert Fraction(r["delta"][v], q) == sd - cur
                        cand = sd >= (1 - Fraction(*phi)) * cur
                        assert bool(r["cand"][v]) == cand
                        checked += 1
    assert checked > 300


def test_lambda_zero_scores_are_adjacency_weights():
    """lambda = 0 (label propagation, Sec. II): D[v] is the neighbouring cluster with the largest total
    edge weight (lowest id on ties), and with phi = 0 v is a candidate iff that weight is at least the
    weight to its own cluster.  a(v, c) comes from a sparse matrix product A @ onehot(C)."""
    rng = np.random.default_rng(5)
    for g in tiny_graphs(20, 6, 14, seed=4):
        vw, p, q = resolved(g, O.VW_UNIT, (0, 1, False))
        C = rng.integers(0, g.n, size=g.n).astype(np.int32)
        A = sp.csr_matrix((g.w.astype(np.int64), g.idx, g.off), shape=(g.n, g.n))
        H = sp.csr_matrix((np.ones(g.n, np.int64), (np.arange(g.n), C)), shape=(g.n, g.n))
        a = (A @ H).toarray()
        r = O.lm_pass(g, vw, p, q, C, phi=(0, 1))
        for v in range(g.n):
            row = a[v].copy()
            own = row[C[v]]
            row[C[v]] = 0
            if row.max() == 0:
                assert not r["cand"][v]
                continue
            assert r["D"][v] == int(np.argmax(row))
            assert bool(r["cand"][v]) == (row.max() >= own)


def test_afterburner_two_singletons_exactly_one_moves():
    g = gg.from_pairs(2, [(0, 1)])
    vw, p, q = resolved(g)
    r = O.lm_pass(g, vw, p, q, [0, 1])
    assert r["cand"].all() and r["keep"].sum() == 1
    assert r["C"][0] == r["C"][1]


def test_afterburner_swap_penalty():
    """u in A wants B and v in B wants A: the later-ordered of the two carries -2 q w'(u, v)."""
    # a1 - u = v - b1 with w(u, v) = 10, clusters A = {a1, u}, B = {v, b1}
    g = gg.from_pairs(4, [(0, 1), (1, 2), (2, 3)], [1, 10, 1])
    vw, p, q = resolved(g, O.VW_UNIT, (0, 1, False))
    C = [0, 0, 3, 3]
    r = O.lm_pass(g, vw, p, q, C, phi=(0, 1))
    assert r["D"][1] == 3 and r["D"][2] == 0
    d = [r["dadj"][v] - r["delta"][v] for v in (1, 2)]
    assert sorted(d) == [-2 * 10 * q, 0]


def test_afterburner_exact_gain_identity():
    """When every candidate is kept (M = L) and every pair of movers is adjacent (complete graphs) or
    lambda = 0 (non-adjacent movers do not interact), the afterburner-adjusted deltas add up to the
    exact change of the objective: 2 sum_{v in M} delta'_v = N(after) - N(before)."""
    rng = random.Random(13)
    hits = 0
    for k in range(400):
        n = rng.randint(3, 7)
        complete = k % 2 == 0
        if complete:
            pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
            g = gg.from_pairs(n, pairs, [rng.randint(1, 9) for _ in pairs])
            lam = rng.choice([(1, 1, True), (1, 20, False), (1, 7, False)])
        else:
            g = gg.random_gnp(n, 0.5, 500 + k, w_max=6)
            lam = (0, 1, False)
        st, vw, p, q = O.setup(g, O.VW_WEIGHTED_DEGREE, lam)
        if st != 0:
            continue
        C = [rng.randrange(n) for _ in range(n)]
        N0 = O.objective(g, vw, p, q, C)
        r = O.lm_pass(g, vw, p, q, C, phi=rng.choice([(3, 4), (0, 1)]))
        if r["nL"] == 0 or r["nM"] != r["nL"]:
            continue
        N1 = O.objective(g, vw, p, q, r["C"])
        assert 2 * sum(r["dadj"][v] for v in range(n) if r["keep"][v]) == N1 - N0
        hits += 1
    assert hits > 50


def test_apply_invariants_and_empty_ids():
    rng = random.Random(17)
    saw_empty = False
    for g in tiny_graphs(40, 5, 12, seed=5):
        vw, p, q = resolved(g, O.VW_UNIT, (1, 2, False))
        C = [rng.randrange(3) for _ in range(g.n)]
        r = O.lm_pass(g, vw, p, q, C, phi=(3, 4))
        newC = r["C"]
        assert ((0 <= newC) & (newC < g.n)).all()
        for v in range(g.n):
            if not r["keep"][v]:
                assert newC[v] == C[v]
            elif r["D"][v] != O.EMPTY:
                assert newC[v] == r["D"][v]
        # every EMPTY mover is alone in a cluster id nobody else holds
        movers = [v for v in range(g.n) if r["keep"][v] and r["D"][v] == O.EMPTY]
        for v in movers:
            saw_empty = True
            assert (newC == newC[v]).sum() == 1
        # EMPTY movers took the smallest unused ids, in vertex order
        others = {int(newC[v]) for v in range(g.n) if v not in movers}
        free = [c for c in range(g.n) if c not in others][:len(movers)]
        assert [int(newC[v]) for v in movers] == free
    assert saw_empty


def test_local_move_monotone_and_deterministic():
    rng = np.random.default_rng(19)
    for g in tiny_graphs(20, 8, 30, seed=6):
        vw, p, q = resolved(g)
        C0 = rng.integers(0, g.n, size=g.n).astype(np.int32)
        C1, N1 = O.local_move(g, vw, p, q, C0)
        C2, N2 = O.local_move(g, vw, p, q, C0)
        assert N1 >= O.objective(g, vw, p, q, C0)
        assert N1 == O.objective(g, vw, p, q, C1)
        assert (C1 == C2).all() and N1 == N2


# ------------------------------------------------------------------------------------------------
# contraction (Alg. 4)
# ------------------------------------------------------------------------------------------------

def _random_map(rng, n, k):
    lab = rng.integers(0, k, size=n)
    _, cmap = np.unique(lab, return_inverse=True)
    return cmap.astype(np.int32), int(cmap.max()) + 1 if n else 0


def test_contract_matches_scipy_triple_product():
    rng = np.random.default_rng(23)
    for g in tiny_graphs(20, 5, 40, seed=7, w_max=9):
        vw, p, q = resolved(g)
        cmap, nc = _random_map(rng, g.n, max(1, g.n // 3))
        s_in = rng.integers(0, 5, size=g.n)
        sq_in = rng.integers(0, 50, size=g.n)
        cg, cvw, cs, csq = O.contract(g, vw, cmap, nc, s_in, sq_in)
        A = sp.csr_matrix((g.w.astype(np.int64), g.idx, g.off), shape=(g.n, g.n))
        P = sp.csr_matrix((np.ones(g.n, np.int64), (np.arange(g.n), cmap)), shape=(g.n, nc))
        M = (P.T @ A @ P).toarray()
        got = np.zeros((nc, nc), np.int64)
        for x in range(nc):
            row = cg.idx[cg.off[x]:cg.off[x + 1]]
            assert (np.diff(row) > 0).all()          # ascending, unique
            assert x not in row                       # no self-loops
            got[x, row] = cg.w[cg.off[x]:cg.off[x + 1]]
        assert (got == M - np.diag(np.diag(M))).all()
        assert (cs == np.diag(M) + P.T @ s_in).all()
        assert (cvw == P.T @ vw).all()
        assert (csq == P.T @ sq_in).all()
        assert got.sum() + cs.sum() == g.w.sum() + s_in.sum()


def test_contract_objective_offset_identity():
    """For any partition P of the coarse vertices, N_fine(project(P)) = N_coarse(P) + K with
    K = q sum_x s(x) - p sum_x (w(x)^2 - sq(x))  (objective offset instead of self-loops, Sec. III-A).
    Checked over a three-level chain."""
    rng = np.random.default_rng(29)
    for g in tiny_graphs(15, 8, 40, seed=8, w_max=4):
        for mode, lam in [(O.VW_WEIGHTED_DEGREE, (1, 1, True)), (O.VW_UNIT, (1, 20, False))]:
            vw, p, q = resolved(g, mode, lam)
            m1, n1 = _random_map(rng, g.n, max(1, g.n // 2))
            g1, w1, s1, sq1 = O.contract(g, vw, m1, n1)
            m2, n2 = _random_map(rng, n1, max(1, n1 // 2))
            g2, w2, s2, sq2 = O.contract(g1, w1, m2, n2, s1, sq1)
            K2 = q * int(s2.sum()) - p * int((w2.astype(object) ** 2).sum() - sq2.astype(object).sum())
            for _ in range(3):
                P2 = rng.integers(0, max(1, n2), size=n2).astype(np.int32)
                fine = P2[m2[m1]]
                assert O.objective(g, vw, p, q, fine) == O.objective(g2, w2, p, q, P2) + K2


def test_contract_special_cases():
    g = gg.random_gnp(12, 0.4, 31, w_max=3)
    vw, p, q = resolved(g)
    ident = np.arange(g.n, dtype=np.int32)
    cg, cvw, cs, csq = O.contract(g, vw, ident, g.n)
    assert (cg.off == g.off).all() and (cg.idx == g.idx).all() and (cg.w == g.w).all()
    comp = np.array(defs.components(g), np.int32)
    cg, cvw, cs, csq = O.contract(g, vw, comp, int(comp.max()) + 1)
    assert cg.nnz == 0 and cs.sum() == g.w.sum()


# ------------------------------------------------------------------------------------------------
# pLeidenR (Alg. 6, Lemmas 1-2)
# ------------------------------------------------------------------------------------------------

def _check_refinement(g, vw, p, q, B, out):
    lam = Fraction(p, q)
    D = defs.Dense(g, vw)
    R, par, root, fk = out["R"], out["parent"], out["root"], out["fkey"]
    Bc = defs.clusters_of(B)
    # parents have smaller ordering values; every tree lies inside one constraint cluster
    for v in range(g.n):
        if par[v] != v:
            assert fk[par[v]] < fk[v]
            assert B[par[v]] == B[v] and D.A[v][par[v]] > 0
    for r, mem in defs.clusters_of(R).items():
        assert len({int(B[v]) for v in mem}) == 1                   # R refines B
        assert defs.connected_within(g, mem)                         # connected
    # re-simulate LeidenR along the ordering: each committed vertex is a legal join; the first vertex of
    # a tree that was not committed violates one of the conditions
    for r in set(root.tolist()):
        tree = sorted([v for v in range(g.n) if root[v] == r], key=lambda v: fk[v])
        X = []
        Bm = Bc[int(B[r])]
        for v in tree:
            ok = (not X) or (D.wprime([v], X, lam) >= 0 and D.wprime(X, Bm, lam) >= 0)
            if X:
                assert D.wprime([v], Bm, lam) >= 0                 # v is well connected (in U)
            if not ok:
                assert all(R[u] == u for u in tree[len(X):])
                break
            assert R[v] == r
            X.append(v)


def test_refine_properties_random():
    rng = np.random.default_rng(37)
    for g in tiny_graphs(30, 6, 40, seed=9, w_max=4):
        for mode, lam in [(O.VW_WEIGHTED_DEGREE, (1, 1, True)), (O.VW_UNIT, (1, 20, False)),
                          (O.VW_UNIT, (1, 3, False))]:
            vw, p, q = resolved(g, mode, lam)
            B = rng.integers(0, max(1, g.n // 4), size=g.n).astype(np.int32)
            for t in range(3):
                _check_refinement(g, vw, p, q, B, O.refine(g, vw, p, q, B, seed=5, t=t))
            Bl, _ = O.local_move(g, vw, p, q, np.arange(g.n, dtype=np.int32))
            _check_refinement(g, vw, p, q, Bl, O.refine(g, vw, p, q, Bl, seed=5, t=0))


def test_refine_reachable_by_sequential_leidenr():
    """Lemma 1: whatever pLeidenR returns, sequential LeidenR can also produce (brute force over all
    visit orders and join choices on graphs with at most 7 vertices)."""
    rng = np.random.default_rng(41)
    cases = 0
    for g in tiny_graphs(25, 4, 7, seed=10, w_max=3):
        for mode, lam in [(O.VW_WEIGHTED_DEGREE, (1, 1, True)), (O.VW_UNIT, (1, 4, False))]:
            vw, p, q = resolved(g, mode, lam)
            B = rng.integers(0, 2, size=g.n).astype(np.int32)
            reach = defs.leidenr_reachable(defs.Dense(g, vw), B, Fraction(p, q))
            for t in range(4):
                R = O.refine(g, vw, p, q, B, seed=9, t=t)["R"]
                canon = tuple(sorted(tuple(sorted(m)) for m in defs.clusters_of(R).values()))
                assert canon in reach
                cases += 1
    assert cases > 100


def test_refine_no_qualifying_edge_gives_singletons():
    # vertex weights 3, unit edges, lambda = 1/2: w'(u, v) = 1 - 9/2 < 0 for every edge
    g = gg.random_gnp(15, 0.5, 43)
    vw = np.full(g.n, 3, np.int64)
    st, vwr, p, q = O.setup(g, O.VW_GIVEN, (1, 2, False), vw)
    out = O.refine(g, vwr, p, q, np.zeros(g.n, np.int32), seed=1, t=0)
    assert (out["R"] == np.arange(g.n)).all()


# ------------------------------------------------------------------------------------------------
# LocalMoveAlt (Sec. V-A)
# ------------------------------------------------------------------------------------------------

def test_lmalt_bruteforce_prefix():
    """Non-node-optimal vertices (ascending id) with destinations fixed up front; every prefix is applied
    and its objective recomputed from Eq. 1; the shortest best prefix must be what is committed."""
    rng = random.Random(47)
    cases = 0
    for g in tiny_graphs(40, 4, 9, seed=11, w_max=4):
        for mode, lam in [(O.VW_WEIGHTED_DEGREE, (1, 1, True)), (O.VW_UNIT, (1, 3, False))]:
            st, vw, p, q = O.setup(g, mode, lam)
            D = defs.Dense(g, vw)
            L = Fraction(p, q)
            C = [rng.randrange(g.n) for _ in range(g.n)]
            movers = []
            for v in range(g.n):
                dst, sd, cur = _expected_destination(D, C, v, L)
                if dst != O.NONE and sd - cur > 0:
                    movers.append((v, dst))
            got, k, kc = O.lmalt(g, vw, p, q, C)
            assert k == len(movers)
            if not movers:
                assert list(got) == C
                continue
            best, bestk = D.lambdacc(C, L), 0
            for i in range(1, len(movers) + 1):
                Ci = list(C)
                for j, (v, dst) in enumerate(movers[:i]):
                    Ci[v] = dst if dst != O.EMPTY else 10 ** 6 + j
                val = D.lambdacc(Ci, L)
                if val > best:
                    best, bestk = val, i
            assert kc == bestk and bestk >= 1
            assert D.lambdacc(list(got), L) == best
            cases += 1
    assert cases > 30


# ------------------------------------------------------------------------------------------------
# full pipelines
# ------------------------------------------------------------------------------------------------

VARIANTS = [O.LOUVAIN, O.PLOUVAIN, O.PLEIDEN, O.PLEIDEN_PLUS]


@pytest.mark.parametrize("variant", VARIANTS)
def test_two_cliques_joined_by_an_edge(variant):
    g = defs_two_cliques(5)
    r = O.cluster(g, variant)
    assert r.status == 0
    assert defs.same_partition(r.labels, [0] * 5 + [1] * 5)


@pytest.mark.parametrize("variant", VARIANTS)
def test_lambda_zero_gives_connected_components(variant):
    """lambda = 0: the objective is the internal edge weight, maximised by the connected components."""
    for k in range(6):
        parts = [gg.random_gnp(6, 0.6, 60 + 3 * k + j) for j in range(3)]
        pairs, wts, base = [], [], 0
        for h in parts:
            for v in range(h.n):
                for j in range(h.off[v], h.off[v + 1]):
                    if h.idx[j] > v:
                        pairs.append((base + v, base + int(h.idx[j])))
                        wts.append(int(h.w[j]))
            base += h.n
        g = gg.from_pairs(base, pairs, wts)
        r = O.cluster(g, variant, lam=(0, 1, False), vw_mode=O.VW_UNIT)
        assert defs.same_partition(r.labels, defs.components(g))


_BELL_CACHE = {}


def _bell_optimum(sizes):
    if sizes not in _BELL_CACHE:
        pairs, base = [], 0
        for s in sizes:
            pairs += [(base + i, base + j) for i in range(s) for j in range(i + 1, s)]
            base += s
        g = gg.from_pairs(base, pairs)
        st, vw, p, q = O.setup(g)
        D = defs.Dense(g, vw)
        lam = Fraction(p, q)
        _BELL_CACHE[sizes] = (g, max(D.lambdacc(C, lam) for C in defs.set_partitions(g.n)))
    return _BELL_CACHE[sizes]


@pytest.mark.parametrize("variant", VARIANTS)
def test_disjoint_cliques_reach_bell_optimum(variant):
    """Disjoint cliques under modularity: the brute-force optimum over all Bell(n) partitions is the
    cliques, and the method must find it."""
    for sizes in [(3, 3, 4), (2, 3, 4), (4, 5), (3, 3, 3)]:
        g, best = _bell_optimum(sizes)
        r = O.cluster(g, variant)
        assert Fraction(r.N, r.q) == best
        assert r.num_clusters == len(sizes)


def test_random_tiny_never_beats_bell_optimum():
    for g in tiny_graphs(8, 5, 8, seed=12):
        st, vw, p, q = O.setup(g)
        if st != 0:
            continue
        D = defs.Dense(g, vw)
        lam = Fraction(p, q)
        best = max(D.lambdacc(C, lam) for C in defs.set_partitions(g.n))
        for variant in VARIANTS:
            r = O.cluster(g, variant)
            assert Fraction(r.N, r.q) == D.lambdacc(list(r.labels), lam) <= best


def test_leiden_connected_and_separated():
    """Leiden guarantees after an iteration (Sec. II-B, Theorem 1): every cluster is connected and any two
    clusters are gamma-separated, w'(C_x, C_y) <= 0.  (pLeiden+ has these only in stable iterations,
    Sec. VI-A, so it is not checked here.)"""
    variant = O.PLEIDEN
    graphs = list(tiny_graphs(10, 20, 80, seed=13, w_max=3)) + [gg.lattice(20, 20, 0.1, 100, 3),
                                                                gg.config1_sbm()]
    for g in graphs:
        for mode, lam in [(O.VW_WEIGHTED_DEGREE, (1, 1, True)), (O.VW_UNIT, (1, 20, False))]:
            r = O.cluster(g, variant, lam=lam, vw_mode=mode)
            assert r.status == 0
            cl = defs.clusters_of(r.labels)
            for mem in cl.values():
                assert defs.connected_within(g, mem)
            st, vw, p, q = O.setup(g, mode, lam)
            Wc = np.bincount(r.labels, weights=vw.astype(np.float64)).astype(np.int64)
            cut = {}
            for v in range(g.n):
                for j in range(g.off[v], g.off[v + 1]):
                    a, b = int(r.labels[v]), int(r.labels[g.idx[j]])
                    if a != b:
                        cut[(a, b)] = cut.get((a, b), 0) + int(g.w[j])
            for (a, b), wab in cut.items():
                assert q * wab - p * int(Wc[a]) * int(Wc[b]) <= 0


def test_config1_quality_and_determinism():
    g = gg.config1_sbm()
    r1 = O.cluster(g, O.LOUVAIN)
    r2 = O.cluster(g, O.LOUVAIN)
    assert (r1.labels == r2.labels).all()
    st, vw, p, q = O.setup(g)
    Q = (r1.N - p * int((vw.astype(object) ** 2).sum())) / (q * int(vw.sum()))
    planted = np.arange(g.n) // 100
    Qp = defs.textbook_modularity(g, planted)
    assert r1.num_clusters == 20 and abs(Q - Qp) < 0.02


# ------------------------------------------------------------------------------------------------
# iteration inputs (Sec. II-B, Sec. IV-D): initial clustering and constraint clustering
# ------------------------------------------------------------------------------------------------

def _node_optimal(g, labels, vw, p, q):
    """Every vertex is node optimal (Sec. II-B): no move to a neighbouring cluster or to a new singleton
    (score 0) strictly improves the objective.  Exact integer scores from the definitions."""
    labels = np.asarray(labels, dtype=np.int64)
    Wc = {}
    for v in range(g.n):
        Wc[int(labels[v])] = Wc.get(int(labels[v]), 0) + int(vw[v])
    for v in range(g.n):
        cv = int(labels[v])
        a = {}
        for j in range(g.off[v], g.off[v + 1]):
            c = int(labels[g.idx[j]])
            a[c] = a.get(c, 0) + int(g.w[j])
        wv = int(vw[v])
        s_cur = q * a.get(cv, 0) - p * wv * (Wc[cv] - wv)
        best = max([q * av - p * wv * Wc[c] for c, av in a.items() if c != cv] + [0])
        if best > s_cur:
            return False
    return True


def test_iterated_pleiden_stable_iteration_is_node_optimal():
    """Feeding pLeiden its own output (Alg. 5 with C_in) until the output repeats: in a stable iteration every
    vertex is node optimal (Sec. II-B), every cluster is connected and clusters are gamma-separated."""
    graphs = [gg.config1_sbm(), gg.random_gnp(300, 0.03, 71, w_max=5), gg.lattice(12, 12, 0.1, 100, 3)]
    for g in graphs:
        for mode, lam in [(O.VW_WEIGHTED_DEGREE, (1, 1, True)), (O.VW_UNIT, (1, 20, False))]:
            st, vw, p, q = O.setup(g, mode, lam)
            r = O.cluster(g, O.PLEIDEN, lam=lam, vw_mode=mode)
            stable = False
            for _ in range(30):
                r2 = O.cluster(g, O.PLEIDEN, lam=lam, vw_mode=mode, init=r.labels)
                assert r2.status == 0 and r2.N >= r.N  # an iteration never loses objective
                if defs.same_partition(r2.labels, r.labels):
                    stable = True
                    break
                r = r2
            assert stable, (g.name, lam)
            assert _node_optimal(g, r.labels, vw, p, q)
            for mem in defs.clusters_of(r.labels).values():
                assert defs.connected_within(g, mem)


def test_louvain_init_is_the_level0_start():
    """Louvain from an initial clustering: the level-0 local move starts from it.  Starting from the
    singletons is the plain run; starting from a node-optimal stable clustering changes nothing at level 0."""
    g = gg.random_gnp(400, 0.02, 81, w_max=4)
    r = O.cluster(g, O.LOUVAIN)
    same = O.cluster(g, O.LOUVAIN, init=np.arange(g.n, dtype=np.int32))
    assert np.array_equal(same.labels, r.labels) and same.N == r.N
    bad = O.cluster(g, O.PLOUVAIN, init=np.full(g.n, g.n, dtype=np.int32))
    assert bad.status == -1


def test_constraint_special_cases():
    """One constraint cluster = no constraint; singleton constraints forbid every merge (all singletons)."""
    for g in [gg.config1_sbm(), gg.random_gnp(500, 0.01, 91, w_max=7)]:
        for mode, lam in [(O.VW_WEIGHTED_DEGREE, (1, 1, True)), (O.VW_UNIT, (1, 20, False))]:
            free = O.cluster(g, O.PLOUVAIN, lam=lam, vw_mode=mode)
            one = O.cluster(g, O.PLOUVAIN, lam=lam, vw_mode=mode, constraint=np.full(g.n, 7, dtype=np.int32))
            assert np.array_equal(one.labels, free.labels) and one.N == free.N
            sing = O.cluster(g, O.PLOUVAIN, lam=lam, vw_mode=mode, constraint=np.arange(g.n, dtype=np.int32))
            assert sing.num_clusters == g.n and sing.levels == 1
    g = gg.config1_sbm()
    assert O.cluster(g, O.PLEIDEN, constraint=np.zeros(g.n, np.int32)).status == -1
    assert O.cluster(g, O.PLOUVAIN, init=np.arange(g.n, dtype=np.int32),
                     constraint=np.zeros(g.n, np.int32)).status == -1


def test_constrained_coarsening_stays_inside_constraint():
    """Without uncoarsening (LOUVAIN) the result is the coarsening's: every cluster lies inside one constraint
    cluster (Sec. IV-D: the constrained coarsening only joins clusters inside a constraint cluster)."""
    rng = np.random.default_rng(5)
    for g in [gg.config1_sbm(), gg.random_gnp(600, 0.01, 95, w_max=3), gg.lattice(15, 15, 0.1, 100, 3)]:
        B = rng.integers(0, 6, size=g.n).astype(np.int32)
        r = O.cluster(g, O.LOUVAIN, constraint=B)
        for mem in defs.clusters_of(r.labels).values():
            assert len({int(B[v]) for v in mem}) == 1


# ------------------------------------------------------------------------------------------------
# symmetry-breaking ablations (Table 2): none, minimum label heuristic
# ------------------------------------------------------------------------------------------------

def test_no_symmetry_breaking_keeps_every_candidate():
    for g in [gg.config1_sbm(), gg.random_gnp(400, 0.02, 61, w_max=5)]:
        r = O.cluster(g, O.PLOUVAIN, opts=O.make_opts(phases=((0, 1, 6),), symmetry=O.SYM_NONE))
        passes = [t for t in r.trace if t[0] == 1]
        assert passes and all(t[4] == t[5] for t in passes)


def test_minimum_label_heuristic_two_singletons():
    """Two adjacent singletons that want each other: in an odd pass (heuristic active) only the vertex moving to
    the lower id moves; in an even pass both move (no symmetry breaking)."""
    g = gg.from_pairs(2, [(0, 1)])
    vw, p, q = resolved(g, O.VW_UNIT, (0, 1, False))
    odd = O.lm_pass(g, vw, p, q, [0, 1], phi=(0, 1), symmetry=O.SYM_MLH, pass_no=1)
    assert list(odd["D"]) == [1, 0] and list(odd["keep"]) == [False, True] and list(odd["C"]) == [0, 0]
    even = O.lm_pass(g, vw, p, q, [0, 1], phi=(0, 1), symmetry=O.SYM_MLH, pass_no=2)
    assert list(even["keep"]) == [True, True] and list(even["C"]) == [1, 0]


def test_minimum_label_heuristic_rule_on_random_graphs():
    rng = np.random.default_rng(8)
    for k, g in enumerate(tiny_graphs(12, 10, 40, seed=21)):
        vw, p, q = resolved(g)
        C = rng.integers(0, g.n, size=g.n).astype(np.int32)
        for pass_no in (1, 2):
            r = O.lm_pass(g, vw, p, q, C, phi=(0, 1), symmetry=O.SYM_MLH, pass_no=pass_no)
            for v in range(g.n):
                if not r["cand"][v]:
                    assert not r["keep"][v]
                elif pass_no == 2:
                    assert r["keep"][v]
                else:
                    assert r["keep"][v] == (r["D"][v] == O.EMPTY or r["D"][v] < C[v])
