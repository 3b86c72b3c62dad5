"""Pins for the oracle's ordering and schedule rules, each against a statement of the paper rather than the
oracle's own code:

* the afterburner order (Sec. IV-A): larger objective deltas first; deltas within epsilon = 0.1 of each other
  are ordered by a hash of the vertex ids (the reading: smaller splitmix64 finaliser first);
* the temperature schedule of the experiments (Sec. VI): six passes, phi = 0.75 for the first four and 0.25
  for the last two;
* the best-so-far clustering of Alg. 2, replaced only when the objective is strictly larger;
* the singleton-tree fix of pLeidenR (Sec. V-B): a root without children takes f_new = 2K - f_old, so that a
  vertex whose chosen edge pointed to a later vertex joins that vertex's tree.

The hash draws are recomputed here in plain Python from the published generator definitions (splitmix64,
MurmurHash3's 32-bit finaliser), checked first against a published test vector.

CPU only (no GPU marker)."""
from __future__ import annotations

import random

import numpy as np

import graphgen as gg
import oracle as O

M64 = (1 << 64) - 1
M32 = (1 << 32) - 1
GOLDEN = 0x9E3779B97F4A7C15


def splitmix_out(z: int) -> int:
    """Output function of splitmix64 (Steele, Lea & Flood, OOPSLA 2014)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def murmur_fin32(h: int) -> int:
    """Finaliser of MurmurHash3 (Appleby), 32-bit."""
    h &= M32
    h = ((h ^ (h >> 16)) * 0x85EBCA6B) & M32
    h = ((h ^ (h >> 13)) * 0xC2B2AE35) & M32
    return h ^ (h >> 16)


def seed_output(seed: int, t: int) -> int:
    """t-th output (from 0) of the splitmix64 generator seeded with seed."""
    return splitmix_out(seed + (t + 1) * GOLDEN)


def test_python_hashes_match_published_vector():
    # splitmix64 seeded with 1234567: its first two outputs as published with the reference generator
    assert seed_output(1234567, 0) == 6457827717110365317
    assert seed_output(1234567, 1) == 3203168211198807973
    assert murmur_fin32(0) == 0
    for x in (1, 2, 12345, 0xDEADBEEF):
        assert murmur_fin32(x) == O.fmix32(x) and splitmix_out(x) == O.fmix64(x)


# ------------------------------------------------------------------------------------------------
# afterburner order: the epsilon window and the hash tie-break
# ------------------------------------------------------------------------------------------------

def _swap_case(alpha: int, beta: int):
    """Two adjacent vertices u in cluster A and v in cluster B that want to swap, on unit vertex weights with
    lambda = 1/1000 (p = 1, q = 1000).  A = {u, a1} plus alpha isolated vertices, B = {v, b1} plus beta; edges
    u-v (10), u-a1 (1), v-b1 (1).  Then
        delta_u = S(u, B) - S(u, A) = (10 q - (2 + beta)) - (q - (1 + alpha)) = 8999 + alpha - beta,
        delta_v = 8999 + beta - alpha,
    so the objective deltas 2 delta / q differ by 4 (alpha - beta) / q.  The ids are chosen so that v's hash is
    smaller than u's: in a tie v goes first, otherwise u (the larger delta) goes first."""
    ids = sorted(range(4), key=lambda x: splitmix_out(x))
    v, u = ids[0], ids[3]  # splitmix(v) < splitmix(u)
    a1, b1 = ids[1], ids[2]
    n = 4 + alpha + beta
    pairs = [(min(u, v), max(u, v)), (min(u, a1), max(u, a1)), (min(v, b1), max(v, b1))]
    w = [10, 1, 1]
    g = gg.from_pairs(n, pairs, w)
    C = np.zeros(n, np.int32)
    C[[u, a1]] = u
    C[[v, b1]] = v
    C[4:4 + alpha] = u
    C[4 + alpha:] = v
    st, vw, p, q = O.setup(g, O.VW_UNIT, (1, 1000, False))
    assert st == 0 and (p, q) == (1, 1000)
    return g, vw, p, q, C, u, v


def test_afterburner_epsilon_window_and_hash_order():
    """Sec. IV-A: candidates are ordered by objective delta, larger first, unless the deltas differ by less than
    epsilon = 0.1, when a hash of the ids decides.  With q = 1000 the objective deltas 2 delta / q differ by
    less than 0.1 exactly when |delta_u - delta_v| < 50.  The earlier vertex of the swapping pair keeps its move;
    the later one carries -2 q w'(u, v) = -19998 and is dropped."""
    penalty = -2 * (10 * 1000 - 1)
    for alpha, first in [(24, "v"), (25, "u"), (26, "u"), (60, "u")]:
        g, vw, p, q, C, u, v = _swap_case(alpha, 0)
        r = O.lm_pass(g, vw, p, q, C, phi=(0, 1), eps=(1, 10))
        assert r["D"][u] == v and r["D"][v] == u
        assert r["delta"][u] - r["delta"][v] == 2 * alpha
        assert r["cand"][u] and r["cand"][v]
        early, late = (v, u) if first == "v" else (u, v)
        assert r["keep"][early] and not r["keep"][late], (alpha, first)
        assert r["dadj"][late] - r["delta"][late] == penalty
        assert r["dadj"][early] == r["delta"][early]


def test_afterburner_ties_follow_hash_for_equal_deltas():
    """Equal deltas are always a tie: the vertex with the smaller hash goes first."""
    g, vw, p, q, C, u, v = _swap_case(0, 0)
    r = O.lm_pass(g, vw, p, q, C, phi=(0, 1), eps=(1, 10))
    assert r["delta"][u] == r["delta"][v]
    assert r["keep"][v] and not r["keep"][u]


# ------------------------------------------------------------------------------------------------
# LocalMovePasses: the temperature schedule and the strict best-so-far rule
# ------------------------------------------------------------------------------------------------

PAPER_SCHEDULE = [(3, 4)] * 4 + [(1, 4)] * 2  # Sec. VI: six passes, phi 0.75 then 0.25


def _passes(g, vw, p, q, C0, schedule, strict=True):
    """Alg. 2 from the pinned single pass: C_out starts as C_in and is replaced only when a pass reaches a
    strictly larger objective (or an equal one when strict is False, the counterfactual); every pass continues
    from C, not from C_out.  Returns C_out, its objective and the per-pass (|L|, |M|, N)."""
    C = np.array(C0, np.int32)
    best, nbest = C.copy(), O.objective(g, vw, p, q, C)
    recs = []
    for i, phi in enumerate(schedule, 1):
        r = O.lm_pass(g, vw, p, q, C, phi=phi, pass_no=i)
        C = r["C"]
        N = O.objective(g, vw, p, q, C)
        recs.append((r["nL"], r["nM"], N))
        if N > nbest or (not strict and N == nbest):
            best, nbest = C.copy(), N
    return best, nbest, recs


def _cases():
    rng = random.Random(101)
    for k in range(260):
        n = rng.randint(6, 16)
        g = gg.random_gnp(n, rng.choice([0.3, 0.45, 0.6]), 9000 + k, w_max=rng.choice([1, 1, 3]))
        mode, lam = rng.choice([(O.VW_UNIT, (0, 1, False)), (O.VW_WEIGHTED_DEGREE, (1, 1, True)),
                                (O.VW_UNIT, (1, 8, False)), (O.VW_UNIT, (1, 3, False))])
        st, vw, p, q = O.setup(g, mode, lam)
        if st != 0:
            continue
        for s in range(3):
            if s == 0:
                C0 = np.arange(n, dtype=np.int32)
            else:
                C0 = np.array([rng.randrange(max(1, n // 3)) for _ in range(n)], np.int32)
            yield g, vw, p, q, C0


def test_local_move_follows_paper_schedule_and_strict_best():
    """The oracle's LocalMovePasses (default options) against Alg. 2 composed from single passes with the
    schedule of Sec. VI and the strict improvement test.  The counterfactuals (phi = 0.25 already in pass 4; a
    non-strict best-so-far test) must change the outcome on some of these graphs, so the pin can tell them
    apart."""
    phi_sensitive = tie_sensitive = total = 0
    alt_schedule = [(3, 4)] * 3 + [(1, 4)] * 3
    for g, vw, p, q, C0 in _cases():
        got, ngot = O.local_move(g, vw, p, q, C0)
        want, nwant, _ = _passes(g, vw, p, q, C0, PAPER_SCHEDULE)
        assert np.array_equal(got, want) and ngot == nwant
        alt, nalt, _ = _passes(g, vw, p, q, C0, alt_schedule)
        phi_sensitive += int(not np.array_equal(alt, want))
        loose, _, _ = _passes(g, vw, p, q, C0, PAPER_SCHEDULE, strict=False)
        tie_sensitive += int(not np.array_equal(loose, want))
        total += 1
    assert total > 300
    assert phi_sensitive >= 5, phi_sensitive
    assert tie_sensitive >= 5, tie_sensitive


def test_pipeline_level0_passes_follow_paper_schedule():
    """Louvain's level-0 LocalMovePasses inside the full pipeline (singleton start): its per-pass trace
    records (|L|, |M|, N) equal Alg. 2 composed from single passes with the schedule of Sec. VI."""
    checked = 0
    for k, (g, vw, p, q, C0) in enumerate(_cases()):
        if k % 3:  # singleton starts only
            continue
        mode = O.VW_UNIT if vw.sum() == g.n else O.VW_WEIGHTED_DEGREE
        lam = (p, q, False) if mode == O.VW_UNIT else (1, 1, True)
        if mode == O.VW_WEIGHTED_DEGREE and (p, q) != O.setup(g, mode, lam)[2:]:
            continue
        r = O.cluster(g, O.LOUVAIN, lam=lam, vw_mode=mode)
        assert r.status == 0
        recs = [tuple(int(x) for x in t[4:7]) for t in r.trace if t[0] == 1 and t[1] == 0 and t[2] == 0]
        _, _, want = _passes(g, vw, p, q, C0, PAPER_SCHEDULE)
        assert recs == [(a, b, c) for a, b, c in want]
        checked += 1
    assert checked > 50


# ------------------------------------------------------------------------------------------------
# pLeidenR: the singleton-tree fix f_new = 2K - f_old
# ------------------------------------------------------------------------------------------------

def _expected_pair_refinement(seed: int, t: int):
    """pLeidenR on the single edge 0-1 (both vertices well connected, w'(0, 1) >= 0), from the paper's steps
    and the readings of its random choices:
      A_v = {0, 1} in id order; H[v] = A_v[splitmix(s_t ^ 2v) mod 2] with s_t the t-th generator output;
      f(v) = fmix32(v ^ high32(s_t)); an edge is kept only towards a smaller f;
      roots without children take f = 2K - 1 - f (K = 2^32) and their own edge is tested again.
    Returns (merged, the flip decided it)."""
    s = seed_output(seed, t)
    H = [[0, 1][splitmix_out(s ^ (2 * v)) % 2] for v in (0, 1)]
    f = [murmur_fin32(v ^ (s >> 32)) for v in (0, 1)]
    par = [H[v] if H[v] != v and f[H[v]] < f[v] else v for v in (0, 1)]
    child = [any(par[x] == v and x != v for x in (0, 1)) for v in (0, 1)]
    merged_before = par[0] == 1 or par[1] == 0
    K = 1 << 32
    flipped = [par[v] == v and not child[v] for v in (0, 1)]
    f2 = [2 * K - 1 - f[v] if flipped[v] else f[v] for v in (0, 1)]
    for v in (0, 1):
        if flipped[v] and H[v] != v and f2[H[v]] < f2[v]:
            par[v] = H[v]
    merged = par[0] == 1 or par[1] == 0
    return merged, merged and not merged_before


def test_refine_singleton_flip_joins_trees():
    """Sec. V-B: a vertex left alone because its chosen edge pointed to a later vertex gets a new order value,
    which reverses the order of the singleton trees and lets its edge through.  On one edge the pair merges
    unless both vertices chose themselves (the only singleton trees the fix leaves, as the paper states)."""
    g = gg.from_pairs(2, [(0, 1)], [10])
    st, vw, p, q = O.setup(g, O.VW_UNIT, (1, 20, False))
    B = np.zeros(2, np.int32)
    flip_decided = 0
    for t in range(96):
        merged, by_flip = _expected_pair_refinement(7, t)
        R = O.refine(g, vw, p, q, B, seed=7, t=t)["R"]
        assert (R[0] == R[1]) == merged, t
        if merged:
            assert R[0] == R[1] in (0, 1)
        else:
            assert list(R) == [0, 1]
        flip_decided += int(by_flip)
    assert flip_decided >= 10, flip_decided
