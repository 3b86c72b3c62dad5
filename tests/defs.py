"""Definitions straight from the paper, in exact rational arithmetic, for pinning the oracle.

These are written from the set-based definitions of Sec. II (w(X), w(X, Y), the signed graph
w'(X, Y) = w(X, Y) - lambda w(X) w(Y minus X), Eq. 1) and deliberately do NOT use the oracle's
integer score form (q a - p w W); a transposed operand or dropped term in either shows up as a
mismatch.  Pure Python: tiny graphs only.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


class Dense:
    """Dense symmetric weight matrix + vertex weights for tiny graphs."""

    def __init__(self, g, vw):
        self.n = g.n
        self.A = [[0] * g.n for _ in range(g.n)]
        for v in range(g.n):
            for j in range(int(g.off[v]), int(g.off[v + 1])):
                self.A[v][int(g.idx[j])] = int(g.w[j]) if g.w is not None else 1
        self.vw = [int(x) for x in vw]

    def wset(self, X):
        return sum(self.vw[v] for v in X)

    def wedge(self, X, Y):
        """w(X, Y) = sum over (u, v) in X x (Y minus X) of w(u, v)."""
        Xs = set(X)
        return sum(self.A[u][v] for u in X for v in Y if v not in Xs)

    def wprime(self, X, Y, lam):
        """w'(X, Y) = w(X, Y) - lambda w(X) w(Y minus X)."""
        Xs = set(X)
        return self.wedge(X, Y) - lam * self.wset(X) * self.wset([v for v in Y if v not in Xs])

    def lambdacc(self, C, lam):
        """Eq. 1: sum over clusters of sum over ordered pairs u != v of w(u,v) - lambda w(u) w(v)."""
        tot = Fraction(0)
        for u in range(self.n):
            for v in range(self.n):
                if u != v and C[u] == C[v]:
                    tot += self.A[u][v] - lam * self.vw[u] * self.vw[v]
        return tot


def clusters_of(C):
    out = {}
    for v, c in enumerate(C):
        out.setdefault(int(c), []).append(v)
    return out


def set_partitions(n):
    """All set partitions of range(n) as restricted-growth label lists (Bell(n) of them)."""
    def rec(i, labels, k):
        if i == n:
            yield list(labels)
            return
        for c in range(k + 1):
            labels.append(c)
            yield from rec(i + 1, labels, max(k, c + 1))
            labels.pop()
    yield from rec(0, [], 0)


def textbook_modularity(g, labels, gamma=1.0):
    """Newman-Girvan weighted modularity, FP64, from the dense adjacency:
    Q = (1/2m) sum_ij [A_ij - gamma k_i k_j / 2m] delta(c_i, c_j), k = weighted degree, 2m = sum k."""
    n = g.n
    A = np.zeros((n, n))
    for v in range(n):
        for j in range(int(g.off[v]), int(g.off[v + 1])):
            A[v, int(g.idx[j])] = float(g.w[j]) if g.w is not None else 1.0
    k = A.sum(axis=1)
    two_m = k.sum()
    same = np.asarray(labels)[:, None] == np.asarray(labels)[None, :]
    return float(((A - gamma * np.outer(k, k) / two_m) * same).sum() / two_m)


def connected_within(g, members):
    """BFS over the subgraph induced by `members`."""
    ms = set(members)
    if not ms:
        return True
    start = next(iter(ms))
    seen = {start}
    stack = [start]
    while stack:
        v = stack.pop()
        for j in range(int(g.off[v]), int(g.off[v + 1])):
            u = int(g.idx[j])
            if u in ms and u not in seen:
                seen.add(u)
                stack.append(u)
    return seen == ms


def components(g):
    lab = [-1] * g.n
    c = 0
    for s in range(g.n):
        if lab[s] >= 0:
            continue
        lab[s] = c
        stack = [s]
        while stack:
            v = stack.pop()
            for j in range(int(g.off[v]), int(g.off[v + 1])):
                u = int(g.idx[j])
                if lab[u] < 0:
                    lab[u] = c
                    stack.append(u)
        c += 1
    return lab


def same_partition(a, b):
    """True iff two label vectors induce the same partition."""
    a = np.asarray(a)
    b = np.asarray(b)
    if a.shape != b.shape:
        return False
    fwd, bwd = {}, {}
    for x, y in zip(a.tolist(), b.tolist()):
        if fwd.setdefault(x, y) != y or bwd.setdefault(y, x) != x:
            return False
    return True


def leidenr_reachable(D: Dense, B, lam, max_n=7):
    """Every clustering sequential LeidenR (Sec. V-B) can produce from singletons under constraint B:
    vertices visited in any order; a visited vertex that is still a singleton may stay, or join an
    adjacent cluster X of its own constraint cluster when it is well connected (w'(v, B[v]) >= 0),
    w'(v, X) >= 0 and w'(X, B[X]) >= 0; non-singletons are skipped.  Returns a set of canonical
    partitions (tuples of frozensets)."""
    n = D.n
    assert n <= max_n
    Bc = clusters_of(B)
    U = [D.wprime([v], Bc[int(B[v])], lam) >= 0 for v in range(n)]
    results = set()
    seen_states = set()

    def canon(C):
        cl = clusters_of(C)
        return tuple(sorted(tuple(sorted(m)) for m in cl.values()))

    def rec(visited, C):
        key = (visited, tuple(C))
        if key in seen_states:
            return
        seen_states.add(key)
        if visited == (1 << n) - 1:
            results.add(canon(C))
            return
        cl = clusters_of(C)
        for v in range(n):
            if visited & (1 << v):
                continue
            nv = visited | (1 << v)
            rec(nv, C)  # stay (or skipped)
            if len(cl[C[v]]) != 1 or not U[v]:
                continue
            for x, X in cl.items():
                if x == C[v] or int(B[X[0]]) != int(B[v]):
                    continue
                if not any(D.A[v][u] for u in X):
                    continue
                if D.wprime([v], X, lam) < 0 or D.wprime(X, Bc[int(B[v])], lam) < 0:
                    continue
                C2 = list(C)
                C2[v] = x
                rec(nv, C2)

    rec(0, list(range(n)))
    return results
