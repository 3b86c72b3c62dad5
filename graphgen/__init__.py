"""Seeded synthetic graph generators shared by the tests, the oracle scripts and the benchmark.

The generators live in ``gen.c`` (counter-based randomness, OpenMP) and are loaded through ctypes.
They hold none of the clustering method's arithmetic: they only draw edges and build a symmetric CSR
(rows ascending, neighbours ascending and unique, no self-loops, duplicates merged by summing
integer weights).

Workload recipes (sizes follow the paper's graph families, Table 1):
  * ``sbm``     planted partition, unit weights (community structure)
  * ``rmat``    R-MAT with quadrant probabilities (a, b, c, d), multiplicity weights (skewed degrees)
  * ``lattice`` 2-D 4-neighbour grid with a fixed fraction of edges deleted, weights uniform in [1, w_max]
  * ``knn``     k = 15 nearest-neighbour graphs of 50-D Gaussian-mixture points (geometric families), weights
                exp(-d^2 / sigma^2) quantised to 1..1000; ``knn_batch_spec`` gives the sizes of the batched
                workload and ``knn_graph_torch`` builds the same graphs with torch tensors on a GPU (a data tool,
                used where brute force on the host would take hours)
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile gen.c into libgraphgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P64 = ctypes.POINTER(ctypes.c_int64)
        P32 = ctypes.POINTER(ctypes.c_int32)
        PP64 = ctypes.POINTER(P64)
        PP32 = ctypes.POINTER(P32)
        lib.gen_sbm.restype = ctypes.c_int64
        lib.gen_sbm.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_uint64, P64, PP64, PP32, PP32]
        lib.gen_rmat.restype = ctypes.c_int64
        lib.gen_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_uint64, P64, PP64, PP32, PP32]
        lib.gen_lattice.restype = ctypes.c_int64
        lib.gen_lattice.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                    ctypes.c_uint64, P64, PP64, PP32, PP32]
        lib.gen_from_pairs.restype = ctypes.c_int64
        lib.gen_from_pairs.argtypes = [ctypes.c_int64, ctypes.c_int64, P32, P32, P32, PP64, PP32, PP32]
        lib.gen_knn_points.restype = None
        lib.gen_knn_points.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                       ctypes.c_uint64, ctypes.POINTER(ctypes.c_int8)]
        lib.gen_knn.restype = None
        lib.gen_knn.argtypes = [ctypes.POINTER(ctypes.c_int8), ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                P32, P64]
        lib.gen_free.restype = None
        lib.gen_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Symmetric CSR: ``off`` int64[n+1], ``idx`` int32[nnz], ``w`` int32[nnz]."""
    n: int
    off: np.ndarray
    idx: np.ndarray
    w: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.off[-1])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (np.int64(self.n), self.off, self.idx, self.w):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def _take(lib, nnz, n, poff, pidx, pw, name) -> Graph:
    if nnz < 0:
        raise MemoryError("graph generation failed (allocation or weight overflow)")
    off = np.ctypeslib.as_array(poff, shape=(n + 1,)).copy()
    idx = np.ctypeslib.as_array(pidx, shape=(max(nnz, 1),))[:nnz].copy()
    w = np.ctypeslib.as_array(pw, shape=(max(nnz, 1),))[:nnz].copy()
    for p in (poff, pidx, pw):
        lib.gen_free(ctypes.cast(p, ctypes.c_void_p))
    return Graph(n=n, off=off, idx=idx, w=w, name=name)


def _outs():
    return (ctypes.c_int64(0), ctypes.POINTER(ctypes.c_int64)(), ctypes.POINTER(ctypes.c_int32)(),
            ctypes.POINTER(ctypes.c_int32)())


def sbm(n_blocks: int, block_size: int, p_in: float, p_out: float, seed: int) -> Graph:
    lib = _load()
    n, po, pi, pw = _outs()
    nnz = lib.gen_sbm(n_blocks, block_size, p_in, p_out, seed, ctypes.byref(n), ctypes.byref(po),
                      ctypes.byref(pi), ctypes.byref(pw))
    return _take(lib, nnz, n.value, po, pi, pw, f"sbm{n_blocks}x{block_size}")


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 2) -> Graph:
    lib = _load()
    n, po, pi, pw = _outs()
    nnz = lib.gen_rmat(scale, edge_factor, a, b, c, seed, ctypes.byref(n), ctypes.byref(po),
                       ctypes.byref(pi), ctypes.byref(pw))
    return _take(lib, nnz, n.value, po, pi, pw, f"rmat{scale}")


def lattice(rows: int, cols: int, del_frac: float = 0.1, w_max: int = 100, seed: int = 3) -> Graph:
    lib = _load()
    n, po, pi, pw = _outs()
    nnz = lib.gen_lattice(rows, cols, del_frac, w_max, seed, ctypes.byref(n), ctypes.byref(po),
                          ctypes.byref(pi), ctypes.byref(pw))
    return _take(lib, nnz, n.value, po, pi, pw, f"lattice{rows}x{cols}")


def from_pairs(n: int, pairs, weights=None, name: str = "pairs") -> Graph:
    """CSR from an undirected pair list; self-loops dropped, duplicates summed."""
    lib = _load()
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    pu = np.ascontiguousarray(pairs[:, 0].astype(np.int32))
    pv = np.ascontiguousarray(pairs[:, 1].astype(np.int32))
    P32 = ctypes.POINTER(ctypes.c_int32)
    if weights is None:
        pw_in = None
    else:
        wa = np.ascontiguousarray(np.asarray(weights, dtype=np.int32))
        pw_in = wa.ctypes.data_as(P32)
    _, po, pi, pw = _outs()
    nnz = lib.gen_from_pairs(n, len(pu), pu.ctypes.data_as(P32), pv.ctypes.data_as(P32), pw_in,
                             ctypes.byref(po), ctypes.byref(pi), ctypes.byref(pw))
    return _take(lib, nnz, n, po, pi, pw, name)


def random_gnp(n: int, p: float, seed: int, w_max: int = 1) -> Graph:
    """Small Erdos-Renyi graph (numpy RNG), weights uniform in [1, w_max]; for tests."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(len(iu)) < p
    pairs = np.stack([iu[keep], ju[keep]], axis=1)
    wts = rng.integers(1, w_max + 1, size=len(pairs)) if w_max > 1 else None
    return from_pairs(n, pairs, wts, name=f"gnp{n}")


def reweight(g: Graph, total: int, seed: int) -> Graph:
    """Same edges as ``g``, new symmetric integer weights uniform in [1, 2 m] scaled so that the sum of all
    CSR entries comes to about ``total`` (and never above it); for tests of large weight totals."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.off))
    up = rows < g.idx
    pairs = np.stack([rows[up], g.idx[up].astype(np.int64)], axis=1)
    m = len(pairs)
    raw = rng.integers(1, 2 * m + 1, size=m).astype(np.float64)
    w = np.maximum(1, np.floor(raw * (total / 2) / raw.sum())).astype(np.int64)
    assert 2 * int(w.sum()) <= total and int(w.max()) < 2 ** 31
    return from_pairs(g.n, pairs, w, name=g.name + "-heavy")


# Named workloads ---------------------------------------------------------------------------------

def config1_sbm() -> Graph:
    """2,000 vertices in 20 blocks of 100, p_in 0.1, p_out 0.002, unit weights, seed 1."""
    return sbm(20, 100, 0.1, 0.002, 1)


def config2_rmat() -> Graph:
    """R-MAT scale 22, edge factor 16, (0.57, 0.19, 0.19, 0.05), seed 2."""
    return rmat(22, 16, 0.57, 0.19, 0.19, 2)


def config3a_lattice() -> Graph:
    """4096 x 4096 lattice, 10 % of edges deleted, weights uniform in [1, 100], seed 3."""
    return lattice(4096, 4096, 0.1, 100, 3)


def config3b_rmat() -> Graph:
    """R-MAT scale 26, edge factor 16, same generator as the scale-22 graph, seed 4."""
    return rmat(26, 16, 0.57, 0.19, 0.19, 4)


# k-nearest-neighbour graphs (batched workload) ----------------------------------------------------

KNN_DIM = 50
KNN_K = 15
_GOLDEN = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def _fmix64_int(z: int) -> int:
    z &= _M64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & _M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def _draw(seed: int, stream: int, ctr: int) -> int:
    key = _fmix64_int(seed ^ _fmix64_int(stream + _GOLDEN))
    return _fmix64_int(key + (ctr + 1) * _GOLDEN)


def knn_batch_spec(count: int = 4096, seed: int = 5, n_min: int = 500, n_max: int = 50000):
    """(n_g, K_g) of graph g: n_g = round(exp(U[ln n_min, ln n_max])), K_g uniform in 5..40 components.
    Draws come from the generator stream 2^32 + g of `seed` (the points use streams 2g and 2g + 1)."""
    import math
    out = []
    for g in range(count):
        u = ((_draw(seed, (1 << 32) + g, 0) >> 11) + 1) / float(1 << 53)
        n = int(round(math.exp(math.log(n_min) + u * (math.log(n_max) - math.log(n_min)))))
        K = 5 + _draw(seed, (1 << 32) + g, 1) % 36
        out.append((n, int(K)))
    return out


def knn_points(n: int, K: int, seed: int, graph: int, dim: int = KNN_DIM) -> np.ndarray:
    """int8[n, dim] Gaussian-mixture points on the 1/8 grid (see gen.c for the integer recipe)."""
    lib = _load()
    out = np.zeros((n, dim), dtype=np.int8)
    lib.gen_knn_points(n, dim, K, seed, graph, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    return out


def knn_weights(d2: np.ndarray, sigma2: float) -> np.ndarray:
    """clamp(floor(1000 exp(-d^2 / sigma^2) + 1/2), 1, 1000)."""
    w = np.floor(1000.0 * np.exp(-d2.astype(np.float64) / sigma2) + 0.5)
    return np.clip(w, 1, 1000).astype(np.int32)


def knn_graph(n: int, K: int, seed: int, graph: int, k: int = KNN_K, dim: int = KNN_DIM) -> Graph:
    """Exact k-NN graph on the host (brute force, for graphs up to a few tens of thousands of vertices):
    sigma^2 = mean squared distance over the directed kNN edges, symmetrised by union with one weight per
    pair (distances are symmetric)."""
    lib = _load()
    pts = knn_points(n, K, seed, graph, dim)
    nbr = np.zeros(n * k, dtype=np.int32)
    d2 = np.zeros(n * k, dtype=np.int64)
    lib.gen_knn(pts.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), n, dim, k,
                nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), d2.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    sigma2 = float(d2.sum()) / float(len(d2))
    u = np.repeat(np.arange(n, dtype=np.int64), k)
    v = nbr.astype(np.int64)
    a, b = np.minimum(u, v), np.maximum(u, v)
    key, first = np.unique(a * n + b, return_index=True)
    w = knn_weights(d2[first], sigma2)
    pairs = np.stack([key // n, key % n], axis=1)
    return from_pairs(n, pairs, w, name=f"knn{n}")


def knn_graph_torch(n: int, K: int, seed: int, graph: int, device, k: int = KNN_K, dim: int = KNN_DIM,
                    rows_per_chunk: int = 2048):
    """The same graph as ``knn_graph``, built with torch on `device`.  Returns (off int64, idx int32, w int32)
    device tensors.  Exact: coordinates are small integers, distances are formed in float64 (exact below
    2^53) and neighbours are ranked by the integer key d^2 * 2^16 + index."""
    import torch
    pts = torch.from_numpy(knn_points(n, K, seed, graph, dim)).to(device)
    x = pts.to(torch.float64)
    sq = (x * x).sum(1)
    nbrs, d2s = [], []
    idx = torch.arange(n, device=device, dtype=torch.int64)
    for r0 in range(0, n, rows_per_chunk):
        r1 = min(n, r0 + rows_per_chunk)
        D = sq[r0:r1, None] + sq[None, :] - 2.0 * (x[r0:r1] @ x.T)
        key = D.round().to(torch.int64) * 65536 + idx[None, :]
        key[torch.arange(r1 - r0, device=device), idx[r0:r1]] = torch.iinfo(torch.int64).max
        top = torch.topk(key, k, dim=1, largest=False, sorted=True).values
        nbrs.append(top & 0xFFFF)
        d2s.append(top >> 16)
        del D, key
    nbr = torch.cat(nbrs).reshape(-1)
    d2 = torch.cat(d2s).reshape(-1)
    sigma2 = float(d2.sum().item()) / float(d2.numel())
    u = idx.repeat_interleave(k)
    a, b = torch.minimum(u, nbr), torch.maximum(u, nbr)
    # both directions of every pair, one weight per pair
    src = torch.cat([a, b])
    dst = torch.cat([b, a])
    dd = torch.cat([d2, d2])
    key = src * n + dst
    order = torch.argsort(key, stable=True)
    key, dd = key[order], dd[order]
    keep = torch.ones_like(key, dtype=torch.bool)
    keep[1:] = key[1:] != key[:-1]
    key, dd = key[keep], dd[keep]
    w = torch.floor(1000.0 * torch.exp(-dd.to(torch.float64) / sigma2) + 0.5).clamp(1, 1000).to(torch.int32)
    rows = key // n
    cols = (key % n).to(torch.int32)
    off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    off[1:] = torch.cumsum(torch.bincount(rows, minlength=n), 0)
    return off, cols.contiguous(), w.contiguous()


# Request stream of the served workload ------------------------------------------------------------

SERVE_OBJECTIVES = [((1, 1, True), 1), ((1, 10, False), 2), ((1, 20, False), 2), ((1, 50, False), 2)]
"""(lambda, vertex-weight mode): modularity (weighted degree), CPM 1/10, 1/20, 1/50 (unit weights)."""


def serve_pool(seed: int = 6, sbm_blocks=(2, 7000), rmat_scales=(12, 20), knn_n=(500, 50000), n_sbm: int = 16,
               n_knn: int = 16):
    """Graph specs the request stream draws from: SBM with b blocks of 100 (p_in 0.1, p_out 3.8 / (n - 100),
    b log-spaced), R-MAT of every scale in the range (edge factor 16), kNN graphs of the batched workload's
    generator (sizes log-uniform).  Returns a list of ("sbm", b) / ("rmat", scale) / ("knn", n, K, index)."""
    import math
    pool = []
    lo, hi = sbm_blocks
    for i in range(n_sbm):
        b = int(round(math.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * i / max(1, n_sbm - 1))))
        pool.append(("sbm", b))
    for s in range(rmat_scales[0], rmat_scales[1] + 1):
        pool.append(("rmat", s))
    for i, (n, K) in enumerate(knn_batch_spec(n_knn, seed, knn_n[0], knn_n[1])):
        pool.append(("knn", n, K, i))
    return pool


def serve_graph(spec, seed: int = 6) -> Graph:
    """Host graph of a pool entry (kNN graphs by host brute force: use small kNN sizes on the host)."""
    if spec[0] == "sbm":
        b = spec[1]
        n = 100 * b
        return sbm(b, 100, 0.1, 3.8 / (n - 100), seed)
    if spec[0] == "rmat":
        return rmat(spec[1], 16, 0.57, 0.19, 0.19, seed)
    _, n, K, i = spec
    return knn_graph(n, K, seed, i)


def serve_requests(count: int, pool_size_by_family, seed: int = 6):
    """Request k: family uniform over (sbm, rmat, knn), a pool entry of that family uniform, objective uniform
    over SERVE_OBJECTIVES, variant pLouvain+ or pLeiden with probability 1/2 each.  Returns a list of
    (family, entry, objective index, variant) with variant 1 = pLouvain+, 2 = pLeiden."""
    out = []
    fams = ["sbm", "rmat", "knn"]
    for k in range(count):
        d = [_draw(seed, (1 << 33) + k, t) for t in range(4)]
        fam = fams[d[0] % 3]
        out.append((fam, int(d[1] % pool_size_by_family[fam]), int(d[2] % len(SERVE_OBJECTIVES)),
                    1 if d[3] % 2 == 0 else 2))
    return out
