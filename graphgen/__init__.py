"""Seeded synthetic graph generators shared by the tests, the oracle scripts and the benchmark.

The generators live in ``gen.c`` (counter-based randomness, OpenMP) and are loaded through ctypes.
They hold none of the clustering method's arithmetic: they only draw edges and build a symmetric CSR
(rows ascending, neighbours ascending and unique, no self-loops, duplicates merged by summing
integer weights).

Workload recipes (sizes follow the paper's graph families, Table 1):
  * ``sbm``     planted partition, unit weights (community structure)
  * ``rmat``    R-MAT with quadrant probabilities (a, b, c, d), multiplicity weights (skewed degrees)
  * ``lattice`` 2-D 4-neighbour grid with a fixed fraction of edges deleted, weights uniform in [1, w_max]
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
