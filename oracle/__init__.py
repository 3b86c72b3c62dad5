"""CPU oracle for synchronous multilevel LambdaCC clustering (pLouvain / Louvain+, pLeiden).

TEST INFRASTRUCTURE ONLY: the plain, exact, single-threaded reference the GPU library is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it.  It shares no code with the GPU library (``paper_2608_01503_amd``); the two meet only in
the seeded generators of ``graphgen``.

Everything is computed in ``lcc_oracle.c`` (gcc, no fast-math, 128-bit integer arithmetic).
This module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lcc_oracle.c")
_HDR = os.path.join(_HERE, "lcc_oracle.h")
_LIB = os.path.join(_HERE, "liblcc_oracle.so")
_lib = None

LOUVAIN, PLOUVAIN, PLEIDEN, PLEIDEN_PLUS = 0, 1, 2, 3
VW_GIVEN, VW_WEIGHTED_DEGREE, VW_UNIT = 0, 1, 2
EMPTY, NONE = -2, -1
STATUS = {0: "OK", -1: "INVALID", -2: "NOT_SYMMETRIC", -3: "SELF_LOOP", -4: "UNSORTED", -5: "WEIGHT",
          -6: "LAMBDA", -7: "OVERFLOW", -8: "OOM"}
TR_LMPASS, TR_LEVEL, TR_LMALT, TR_REFINE = 1, 2, 3, 4


def build(force: bool = False) -> str:
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_HDR))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class Opts(ctypes.Structure):
    _fields_ = [("pass_limit", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("phi_num", ctypes.c_uint32 * 8), ("phi_den", ctypes.c_uint32 * 8),
                ("phi_until", ctypes.c_uint32 * 8), ("eps_num", ctypes.c_uint32),
                ("eps_den", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("max_levels", ctypes.c_int32),
                ("symmetry", ctypes.c_int32)]


SYM_AFTERBURNER, SYM_NONE, SYM_MLH = 0, 1, 2


def make_opts(pass_limit=6, phases=((3, 4, 4), (1, 4, 6)), eps=(1, 10), seed=1, max_levels=64,
              symmetry=SYM_AFTERBURNER) -> Opts:
    """Options: ``phases`` is a list of (phi_num, phi_den, last_pass); ``symmetry`` an ORC_SYM_* mode."""
    o = Opts()
    o.pass_limit = pass_limit
    o.n_phi = len(phases)
    for k, (a, b, u) in enumerate(phases):
        o.phi_num[k], o.phi_den[k], o.phi_until[k] = a, b, u
    o.eps_num, o.eps_den = eps
    o.seed = seed
    o.max_levels = max_levels
    o.symmetry = symmetry
    return o


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t)) if a is not None else None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, u64, i32, u32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32
        P = ctypes.POINTER
        g = [i64, P(i64), P(i32), P(i32), P(i64)]
        lib.orc_cluster.restype = ctypes.c_int
        lib.orc_cluster.argtypes = g + [ctypes.c_int, u64, u64, ctypes.c_int, ctypes.c_int, P(Opts), P(i32),
                                        P(i64), P(i64), i64, P(i64)]
        lib.orc_cluster_ex.restype = ctypes.c_int
        lib.orc_cluster_ex.argtypes = g + [ctypes.c_int, u64, u64, ctypes.c_int, ctypes.c_int, P(Opts), P(i32),
                                           P(i32), P(i32), P(i64), P(i64), i64, P(i64)]
        lib.orc_setup.restype = ctypes.c_int
        lib.orc_setup.argtypes = g + [ctypes.c_int, u64, u64, ctypes.c_int, P(i64), P(u64)]
        lib.orc_objective.restype = None
        lib.orc_objective.argtypes = g + [u64, u64, P(i32), P(i64)]
        lib.orc_lm_pass.restype = None
        lib.orc_lm_pass.argtypes = g + [u64, u64, u32, u32, u32, u32, ctypes.c_int32, ctypes.c_int32, P(i32), P(i32),
                                        P(i64), P(u64), P(i64),
                                        P(u64), P(ctypes.c_uint8), P(ctypes.c_uint8), P(i64)]
        lib.orc_local_move.restype = None
        lib.orc_local_move.argtypes = g + [u64, u64, P(Opts), P(i32), P(i64)]
        lib.orc_contract.restype = i64
        lib.orc_contract.argtypes = g + [P(i64), P(i64), P(i32), i64, P(i64), P(i32), P(i32), P(i64), P(i64),
                                         P(i64)]
        lib.orc_refine.restype = None
        lib.orc_refine.argtypes = g + [u64, u64, P(i32), u64, u64, P(i32), P(i32), P(i32), P(i64)]
        lib.orc_lmalt.restype = None
        lib.orc_lmalt.argtypes = g + [u64, u64, P(i32), P(i64)]
        lib.orc_fmix64.restype = u64
        lib.orc_fmix64.argtypes = [u64]
        lib.orc_fmix32.restype = u32
        lib.orc_fmix32.argtypes = [u32]
        _lib = lib
    return _lib


def _garrays(g, vw=None):
    off = np.ascontiguousarray(g.off, dtype=np.int64)
    idx = np.ascontiguousarray(g.idx, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.int32) if g.w is not None else None
    vwa = np.ascontiguousarray(vw, dtype=np.int64) if vw is not None else None
    keep = (off, idx, w, vwa)
    return keep, [g.n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32), _p(w, ctypes.c_int32),
                  _p(vwa, ctypes.c_int64)]


def _i128(hi, lo) -> int:
    return (int(hi) << 64) + (int(lo) & 0xFFFFFFFFFFFFFFFF)


@dataclass
class Result:
    status: int
    labels: np.ndarray | None = None
    num_clusters: int = 0
    N: int = 0            # objective numerator; lambdaCC = N / q
    p: int = 0
    q: int = 0
    levels: int = 0
    flags: int = 0
    trace: np.ndarray | None = field(default=None, repr=False)


def cluster(g, variant=PLOUVAIN, lam=(1, 1, True), vw_mode=VW_WEIGHTED_DEGREE, vw=None, opts=None,
            trace_cap=1 << 16, init=None, constraint=None) -> Result:
    """Full clustering.  ``lam`` = (num, den, over_total_weight): lambda = num/den or num/(den W).
    ``init``: starting clustering (pLeiden: Alg. 5's C_in; Louvain: the level-0 local move's start).
    ``constraint``: Louvain / Louvain+ coarsening confined to the constraint clusters (Sec. IV-D)."""
    lib = _load()
    keep, ga = _garrays(g, vw)
    labels = np.zeros(max(g.n, 1), dtype=np.int32)
    res = np.zeros(8, dtype=np.int64)
    tr = np.zeros(8 * trace_cap, dtype=np.int64)
    tcount = ctypes.c_int64(0)
    o = opts if opts is not None else make_opts()
    ia = np.ascontiguousarray(init, dtype=np.int32) if init is not None else None
    ca = np.ascontiguousarray(constraint, dtype=np.int32) if constraint is not None else None
    st = lib.orc_cluster_ex(*ga, vw_mode, lam[0], lam[1], int(bool(lam[2])), variant, ctypes.byref(o),
                            _p(ia, ctypes.c_int32), _p(ca, ctypes.c_int32),
                            _p(labels, ctypes.c_int32), _p(res, ctypes.c_int64), _p(tr, ctypes.c_int64),
                            trace_cap, ctypes.byref(tcount))
    del keep
    if st != 0:
        return Result(status=st)
    nt = min(tcount.value, trace_cap)
    return Result(status=0, labels=labels[:g.n].copy(), num_clusters=int(res[0]), N=_i128(res[1], res[2]),
                  q=int(res[5]), p=int(res[6]), levels=int(res[3]), flags=int(res[4]),
                  trace=tr[:8 * nt].reshape(nt, 8).copy())


def setup(g, vw_mode=VW_WEIGHTED_DEGREE, lam=(1, 1, True), vw=None):
    """Returns (status, vw, p, q)."""
    lib = _load()
    keep, ga = _garrays(g, vw)
    vout = np.zeros(max(g.n, 1), dtype=np.int64)
    pq = np.zeros(2, dtype=np.uint64)
    st = lib.orc_setup(*ga, vw_mode, lam[0], lam[1], int(bool(lam[2])), _p(vout, ctypes.c_int64),
                       _p(pq, ctypes.c_uint64))
    del keep
    return st, vout[:g.n].copy(), int(pq[0]), int(pq[1])


def objective(g, vw, p, q, C) -> int:
    lib = _load()
    keep, ga = _garrays(g, vw)
    C = np.ascontiguousarray(C, dtype=np.int32)
    out = np.zeros(2, dtype=np.int64)
    lib.orc_objective(*ga, p, q, _p(C, ctypes.c_int32), _p(out, ctypes.c_int64))
    del keep
    return _i128(out[0], out[1])


def lm_pass(g, vw, p, q, C, phi=(3, 4), eps=(1, 10), symmetry=0, pass_no=1):
    """One synchronous pass; returns dict with the new C and the per-vertex decisions."""
    lib = _load()
    keep, ga = _garrays(g, vw)
    n = max(g.n, 1)
    C = np.array(C, dtype=np.int32, copy=True)
    D = np.zeros(n, np.int32)
    dh = np.zeros(n, np.int64)
    dl = np.zeros(n, np.uint64)
    ah = np.zeros(n, np.int64)
    al = np.zeros(n, np.uint64)
    cand = np.zeros(n, np.uint8)
    kp = np.zeros(n, np.uint8)
    cnt = np.zeros(2, np.int64)
    lib.orc_lm_pass(*ga, p, q, phi[0], phi[1], eps[0], eps[1], symmetry, pass_no, _p(C, ctypes.c_int32), _p(D, ctypes.c_int32),
                    _p(dh, ctypes.c_int64), _p(dl, ctypes.c_uint64), _p(ah, ctypes.c_int64), _p(al, ctypes.c_uint64), _p(cand, ctypes.c_uint8),
                    _p(kp, ctypes.c_uint8), _p(cnt, ctypes.c_int64))
    del keep
    delta = [_i128(h, l) for h, l in zip(dh[:g.n], dl[:g.n])]
    dadj = [_i128(h, l) for h, l in zip(ah[:g.n], al[:g.n])]
    return dict(C=C[:g.n], D=D[:g.n], delta=delta, dadj=dadj, cand=cand[:g.n].astype(bool), keep=kp[:g.n].astype(bool),
                nL=int(cnt[0]), nM=int(cnt[1]))


def local_move(g, vw, p, q, C, opts=None):
    lib = _load()
    keep, ga = _garrays(g, vw)
    C = np.array(C, dtype=np.int32, copy=True)
    out = np.zeros(2, np.int64)
    o = opts if opts is not None else make_opts()
    lib.orc_local_move(*ga, p, q, ctypes.byref(o), _p(C, ctypes.c_int32), _p(out, ctypes.c_int64))
    del keep
    return C, _i128(out[0], out[1])


def contract(g, vw, cmap, nc, s=None, sq=None):
    """Returns (coarse Graph-like tuple (n, off, idx, w), cvw, cs, csq)."""
    lib = _load()
    keep, ga = _garrays(g, vw)
    cmap = np.ascontiguousarray(cmap, dtype=np.int32)
    sa = np.ascontiguousarray(s, dtype=np.int64) if s is not None else None
    sqa = np.ascontiguousarray(sq, dtype=np.int64) if sq is not None else None
    nnz = max(int(g.off[-1]), 1)
    coff = np.zeros(nc + 1, np.int64)
    cidx = np.zeros(nnz, np.int32)
    cw = np.zeros(nnz, np.int32)
    cvw = np.zeros(max(nc, 1), np.int64)
    cs = np.zeros(max(nc, 1), np.int64)
    csq = np.zeros(max(nc, 1), np.int64)
    e = lib.orc_contract(*ga, _p(sa, ctypes.c_int64), _p(sqa, ctypes.c_int64), _p(cmap, ctypes.c_int32), nc,
                         _p(coff, ctypes.c_int64), _p(cidx, ctypes.c_int32), _p(cw, ctypes.c_int32),
                         _p(cvw, ctypes.c_int64), _p(cs, ctypes.c_int64), _p(csq, ctypes.c_int64))
    del keep
    from graphgen import Graph
    return Graph(n=nc, off=coff, idx=cidx[:e].copy(), w=cw[:e].copy(), name="coarse"), cvw[:nc], cs[:nc], csq[:nc]


def refine(g, vw, p, q, B, seed=1, t=0):
    """pLeidenR; returns dict(R, parent, root, fkey)."""
    lib = _load()
    keep, ga = _garrays(g, vw)
    n = max(g.n, 1)
    B = np.ascontiguousarray(B, dtype=np.int32)
    R = np.zeros(n, np.int32)
    par = np.zeros(n, np.int32)
    root = np.zeros(n, np.int32)
    fk = np.zeros(n, np.int64)
    lib.orc_refine(*ga, p, q, _p(B, ctypes.c_int32), seed, t, _p(R, ctypes.c_int32), _p(par, ctypes.c_int32),
                   _p(root, ctypes.c_int32), _p(fk, ctypes.c_int64))
    del keep
    return dict(R=R[:g.n], parent=par[:g.n], root=root[:g.n], fkey=fk[:g.n])


def lmalt(g, vw, p, q, C):
    lib = _load()
    keep, ga = _garrays(g, vw)
    C = np.array(C, dtype=np.int32, copy=True)
    cnt = np.zeros(2, np.int64)
    lib.orc_lmalt(*ga, p, q, _p(C, ctypes.c_int32), _p(cnt, ctypes.c_int64))
    del keep
    return C, int(cnt[0]), int(cnt[1])


def fmix64(x: int) -> int:
    return int(_load().orc_fmix64(x))


def fmix32(x: int) -> int:
    return int(_load().orc_fmix32(x))
