"""Thin Python binding of the C-ABI in include/lcc.h (ctypes marshalling only).

Every step of the clustering runs in the HIP library liblcc.so; this module only converts arguments.  If
the library is missing it raises -- there is no Python or CPU fallback.  Torch supplies device memory (its
caching allocator is passed to the library as the allocator callbacks) and streams.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblcc.so")

# enums of include/lcc.h
LCC_OK = 0
STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "NOT_SYMMETRIC", -3: "SELF_LOOP", -4: "UNSORTED", -5: "WEIGHT",
                -6: "LAMBDA", -7: "OVERFLOW", -8: "OOM", -9: "DEVICE", -10: "BUSY", -11: "NOT_FOUND"}
LCC_LOUVAIN, LCC_PLOUVAIN, LCC_PLEIDEN, LCC_PLEIDEN_PLUS = 0, 1, 2, 3
LCC_VW_GIVEN, LCC_VW_WEIGHTED_DEGREE, LCC_VW_UNIT = 0, 1, 2
LCC_MEM_HOST, LCC_MEM_DEVICE = 0, 1
LCC_FLAG_LEVEL_CAP, LCC_FLAG_REFINE_NO_PROGRESS = 1, 2
LCC_NOALLOC_SCRATCH_BYTES = 128 << 20

EXPORTED = ["lcc_create", "lcc_destroy", "lcc_default_options", "lcc_workspace_bytes", "lcc_cluster",
            "lcc_cluster_ex", "lcc_cluster_noalloc", "lcc_cluster_batch", "lcc_objective", "lcc_objective_device",
            "lcc_server_create", "lcc_submit", "lcc_poll", "lcc_server_destroy", "lcc_profile_enable", "lcc_profile_read", "lcc_status_string", "lcc_last_error",
            "lcc_default_tuning", "lcc_set_tuning", "lcc_get_tuning", "lcc_autotune"]

# kernel families of lcc_profile_enable (bit = index) and the kernel each one times
PROFILE_FAMILIES = ["enum_b0", "enum_b1", "enum_b2", "enum_b3", "enum_b4", "enum_b5", "enum_b6", "enum_b7",
                    "single", "afterburner"]
# (buckets 0-2 share one launch, timed as family enum_b0; enum_b1 and enum_b2 stay empty)
FAMILY_KERNELS = {"enum_b0": "k_enum_grps", "enum_b3": "k_enum_grp<32>", "enum_b4": "k_enum_wave<256>",
                  "enum_b5": "k_enum_blk<128, 2048>",
                  "enum_b6": "k_enum_blk<512, 8192>+k_enum_blk<1024, 16384>",
                  "enum_b7": "k_hub_insert+k_hub_scan+k_hub_final",
                  "single": "k_single_*"}


class lcc_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("offsets", ctypes.c_void_p),
                ("offsets_bits", ctypes.c_int32), ("indices", ctypes.c_void_p), ("edge_w", ctypes.c_void_p),
                ("vertex_w", ctypes.c_void_p), ("vw_mode", ctypes.c_int), ("mem", ctypes.c_int)]


class lcc_lambda(ctypes.Structure):
    _fields_ = [("num", ctypes.c_uint64), ("den", ctypes.c_uint64), ("over_total_weight", ctypes.c_int32)]


class lcc_trace(ctypes.Structure):
    _fields_ = [("records", ctypes.c_void_p), ("capacity", ctypes.c_int64), ("count", ctypes.c_int64)]


class lcc_options(ctypes.Structure):
    _fields_ = [("pass_limit", ctypes.c_int32), ("n_phi", ctypes.c_int32), ("phi_num", ctypes.c_uint32 * 8),
                ("phi_den", ctypes.c_uint32 * 8), ("phi_until", ctypes.c_uint32 * 8), ("eps_num", ctypes.c_uint32),
                ("eps_den", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("max_levels", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("trace", ctypes.POINTER(lcc_trace)), ("symmetry", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_OPTION_FIELDS = {f[0] for f in lcc_options._fields_} - {"n_phi", "phi_num", "phi_den", "phi_until", "eps_num",
                                                           "eps_den", "reserved"}

LCC_SYM_AFTERBURNER, LCC_SYM_NONE, LCC_SYM_MLH = 0, 1, 2


class lcc_tuning(ctypes.Structure):
    _fields_ = [("bucket_max", ctypes.c_int64 * 7), ("grid_cap", ctypes.c_int32), ("hash_shift", ctypes.c_int32)]


class lcc_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class lcc_result(ctypes.Structure):
    _fields_ = [("num_clusters", ctypes.c_int64), ("objective", ctypes.c_double), ("modularity", ctypes.c_double),
                ("obj_num_hi", ctypes.c_int64), ("obj_num_lo", ctypes.c_uint64), ("obj_den", ctypes.c_uint64),
                ("levels", ctypes.c_int32), ("flags", ctypes.c_uint32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def load():
    """Load liblcc.so (built by paper_2608_01503_amd/build.py).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    # torch first: its HIP runtime must be the one loaded into the process (liblcc.so links the same soname
    # and then binds to it); loading liblcc.so first would pull in a second runtime under torch
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    v, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
    st = ctypes.c_int
    lib.lcc_create.restype = st
    lib.lcc_create.argtypes = [ctypes.c_int, ALLOC_FN, FREE_FN, v, P(v)]
    lib.lcc_destroy.restype = st
    lib.lcc_destroy.argtypes = [v]
    lib.lcc_default_options.restype = None
    lib.lcc_default_options.argtypes = [P(lcc_options)]
    lib.lcc_workspace_bytes.restype = st
    lib.lcc_workspace_bytes.argtypes = [i64, i64, ctypes.c_int, P(ctypes.c_size_t)]
    lib.lcc_cluster.restype = st
    lib.lcc_cluster.argtypes = [v, P(lcc_graph), lcc_lambda, ctypes.c_int, P(lcc_options), v, v, P(lcc_result)]
    lib.lcc_cluster_noalloc.restype = st
    lib.lcc_cluster_noalloc.argtypes = [v, P(lcc_graph), lcc_lambda, ctypes.c_int, P(lcc_options), v, v,
                                        P(lcc_result)]
    lib.lcc_cluster_ex.restype = st
    lib.lcc_cluster_ex.argtypes = [v, P(lcc_graph), lcc_lambda, ctypes.c_int, P(lcc_options), v, v, v, v,
                                   P(lcc_result)]
    lib.lcc_cluster_batch.restype = st
    lib.lcc_cluster_batch.argtypes = [v, P(lcc_graph), P(lcc_lambda), P(ctypes.c_int), i64, P(lcc_options), v,
                                      P(v), P(lcc_result)]
    lib.lcc_objective.restype = st
    lib.lcc_objective.argtypes = [P(lcc_graph), lcc_lambda, v, P(lcc_result)]
    lib.lcc_objective_device.restype = st
    lib.lcc_objective_device.argtypes = [v, P(lcc_graph), lcc_lambda, v, v, P(lcc_result)]
    lib.lcc_server_create.restype = st
    lib.lcc_server_create.argtypes = [v, ctypes.c_size_t, P(v)]
    lib.lcc_submit.restype = st
    lib.lcc_submit.argtypes = [v, P(lcc_graph), lcc_lambda, ctypes.c_int, P(lcc_options), P(u64)]
    lib.lcc_poll.restype = st
    lib.lcc_poll.argtypes = [v, u64, P(ctypes.c_int), v, P(lcc_result)]
    lib.lcc_server_destroy.restype = st
    lib.lcc_server_destroy.argtypes = [v]
    lib.lcc_profile_enable.restype = st
    lib.lcc_profile_enable.argtypes = [v, u64]
    lib.lcc_profile_read.restype = st
    lib.lcc_profile_read.argtypes = [v, P(lcc_kernel_stat), ctypes.c_int32, P(ctypes.c_int32), ctypes.c_int32]
    lib.lcc_default_tuning.restype = None
    lib.lcc_default_tuning.argtypes = [P(lcc_tuning)]
    lib.lcc_set_tuning.restype = st
    lib.lcc_set_tuning.argtypes = [v, P(lcc_tuning)]
    lib.lcc_get_tuning.restype = st
    lib.lcc_get_tuning.argtypes = [v, P(lcc_tuning)]
    lib.lcc_autotune.restype = st
    lib.lcc_autotune.argtypes = [v, P(lcc_graph), P(lcc_lambda), P(ctypes.c_int), i64, P(lcc_options), v,
                                 ctypes.c_int32, P(lcc_tuning), P(ctypes.c_double)]
    lib.lcc_status_string.restype = ctypes.c_char_p
    lib.lcc_status_string.argtypes = [ctypes.c_int]
    lib.lcc_last_error.restype = ctypes.c_char_p
    lib.lcc_last_error.argtypes = []
    _lib = lib
    return lib


class LccError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(st: int):
    if st != LCC_OK:
        raise LccError(st, (load().lcc_last_error() or b"").decode())


# ------------------------------------------------------------------------------------------------
# same-named thin wrappers
# ------------------------------------------------------------------------------------------------

def lcc_default_options(**kw) -> lcc_options:
    o = lcc_options()
    load().lcc_default_options(ctypes.byref(o))
    for k, val in kw.items():
        if k == "phases":
            o.n_phi = len(val)
            for j, (a, b, u) in enumerate(val):
                o.phi_num[j], o.phi_den[j], o.phi_until[j] = a, b, u
        elif k == "eps":
            o.eps_num, o.eps_den = val
        elif k in _OPTION_FIELDS:
            setattr(o, k, val)
        else:
            raise TypeError(f"unknown option {k!r}")
    return o


def lcc_default_tuning(bucket_max=None, grid_cap=None, hash_shift=None) -> lcc_tuning:
    """The default launch tuning, with the given fields replaced (bucket_max: 7 bounds)."""
    t = lcc_tuning()
    load().lcc_default_tuning(ctypes.byref(t))
    if bucket_max is not None:
        for k, b in enumerate(bucket_max):
            t.bucket_max[k] = int(b)
    if grid_cap is not None:
        t.grid_cap = int(grid_cap)
    if hash_shift is not None:
        t.hash_shift = int(hash_shift)
    return t


def tuning_dict(t: lcc_tuning) -> dict:
    return {"bucket_max": [int(x) for x in t.bucket_max], "grid_cap": int(t.grid_cap),
            "hash_shift": int(t.hash_shift)}


def lcc_workspace_bytes(n: int, nnz: int, variant: int = LCC_PLOUVAIN) -> int:
    out = ctypes.c_size_t(0)
    _check(load().lcc_workspace_bytes(n, nnz, variant, ctypes.byref(out)))
    return out.value


def lcc_status_string(st: int) -> str:
    return load().lcc_status_string(st).decode()


def lcc_last_error() -> str:
    return (load().lcc_last_error() or b"").decode()


def _ptr(a):
    """Device pointer of a torch tensor or host pointer of a numpy array (None -> NULL)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _is_device(a) -> bool:
    return hasattr(a, "is_cuda") and a.is_cuda


def make_graph(off, idx, w=None, vw=None, vw_mode=LCC_VW_WEIGHTED_DEGREE):
    """lcc_graph over torch CUDA tensors (device) or numpy arrays (host); all arrays in one memory space."""
    dev = _is_device(off)
    n = int(off.shape[0]) - 1
    nnz = int(idx.shape[0])
    bits = 64 if str(off.dtype).endswith("int64") else 32
    g = lcc_graph(n=n, nnz=nnz, offsets=_ptr(off), offsets_bits=bits, indices=_ptr(idx), edge_w=_ptr(w),
                  vertex_w=_ptr(vw), vw_mode=vw_mode, mem=LCC_MEM_DEVICE if dev else LCC_MEM_HOST)
    g._keep = (off, idx, w, vw)
    return g


def lam_of(lam) -> lcc_lambda:
    """(num, den, over_total_weight) -> lcc_lambda."""
    return lcc_lambda(num=int(lam[0]), den=int(lam[1]), over_total_weight=int(bool(lam[2])))


@dataclass
class Result:
    num_clusters: int
    objective: float
    modularity: float
    N: int            # exact objective numerator (lambdaCC = N / obj_den)
    obj_den: int
    levels: int
    flags: int
    trace: np.ndarray | None = field(default=None, repr=False)


def _result(r: lcc_result, trace=None) -> Result:
    N = (int(r.obj_num_hi) << 64) + int(r.obj_num_lo)
    return Result(num_clusters=int(r.num_clusters), objective=float(r.objective), modularity=float(r.modularity),
                  N=N, obj_den=int(r.obj_den), levels=int(r.levels), flags=int(r.flags), trace=trace)


class Context:
    """One lcc_ctx on a HIP device.  allocator: "torch" (torch's caching allocator), "hip" (hipMalloc), or a
    pair of callables (alloc(nbytes) -> device pointer as int, or None when out of memory; free(pointer))."""

    def __init__(self, device: int = 0, allocator="torch"):
        lib = load()
        self.device = device
        self._alloc_cb = ALLOC_FN(0)
        self._free_cb = FREE_FN(0)
        if isinstance(allocator, tuple):
            user_alloc, user_free = allocator

            def _ua(nbytes, user):
                try:
                    return user_alloc(int(nbytes))
                except Exception:  # reported by the library as LCC_ERR_OOM
                    return None

            def _uf(p, user):
                try:
                    user_free(p)
                except Exception:
                    pass

            self._alloc_cb = ALLOC_FN(_ua)
            self._free_cb = FREE_FN(_uf)
        elif allocator == "torch":
            import torch

            def _a(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device)
                except Exception:  # out of memory is reported by the library as LCC_ERR_OOM
                    return None

            def _f(p, user):
                try:
                    torch.cuda.caching_allocator_delete(p)
                except Exception:  # interpreter shutdown: torch is already torn down, the process frees it
                    pass

            self._alloc_cb = ALLOC_FN(_a)
            self._free_cb = FREE_FN(_f)
        h = ctypes.c_void_p()
        _check(lib.lcc_create(device, self._alloc_cb, self._free_cb, None, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load().lcc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cluster(self, graph: lcc_graph, lam=(1, 1, True), variant=LCC_PLOUVAIN, opts: lcc_options | None = None,
                labels_out=None, stream=None, trace_capacity: int = 0, init=None, constraint=None,
                noalloc: bool = False):
        """Cluster one graph.  Returns (labels, Result).  labels_out defaults to a new int32 array in the
        graph's memory space (torch tensor on the device, numpy on the host).  init / constraint: optional
        int32 arrays in the graph's memory space (lcc_cluster_ex).  noalloc: lcc_cluster_noalloc."""
        lib = load()
        if noalloc and (init is not None or constraint is not None):
            raise ValueError("lcc_cluster_noalloc takes no initial or constraint clustering")
        n = graph.n
        if labels_out is None:
            if graph.mem == LCC_MEM_DEVICE:
                import torch
                labels_out = torch.empty(max(n, 1), dtype=torch.int32, device=f"cuda:{self.device}")
            else:
                labels_out = np.zeros(max(n, 1), dtype=np.int32)
        o = opts if opts is not None else lcc_default_options()
        tr = None
        rec = None
        if trace_capacity:
            rec = np.zeros(8 * trace_capacity, dtype=np.int64)
            tr = lcc_trace(records=rec.ctypes.data, capacity=trace_capacity, count=0)
            o.trace = ctypes.pointer(tr)
        res = lcc_result()
        st = _stream_handle(stream, graph)
        if noalloc:
            _check(lib.lcc_cluster_noalloc(self.handle, ctypes.byref(graph), lam_of(lam), variant, ctypes.byref(o),
                                           st, _ptr(labels_out), ctypes.byref(res)))
        elif init is None and constraint is None:
            _check(lib.lcc_cluster(self.handle, ctypes.byref(graph), lam_of(lam), variant, ctypes.byref(o), st,
                                   _ptr(labels_out), ctypes.byref(res)))
        else:
            _check(lib.lcc_cluster_ex(self.handle, ctypes.byref(graph), lam_of(lam), variant, ctypes.byref(o), st,
                                      _ptr(init), _ptr(constraint), _ptr(labels_out), ctypes.byref(res)))
        trace = None
        if tr is not None:
            cnt = min(tr.count, trace_capacity)
            trace = rec[:8 * cnt].reshape(cnt, 8).copy()
            o.trace = None
        return labels_out[:n], _result(res, trace)

    def cluster_batch(self, graphs, lams, variants, opts=None, labels_out=None, stream=None):
        lib = load()
        k = len(graphs)
        G = (lcc_graph * k)(*graphs)
        L = (lcc_lambda * k)(*[lam_of(x) for x in lams])
        V = (ctypes.c_int * k)(*variants)
        if labels_out is None:
            labels_out = []
            for g in graphs:
                if g.mem == LCC_MEM_DEVICE:
                    import torch
                    labels_out.append(torch.empty(max(g.n, 1), dtype=torch.int32, device=f"cuda:{self.device}"))
                else:
                    labels_out.append(np.zeros(max(g.n, 1), dtype=np.int32))
        P = (ctypes.c_void_p * k)(*[_ptr(x) for x in labels_out])
        R = (lcc_result * k)()
        o = opts if opts is not None else lcc_default_options()
        st = _stream_handle(stream, graphs[0] if graphs else None)
        _check(lib.lcc_cluster_batch(self.handle, G, L, V, k, ctypes.byref(o), st, P, R))
        return [lab[:g.n] for lab, g in zip(labels_out, graphs)], [_result(R[i]) for i in range(k)]

    def set_tuning(self, t: lcc_tuning):
        _check(load().lcc_set_tuning(self.handle, ctypes.byref(t)))

    def get_tuning(self) -> lcc_tuning:
        t = lcc_tuning()
        _check(load().lcc_get_tuning(self.handle, ctypes.byref(t)))
        return t

    def autotune(self, graphs, lams, variants, opts=None, stream=None, trials: int = 1):
        """Run the library's autotuner on these graphs; the chosen tuning stays on the context.
        Returns (tuning, ms per run)."""
        lib = load()
        k = len(graphs)
        G = (lcc_graph * k)(*graphs)
        L = (lcc_lambda * k)(*[lam_of(x) for x in lams])
        V = (ctypes.c_int * k)(*variants)
        o = opts if opts is not None else lcc_default_options()
        best = lcc_tuning()
        ms = ctypes.c_double(0.0)
        _check(lib.lcc_autotune(self.handle, G, L, V, k, ctypes.byref(o), _stream_handle(stream, graphs[0]),
                                int(trials), ctypes.byref(best), ctypes.byref(ms)))
        return best, ms.value

    def profile_enable(self, families):
        """Time the named kernel families (see PROFILE_FAMILIES) in subsequent calls; [] disables."""
        mask = 0
        for f in families:
            mask |= 1 << PROFILE_FAMILIES.index(f)
        _check(load().lcc_profile_enable(self.handle, mask))

    def profile_read(self, reset: bool = False) -> dict:
        """{family: (launches, total_ms, algorithmic_bytes)}"""
        cap = len(PROFILE_FAMILIES)
        arr = (lcc_kernel_stat * cap)()
        cnt = ctypes.c_int32(0)
        _check(load().lcc_profile_read(self.handle, arr, cap, ctypes.byref(cnt), int(reset)))
        return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms), float(arr[i].bytes))
                for i in range(min(cnt.value, cap))}

    def objective(self, graph: lcc_graph, labels, lam=(1, 1, True), stream=None) -> Result:
        res = lcc_result()
        _check(load().lcc_objective_device(self.handle, ctypes.byref(graph), lam_of(lam), _ptr(labels),
                                    _stream_handle(stream, graph), ctypes.byref(res)))
        return _result(res)


def lcc_objective(graph: lcc_graph, labels, lam=(1, 1, True)) -> Result:
    """Exact objective of `labels` (numpy int32) on a host graph (numpy arrays), evaluated by the library on the
    host in 128-bit integers."""
    res = lcc_result()
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    _check(load().lcc_objective(ctypes.byref(graph), lam_of(lam), _ptr(lab), ctypes.byref(res)))
    return _result(res)


def _stream_handle(stream, graph):
    if stream is not None:
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    if graph is not None and graph.mem == LCC_MEM_DEVICE:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return None


class Server:
    """Continuous-batching server (lcc_server_*) over a context."""

    def __init__(self, ctx: Context, hbm_budget: int):
        h = ctypes.c_void_p()
        _check(load().lcc_server_create(ctx.handle, hbm_budget, ctypes.byref(h)))
        self.handle = h
        self._ctx = ctx

    def submit(self, graph: lcc_graph, lam=(1, 1, True), variant=LCC_PLOUVAIN, opts=None) -> int:
        t = ctypes.c_uint64(0)
        o = ctypes.byref(opts) if opts is not None else None
        _check(load().lcc_submit(self.handle, ctypes.byref(graph), lam_of(lam), variant, o, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, n: int):
        done = ctypes.c_int(0)
        labels = np.zeros(max(n, 1), dtype=np.int32)
        res = lcc_result()
        _check(load().lcc_poll(self.handle, ticket, ctypes.byref(done), labels.ctypes.data, ctypes.byref(res)))
        if not done.value:
            return None
        return labels[:n], _result(res)

    def close(self):
        if getattr(self, "handle", None):
            load().lcc_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
