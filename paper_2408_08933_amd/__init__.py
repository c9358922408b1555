"""Python binding of the MI355X RoarGraph library (libroargraph.so).

Argument marshalling only: every step of construction and search runs in
the library (HIP kernels on gfx950 plus its native host code).  PyTorch
supplies device memory and the current HIP stream.  Names follow the C ABI
in include/roargraph.h.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RG_LIB", os.path.join(_HERE, "libroargraph.so"))

RG_OK, RG_EINVAL, RG_ENOMEM, RG_EDEVICE, RG_EAGAIN, RG_ECORRUPT, RG_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
RG_METRIC_IP = 0
RG_STORE_FP32, RG_STORE_BF16, RG_STORE_FP8E4M3 = 0, 1, 2
RG_STAGE_PROJECTED, RG_STAGE_BIPARTITE = 1, 2
NONE = 0xFFFFFFFF
MAX_L = 512


class RGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"roargraph error {code}: {msg}")
        self.code = code


class rg_build_opts(ctypes.Structure):
    _fields_ = [("L_build", ctypes.c_int32), ("m_pj", ctypes.c_int32), ("m_ce", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("knn_slack", ctypes.c_int32), ("keep_stages", ctypes.c_int32)]


class rg_server_limits(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("hbm_pool_bytes", ctypes.c_int64),
                ("hops_per_step", ctypes.c_int32), ("max_L", ctypes.c_int32), ("hash_bits", ctypes.c_int32)]


class rg_result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("k", ctypes.c_int32), ("status", ctypes.c_int32),
                ("hops", ctypes.c_uint32), ("evals", ctypes.c_uint32),
                ("ids", ctypes.c_uint32 * MAX_L), ("dists", ctypes.c_float * MAX_L),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


_lib = None
P, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
PP = ctypes.POINTER(ctypes.c_void_p)
_SIGS = {
    "rg_build": (i32, [P, i64, i32, P, i64, i32, i32, i32, ctypes.POINTER(rg_build_opts), P, PP]),
    "rg_index_from_csr": (i32, [P, i64, i32, P, P, u32, i32, P, PP]),
    "rg_build_from_knn": (i32, [P, i64, i32, P, P, i64, i32, i32, ctypes.POINTER(rg_build_opts), PP]),
    "rg_index_graph": (i32, [P, PP, PP, ctypes.POINTER(i64), ctypes.POINTER(u32)]),
    "rg_index_stage_graph": (i32, [P, i32, PP, PP, ctypes.POINTER(i64), ctypes.POINTER(u32)]),
    "rg_index_bipartite": (i32, [P, PP, PP, ctypes.POINTER(i64), PP, PP, ctypes.POINTER(i64)]),
    "rg_insert": (i32, [P, P, i64, i32, P]),
    "rg_delete": (i32, [P, P, i64, P]),
    "rg_index_tombstones": (i32, [P, PP, ctypes.POINTER(i64)]),
    "rg_index_info": (i32, [P, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32),
                            ctypes.POINTER(i32), ctypes.POINTER(i64)]),
    "rg_index_set_storage": (i32, [P, i32, P]),
    "rg_search": (i32, [P, P, i64, i32, i32, P, P, P, P, P]),
    "rg_search_noalloc": (i32, [P, P, i64, i32, i32, P, P, P, P, P]),
    "rg_search_hashbits": (i32, [P, P, i64, i32, i32, P, P, P, P, i32, P]),
    "rg_knn": (i32, [P, i64, P, i64, i32, i32, P, P, P]),
    "rg_knn_candidates": (i32, [P, i64, P, i64, i32, i32, P, P, P]),
    "rg_knn_candidates_f16": (i32, [P, i64, P, i64, i32, i32, P, P, P]),
    "rg_knn_last_stats": (i32, [ctypes.POINTER(i64)] * 3),
    "rg_measure_peaks": (i32, [ctypes.POINTER(ctypes.c_double)] * 3 + [P]),
    "rg_index_build_stats": (i32, [P] + [ctypes.POINTER(ctypes.c_double)] * 4 + [ctypes.POINTER(i64)]),
    "rg_index_storage_ptrs": (i32, [P, PP, PP, PP, ctypes.POINTER(i32)]),
    "rg_save": (i32, [P, ctypes.c_char_p]),
    "rg_load": (i32, [ctypes.c_char_p, P, PP]),
    "rg_free": (None, [P]),
    "rg_device_copy": (i32, [P, P, i64, P]),
    "rg_last_error": (ctypes.c_char_p, []),
    "rg_server_create": (i32, [P, ctypes.POINTER(rg_server_limits), PP]),
    "rg_server_submit": (i32, [P, P, i32, i32, ctypes.c_uint64]),
    "rg_server_poll": (i32, [P, ctypes.POINTER(rg_result), i32, ctypes.POINTER(i32)]),
    "rg_server_submit_batch": (i32, [P, P, P, P, P, i32, ctypes.POINTER(i32)]),
    "rg_server_stats": (i32, [P] + [ctypes.POINTER(ctypes.c_uint64)] * 4),
    "rg_server_now": (ctypes.c_double, [P]),
    "rg_server_slots": (i32, [P]),
    "rg_server_destroy": (None, [P]),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def _check(rc):
    if rc != RG_OK:
        raise RGError(rc, lib().rg_last_error().decode(errors="replace"))


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f32(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.dim() == 2
            and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous 2-D float32 CUDA tensor")
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def as_u32(t) -> np.ndarray:
    """Device int32 tensor holding uint32 ids -> numpy uint32."""
    return t.cpu().numpy().view(np.uint32)


class Index:
    """Owns an rg_index handle."""

    def __init__(self, handle, keep=None, on_device=True):
        self.h = handle
        self._keep = keep
        self.on_device = on_device   # False: built on the host alone (rg_build_from_knn)

    def _st(self, stream):
        return _stream(stream) if self.on_device else ctypes.c_void_p(None)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:   # at interpreter exit the library may already be gone
            _lib.rg_free(h)
        self.h = None

    def graph(self):
        off, idx = ctypes.c_void_p(), ctypes.c_void_p()
        nnz, entry = i64(), u32()
        _check(lib().rg_index_graph(self.h, ctypes.byref(off), ctypes.byref(idx), ctypes.byref(nnz),
                                    ctypes.byref(entry)))
        n = self.info()["n"]
        o = np.ctypeslib.as_array(ctypes.cast(off, ctypes.POINTER(ctypes.c_int64)), (n + 1,)).copy()
        if nnz.value:
            x = np.ctypeslib.as_array(ctypes.cast(idx, ctypes.POINTER(ctypes.c_uint32)), (nnz.value,)).copy()
        else:
            x = np.zeros(0, np.uint32)
        return o, x, int(entry.value)

    def stage_graph(self, stage):
        """(offsets, indices, entry) copies of RG_STAGE_PROJECTED or RG_STAGE_BIPARTITE."""
        off, idx = ctypes.c_void_p(), ctypes.c_void_p()
        nnz, entry = i64(), u32()
        _check(lib().rg_index_stage_graph(self.h, int(stage), ctypes.byref(off), ctypes.byref(idx), ctypes.byref(nnz),
                                          ctypes.byref(entry)))
        n = self.info()["n"]
        o = np.ctypeslib.as_array(ctypes.cast(off, ctypes.POINTER(ctypes.c_int64)), (n + 1,)).copy()
        x = (np.ctypeslib.as_array(ctypes.cast(idx, ctypes.POINTER(ctypes.c_uint32)), (nnz.value,)).copy()
             if nnz.value else np.zeros(0, np.uint32))
        return o, x, int(entry.value)

    def bipartite(self):
        """(bridge_offsets, bridges, nout_offsets, nout) copies of G_bi (N_out lists include inserted rows)."""
        bo, bi, no, nx = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        nb, nt = i64(), i64()
        _check(lib().rg_index_bipartite(self.h, ctypes.byref(bo), ctypes.byref(bi), ctypes.byref(nb), ctypes.byref(no),
                                        ctypes.byref(nx), ctypes.byref(nt)))
        b_off = np.ctypeslib.as_array(ctypes.cast(bo, ctypes.POINTER(ctypes.c_int64)), (nb.value + 1,)).copy()
        b_idx = np.ctypeslib.as_array(ctypes.cast(bi, ctypes.POINTER(ctypes.c_uint32)), (nt.value,)).copy()
        n_off = np.ctypeslib.as_array(ctypes.cast(no, ctypes.POINTER(ctypes.c_int64)), (nt.value + 1,)).copy()
        nout = np.ctypeslib.as_array(ctypes.cast(nx, ctypes.POINTER(ctypes.c_uint32)), (int(n_off[-1]),)).copy()
        return b_off, b_idx, n_off, nout

    def insert(self, vectors, L=0, stream=None):
        """Insert host vectors (nv x d); returns their new ids."""
        V = np.ascontiguousarray(vectors, dtype=np.float32)
        n0 = self.info()["n"]
        _check(lib().rg_insert(self.h, V.ctypes.data_as(P), V.shape[0], int(L), self._st(stream)))
        return np.arange(n0, n0 + V.shape[0], dtype=np.uint32)

    def delete(self, ids, stream=None):
        a = np.ascontiguousarray(ids, dtype=np.uint32)
        _check(lib().rg_delete(self.h, a.ctypes.data_as(P), a.size, self._st(stream)))

    def tombstones(self):
        """(bitmap words copy or None, number deleted)."""
        b, c = ctypes.c_void_p(), i64()
        _check(lib().rg_index_tombstones(self.h, ctypes.byref(b), ctypes.byref(c)))
        if not b.value:
            return None, c.value
        n = self.info()["n"]
        return np.ctypeslib.as_array(ctypes.cast(b, ctypes.POINTER(ctypes.c_uint32)), ((n + 31) // 32,)).copy(), c.value

    def info(self):
        n, d, pitch, ell, b = i64(), i32(), i32(), i32(), i64()
        _check(lib().rg_index_info(self.h, ctypes.byref(n), ctypes.byref(d), ctypes.byref(pitch),
                                   ctypes.byref(ell), ctypes.byref(b)))
        return {"n": n.value, "d": d.value, "pitch": pitch.value, "ell": ell.value, "device_bytes": b.value}

    def build_stats(self):
        v = [ctypes.c_double() for _ in range(4)]
        r = i64()
        _check(lib().rg_index_build_stats(self.h, *[ctypes.byref(x) for x in v], ctypes.byref(r)))
        return {"t_knn": v[0].value, "t_project": v[1].value, "t_enhance": v[2].value,
                "t_total": v[3].value, "repairs": r.value}

    def storage_ptrs(self):
        b, f, s = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        p8 = i32()
        _check(lib().rg_index_storage_ptrs(self.h, ctypes.byref(b), ctypes.byref(f), ctypes.byref(s),
                                           ctypes.byref(p8)))
        return b.value, f.value, s.value, p8.value


def rg_build(base, train, Nq, M, L_build=0, m_pj=0, m_ce=0, threads=0, knn_slack=0, keep_stages=False,
             stream=None) -> Index:
    base, train = _dev_f32(base, "base"), _dev_f32(train, "train")
    o = rg_build_opts(L_build, m_pj, m_ce, threads, knn_slack, int(bool(keep_stages)))
    h = ctypes.c_void_p()
    _check(lib().rg_build(_ptr(base), base.shape[0], base.shape[1], _ptr(train), train.shape[0], int(Nq), int(M),
                          RG_METRIC_IP, ctypes.byref(o), _stream(stream), ctypes.byref(h)))
    return Index(h)


def rg_build_from_knn(base_host, knn_host, Nq, M, L_build=0, m_pj=0, m_ce=0, threads=0, keep_stages=False,
                      train_host=None) -> Index:
    """Host-only construction from precomputed kNN lists (numpy inputs)."""
    X = np.ascontiguousarray(base_host, dtype=np.float32)
    K = np.ascontiguousarray(knn_host, dtype=np.uint32)
    if K.ndim != 2 or K.shape[1] != Nq:
        raise ValueError("knn_host must be nt x Nq")
    Tp = None
    if train_host is not None:
        Tr = np.ascontiguousarray(train_host, dtype=np.float32)
        if Tr.shape != (K.shape[0], X.shape[1]):
            raise ValueError("train_host must be nt x d")
        Tp = Tr.ctypes.data_as(P)
    o = rg_build_opts(L_build, m_pj, m_ce, threads, 0, int(bool(keep_stages)))
    h = ctypes.c_void_p()
    _check(lib().rg_build_from_knn(X.ctypes.data_as(P), X.shape[0], X.shape[1], K.ctypes.data_as(P), Tp, K.shape[0],
                                   int(Nq), int(M), ctypes.byref(o), ctypes.byref(h)))
    return Index(h, on_device=False)


def rg_index_from_csr(base, offsets, indices, entry, stream=None) -> Index:
    base = _dev_f32(base, "base")
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(indices, dtype=np.uint32)
    if idx.size == 0:
        idx = np.zeros(1, np.uint32)
    h = ctypes.c_void_p()
    _check(lib().rg_index_from_csr(_ptr(base), base.shape[0], base.shape[1], off.ctypes.data_as(P),
                                   idx.ctypes.data_as(P), int(entry), RG_METRIC_IP, _stream(stream), ctypes.byref(h)))
    return Index(h)


def rg_index_set_storage(index: Index, storage: int, stream=None):
    _check(lib().rg_index_set_storage(index.h, int(storage), _stream(stream)))


def rg_search(index: Index, queries, k, L, stats=False, hash_bits=None, stream=None):
    """Returns (ids int32-as-uint32, dists float32[, hops, evals]) device tensors."""
    import torch
    queries = _dev_f32(queries, "queries")
    nq = queries.shape[0]
    dev = queries.device
    ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    ds = torch.empty((nq, k), dtype=torch.float32, device=dev)
    hops = torch.empty(nq, dtype=torch.int32, device=dev) if stats else None
    ev = torch.empty(nq, dtype=torch.int32, device=dev) if stats else None
    hp = _ptr(hops) if stats else None
    ep = _ptr(ev) if stats else None
    if hash_bits is None:
        _check(lib().rg_search(index.h, _ptr(queries), nq, int(k), int(L), _ptr(ids), _ptr(ds), hp, ep,
                               _stream(stream)))
    else:
        _check(lib().rg_search_hashbits(index.h, _ptr(queries), nq, int(k), int(L), _ptr(ids), _ptr(ds), hp, ep,
                                        int(hash_bits), _stream(stream)))
    return (ids, ds, hops, ev) if stats else (ids, ds)


def _out_buffers(queries, k, ids, ds, hops, ev):
    """The output tensors must hold what the search writes: nq x k ids
    (int32) and distances (float32), nq hops and evals (int32)."""
    import torch
    queries = _dev_f32(queries, "queries")
    nq = queries.shape[0]
    for t, name, dt, n in ((ids, "ids", torch.int32, nq * max(int(k), 0)),
                           (ds, "dists", torch.float32, nq * max(int(k), 0)),
                           (hops, "hops", torch.int32, nq), (ev, "evals", torch.int32, nq)):
        if t is None and name in ("hops", "evals"):
            continue
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()
                and t.numel() >= n):
            raise ValueError(f"{name} must be a contiguous {dt} CUDA tensor of at least {n} elements")
    return queries


def rg_search_into(index: Index, queries, k, L, ids, ds, hops=None, ev=None, stream=None):
    """rg_search writing into preallocated device tensors (no allocation)."""
    queries = _out_buffers(queries, k, ids, ds, hops, ev)
    _check(lib().rg_search(index.h, _ptr(queries), queries.shape[0], int(k), int(L), _ptr(ids), _ptr(ds),
                           _ptr(hops) if hops is not None else None, _ptr(ev) if ev is not None else None,
                           _stream(stream)))


def rg_search_noalloc_into(index: Index, queries, k, L, ids, ds, hops=None, ev=None, stream=None):
    """The allocation-free search into preallocated device tensors."""
    queries = _out_buffers(queries, k, ids, ds, hops, ev)
    _check(lib().rg_search_noalloc(index.h, _ptr(queries), queries.shape[0], int(k), int(L), _ptr(ids), _ptr(ds),
                                   _ptr(hops) if hops is not None else None,
                                   _ptr(ev) if ev is not None else None, _stream(stream)))


def rg_knn(queries, base, k, stream=None):
    import torch
    queries, base = _dev_f32(queries, "queries"), _dev_f32(base, "base")
    nq = queries.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
    ds = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
    _check(lib().rg_knn(_ptr(queries), nq, _ptr(base), base.shape[0], base.shape[1], int(k), _ptr(ids), _ptr(ds),
                        _stream(stream)))
    return ids, ds


def rg_knn_candidates(queries, base, K, stream=None):
    import torch
    queries, base = _dev_f32(queries, "queries"), _dev_f32(base, "base")
    nq = queries.shape[0]
    ids = torch.empty((nq, K), dtype=torch.int32, device=queries.device)
    sc = torch.empty((nq, K), dtype=torch.float32, device=queries.device)
    _check(lib().rg_knn_candidates(_ptr(queries), nq, _ptr(base), base.shape[0], base.shape[1], int(K), _ptr(ids),
                                   _ptr(sc), _stream(stream)))
    return ids, sc


def rg_knn_candidates_f16(queries, base, K, stream=None):
    import torch
    queries, base = _dev_f32(queries, "queries"), _dev_f32(base, "base")
    nq = queries.shape[0]
    ids = torch.empty((nq, K), dtype=torch.int32, device=queries.device)
    sc = torch.empty((nq, K), dtype=torch.float32, device=queries.device)
    _check(lib().rg_knn_candidates_f16(_ptr(queries), nq, _ptr(base), base.shape[0], base.shape[1], int(K),
                                       _ptr(ids), _ptr(sc), _stream(stream)))
    return ids, sc


def rg_knn_last_stats():
    """Rows of this thread's last kNN certified from FP16 candidates, from
    FP32 candidates and by the host scan."""
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().rg_knn_last_stats(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return {"f16": a.value, "f32": b.value, "host": c.value}


def rg_measure_peaks(stream=None):
    """Measured HBM read bandwidth (GB/s) and FP16 / FP32 MFMA throughput
    (TFLOP/s) of the current device."""
    v = [ctypes.c_double() for _ in range(3)]
    _check(lib().rg_measure_peaks(*[ctypes.byref(x) for x in v], _stream(stream)))
    return {"hbm_read_GBps": v[0].value, "mfma_f16_TFLOPs": v[1].value, "mfma_f32_TFLOPs": v[2].value}


def rg_device_copy(dst, src, stream=None):
    """Plain copy kernel of dst.numel()*itemsize bytes (traffic calibration)."""
    nbytes = src.numel() * src.element_size()
    _check(lib().rg_device_copy(_ptr(dst), _ptr(src), nbytes, _stream(stream)))


def rg_save(index: Index, path: str):
    _check(lib().rg_save(index.h, path.encode()))


def rg_load(path: str, stream=None) -> Index:
    h = ctypes.c_void_p()
    _check(lib().rg_load(path.encode(), _stream(stream), ctypes.byref(h)))
    return Index(h)


class Server:
    """Continuous-batching search server over an Index (rg_server_*)."""

    def __init__(self, index: Index, max_slots=0, hbm_pool_bytes=0, hops_per_step=32, max_L=512, hash_bits=0):
        self.index = index
        lim = rg_server_limits(max_slots, hbm_pool_bytes, hops_per_step, max_L, hash_bits)
        h = ctypes.c_void_p()
        _check(lib().rg_server_create(index.h, ctypes.byref(lim), ctypes.byref(h)))
        self.h = h
        self._buf = (rg_result * 1024)()

    def submit(self, q: np.ndarray, k: int, L: int, tag: int) -> int:
        q = np.ascontiguousarray(q, dtype=np.float32)
        rc = lib().rg_server_submit(self.h, q.ctypes.data_as(P), int(k), int(L), int(tag))
        if rc not in (RG_OK, RG_EAGAIN):
            _check(rc)
        return rc

    def submit_batch(self, Q: np.ndarray, k, L, tags) -> int:
        """Queue len(Q) requests; returns how many were accepted."""
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        k = np.ascontiguousarray(k, dtype=np.int32)
        L = np.ascontiguousarray(L, dtype=np.int32)
        t = np.ascontiguousarray(tags, dtype=np.uint64)
        acc = i32()
        rc = lib().rg_server_submit_batch(self.h, Q.ctypes.data_as(P), k.ctypes.data_as(P), L.ctypes.data_as(P),
                                          t.ctypes.data_as(P), len(Q), ctypes.byref(acc))
        if rc not in (RG_OK, RG_EAGAIN):
            _check(rc)
        return acc.value

    def poll(self):
        n = i32()
        _check(lib().rg_server_poll(self.h, self._buf, len(self._buf), ctypes.byref(n)))
        out = []
        for i in range(n.value):
            r = self._buf[i]
            k = r.k
            out.append({"tag": r.tag, "k": k, "status": r.status, "hops": r.hops, "evals": r.evals,
                        "ids": np.frombuffer(r.ids, dtype=np.uint32, count=k).copy(),
                        "dists": np.frombuffer(r.dists, dtype=np.float32, count=k).copy(),
                        "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done})
        return out

    def now(self) -> float:
        return lib().rg_server_now(self.h)

    def slots(self) -> int:
        return lib().rg_server_slots(self.h)

    def stats(self):
        v = [ctypes.c_uint64() for _ in range(4)]
        _check(lib().rg_server_stats(self.h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("submitted", "admitted", "completed", "steps"), (x.value for x in v)))

    def close(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.rg_server_destroy(h)
        self.h = None

    def __del__(self):
        self.close()
