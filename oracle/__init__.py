"""Python view of the RoarGraph oracle (TEST INFRASTRUCTURE ONLY).

The oracle is plain C in FP64 (roar_oracle.c).  Only tests, the smoke check
and the benchmark's CPU-baseline leg may import this module; the library
under paper_2408_08933_amd never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "roar_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NONE = 0xFFFFFFFF

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-shared", "-fPIC", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, u32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    sig = {
        "or_dist": (f64, [P, P, i32]),
        "or_knn": (None, [P, i64, i32, P, i64, i32, P, P]),
        "or_medoid": (u32, [P, i64, i32]),
        "or_medoid_masked": (u32, [P, i64, i32, P]),
        "or_acquire": (i32, [P, i32, u32, P, i32, i32, i32, P]),
        "or_search": (None, [P, i64, i32, P, P, u32, P, i64, i32, i32, P, P, P, P, P]),
        "or_search_rerank": (None, [P, P, i64, i32, P, P, u32, P, i64, i32, i32, P, P, P, P, P]),
        "or_search_perturbed": (None, [P, i64, i32, P, P, u32, P, i64, i32, i32, f64, ctypes.c_uint64, P, P, P, P]),
        "or_search_rerank_perturbed": (None, [P, P, i64, i32, P, P, u32, P, i64, i32, i32, f64, ctypes.c_uint64,
                                              P, P, P, P]),
        "or_bf16": (ctypes.c_float, [ctypes.c_float]),
        "or_quant_bf16": (None, [P, i64, P]),
        "or_e4m3_value": (f64, [ctypes.c_uint8]),
        "or_e4m3_encode": (ctypes.c_uint8, [f64]),
        "or_quant_fp8": (None, [P, i64, i32, P, P, P]),
        "or_recall": (f64, [P, i32, P, i32, i64, i32]),
        "or_build": (P, [P, i64, i32, P, i64, i32, i32, i32, i32, i32]),
        "or_repair": (i64, [i64, i32, u32, P, P, P, P, i64]),
        "or_set_threads": (None, [i32]),
        "or_graph_n": (i64, [P]),
        "or_graph_entry": (u32, [P]),
        "or_graph_repairs": (i64, [P]),
        "or_graph_ok": (ctypes.c_int, [P]),
        "or_graph_off": (P, [P, ctypes.c_int]),
        "or_graph_idx": (P, [P, ctypes.c_int]),
        "or_graph_pivot": (P, [P]),
        "or_graph_nout": (P, [P]),
        "or_graph_cx": (P, [P]),
        "or_graph_cx_n": (P, [P]),
        "or_graph_free": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def dist(a, b) -> float:
    a, b = _f32(a), _f32(b)
    return _load().or_dist(_p(a), _p(b), a.shape[-1])


def knn(X, Q, k):
    """Exact k nearest base rows of every query in (delta, id) order."""
    X, Q = _f32(X), _f32(Q)
    nq = Q.shape[0]
    ids = np.empty((nq, k), np.uint32)
    ds = np.empty((nq, k), np.float64)
    _load().or_knn(_p(X), X.shape[0], X.shape[1], _p(Q), nq, k, _p(ids), _p(ds))
    return ids, ds


def medoid(X, mask=None) -> int:
    """Row nearest (L2) to the mean of all rows; with a mask, among the
    masked rows only (all rows if none is masked); lower id on ties."""
    X = _f32(X)
    if mask is None:
        return int(_load().or_medoid(_p(X), X.shape[0], X.shape[1]))
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    if not m.any():
        return int(_load().or_medoid(_p(X), X.shape[0], X.shape[1]))
    return int(_load().or_medoid_masked(_p(X), X.shape[0], X.shape[1], _p(m)))


def bipartite_routing(b_offsets, b_indices, nout):
    """Greedy routing on the query-base bipartite graph G_bi (Sec. 4.2.1):
    from base node x to the query nodes x links to (the queries whose pivot
    is x, ascending), then to those queries' base out-neighbours N_out(t).
    Returns CSR rows over base nodes: row x = N_out(t) for each bridge t of x,
    concatenated; a search visits a repeated node once.  Plain loop."""
    n = len(b_offsets) - 1
    off = np.zeros(n + 1, np.int64)
    rows = []
    for x in range(n):
        r = [np.asarray(nout[int(t)], np.uint32) for t in b_indices[b_offsets[x]:b_offsets[x + 1]]]
        r = np.concatenate(r) if r else np.zeros(0, np.uint32)
        rows.append(r)
        off[x + 1] = off[x] + len(r)
    idx = np.concatenate(rows) if off[-1] else np.zeros(0, np.uint32)
    return off, idx.astype(np.uint32)


def acquire(X, x, C, m, fill):
    X = _f32(X)
    C = np.ascontiguousarray(C, dtype=np.uint32)
    res = np.empty(max(m, 1), np.uint32)
    n = _load().or_acquire(_p(X), X.shape[1], int(x), _p(C), len(C), int(m), int(fill), _p(res))
    return res[:n].copy()


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops (0: the default)."""
    _load().or_set_threads(int(n))


def search(X, offsets, indices, entry, Q, k, L, with_stats=True, with_margins=True):
    """Beam search; returns ids, FP64 distances, hops, evals and each query's
    decision margin: the smallest (delta_b - delta_a) / (S_a + S_b), with
    S = sum_i |q_i x_i|, over the pairs whose order decides the search."""
    X, Q = _f32(X), _f32(Q)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(indices, dtype=np.uint32)
    if idx.size == 0:
        idx = np.zeros(1, np.uint32)
    nq = Q.shape[0]
    ids = np.empty((nq, k), np.uint32)
    ds = np.empty((nq, k), np.float64)
    hops = np.empty(nq, np.uint32)
    ev = np.empty(nq, np.uint32)
    gaps = np.full(nq, np.nan)
    _load().or_search(_p(X), X.shape[0], X.shape[1], _p(off), _p(idx), int(entry), _p(Q), nq,
                      int(k), int(L), _p(ids), _p(ds), _p(hops), _p(ev), _p(gaps) if with_margins else None)
    return ids, ds, hops, ev, gaps


def search_rerank(Xq, X, offsets, indices, entry, Q, k, L):
    """Search over reduced-precision rows Xq, rerank the final queue on X."""
    Xq, X, Q = _f32(Xq), _f32(X), _f32(Q)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(indices, dtype=np.uint32)
    nq = Q.shape[0]
    ids = np.empty((nq, k), np.uint32)
    ds = np.empty((nq, k), np.float64)
    hops = np.empty(nq, np.uint32)
    ev = np.empty(nq, np.uint32)
    gaps = np.empty(nq, np.float64)
    _load().or_search_rerank(_p(Xq), _p(X), X.shape[0], X.shape[1], _p(off), _p(idx), int(entry),
                             _p(Q), nq, int(k), int(L), _p(ids), _p(ds), _p(hops), _p(ev), _p(gaps))
    return ids, ds, hops, ev, gaps


def repair(rows, M, entry, cand):
    """Reachability repair of a graph given as lists of out-neighbours, with
    each node's enhancement candidates `cand` (lists); returns the repaired
    rows (sorted by id, repair edges appended) and the number of edges added."""
    n = len(rows)
    a = np.zeros((n, M), np.uint32)
    deg = np.zeros(n, np.int32)
    for x, r in enumerate(rows):
        assert len(r) <= M
        a[x, :len(r)] = r
        deg[x] = len(r)
    stride = max(1, max((len(c) for c in cand), default=1))
    cx = np.zeros((n, stride), np.uint32)
    cn = np.zeros(n, np.int32)
    for x, c in enumerate(cand):
        cx[x, :len(c)] = c
        cn[x] = len(c)
    added = _load().or_repair(n, int(M), int(entry), _p(a), _p(deg), _p(cx), _p(cn), stride)
    if added < 0:
        raise RuntimeError("repair: no reached node has a free slot")
    return [a[x, :deg[x]].tolist() for x in range(n)], int(added)


def search_perturbed(X, offsets, indices, entry, Q, k, L, eps, seed, Xq=None):
    """The search (or, with Xq, the search over Xq and the rerank on X) with
    every distance moved by eps * sign * S(q, x), sign in {-1, 0, +1} drawn
    per node from the seed; returns ids, distances, hops, evals."""
    X, Q = _f32(X), _f32(Q)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(indices, dtype=np.uint32)
    if idx.size == 0:
        idx = np.zeros(1, np.uint32)
    nq = Q.shape[0]
    ids = np.empty((nq, k), np.uint32)
    ds = np.empty((nq, k), np.float64)
    hops = np.empty(nq, np.uint32)
    ev = np.empty(nq, np.uint32)
    if Xq is None:
        _load().or_search_perturbed(_p(X), X.shape[0], X.shape[1], _p(off), _p(idx), int(entry), _p(Q), nq,
                                    int(k), int(L), float(eps), int(seed), _p(ids), _p(ds), _p(hops), _p(ev))
    else:
        Xq = _f32(Xq)
        _load().or_search_rerank_perturbed(_p(Xq), _p(X), X.shape[0], X.shape[1], _p(off), _p(idx), int(entry),
                                           _p(Q), nq, int(k), int(L), float(eps), int(seed), _p(ids), _p(ds),
                                           _p(hops), _p(ev))
    return ids, ds, hops, ev


def bf16(x):
    x = _f32(x)
    out = np.empty_like(x)
    _load().or_quant_bf16(_p(x), x.size, _p(out))
    return out


def e4m3_value(code: int) -> float:
    return _load().or_e4m3_value(int(code))


def e4m3_encode(y: float) -> int:
    return int(_load().or_e4m3_encode(float(y)))


def quant_fp8(X):
    X = _f32(X)
    n, d = X.shape
    codes = np.empty((n, d), np.uint8)
    scales = np.empty(n, np.float32)
    deq = np.empty((n, d), np.float32)
    _load().or_quant_fp8(_p(X), n, d, _p(codes), _p(scales), _p(deq))
    return codes, scales, deq


def recall(res_ids, gt_ids, k):
    r = np.ascontiguousarray(res_ids, dtype=np.uint32)
    g = np.ascontiguousarray(gt_ids, dtype=np.uint32)
    return _load().or_recall(_p(r), r.shape[1], _p(g), g.shape[1], r.shape[0], int(k))


class Graph:
    """Result of the oracle's index construction, copied out of C memory."""

    def __init__(self, X, T, Nq, M, L=500, m_pj=0, m_ce=0):
        X, T = _f32(X), _f32(T)
        lib = _load()
        n, d = X.shape
        h = lib.or_build(_p(X), n, d, _p(T), T.shape[0], int(Nq), int(M), int(L), int(m_pj), int(m_ce))
        if not h:
            raise ValueError("oracle build rejected its arguments")
        try:
            if not lib.or_graph_ok(h):
                raise RuntimeError("oracle build: reachability repair found no free slot")
            self.n, self.d, self.Nq, self.M, self.L = n, d, Nq, M, L
            self.entry = int(lib.or_graph_entry(h))
            self.repairs = int(lib.or_graph_repairs(h))

            def csr(which, nrows):
                off = np.ctypeslib.as_array(ctypes.cast(lib.or_graph_off(h, which),
                                                        ctypes.POINTER(ctypes.c_int64)), (nrows + 1,)).copy()
                nnz = int(off[-1])
                idx = np.ctypeslib.as_array(ctypes.cast(lib.or_graph_idx(h, which),
                                                        ctypes.POINTER(ctypes.c_uint32)), (max(nnz, 1),))[:nnz].copy()
                return off, idx

            self.offsets, self.indices = csr(0, n)
            self.pj_offsets, self.pj_indices = csr(1, n)
            self.ce_offsets, self.ce_indices = csr(2, n)
            self.b_offsets, self.b_indices = csr(3, n)
            nt = T.shape[0]
            self.pivot = np.ctypeslib.as_array(ctypes.cast(lib.or_graph_pivot(h), ctypes.POINTER(ctypes.c_uint32)), (nt,)).copy()
            self.nout = np.ctypeslib.as_array(ctypes.cast(lib.or_graph_nout(h), ctypes.POINTER(ctypes.c_uint32)), (nt * (Nq - 1),)).copy().reshape(nt, Nq - 1)
            self.cx_n = np.ctypeslib.as_array(ctypes.cast(lib.or_graph_cx_n(h), ctypes.POINTER(ctypes.c_int32)), (n,)).copy()
            self.cx = np.ctypeslib.as_array(ctypes.cast(lib.or_graph_cx(h), ctypes.POINTER(ctypes.c_uint32)), (n * L,)).copy().reshape(n, L)
        finally:
            lib.or_graph_free(h)

    def rows(self, which="final"):
        off, idx = {"final": (self.offsets, self.indices), "pj": (self.pj_offsets, self.pj_indices),
                    "ce": (self.ce_offsets, self.ce_indices)}[which]
        return [idx[off[i]:off[i + 1]] for i in range(self.n)]
