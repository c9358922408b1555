"""GPU parity: every entry point of the C ABI against the FP64 oracle on the
same seeded inputs.  Run on an MI355X (-m gpu)."""
import os
import sys
import tempfile

import numpy as np
import pytest

import datagen
from parity import NONE, compare, oracle_explainer

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rg = pytest.importorskip("paper_2408_08933_amd")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rg.lib()
    return torch.device("cuda:0")


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


@pytest.fixture(scope="module")
def c1(oracle_lib):
    """Tiny OOD workload: d=64, 10k base, 10k training, 1k test; Nq=32, M=32."""
    g = datagen.Generator(1)
    X, Tr, Q = g.base(), g.train(), g.test()
    G = oracle_lib.Graph(X, Tr, 32, 32, 500)
    return X, Tr, Q, G


# ---------------------------------------------------------------------------
# kNN
# ---------------------------------------------------------------------------
# d = 33 and 95 leave a last coordinate slice of 1 and 31 (slices are 32 wide)
@pytest.mark.parametrize("nq,n,d,K", [(300, 3000, 64, 48), (257, 1999, 200, 40), (130, 700, 37, 33),
                                      (5, 128, 16, 128), (1000, 10000, 512, 112), (64, 2000, 33, 20),
                                      (70, 1500, 95, 30)])
def test_knn_candidates_are_fp32_topk(dev, nq, n, d, K):
    say(f"knn_candidates nq={nq} n={n} d={d} K={K}")
    rng = np.random.default_rng(nq + n + d)
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = rng.standard_normal((nq, d)).astype(np.float32)
    ids, sc = rg.rg_knn_candidates(T(Q, dev), T(X, dev), K)
    torch.cuda.synchronize()
    ids, sc = rg.as_u32(ids), sc.cpu().numpy().astype(np.float64)
    S = Q.astype(np.float64) @ X.astype(np.float64).T
    u = 2.0 ** -24
    tau = (d + 1) * u / (1 - (d + 1) * u) * np.linalg.norm(Q, axis=1)[:, None] * np.linalg.norm(X, axis=1).max()
    assert (ids < n).all()
    assert all(len(set(r.tolist())) == K for r in ids)
    got = np.take_along_axis(S, ids.astype(np.int64), axis=1)
    assert (np.abs(got - sc) <= tau).all()                    # each score is its pair's FP32 score
    assert (np.diff(sc, axis=1) <= 0).all()                     # descending
    kth_true = -np.sort(-S, axis=1)[:, K - 1]
    # anything left out scores no better than the K-th kept one (up to rounding)
    for q in range(nq):
        out = np.setdiff1d(np.arange(n), ids[q].astype(np.int64))
        assert (S[q, out] <= sc[q, K - 1] + 2 * tau[q, 0]).all()
        assert got[q].min() >= kth_true[q] - 2 * tau[q, 0]


def test_knn_certification_retries_on_ties(dev, oracle_lib):
    # 40 identical rows nearest to every query: the first candidate list
    # (k + 16 = 26) ends inside the tie, so certification fails and the rows
    # are retried with 52 candidates, which reach past it.  The exact answer
    # is the k lowest ids of the tied rows.
    rng = np.random.default_rng(11)
    n, d, k = 3000, 24, 10
    X = rng.standard_normal((n, d)).astype(np.float32) * 0.1
    v = rng.standard_normal(d).astype(np.float32)
    tied = np.sort(rng.choice(n, 40, replace=False))
    X[tied] = v
    Q = (v[None, :] + 0.01 * rng.standard_normal((50, d))).astype(np.float32)
    say("rg_knn with a 40-row tie, k=10")
    ids, ds = rg.rg_knn(T(Q, dev), T(X, dev), k)
    torch.cuda.synchronize()
    oi, od = oracle_lib.knn(X, Q, k)
    assert np.array_equal(rg.as_u32(ids), oi)
    assert (rg.as_u32(ids) == tied[:k]).all()
    assert np.array_equal(ds.cpu().numpy(), od.astype(np.float32))


def test_knn_tie_wider_than_any_candidate_list(dev, oracle_lib):
    # a tie of 300 rows cannot be certified with at most 256 candidates; the
    # rows are scanned in full on the host and the answer is still exact
    rng = np.random.default_rng(12)
    X = rng.standard_normal((2000, 16)).astype(np.float32) * 0.1
    X[:300] = 1.0
    Q = np.ones((4, 16), np.float32)
    say("rg_knn with a 300-row tie, k=10")
    ids, ds = rg.rg_knn(T(Q, dev), T(X, dev), 10)
    torch.cuda.synchronize()
    st = rg.rg_knn_last_stats()
    oi, od = oracle_lib.knn(X, Q, 10)
    assert np.array_equal(rg.as_u32(ids), oi) and (oi == np.arange(10)).all()
    assert np.array_equal(ds.cpu().numpy(), od.astype(np.float32))
    assert st == {"f16": 0, "f32": 0, "host": 4}


def _fp16_scores(Q, X):
    """Exact sums of the products of the FP16-rounded inputs (the FP16
    pass's scores before FP32 accumulation), and the sums of their
    magnitudes."""
    q = torch.from_numpy(Q).half().double().numpy()
    x = torch.from_numpy(X).half().double().numpy()
    return q @ x.T, np.abs(q) @ np.abs(x).T


# d = 16 and 200 are not multiples of 32 (zero padded); nq and n ragged
@pytest.mark.parametrize("nq,n,d,K", [(300, 3000, 64, 48), (257, 1999, 200, 40), (5, 128, 16, 128),
                                      (1000, 10000, 512, 200), (70, 1500, 95, 30)])
def test_knn_candidates_f16_are_fp16_topk(dev, nq, n, d, K):
    say(f"knn_candidates_f16 nq={nq} n={n} d={d} K={K}")
    rng = np.random.default_rng(nq + n + d + 1)
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = rng.standard_normal((nq, d)).astype(np.float32)
    ids, sc = rg.rg_knn_candidates_f16(T(Q, dev), T(X, dev), K)
    torch.cuda.synchronize()
    ids, sc = rg.as_u32(ids), sc.cpu().numpy().astype(np.float64)
    S16, A16 = _fp16_scores(Q, X)
    dp = (d + 31) // 32 * 32
    gacc = 2 * dp * 2.0 ** -24 / (1 - 2 * dp * 2.0 ** -24)   # FP32 accumulation, any order, truncating adds
    assert (ids < n).all()
    assert all(len(set(r.tolist())) == K for r in ids)
    got = np.take_along_axis(S16, ids.astype(np.int64), axis=1)
    tau = gacc * np.take_along_axis(A16, ids.astype(np.int64), axis=1)
    assert (np.abs(got - sc) <= tau).all()                   # each score is its pair's FP16-product sum
    assert (np.diff(sc, axis=1) <= 0).all()                  # descending
    for q in range(nq):
        out = np.setdiff1d(np.arange(n), ids[q].astype(np.int64))
        # nothing left out beats the K-th kept score beyond both roundings
        assert (S16[q, out] <= sc[q, K - 1] + gacc * (A16[q, out] + A16[q].max())).all()


@pytest.mark.parametrize("nq,k", [(1000, 10), (37, 100), (129, 1)])
def test_knn_exact_through_fp16_candidates(dev, oracle_lib, c1, nq, k):
    X, Tr, Q, G = c1
    Qs = np.concatenate([Q, Tr])[:nq]
    say(f"rg_knn (FP16 candidates) nq={nq} k={k}")
    ids, ds = rg.rg_knn(T(Qs, dev), T(X, dev), k)
    torch.cuda.synchronize()
    st = rg.rg_knn_last_stats()
    say(f"  certified rows: {st}")
    oi, od = oracle_lib.knn(X, Qs, k)
    assert np.array_equal(rg.as_u32(ids), oi)
    assert np.array_equal(ds.cpu().numpy(), od.astype(np.float32))
    assert st["f16"] + st["f32"] + st["host"] == nq and st["f16"] >= 0.99 * nq


def test_knn_values_beyond_fp16_range_use_fp32(dev, oracle_lib):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((3000, 32)).astype(np.float32)
    X[7, 3] = 1e5
    Q = rng.standard_normal((50, 32)).astype(np.float32)
    ids, ds = rg.rg_knn(T(Q, dev), T(X, dev), 10)
    torch.cuda.synchronize()
    st = rg.rg_knn_last_stats()
    oi, od = oracle_lib.knn(X, Q, 10)
    assert np.array_equal(rg.as_u32(ids), oi) and st["f16"] == 0 and st["f32"] == 50
    with pytest.raises(rg.RGError):
        rg.rg_knn_candidates_f16(T(Q, dev), T(X, dev), 10)


def test_knn_multi_launch_and_thin_last_wave(dev, oracle_lib):
    # 200k query rows: more query tiles than one launch takes (1,024) and a
    # last wave too thin to fill the device, which runs with the base split
    # across workgroups; both candidate kernels, sampled rows checked
    g = datagen.Generator(1, n=60_000, n_train=200_000, n_test=1)
    X, Tr = g.base(), g.train()
    say("rg_knn 200k x 60k x 64, k=32")
    ids, ds = rg.rg_knn(T(Tr, dev), T(X, dev), 32)
    torch.cuda.synchronize()
    st = rg.rg_knn_last_stats()
    say(f"  certified rows: {st}")
    assert st["f16"] + st["f32"] + st["host"] == len(Tr)
    pick = np.unique(np.concatenate([np.arange(0, len(Tr), 997), np.arange(len(Tr) - 300, len(Tr))]))
    oi, od = oracle_lib.knn(X, Tr[pick], 32)
    got = rg.as_u32(ids)[pick]
    assert np.array_equal(got, oi)
    assert np.array_equal(ds.cpu().numpy()[pick], od.astype(np.float32))
    say("rg_knn_candidates (FP32) 200k x 60k x 64, K=40")
    cid, csc = rg.rg_knn_candidates(T(Tr, dev), T(X, dev), 40)
    torch.cuda.synchronize()
    cid, csc = rg.as_u32(cid)[pick].astype(np.int64), csc.cpu().numpy()[pick].astype(np.float64)
    S = Tr[pick].astype(np.float64) @ X.astype(np.float64).T
    u = 2.0 ** -24
    tau = 65 * u / (1 - 65 * u) * np.linalg.norm(Tr[pick], axis=1)[:, None] * np.linalg.norm(X, axis=1).max()
    assert (np.abs(np.take_along_axis(S, cid, axis=1) - csc) <= tau).all()
    kth = -np.sort(-S, axis=1)[:, 39]
    assert (np.take_along_axis(S, cid, axis=1).min(axis=1) >= kth - 2 * tau[:, 0]).all()


def test_knn_rejects_bad_k(dev):
    X = torch.zeros((10, 4), device=dev)
    with pytest.raises(rg.RGError):
        rg.rg_knn(X, X, 11)


# ---------------------------------------------------------------------------
# search on the oracle's graph
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1_index(dev, c1):
    X, Tr, Q, G = c1
    return rg.rg_index_from_csr(T(X, dev), G.offsets, G.indices, G.entry)


@pytest.mark.parametrize("L", [16, 32, 64, 128])
def test_search_parity_c1(dev, oracle_lib, c1, c1_index, L):
    X, Tr, Q, G = c1
    say(f"search c1 k=10 L={L}")
    ids, ds, hops, ev = rg.rg_search(c1_index, T(Q, dev), 10, L, stats=True)
    torch.cuda.synchronize()
    oi, od, oh, oe, gaps = oracle_lib.search(X, G.offsets, G.indices, G.entry, Q, 10, L)
    # c1 runs on the persistent kernel's exact visited bitmap: a certified
    # query scores exactly the oracle's rows and expands as many nodes
    r = compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Q, X, label=f"c1 L={L}",
                gpu_evals=ev.cpu().numpy(), or_evals=oe, exact_visits=True,
                explain=oracle_explainer(oracle_lib, X, G.offsets, G.indices, G.entry, Q, 10, L))
    h = hops.cpu().numpy()
    sure = gaps > r["gamma"]
    assert sure.mean() >= 0.8, f"only {sure.mean():.2%} of queries certified"
    assert np.array_equal(h[sure], oh[sure].astype(np.int64))


def test_search_k_larger_than_L_and_ragged(dev, oracle_lib, c1, c1_index):
    X, Tr, Q, G = c1
    Qs = Q[:77]
    for k, L in ((100, 32), (1, 1), (7, 13), (512, 512)):
        say(f"search c1 ragged nq=77 k={k} L={L}")
        ids, ds = rg.rg_search(c1_index, T(Qs, dev), k, L)
        torch.cuda.synchronize()
        oi, od, _, _, gaps = oracle_lib.search(X, G.offsets, G.indices, G.entry, Qs, k, L)
        compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Qs, X, label=f"k={k} L={L}",
                explain=oracle_explainer(oracle_lib, X, G.offsets, G.indices, G.entry, Qs, k, L))


def test_visited_table_size_does_not_change_results(dev, c1, c1_index):
    X, Tr, Q, G = c1
    say("search c1 hash_bits 8 vs 15, L=128")
    a = rg.rg_search(c1_index, T(Q, dev), 10, 128, stats=True, hash_bits=8)
    b = rg.rg_search(c1_index, T(Q, dev), 10, 128, stats=True, hash_bits=15)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    assert (a[3] >= b[3]).all() and (a[3] > b[3]).any()   # the small table forgets and rescores


def test_search_repeatable(dev, c1, c1_index):
    X, Tr, Q, G = c1
    a = rg.rg_search(c1_index, T(Q, dev), 10, 64)
    b = rg.rg_search(c1_index, T(Q, dev), 10, 64)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_search_special_graphs(dev, oracle_lib):
    rng = np.random.default_rng(7)
    n, d = 120, 24
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = rng.standard_normal((33, d)).astype(np.float32)
    gt, gd = oracle_lib.knn(X, Q, 10)
    # complete graph (degree n-1 = 119 <= 128): exact for any L >= k
    rows = [np.array([j for j in range(n) if j != i], np.uint32) for i in range(n)]
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    ix = rg.rg_index_from_csr(T(X, dev), off, np.concatenate(rows), 5)
    for L in (10, 40):
        say(f"complete graph L={L}")
        ids, ds = rg.rg_search(ix, T(Q, dev), 10, L)
        torch.cuda.synchronize()
        assert np.array_equal(rg.as_u32(ids), gt)
    # random connected graph with L >= n: exact
    off2, idx2 = datagen.random_graph(n, 6, seed=3)
    ix2 = rg.rg_index_from_csr(T(X, dev), off2, idx2, 0)
    say("random graph L >= n")
    ids, ds = rg.rg_search(ix2, T(Q, dev), 10, 128)
    torch.cuda.synchronize()
    assert np.array_equal(rg.as_u32(ids), gt)
    # single node: padding
    ix3 = rg.rg_index_from_csr(T(X[:1], dev), np.zeros(2, np.int64), np.zeros(0, np.uint32), 0)
    ids, ds = rg.rg_search(ix3, T(Q[:3], dev), 4, 2)
    torch.cuda.synchronize()
    i3 = rg.as_u32(ids)
    assert (i3[:, 0] == 0).all() and (i3[:, 1:] == NONE).all() and torch.isinf(ds[:, 1:]).all()
    # zero queries is a no-op
    rg.rg_search(ix3, torch.zeros((0, d), device=dev), 4, 2)


def test_search_rejects_bad_args(dev, c1_index):
    q = torch.zeros((2, 64), device=dev)
    for k, L in ((0, 10), (10, 0), (1025, 10), (10, 1025)):
        with pytest.raises(rg.RGError):
            rg.rg_search(c1_index, q, k, L)


# Queues longer than 512 entries run in the long-queue kernels (twice the
# queue entries per lane in the merge and the rerank).  Both visited sets
# (the persistent kernel's exact bitmap, the LDS table) against the oracle,
# for every storage form, at L just above 512, at the 1024 maximum, and
# with k above 512; the two kernels return the same results.
@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp8"])
def test_long_queue_parity(dev, oracle_lib, c1, storage):
    X, Tr, Q, G = c1
    Qs = Q[:150]
    ix = rg.rg_index_from_csr(T(X, dev), G.offsets, G.indices, G.entry)
    Xq = None
    if storage != "fp32":
        rg.rg_index_set_storage(ix, rg.RG_STORE_BF16 if storage == "bf16" else rg.RG_STORE_FP8E4M3)
        Xq = oracle_lib.bf16(X) if storage == "bf16" else oracle_lib.quant_fp8(X)[2]
    nq = Qs.shape[0]
    for k, L in ((10, 513), (10, 1024), (700, 600), (1024, 1)):
        say(f"long queue {storage} k={k} L={L}")
        # exact bitmap: the persistent kernel
        ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
        ds = torch.empty((nq, k), dtype=torch.float32, device=dev)
        hops = torch.empty(nq, dtype=torch.int32, device=dev)
        ev = torch.empty(nq, dtype=torch.int32, device=dev)
        rg.rg_search_noalloc_into(ix, T(Qs, dev), k, L, ids, ds, hops, ev)
        # LDS tables of 2^8..2^10 entries: the table kernel, which forgets and
        # rescores; rg_search's own choice (for FP32 on this small graph, the
        # bitmap) returns the same results
        evs = {}
        for hb in (8, 9, 10):
            tids, tds, _, tev = rg.rg_search(ix, T(Qs, dev), k, L, stats=True, hash_bits=hb)
            torch.cuda.synchronize()
            assert torch.equal(ids, tids) and torch.equal(ds, tds), f"{storage} k={k} L={L} 2^{hb}: kernels differ"
            evs[hb] = tev
        dids, dds, _, d_ev = rg.rg_search(ix, T(Qs, dev), k, L, stats=True)
        torch.cuda.synchronize()
        assert torch.equal(ids, dids) and torch.equal(ds, dds), f"{storage} k={k} L={L}: default differs"
        if storage != "fp32":   # the LDS table, at one of the three sizes
            assert any(torch.equal(d_ev, e) for e in evs.values())
        if Xq is None:
            oi, od, oh, oe, gaps = oracle_lib.search(X, G.offsets, G.indices, G.entry, Qs, k, L)
            r = compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Qs, X, label=f"fp32 k={k} L={L}",
                        gpu_evals=ev.cpu().numpy(), or_evals=oe, exact_visits=True,
                        explain=oracle_explainer(oracle_lib, X, G.offsets, G.indices, G.entry, Qs, k, L))
            sure = gaps > r["gamma"]
            assert np.array_equal(hops.cpu().numpy()[sure], oh[sure].astype(np.int64))
        else:
            oi, od, _, _, gaps = oracle_lib.search_rerank(Xq, X, G.offsets, G.indices, G.entry, Qs, k, L)
            compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Qs, X, label=f"{storage} k={k} L={L}",
                    storage=storage,
                    explain=oracle_explainer(oracle_lib, X, G.offsets, G.indices, G.entry, Qs, k, L, Xq=Xq))


# ---------------------------------------------------------------------------
# build
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1_built(dev, c1):
    X, Tr, Q, G = c1
    say("rg_build c1 (10k x 64, Nq=32, M=32, L=500), stage graphs kept")
    return rg.rg_build(T(X, dev), T(Tr, dev), 32, 32, L_build=500, keep_stages=True)


def test_build_bit_exact_c1(c1, c1_built):
    X, Tr, Q, G = c1
    off, idx, entry = c1_built.graph()
    assert entry == G.entry
    assert np.array_equal(off, G.offsets) and np.array_equal(idx, G.indices)
    assert c1_built.build_stats()["repairs"] == G.repairs


def test_build_bit_exact_wide_lists(dev, oracle_lib):
    # M = 128 at d = 200: the enhancement selection keeps up to 63 rows per
    # node, more than fit in LDS, so the device reads them from HBM
    g = datagen.Generator(2, n=3000, n_train=3000, n_test=10, d=200)
    X, Tr = g.base(), g.train()
    say("rg_build 3000 x 200, Nq=48, M=128, L=200")
    ix = rg.rg_build(T(X, dev), T(Tr, dev), 48, 128, L_build=200)
    G = oracle_lib.Graph(X, Tr, 48, 128, 200)
    off, idx, entry = ix.graph()
    assert entry == G.entry and np.array_equal(off, G.offsets) and np.array_equal(idx, G.indices)


def test_build_bit_exact_three_enhancement_batches(dev, oracle_lib):
    # 70k rows: the device enhancement runs in batches of 32,768 nodes (three
    # here, the last one ragged) and the kNN in FP16 candidates over
    # 547 query tiles; the graph must equal the oracle's bit for bit
    g = datagen.Generator(1, n=70_000, n_train=70_000, n_test=1)
    X, Tr = g.base(), g.train()
    say("oracle build 70k x 64, Nq=32, M=32, L=200")
    G = oracle_lib.Graph(X, Tr, 32, 32, 200)
    say("rg_build 70k x 64")
    ix = rg.rg_build(T(X, dev), T(Tr, dev), 32, 32, L_build=200)
    st = rg.rg_knn_last_stats()
    say(f"  kNN rows certified: {st}")
    off, idx, entry = ix.graph()
    assert entry == G.entry
    assert np.array_equal(off, G.offsets) and np.array_equal(idx, G.indices)
    assert ix.build_stats()["repairs"] == G.repairs


def test_build_stage_graphs_c1(oracle_lib, c1, c1_built):
    X, Tr, Q, G = c1
    b_off, b_idx, n_off, nout = c1_built.bipartite()
    assert np.array_equal(b_off, G.b_offsets) and np.array_equal(b_idx, G.b_indices)
    assert np.array_equal(nout.reshape(G.nout.shape), G.nout) and n_off[-1] == G.nout.size
    off, idx, entry = c1_built.stage_graph(rg.RG_STAGE_PROJECTED)
    assert np.array_equal(off, G.pj_offsets) and entry == G.entry
    assert np.array_equal(idx, np.concatenate([np.sort(r) for r in G.rows("pj")]))
    ro, ri = oracle_lib.bipartite_routing(G.b_offsets, G.b_indices, G.nout)
    off, idx, entry = c1_built.stage_graph(rg.RG_STAGE_BIPARTITE)
    assert np.array_equal(off, ro) and np.array_equal(idx, ri)
    assert entry == oracle_lib.medoid(X, mask=np.diff(G.b_offsets) > 0)


@pytest.mark.parametrize("stage", ["projected", "bipartite"])
def test_search_stage_graph_parity(dev, oracle_lib, c1, stage):
    # the ablation's graphs (Sec. 5.4): G_pj and routing on G_bi through
    # query nodes; G_bi rows are |B(x)| * (Nq - 1) long, past the ELL width
    X, Tr, Q, G = c1
    if stage == "projected":
        off, idx, entry = G.pj_offsets, G.pj_indices, G.entry
    else:
        off, idx = oracle_lib.bipartite_routing(G.b_offsets, G.b_indices, G.nout)
        entry = oracle_lib.medoid(X, mask=np.diff(G.b_offsets) > 0)
    ix = rg.rg_index_from_csr(T(X, dev), off, idx, entry)
    if stage == "bipartite":
        assert np.diff(off).max() > 128 and ix.info()["ell"] == 0   # held and searched as CSR
    for k, L in ((10, 32), (10, 128), (100, 100)):
        say(f"search on {stage} graph k={k} L={L}")
        ids, ds = rg.rg_search(ix, T(Q, dev), k, L)
        torch.cuda.synchronize()
        oi, od, _, _, gaps = oracle_lib.search(X, off, idx, entry, Q, k, L)
        compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Q, X, label=f"{stage} k={k} L={L}",
                explain=oracle_explainer(oracle_lib, X, off, idx, entry, Q, k, L))


def test_search_wide_csr_rows(dev, oracle_lib):
    # rows of 200..700 neighbours (several 128-id chunks, ragged last chunk):
    # every entry point that searches (persistent, LDS table, serving)
    rng = np.random.default_rng(21)
    n, d = 3000, 40
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = rng.standard_normal((150, d)).astype(np.float32)
    deg = rng.integers(200, 701, n)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(deg)
    idx = np.concatenate([rng.choice(n, int(g), replace=False) for g in deg]).astype(np.uint32)
    ix = rg.rg_index_from_csr(T(X, dev), off, idx, 17)
    assert ix.info()["ell"] == 0
    for k, L in ((10, 20), (10, 64), (50, 200)):
        say(f"wide csr k={k} L={L}")
        ids, ds, hops, ev = rg.rg_search(ix, T(Q, dev), k, L, stats=True)
        torch.cuda.synchronize()
        oi, od, oh, oe, gaps = oracle_lib.search(X, off, idx, 17, Q, k, L)
        compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Q, X, label=f"wide k={k} L={L}",
                gpu_evals=ev.cpu().numpy(), or_evals=oe, exact_visits=True,
                explain=oracle_explainer(oracle_lib, X, off, idx, 17, Q, k, L))
        b = rg.rg_search(ix, T(Q, dev), k, L, stats=True, hash_bits=9)
        torch.cuda.synchronize()
        assert torch.equal(b[0], ids) and torch.equal(b[1], ds) and torch.equal(b[2], hops)
    # serving on the same index gives each request's rg_search result
    srv = rg.Server(ix, max_slots=64, hops_per_step=8)
    for i in range(40):
        assert srv.submit(Q[i], 10, 64, i) == rg.RG_OK
    got = {}
    import time
    t0 = time.time()
    while len(got) < 40 and time.time() - t0 < 60:
        for r in srv.poll():
            got[r["tag"]] = r
        time.sleep(0.001)
    srv.close()
    assert len(got) == 40
    ids, ds = rg.rg_search(ix, T(Q[:40], dev), 10, 64)
    torch.cuda.synchronize()
    a = rg.as_u32(ids)
    for i in range(40):
        assert np.array_equal(got[i]["ids"], a[i])


def test_recall_on_built_index(dev, oracle_lib, c1, c1_built):
    X, Tr, Q, G = c1
    gt, _ = oracle_lib.knn(X, Q, 10)
    rec = []
    for L in (16, 32, 64, 128):
        ids, _ = rg.rg_search(c1_built, T(Q, dev), 10, L)
        torch.cuda.synchronize()
        rec.append(oracle_lib.recall(rg.as_u32(ids), gt, 10))
    say(f"recall@10 over L=16..128: {rec}")
    assert rec[-1] >= 0.9 and rec[0] < rec[-1]


def test_save_load_roundtrip(dev, c1, c1_built):
    X, Tr, Q, G = c1
    with tempfile.TemporaryDirectory() as td:
        p = os.path.join(td, "c1.rgidx")
        rg.rg_save(c1_built, p)
        ix = rg.rg_load(p)
        a, b = c1_built.graph(), ix.graph()
        assert all(np.array_equal(x, y) for x, y in zip(a[:2], b[:2])) and a[2] == b[2]
        r1 = rg.rg_search(c1_built, T(Q[:50], dev), 10, 32)
        r2 = rg.rg_search(ix, T(Q[:50], dev), 10, 32)
        torch.cuda.synchronize()
        assert torch.equal(r1[0], r2[0]) and torch.equal(r1[1], r2[1])
        raw = bytearray(open(p, "rb").read())
        raw[100] ^= 0x40
        open(p, "wb").write(bytes(raw))
        with pytest.raises(rg.RGError) as e:
            rg.rg_load(p)
        assert e.value.code == rg.RG_ECORRUPT


def test_save_load_several_chunks(dev):
    # rg_save copies the padded device rows back 16,384 at a time: 40,000
    # rows of d = 72 (pitch 80) take three copies, the last one ragged.  The
    # loaded index must answer every query exactly as the saved one.
    n, d = 40_000, 72
    rng = np.random.default_rng(17)
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = rng.standard_normal((64, d)).astype(np.float32)
    off, idx = datagen.random_graph_fast(n, 16, seed=5)
    ix = rg.rg_index_from_csr(T(X, dev), off, idx, 0)
    with tempfile.TemporaryDirectory() as td:
        p = os.path.join(td, "r.rgidx")
        rg.rg_save(ix, p)
        ix2 = rg.rg_load(p)
    a, b = ix.graph(), ix2.graph()
    assert all(np.array_equal(x, y) for x, y in zip(a[:2], b[:2])) and a[2] == b[2]
    r1 = rg.rg_search(ix, T(Q, dev), 10, 200)
    r2 = rg.rg_search(ix2, T(Q, dev), 10, 200)
    torch.cuda.synchronize()
    assert torch.equal(r1[0], r2[0]) and torch.equal(r1[1], r2[1])
    # the distances the loaded index returns are those of the original rows
    # (rows from every copy chunk come back)
    ids = rg.as_u32(r2[0])
    assert ids.max() >= 2 * 16384
    got = r2[1].cpu().numpy().astype(np.float64)
    for q in range(len(Q)):
        want = -(X[ids[q]].astype(np.float64) @ Q[q].astype(np.float64))
        assert np.allclose(got[q], want, rtol=0, atol=1e-4)


# ---------------------------------------------------------------------------
# reduced-precision storage
# ---------------------------------------------------------------------------
def test_quantized_rows_match_oracle(dev, oracle_lib, c1):
    X, Tr, Q, G = c1
    ix = rg.rg_index_from_csr(T(X, dev), G.offsets, G.indices, G.entry)
    rg.rg_index_set_storage(ix, rg.RG_STORE_BF16)
    rg.rg_index_set_storage(ix, rg.RG_STORE_FP8E4M3)
    pb, pf, ps, p8 = ix.storage_ptrs()
    info = ix.info()
    n, d, pitch = info["n"], info["d"], info["pitch"]
    bits = torch.empty((n, pitch), dtype=torch.int16, device=dev)
    codes = torch.empty((n, p8), dtype=torch.uint8, device=dev)
    scales = torch.empty(n, dtype=torch.float32, device=dev)
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    for dst, src, nb in ((bits, pb, n * pitch * 2), (codes, pf, n * p8), (scales, ps, n * 4)):
        assert hip.hipMemcpy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src), ctypes.c_size_t(nb), 3) == 0
    torch.cuda.synchronize()
    b16 = (bits.cpu().numpy()[:, :d].astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
    assert np.array_equal(b16, oracle_lib.bf16(X))
    oc, os_, _ = oracle_lib.quant_fp8(X)
    c = codes.cpu().numpy()
    assert np.array_equal(c[:, :d], oc)
    assert np.array_equal(scales.cpu().numpy(), os_)
    # each E4M3 row carries its scale after the codes (4-byte aligned); the
    # rest of the row is zero
    s_off = (d + 3) // 4 * 4
    assert p8 == ((s_off + 4 + 15) // 16 * 16 + 127) // 128 * 128
    assert np.array_equal(c[:, s_off:s_off + 4].copy().view(np.float32)[:, 0], os_)
    assert not c[:, d:s_off].any() and not c[:, s_off + 4:].any()


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
def test_precision_search_parity(dev, oracle_lib, c1, storage):
    X, Tr, Q, G = c1
    ix = rg.rg_index_from_csr(T(X, dev), G.offsets, G.indices, G.entry)
    st = rg.RG_STORE_BF16 if storage == "bf16" else rg.RG_STORE_FP8E4M3
    rg.rg_index_set_storage(ix, st)
    Xq = oracle_lib.bf16(X) if storage == "bf16" else oracle_lib.quant_fp8(X)[2]
    for k, L in ((10, 64), (100, 128)):
        say(f"precision {storage} k={k} L={L}")
        ids, ds = rg.rg_search(ix, T(Q, dev), k, L)
        torch.cuda.synchronize()
        oi, od, _, _, gaps = oracle_lib.search_rerank(Xq, X, G.offsets, G.indices, G.entry, Q, k, L)
        compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Q, X, label=f"{storage} k={k} L={L}",
                storage=storage,
                explain=oracle_explainer(oracle_lib, X, G.offsets, G.indices, G.entry, Q, k, L, Xq=Xq))


def test_fp32_search_on_the_lds_table_path(dev, oracle_lib):
    # n/8 bytes of bitmap per query (2,500) above 5% of the expected row
    # bytes (40 L rows of 4d bytes: 1,280 at d = 16, L = 10): rg_search runs
    # FP32 rows on the LDS-table kernel; same results as the exact 2^15
    # table, and the oracle's within the FP32 tolerance
    rng = np.random.default_rng(21)
    n, d = 20000, 16
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = rng.standard_normal((80, d)).astype(np.float32)
    off, idx = datagen.random_graph(n, 100, seed=21)
    ix = rg.rg_index_from_csr(T(X, dev), off, idx, 0)
    say("fp32 LDS-table path n=20000 d=16 degree 100 k=10 L=10")
    a = rg.rg_search(ix, T(Q, dev), 10, 10, stats=True)
    b = rg.rg_search(ix, T(Q, dev), 10, 10, stats=True, hash_bits=15)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    # ~100 new rows per expansion overflow the 2^10 table, which forgets and
    # rescores: only the LDS-table kernel counts more evaluations
    assert (a[3] >= b[3]).all() and (a[3] > b[3]).any()
    oi, od, _, _, gaps = oracle_lib.search(X, off, idx, 0, Q, 10, 10)
    compare(rg.as_u32(a[0]), a[1].cpu().numpy(), oi, od, gaps, Q, X, label="fp32 LDS-table path",
            explain=oracle_explainer(oracle_lib, X, off, idx, 0, Q, 10, 10))


@pytest.mark.parametrize("d", [7, 37, 129, 255, 700, 1024])
def test_search_every_dimension_class(dev, oracle_lib, d):
    # odd d, d just past a class limit, and the largest class, for all three
    # storage forms (each form reads its rows in its own chunk shape)
    rng = np.random.default_rng(d)
    n = 3000
    X = (rng.standard_normal((n, d)) * rng.uniform(0.2, 2.0, d)).astype(np.float32)
    Q = rng.standard_normal((60, d)).astype(np.float32)
    off, idx = datagen.random_graph(n, 12, seed=d)
    ix = rg.rg_index_from_csr(T(X, dev), off, idx, 3)
    for storage, st in (("fp32", rg.RG_STORE_FP32), ("bf16", rg.RG_STORE_BF16), ("fp8", rg.RG_STORE_FP8E4M3)):
        rg.rg_index_set_storage(ix, st)
        say(f"d={d} {storage} k=10 L=48")
        ids, ds = rg.rg_search(ix, T(Q, dev), 10, 48)
        torch.cuda.synchronize()
        Xq = None
        if storage == "fp32":
            oi, od, _, _, gaps = oracle_lib.search(X, off, idx, 3, Q, 10, 48)
        else:
            Xq = oracle_lib.bf16(X) if storage == "bf16" else oracle_lib.quant_fp8(X)[2]
            oi, od, _, _, gaps = oracle_lib.search_rerank(Xq, X, off, idx, 3, Q, 10, 48)
        compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Q, X, label=f"d={d} {storage}", storage=storage,
                explain=oracle_explainer(oracle_lib, X, off, idx, 3, Q, 10, 48, Xq=Xq))


# ---------------------------------------------------------------------------
# full-size shape: 1M x 200 rows on a random graph, sampled queries
# ---------------------------------------------------------------------------
def test_full_size_sampled(dev, oracle_lib):
    g = datagen.Generator(2, n=1_000_000, n_train=1, n_test=48)
    say("full size: generating 1M x 200 base and a degree-48 random graph")
    X, Q = g.base(), g.test()
    off, idx = datagen.random_graph_fast(X.shape[0], 48, seed=5)
    ix = rg.rg_index_from_csr(T(X, dev), off, idx, 0)
    for k, L in ((10, 64), (10, 200)):
        say(f"full size search k={k} L={L}")
        ids, ds, hops, ev = rg.rg_search(ix, T(Q, dev), k, L, stats=True)
        torch.cuda.synchronize()
        oi, od, oh, oe, gaps = oracle_lib.search(X, off, idx, 0, Q, k, L)
        # rg_search keeps the exact bitmap while n/8 bytes stay under 5% of
        # 40 L rows of 4d bytes (L = 200 here); at L = 64 it takes the LDS
        # table, which may rescore forgotten rows
        bitmap = X.shape[0] / 8 <= 0.05 * 40 * max(L, k) * 4 * X.shape[1]
        compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Q, X, label=f"1M L={L}",
                gpu_evals=ev.cpu().numpy(), or_evals=oe, exact_visits=bitmap,
                explain=oracle_explainer(oracle_lib, X, off, idx, 0, Q, k, L))
