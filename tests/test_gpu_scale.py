"""Full-size shapes of the other workloads, on seeded random graphs (the
oracle cannot build indexes this large in a test): CLIP-like 2M x 512 with
BF16 storage, 10M x 200 FP32, and 8M x 512 with FP8-E4M3 storage.  Sampled
queries are compared with the oracle's search on the same graph.  At 8M x 512
the FP8 case checks properties that hold at any size (codes of sampled rows,
exact FP32 rerank distances); its oracle parity runs at 500k x 512."""
import sys

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


def test_clip_like_2m_d512_bf16(dev, oracle_lib):
    g = datagen.Generator(3, n=2_000_000, n_train=1, n_test=24)
    say("clip-like: 2M x 512 base, degree-48 random graph")
    X, Q = g.base(), g.test()
    off, idx = datagen.random_graph_fast(X.shape[0], 48, seed=31)
    ix = rg.rg_index_from_csr(torch.from_numpy(X).to(dev), off, idx, 0)
    rg.rg_index_set_storage(ix, rg.RG_STORE_BF16)
    Xq = oracle_lib.bf16(X)
    for k, L in ((10, 64), (100, 128)):
        say(f"clip-like bf16 k={k} L={L}")
        ids, ds = rg.rg_search(ix, torch.from_numpy(Q).to(dev), k, L)
        torch.cuda.synchronize()
        oi, od, _, _, gaps = oracle_lib.search_rerank(Xq, X, off, idx, 0, Q, k, L)
        compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Q, X, label=f"2M d512 bf16 k={k} L={L}",
                storage="bf16", explain=oracle_explainer(oracle_lib, X, off, idx, 0, Q, k, L, Xq=Xq))


def test_t2i_like_10m_d200_fp32(dev, oracle_lib):
    g = datagen.Generator(4, n=10_000_000, n_train=1, n_test=24)
    say("serving shape: 10M x 200 base, degree-32 random graph")
    X, Q = g.base(), g.test()
    off, idx = datagen.random_graph_fast(X.shape[0], 32, seed=41)
    ix = rg.rg_index_from_csr(torch.from_numpy(X).to(dev), off, idx, 0)
    for k, L in ((10, 64), (100, 200)):
        say(f"10M fp32 k={k} L={L}")
        ids, ds = rg.rg_search(ix, torch.from_numpy(Q).to(dev), k, L)
        torch.cuda.synchronize()
        oi, od, _, _, gaps = oracle_lib.search(X, off, idx, 0, Q, k, L)
        compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Q, X, label=f"10M d200 k={k} L={L}",
                explain=oracle_explainer(oracle_lib, X, off, idx, 0, Q, k, L))


def test_fp8_8m_d512_properties(dev, oracle_lib):
    g = datagen.Generator(5, n=8_000_000, n_train=1, n_test=64)
    say("fp8 shape: 8M x 512 base, degree-32 random graph")
    X, Q = g.base(), g.test()
    off, idx = datagen.random_graph_fast(X.shape[0], 32, seed=51)
    Xt = torch.from_numpy(X).to(dev)
    ix = rg.rg_index_from_csr(Xt, off, idx, 0)
    Qt = torch.from_numpy(Q).to(dev)
    rg.rg_index_set_storage(ix, rg.RG_STORE_FP8E4M3)
    # codes and scales of sampled rows equal the oracle's quantiser
    _, pf, ps, p8 = ix.storage_ptrs()
    rows = np.random.default_rng(5).choice(X.shape[0], 512, replace=False)
    codes = torch.empty((X.shape[0], p8), dtype=torch.uint8, device=dev)
    scales = torch.empty(X.shape[0], dtype=torch.float32, device=dev)
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    assert hip.hipMemcpy(ctypes.c_void_p(codes.data_ptr()), ctypes.c_void_p(pf),
                         ctypes.c_size_t(X.shape[0] * p8), 3) == 0
    assert hip.hipMemcpy(ctypes.c_void_p(scales.data_ptr()), ctypes.c_void_p(ps), ctypes.c_size_t(X.shape[0] * 4),
                         3) == 0
    torch.cuda.synchronize()
    oc, osc, _ = oracle_lib.quant_fp8(X[rows])
    assert np.array_equal(codes[torch.from_numpy(rows).to(dev)].cpu().numpy()[:, :X.shape[1]], oc)
    assert np.array_equal(scales.cpu().numpy()[rows], osc)
    del codes, scales
    # search + FP32 rerank: returned distances are the exact FP32-row distances
    ids, ds = rg.rg_search(ix, Qt, 10, 128)
    torch.cuda.synchronize()
    a, dd = rg.as_u32(ids), ds.cpu().numpy().astype(np.float64)
    assert (a != NONE).all() and (np.diff(dd, axis=1) >= 0).all()
    exact = -np.einsum("qkd,qd->qk", X[a.astype(np.int64)].astype(np.float64), Q.astype(np.float64))
    tol = 1e-5 * np.linalg.norm(Q, axis=1)[:, None] * np.linalg.norm(X[rows], axis=1).max() * 1.5
    assert (np.abs(dd - exact) <= tol).all()


def test_fp8_500k_d512_oracle_parity(dev, oracle_lib):
    # the CLIP-like law at d = 512 with FP8 storage, sampled queries vs the
    # oracle's search over its own dequantised rows and FP32 rerank
    g = datagen.Generator(5, n=500_000, n_train=1, n_test=32)
    say("fp8 parity: 500k x 512 base, degree-32 random graph")
    X, Q = g.base(), g.test()
    off, idx = datagen.random_graph_fast(X.shape[0], 32, seed=52)
    ix = rg.rg_index_from_csr(torch.from_numpy(X).to(dev), off, idx, 0)
    rg.rg_index_set_storage(ix, rg.RG_STORE_FP8E4M3)
    Xq = oracle_lib.quant_fp8(X)[2]
    for k, L in ((10, 64), (100, 128)):
        say(f"fp8 500k k={k} L={L}")
        ids, ds = rg.rg_search(ix, torch.from_numpy(Q).to(dev), k, L)
        torch.cuda.synchronize()
        oi, od, _, _, gaps = oracle_lib.search_rerank(Xq, X, off, idx, 0, Q, k, L)
        compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Q, X, label=f"500k d512 fp8 k={k} L={L}",
                storage="fp8", explain=oracle_explainer(oracle_lib, X, off, idx, 0, Q, k, L, Xq=Xq))
