"""Index updates on the GPU (the paper's update section): insertion through
the saved bipartite graph with the device's canonical searches, and
tombstone deletion in rg_search and the server, against the oracle."""
import sys
import time

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


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


@pytest.fixture(scope="module")
def setup(oracle_lib):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle.updates import Updatable
    dev = torch.device("cuda:0")
    g = datagen.Generator(1, n=4000, n_train=4000, n_test=300)
    X, Tr, Q = g.base(), g.train(), g.test()
    Nq, M, L = 24, 24, 200
    say("updates: build n=4000 d=64 with stages kept")
    ix = rg.rg_build(T(X, dev), T(Tr, dev), Nq, M, L_build=L, keep_stages=True)
    G = oracle_lib.Graph(X, Tr, Nq, M, L)
    st = Updatable.from_graph(G, X, Tr)
    V = np.concatenate([g.in_distribution(150), g.requests(150, 1.0)[1]])
    for a, b in ((0, 120), (120, 121), (121, 300)):
        say(f"insert rows {a}..{b}")
        ix.insert(V[a:b], L=128)
        st.insert(V[a:b], L=128)
    return dev, Q, ix, st


def test_insert_graph_bit_exact(setup):
    dev, Q, ix, st = setup
    off, idx, entry = ix.graph()
    o2, i2 = st.csr()
    assert np.array_equal(off, o2) and np.array_equal(idx, i2) and entry == st.entry
    _, _, n_off, nout = ix.bipartite()
    assert [nout[n_off[t]:n_off[t + 1]].tolist() for t in range(len(st.nout))] == st.nout
    assert ix.info()["n"] == st.n


def test_search_after_insert(setup, oracle_lib):
    dev, Q, ix, st = setup
    off, idx = st.csr()
    for k, L in ((10, 64), (100, 128)):
        say(f"search after insert k={k} L={L}")
        ids, ds = rg.rg_search(ix, T(Q, dev), k, L)
        torch.cuda.synchronize()
        oi, od, _, _, gaps = oracle_lib.search(st.X, off, idx, st.entry, Q, k, L)
        compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Q, st.X, label=f"after insert k={k} L={L}",
                explain=oracle_explainer(oracle_lib, st.X, off, idx, st.entry, Q, k, L))
    # new rows are found: each inserted row searched for itself comes back first
    V = st.X[4000:]
    ids, _ = rg.rg_search(ix, T(V, dev), 1, 64)
    torch.cuda.synchronize()
    hit = (rg.as_u32(ids)[:, 0] == np.arange(4000, st.n)).mean()
    say(f"inserted rows found as their own nearest: {hit:.3f}")
    assert hit >= 0.95


def test_insert_with_bf16_storage(setup, oracle_lib):
    dev, Q, ix, st = setup
    rg.rg_index_set_storage(ix, rg.RG_STORE_BF16)
    try:
        V = st.X[4000:4010] * 0.5 + st.X[:10] * 0.5
        ix.insert(V, L=128)
        st.insert(V, L=128)
        off, idx = st.csr()
        o2, i2, _ = ix.graph()
        assert np.array_equal(o2, off) and np.array_equal(i2, idx)
        say("bf16 search after insert k=10 L=64")
        ids, ds = rg.rg_search(ix, T(Q, dev), 10, 64)
        torch.cuda.synchronize()
        Xq = oracle_lib.bf16(st.X)
        oi, od, _, _, gaps = oracle_lib.search_rerank(Xq, st.X, off, idx, st.entry, Q, 10, 64)
        compare(rg.as_u32(ids), ds.cpu().numpy(), oi, od, gaps, Q, st.X, label="bf16 after insert", storage="bf16",
                explain=oracle_explainer(oracle_lib, st.X, off, idx, st.entry, Q, 10, 64, Xq=Xq))
    finally:
        rg.rg_index_set_storage(ix, rg.RG_STORE_FP32)


def _check_tombstoned(gpu_i, gpu_d, or_i, or_d, Q, X, dead):
    tol = 1e-5 * np.linalg.norm(Q, axis=1)[:, None] * np.linalg.norm(X, axis=1).max()
    assert not np.isin(gpu_i[gpu_i != NONE], dead).any()
    assert np.array_equal(gpu_i == NONE, or_i == NONE)
    both = or_i != NONE
    assert (np.abs(gpu_d.astype(np.float64)[both] - or_d[both]) <= np.broadcast_to(tol, or_d.shape)[both]).all()
    agree = np.mean([len(np.intersect1d(a[a != NONE], b[b != NONE])) / max(1, (b != NONE).sum())
                     for a, b in zip(gpu_i, or_i)])
    assert agree >= 0.97, agree
    return agree


def test_tombstones_in_search_and_serving(setup):
    dev, Q, ix, st = setup
    rng = np.random.default_rng(9)
    # delete many of the queries' true neighbours so the skip matters
    ids0, _ = rg.rg_search(ix, T(Q, dev), 10, 64)
    torch.cuda.synchronize()
    near = np.unique(rg.as_u32(ids0)[:, :3])
    dead = np.unique(np.concatenate([near, rng.choice(st.n, 300, replace=False)])).astype(np.uint32)
    ix.delete(dead)
    st.delete(dead)
    assert ix.tombstones()[1] == len(dead)
    for k, L in ((10, 32), (10, 128), (50, 60)):
        say(f"tombstoned search k={k} L={L} ({len(dead)} deleted)")
        gi, gd = rg.rg_search(ix, T(Q, dev), k, L)
        torch.cuda.synchronize()
        oi, od = st.search(Q, k, L)
        a = _check_tombstoned(rg.as_u32(gi), gd.cpu().numpy(), oi, od, Q, st.X, dead)
        say(f"  agreement {a:.4f}")
    # the server returns each request's rg_search result
    srv = rg.Server(ix, max_slots=64, hops_per_step=8)
    for i in range(60):
        assert srv.submit(Q[i], 10, 64, i) == rg.RG_OK
    got = {}
    t0 = time.time()
    while len(got) < 60 and time.time() - t0 < 60:
        for r in srv.poll():
            got[r["tag"]] = r
        time.sleep(0.001)
    srv.close()
    assert len(got) == 60
    gi, _ = rg.rg_search(ix, T(Q[:60], dev), 10, 64)
    torch.cuda.synchronize()
    gi = rg.as_u32(gi)
    for i in range(60):
        assert np.array_equal(got[i]["ids"], gi[i])
    # everything deleted: padding only
    ix.delete(np.arange(st.n))
    gi, gd = rg.rg_search(ix, T(Q[:5], dev), 10, 20)
    torch.cuda.synchronize()
    assert (rg.as_u32(gi) == NONE).all() and torch.isinf(gd).all()
