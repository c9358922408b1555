"""The library's host construction (rg_build_from_knn) against the oracle,
and the C ABI surface.  CPU only: no HIP call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

import datagen
import paper_2408_08933_amd as rg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_declared_symbol_is_exported():
    hdr = open(os.path.join(ROOT, "include", "roargraph.h")).read()
    names = set(re.findall(r"^[a-z_0-9 \*]*\b(rg_[a-z_0-9]+)\s*\(", hdr, flags=re.M))
    assert len(names) >= 23
    lib = ctypes.CDLL(rg.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def _compare(X, T, Nq, M, L, oracle_lib, threads=0, m_pj=0, m_ce=0):
    G = oracle_lib.Graph(X, T, Nq, M, L, m_pj, m_ce)
    knn, _ = oracle_lib.knn(X, T, Nq)
    ix = rg.rg_build_from_knn(X, knn, Nq, M, L_build=L, threads=threads, m_pj=m_pj, m_ce=m_ce)
    off, idx, entry = ix.graph()
    assert entry == G.entry
    assert np.array_equal(off, G.offsets)
    assert np.array_equal(idx, G.indices)
    assert ix.build_stats()["repairs"] == G.repairs
    return G, ix


def test_hand_worked_five_points(oracle_lib):
    import json, math
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "projection_5pt.json")))
    u = lambda a: [math.cos(math.radians(a)), math.sin(math.radians(a))]
    X = np.array([u(a) for a in g["base_angles_deg"]], np.float32)
    T = np.array([u(a) for a in g["train_angles_deg"]], np.float32)
    knn, _ = oracle_lib.knn(X, T, g["Nq"])
    ix = rg.rg_build_from_knn(X, knn, g["Nq"], g["M"], L_build=g["L"])
    off, idx, entry = ix.graph()
    assert [idx[off[i]:off[i + 1]].tolist() for i in range(5)] == g["final_rows"]
    assert entry == g["entry"]


def test_hand_worked_six_points(oracle_lib):
    import json, math
    g0 = json.load(open(os.path.join(ROOT, "tests", "golden", "enhancement_6pt.json")))
    u = lambda a: [math.cos(math.radians(a)), math.sin(math.radians(a))]
    for g in (g0, dict(g0, **g0["variant_p5_235"])):
        X = np.array([u(a) for a in g["base_angles_deg"]], np.float32)
        T = np.array([u(a) for a in g["train_angles_deg"]], np.float32)
        knn, _ = oracle_lib.knn(X, T, g["Nq"])
        ix = rg.rg_build_from_knn(X, knn, g["Nq"], g["M"], L_build=g["L"], keep_stages=True)
        off, idx, entry = ix.graph()
        assert [idx[off[i]:off[i + 1]].tolist() for i in range(len(X))] == g["final_rows"]
        assert entry == g["entry"]
        assert ix.build_stats()["repairs"] == g["repairs"]


def test_hand_worked_reverse_update(oracle_lib):
    import json, math
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "enhancement_reverse.json")))
    u = lambda a: [math.cos(math.radians(a)), math.sin(math.radians(a))]
    b = g["base"]
    X = np.array([[r * c for c in u(a)] for a, r in zip(b["angles_deg"], b["norms"])], np.float32)
    T = np.array([u(a) for a in g["train_angles_deg"]], np.float32)
    knn, _ = oracle_lib.knn(X, T, g["Nq"])
    ix = rg.rg_build_from_knn(X, knn, g["Nq"], g["M"], L_build=g["L"])
    off, idx, entry = ix.graph()
    assert [idx[off[i]:off[i + 1]].tolist() for i in range(len(X))] == g["final_rows"]
    assert entry == g["entry"]
    assert ix.build_stats()["repairs"] == g["repairs"]


@pytest.mark.parametrize("cfg,n,Nq,M,L", [(1, 1200, 16, 16, 100), (1, 3000, 32, 32, 200), (2, 1500, 24, 20, 120)])
def test_library_graph_bit_exact_with_oracle(oracle_lib, cfg, n, Nq, M, L):
    gen = datagen.Generator(cfg, n=n, n_train=n, n_test=10, d=48 if cfg == 2 else None)
    _compare(gen.base(), gen.train(), Nq, M, L, oracle_lib)


def test_thread_count_does_not_change_graph(oracle_lib):
    gen = datagen.Generator(1, n=1500, n_train=1500, n_test=10)
    X, T = gen.base(), gen.train()
    knn, _ = oracle_lib.knn(X, T, 16)
    a = rg.rg_build_from_knn(X, knn, 16, 16, L_build=100, threads=1).graph()
    b = rg.rg_build_from_knn(X, knn, 16, 16, L_build=100, threads=7).graph()
    assert all(np.array_equal(x, y) for x, y in zip(a[:2], b[:2])) and a[2] == b[2]


def test_paper_literal_degree_split(oracle_lib):
    # both phases at the same bound (the paper uses one M for both, Sec. 5.1)
    gen = datagen.Generator(1, n=1000, n_train=1000, n_test=10)
    _compare(gen.base(), gen.train(), 16, 21, 100, oracle_lib, m_pj=10, m_ce=10)


def test_training_set_smaller_than_base(oracle_lib):
    # |T| = 0.1 |X| (the query-set-size study, Sec. 5.5)
    gen = datagen.Generator(1, n=2000, n_train=200, n_test=10)
    _compare(gen.base(), gen.train(), 16, 16, 100, oracle_lib)


def test_build_from_knn_rejects_bad_input():
    X = np.zeros((10, 4), np.float32)
    with pytest.raises(rg.RGError):
        rg.rg_build_from_knn(X, np.zeros((5, 2), np.uint32), 2, 2)        # M < 3
    with pytest.raises(rg.RGError):
        rg.rg_build_from_knn(X, np.full((5, 2), 99, np.uint32), 2, 8)     # ids out of range


@pytest.mark.parametrize("cfg,n,nt,Nq,M,L", [(1, 1500, 1500, 16, 16, 100), (1, 2000, 300, 24, 20, 120)])
def test_stage_graphs_bit_exact_with_oracle(oracle_lib, cfg, n, nt, Nq, M, L):
    # the graphs the ablation searches: G_bi (bridges, N_out lists and the
    # routing rows through query nodes) and G_pj, against the oracle's build
    gen = datagen.Generator(cfg, n=n, n_train=nt, n_test=10)
    X, T = gen.base(), gen.train()
    G = oracle_lib.Graph(X, T, Nq, M, L)
    knn, _ = oracle_lib.knn(X, T, Nq)
    ix = rg.rg_build_from_knn(X, knn, Nq, M, L_build=L, keep_stages=True)
    b_off, b_idx, n_off, nout = ix.bipartite()
    assert np.array_equal(b_off, G.b_offsets) and np.array_equal(b_idx, G.b_indices)
    assert np.array_equal(n_off, np.arange(nt + 1) * (Nq - 1)) and np.array_equal(nout.reshape(nt, Nq - 1), G.nout)
    off, idx, entry = ix.stage_graph(rg.RG_STAGE_PROJECTED)
    pj_sorted = np.concatenate([np.sort(r) for r in G.rows("pj")])
    assert np.array_equal(off, G.pj_offsets) and np.array_equal(idx, pj_sorted) and entry == G.entry
    ro, ri = oracle_lib.bipartite_routing(G.b_offsets, G.b_indices, G.nout)
    off, idx, entry = ix.stage_graph(rg.RG_STAGE_BIPARTITE)
    assert np.array_equal(off, ro) and np.array_equal(idx, ri)
    assert entry == oracle_lib.medoid(X, mask=np.diff(G.b_offsets) > 0)
    # the final graph is unchanged by keeping the stages
    a = ix.graph()
    assert np.array_equal(a[0], G.offsets) and np.array_equal(a[1], G.indices) and a[2] == G.entry


def test_stage_graphs_need_keep_stages(oracle_lib):
    gen = datagen.Generator(1, n=300, n_train=300, n_test=10)
    X = gen.base()
    knn, _ = oracle_lib.knn(X, gen.train(), 8)
    ix = rg.rg_build_from_knn(X, knn, 8, 8, L_build=50)
    with pytest.raises(rg.RGError):
        ix.stage_graph(rg.RG_STAGE_PROJECTED)
    with pytest.raises(rg.RGError):
        ix.bipartite()


# --------------------------------------------------------------------------
# updates (Sec. 6): the library's insertion and tombstones against the oracle
# --------------------------------------------------------------------------
def _unit2(a):
    import math
    return [math.cos(math.radians(a)), math.sin(math.radians(a))]


def test_insert_hand_worked_five_points(oracle_lib):
    import json
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "projection_5pt.json")))
    u = json.load(open(os.path.join(ROOT, "tests", "golden", "updates_5pt.json")))
    X = np.array([_unit2(a) for a in g["base_angles_deg"]], np.float32)
    T = np.array([_unit2(a) for a in g["train_angles_deg"]], np.float32)
    knn, _ = oracle_lib.knn(X, T, g["Nq"])
    ix = rg.rg_build_from_knn(X, knn, g["Nq"], g["M"], L_build=g["L"], keep_stages=True, train_host=T)
    for i, a in enumerate(u["inserts_deg"]):
        assert ix.insert(np.array([_unit2(a)], np.float32)).tolist() == [5 + i]
    off, idx, entry = ix.graph()
    assert [idx[off[i]:off[i + 1]].tolist() for i in range(len(off) - 1)] == u["final_rows"]
    _, _, n_off, nout = ix.bipartite()
    assert [nout[n_off[t]:n_off[t + 1]].tolist() for t in range(2)] == u["final_nout"]


@pytest.mark.parametrize("batches", [[70, 50], [1, 1, 30]])
def test_insert_bit_exact_with_oracle(oracle_lib, batches):
    from oracle.updates import Updatable
    gen = datagen.Generator(1, n=1500, n_train=1500, n_test=120)
    X, T, Q = gen.base(), gen.train(), gen.test()
    Nq, M, L = 16, 16, 120
    G = oracle_lib.Graph(X, T, Nq, M, L)
    knn, _ = oracle_lib.knn(X, T, Nq)
    ix = rg.rg_build_from_knn(X, knn, Nq, M, L_build=L, keep_stages=True, train_host=T)
    st = Updatable.from_graph(G, X, T)
    V = np.concatenate([gen.in_distribution(60), Q])[:sum(batches)]
    s0 = 0
    for b in batches:
        ix.insert(V[s0:s0 + b], L=64)
        st.insert(V[s0:s0 + b], L=64)
        s0 += b
    off, idx, entry = ix.graph()
    o2, i2 = st.csr()
    assert np.array_equal(off, o2) and np.array_equal(idx, i2) and entry == st.entry
    _, _, n_off, nout = ix.bipartite()
    assert [nout[n_off[t]:n_off[t + 1]].tolist() for t in range(len(st.nout))] == st.nout


def test_insert_rows_sharing_a_bridge_query(oracle_lib):
    # near-copies of a few vectors in one call share their bridge training
    # query, so each later copy's own list must see the copies linked before
    from oracle.updates import Updatable
    gen = datagen.Generator(1, n=1200, n_train=1200, n_test=40)
    X, T, Q = gen.base(), gen.train(), gen.test()
    Nq, M, L = 16, 16, 100
    G = oracle_lib.Graph(X, T, Nq, M, L)
    knn, _ = oracle_lib.knn(X, T, Nq)
    ix = rg.rg_build_from_knn(X, knn, Nq, M, L_build=L, keep_stages=True, train_host=T)
    st = Updatable.from_graph(G, X, T)
    rng = np.random.default_rng(5)
    V = (np.repeat(Q[:4], 12, axis=0) + 1e-3 * rng.standard_normal((48, X.shape[1]))).astype(np.float32)
    ix.insert(V, L=64)
    st.insert(V, L=64)
    off, idx, entry = ix.graph()
    o2, i2 = st.csr()
    assert np.array_equal(off, o2) and np.array_equal(idx, i2)
    _, _, n_off, nout = ix.bipartite()
    lists = [nout[n_off[t]:n_off[t + 1]].tolist() for t in range(len(st.nout))]
    assert lists == st.nout
    assert max(sum(1 for u in r if u >= 1200) for r in lists) >= 2   # some query gained several new rows


def test_insert_needs_stages_and_training_queries(oracle_lib):
    gen = datagen.Generator(1, n=300, n_train=300, n_test=10)
    X, T = gen.base(), gen.train()
    knn, _ = oracle_lib.knn(X, T, 8)
    v = X[:2] + 0.01
    with pytest.raises(rg.RGError):
        rg.rg_build_from_knn(X, knn, 8, 8, L_build=50).insert(v)
    with pytest.raises(rg.RGError):
        rg.rg_build_from_knn(X, knn, 8, 8, L_build=50, keep_stages=True).insert(v)
    ix = rg.rg_build_from_knn(X, knn, 8, 8, L_build=50, keep_stages=True, train_host=T)
    assert ix.insert(np.zeros((0, X.shape[1]), np.float32)).size == 0
    with pytest.raises(rg.RGError):
        ix.insert(v, L=513)


def test_delete_marks_tombstones(oracle_lib):
    gen = datagen.Generator(1, n=300, n_train=300, n_test=10)
    X, T = gen.base(), gen.train()
    knn, _ = oracle_lib.knn(X, T, 8)
    ix = rg.rg_build_from_knn(X, knn, 8, 8, L_build=50)
    assert ix.tombstones() == (None, 0)
    ix.delete([3, 40, 3, 299])
    bits, cnt = ix.tombstones()
    assert cnt == 3
    dead = [i for i in range(300) if (bits[i >> 5] >> (i & 31)) & 1]
    assert dead == [3, 40, 299]
    with pytest.raises(rg.RGError):
        ix.delete([300])


def test_failed_insert_leaves_the_index_unchanged(oracle_lib):
    # a rejected call (a non-finite value) must not touch rows, graph or the
    # bipartite lists; a later valid insert behaves as on a fresh index
    gen = datagen.Generator(1, n=400, n_train=400, n_test=10)
    X, T = gen.base(), gen.train()
    knn, _ = oracle_lib.knn(X, T, 8)
    ix = rg.rg_build_from_knn(X, knn, 8, 8, L_build=50, keep_stages=True, train_host=T)
    ref = rg.rg_build_from_knn(X, knn, 8, 8, L_build=50, keep_stages=True, train_host=T)
    before = ix.graph(), ix.bipartite(), ix.info()["n"]
    bad = X[:3] + 0.01
    bad[1, 5] = np.nan
    with pytest.raises(rg.RGError) as e:
        ix.insert(bad)
    assert e.value.code == rg.RG_EINVAL
    after = ix.graph(), ix.bipartite(), ix.info()["n"]
    assert after[2] == before[2]
    assert all(np.array_equal(a, b) for a, b in zip(after[0][:2], before[0][:2])) and after[0][2] == before[0][2]
    assert all(np.array_equal(a, b) for a, b in zip(after[1], before[1]))
    good = X[:3] + 0.01
    ix.insert(good)
    ref.insert(good)
    assert all(np.array_equal(a, b) for a, b in zip(ix.graph()[:2], ref.graph()[:2]))
