"""Pins for the FP64 oracle: each test checks it against something the paper
or plain mathematics fixes (closed forms, hand-worked geometry, brute force
on integer data, special cases of the search, an independent library's
number formats), never against a retyped copy of its own formula."""
import json
import math
import os

import numpy as np
import pytest

import datagen
from oracle import NONE

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def unit2(deg):
    r = math.radians(deg)
    return [math.cos(r), math.sin(r)]


# --------------------------------------------------------------------------
# distance (Def. 1, inner product)
# --------------------------------------------------------------------------
def test_dist_integer_exact(oracle_lib):
    rng = np.random.default_rng(1)
    for d in (1, 3, 64, 200):
        a = rng.integers(-50, 50, size=d)
        b = rng.integers(-50, 50, size=d)
        exact = -sum(int(x) * int(y) for x, y in zip(a, b))
        assert oracle_lib.dist(a, b) == float(exact)


def test_dist_selects_index(oracle_lib):
    # a one-hot vector picks exactly coordinate i of the other operand
    b = np.arange(1, 17, dtype=np.float32)
    for i in range(16):
        a = np.zeros(16, np.float32)
        a[i] = 1
        assert oracle_lib.dist(a, b) == -(i + 1)


def test_dist_self_and_orthogonal(oracle_lib):
    x = np.array([3, 4], np.float32)
    assert oracle_lib.dist(x, x) == -25.0
    assert oracle_lib.dist([1, 0], [0, 7]) == 0.0


def test_dist_sums_in_increasing_index_order(oracle_lib):
    # 2^53 + 1 rounds back to 2^53 in double; summed left to right the 1 is
    # lost (-> 0), summed right to left it survives (-> -1).
    a = np.array([2.0 ** 53, 1.0, -(2.0 ** 53)], np.float32)
    assert oracle_lib.dist(a, np.ones(3, np.float32)) == 0.0
    assert oracle_lib.dist(a[::-1].copy(), np.ones(3, np.float32)) == -1.0


# --------------------------------------------------------------------------
# exact kNN (Def. 1), ties by id
# --------------------------------------------------------------------------
def test_knn_matches_sort_on_integer_data(oracle_lib):
    rng = np.random.default_rng(2)
    X = rng.integers(-3, 4, size=(300, 5)).astype(np.float32)
    Q = rng.integers(-3, 4, size=(40, 5)).astype(np.float32)
    ids, ds = oracle_lib.knn(X, Q, 17)
    S = -(Q.astype(np.int64) @ X.astype(np.int64).T)  # exact integer distances
    for q in range(len(Q)):
        order = np.lexsort((np.arange(len(X)), S[q]))[:17]  # by distance, then id
        assert list(ids[q]) == list(order)
        assert list(ds[q]) == list(S[q][order].astype(float))


def test_knn_k_equals_n_and_padding(oracle_lib):
    X = np.array([[1, 0], [0, 1], [1, 1]], np.float32)
    ids, ds = oracle_lib.knn(X, np.array([[2, 1]], np.float32), 5)
    assert list(ids[0][:3]) == [2, 0, 1]
    assert list(ds[0][:3]) == [-3.0, -2.0, -1.0]
    assert ids[0][3] == oracle_lib.NONE and math.isinf(ds[0][4])


# --------------------------------------------------------------------------
# medoid reading: nearest (L2) to the mean, lower id on ties
# --------------------------------------------------------------------------
def test_medoid(oracle_lib):
    assert oracle_lib.medoid(np.array([[0], [1], [2], [10]], np.float32)) == 2  # mean 3.25
    assert oracle_lib.medoid(np.array([[0], [2]], np.float32)) == 0  # tie -> lower id
    assert oracle_lib.medoid(np.array([[5, 5]], np.float32)) == 0


# medoid with the projected-graph mask (R9): the mean is over ALL rows, the
# choice among the masked rows only, lower id on ties
def test_medoid_mask(oracle_lib):
    # mean of all rows 5.6: row 2 (7); the mean of the masked rows (2.67)
    # would give row 1
    X = np.array([[0], [1], [7], [10], [10]], np.float32)
    assert oracle_lib.medoid(X, mask=np.array([1, 1, 1, 0, 0], bool)) == 2
    # mean 4.5: unmasked, rows 1 and 2 tie (lower id 1); masked to rows 0
    # and 3, which tie at 4.5 from the mean -> row 0
    X = np.array([[0], [4], [5], [9]], np.float32)
    assert oracle_lib.medoid(X) == 1
    assert oracle_lib.medoid(X, mask=np.array([1, 0, 0, 1], bool)) == 0
    assert oracle_lib.medoid(X, mask=np.array([0, 0, 0, 1], bool)) == 3
    # an empty mask selects from all rows
    assert oracle_lib.medoid(X, mask=np.zeros(4, bool)) == 1


# --------------------------------------------------------------------------
# AcquireNeighbors (Algorithm 3) on hand geometry
# --------------------------------------------------------------------------
def test_acquire_fan_both_sides(oracle_lib):
    # x at 0 deg; candidates at +30, -35, +40, +100 deg on the unit circle.
    # Under -IP, c is kept iff angle(x,c) < angle(c,p) for every kept p.
    X = np.array([unit2(a) for a in (0, 30, -35, 40, 100)], np.float32)
    C = [4, 3, 2, 1, 1, 0]  # shuffled, with a duplicate and x itself
    assert list(oracle_lib.acquire(X, 0, C, 4, 0)) == [1, 2]      # 40 occluded by 30, 100 by 30
    assert list(oracle_lib.acquire(X, 0, C, 3, 1)) == [1, 2, 3]   # fill in rank order
    assert list(oracle_lib.acquire(X, 0, C, 4, 1)) == [1, 2, 3, 4]
    assert list(oracle_lib.acquire(X, 0, C, 1, 1)) == [1]
    assert list(oracle_lib.acquire(X, 0, [], 3, 1)) == []


def test_acquire_pivot_xyz_example(oracle_lib):
    # Sec. 4.2.3: pivot P; X is kept; Y is closer to X than to P and is
    # skipped; Z is kept; with degree limit 3 the fill brings Y back.
    P, Xn, Y, Z = unit2(0), unit2(20), unit2(35), unit2(-40)
    X = np.array([P, Xn, Y, Z], np.float32)
    assert list(oracle_lib.acquire(X, 0, [1, 2, 3], 3, 0)) == [1, 3]
    assert list(oracle_lib.acquire(X, 0, [1, 2, 3], 3, 1)) == [1, 3, 2]
    assert list(oracle_lib.acquire(X, 0, [1, 2, 3], 2, 1)) == [1, 3]


def test_acquire_collinear_inner_product(oracle_lib):
    # 1-D, delta(a,b) = -ab.  x = 1; candidates 3, 2, -1: 3 first; 2 fails
    # (-2 < -6 false); -1 passes (1 < 3).
    X = np.array([[1], [3], [2], [-1]], np.float32)
    assert list(oracle_lib.acquire(X, 0, [2, 3, 1], 5, 0)) == [1, 3]


def test_acquire_strict_rule_ties_exclude(oracle_lib):
    # delta(x,c) == delta(c,p) must exclude c (strict <)
    X = np.array([[1, 0], [1, 0], [1, 0]], np.float32)  # all identical vectors
    assert list(oracle_lib.acquire(X, 0, [1, 2], 3, 0)) == [1]


# --------------------------------------------------------------------------
# hand-worked construction
# --------------------------------------------------------------------------
def test_build_hand_worked_five_points(oracle_lib):
    g = json.load(open(os.path.join(GOLDEN, "projection_5pt.json")))
    X = np.array([unit2(a) for a in g["base_angles_deg"]], np.float32)
    T = np.array([unit2(a) for a in g["train_angles_deg"]], np.float32)
    G = oracle_lib.Graph(X, T, g["Nq"], g["M"], g["L"])
    assert [sorted(r.tolist()) for r in G.rows("pj")] == [sorted(r) for r in g["pj_rows"]]
    assert [sorted(r.tolist()) for r in G.rows("ce")] == [sorted(r) for r in g["ce_rows"]]
    assert [r.tolist() for r in G.rows("final")] == g["final_rows"]
    assert G.entry == g["entry"]
    assert G.repairs == g["repairs"]
    assert list(G.pivot) == [0, 3]


def test_enhancement_hand_worked_six_points(oracle_lib):
    # two enhancement edges per node and a queue of 3: truncated searches,
    # occlusion without fill, reverse updates that re-prune copied rows
    # (the variant moves P5 so that its own selection drops a candidate)
    g0 = json.load(open(os.path.join(GOLDEN, "enhancement_6pt.json")))
    for g in (g0, dict(g0, **g0["variant_p5_235"])):
        X = np.array([unit2(a) for a in g["base_angles_deg"]], np.float32)
        T = np.array([unit2(a) for a in g["train_angles_deg"]], np.float32)
        G = oracle_lib.Graph(X, T, g["Nq"], g["M"], g["L"])
        assert G.pivot.tolist() == g0["pivot"]
        assert [sorted(r.tolist()) for r in G.rows("pj")] == g["pj_rows"]
        assert G.entry == g["entry"]
        assert [G.cx[x, :G.cx_n[x]].tolist() for x in range(len(X))] == g["enhancement_candidates"]
        assert [sorted(r.tolist()) for r in G.rows("ce")] == g["ce_rows"]
        assert [r.tolist() for r in G.rows("final")] == g["final_rows"]
        assert G.repairs == g["repairs"]


def test_enhancement_reverse_update_hand_worked(oracle_lib):
    # a half-norm node no search reaches, processed last: its reverse update
    # into a row with room drops it (AcquireNeighbors without fill)
    g = json.load(open(os.path.join(GOLDEN, "enhancement_reverse.json")))
    b = g["base"]
    X = np.array([[r * c for c in unit2(a)] for a, r in zip(b["angles_deg"], b["norms"])], np.float32)
    T = np.array([unit2(a) for a in g["train_angles_deg"]], np.float32)
    G = oracle_lib.Graph(X, T, g["Nq"], g["M"], g["L"])
    assert G.pivot.tolist() == g["pivot"]
    assert [sorted(r.tolist()) for r in G.rows("pj")] == g["pj_rows"]
    assert G.entry == g["entry"]
    assert [G.cx[x, :G.cx_n[x]].tolist() for x in range(len(X))] == g["enhancement_candidates"]
    assert [sorted(r.tolist()) for r in G.rows("ce")] == g["ce_rows"]
    assert [r.tolist() for r in G.rows("final")] == g["final_rows"]
    assert G.repairs == g["repairs"]


def test_projection_cutoff_hand_worked(oracle_lib):
    # overlapping bridge lists beyond L: distinct count before each list,
    # rank by distance to the pivot, truncate to L (Algorithm 2)
    g = json.load(open(os.path.join(GOLDEN, "projection_cutoff.json")))
    b = g["base"]
    X = np.array([[r * c for c in unit2(a)] for a, r in zip(b["angles_deg"], b["norms"])], np.float32)
    T = np.array([unit2(a) for a in g["train_angles_deg"]], np.float32)
    G = oracle_lib.Graph(X, T, g["Nq"], g["M"], g["L"])
    assert G.pivot.tolist() == g["pivot"]
    assert G.nout.tolist() == g["nout"]
    assert [r.tolist() for r in G.rows("pj")] == g["pj_rows"]


def test_repair_fallback_hand_worked(oracle_lib):
    g = json.load(open(os.path.join(GOLDEN, "repair_fallback.json")))
    rows, added = oracle_lib.repair(g["rows"], g["M"], g["entry"], g["candidates"])
    assert rows == g["repaired_rows"]
    assert added == g["repairs"]


def test_repair_reaches_everything_on_random_graphs(oracle_lib):
    # invariant: after the repair every node is reachable and no row exceeds M
    rng = np.random.default_rng(11)
    for trial in range(20):
        n, M = 40, 4
        rows = [sorted(set(rng.integers(0, n, size=int(rng.integers(0, 3))).tolist()) - {x}) for x in range(n)]
        cand = [rng.permutation(n)[:5].tolist() for _ in range(n)]
        out, _ = oracle_lib.repair(rows, M, 0, cand)
        assert max(len(r) for r in out) <= M
        seen, todo = {0}, [0]
        while todo:
            v = todo.pop()
            for w in out[v]:
                if w not in seen:
                    seen.add(w)
                    todo.append(w)
        assert len(seen) == n


def test_bipartite_routing_hand_worked(oracle_lib):
    # greedy routing on G_bi through query nodes (Sec. 4.2.1), by hand
    g = json.load(open(os.path.join(GOLDEN, "projection_5pt.json")))
    X = np.array([unit2(a) for a in g["base_angles_deg"]], np.float32)
    T = np.array([unit2(a) for a in g["train_angles_deg"]], np.float32)
    G = oracle_lib.Graph(X, T, g["Nq"], g["M"], g["L"])
    off, idx = oracle_lib.bipartite_routing(G.b_offsets, G.b_indices, G.nout)
    assert [idx[off[i]:off[i + 1]].tolist() for i in range(5)] == g["bi_rows"]
    entry = oracle_lib.medoid(X, mask=np.diff(G.b_offsets) > 0)
    assert entry == g["bi_entry"]
    s = g["bi_search"]
    q = np.array([unit2(s["query_deg"])], np.float32)
    ids, _, _, _, _ = oracle_lib.search(X, off, idx, entry, q, s["k"], s["L"])
    assert ids[0].tolist() == s["ids"]


def test_bipartite_routing_rows_are_two_hop_sets(oracle_lib, small_graph):
    # every routed neighbour of x is an out-neighbour of a query node that x
    # links to, and each such out-neighbour appears
    X, T, Q, G = small_graph
    off, idx = oracle_lib.bipartite_routing(G.b_offsets, G.b_indices, G.nout)
    for x in range(0, G.n, 7):
        ts = [int(t) for t in range(len(G.pivot)) if G.pivot[t] == x]
        want = sorted(set(int(u) for t in ts for u in G.nout[t]))
        assert sorted(set(idx[off[x]:off[x + 1]].tolist())) == want
        assert off[x + 1] - off[x] == len(ts) * (G.Nq - 1)


# --------------------------------------------------------------------------
# construction invariants on the tiny OOD workload law
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_graph(oracle_lib):
    gen = datagen.Generator(1, n=1500, n_train=1500, n_test=200)
    X, T, Q = gen.base(), gen.train(), gen.test()
    G = oracle_lib.Graph(X, T, 16, 16, 120)
    return X, T, Q, G


def _bfs(off, idx, start, n):
    seen = np.zeros(n, bool)
    seen[start] = True
    st = [start]
    while st:
        v = st.pop()
        for u in idx[off[v]:off[v + 1]]:
            if not seen[u]:
                seen[u] = True
                st.append(int(u))
    return seen


def test_bipartite_invariants(oracle_lib, small_graph):
    X, T, Q, G = small_graph
    ids, _ = oracle_lib.knn(X, T, G.Nq)
    assert (G.pivot == ids[:, 0]).all()                       # pivot = nearest base row
    assert (G.nout == ids[:, 1:]).all()                       # N_out minus the pivot
    assert G.b_offsets[-1] == len(T)                          # sum |B(x)| = |T|
    for x in range(G.n):
        ts = G.b_indices[G.b_offsets[x]:G.b_offsets[x + 1]]
        assert (G.pivot[ts] == x).all() and (np.diff(ts.astype(np.int64)) > 0).all()


def test_graph_invariants(oracle_lib, small_graph):
    X, T, Q, G = small_graph
    m_pj, m_ce = G.M // 2, (G.M - 1) // 2
    pj, ce, fin = G.rows("pj"), G.rows("ce"), G.rows("final")
    for x in range(G.n):
        assert len(pj[x]) <= m_pj and len(ce[x]) <= m_ce and len(fin[x]) <= G.M
        for r in (pj[x], ce[x], fin[x]):
            assert x not in r and len(set(r.tolist())) == len(r)
        assert set(pj[x].tolist()) <= set(fin[x].tolist())
        assert (np.diff(fin[x].astype(np.int64)) > 0).all()
    assert _bfs(G.offsets, G.indices, G.entry, G.n).all()      # every node reachable
    assert len(pj[G.entry]) > 0
    # projection leaves nodes without out-edges, enhancement + repair fix them
    assert sum(len(r) == 0 for r in pj) > 0
    assert all(len(r) > 0 for r in fin)


def test_build_rejects_bad_args(oracle_lib):
    X = np.zeros((4, 2), np.float32)
    with pytest.raises(ValueError):
        oracle_lib.Graph(X, X, 1, 8)   # Nq < 2
    with pytest.raises(ValueError):
        oracle_lib.Graph(X, X, 3, 2)   # M < 3


# --------------------------------------------------------------------------
# beam search (Sec. 4.3): special cases
# --------------------------------------------------------------------------
def _complete(n):
    rows = [[j for j in range(n) if j != i] for i in range(n)]
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    return off, np.array(sum(rows, []), np.uint32)


def test_search_complete_graph_is_exact(oracle_lib):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((60, 8)).astype(np.float32)
    Q = rng.standard_normal((25, 8)).astype(np.float32)
    off, idx = _complete(60)
    gt, gd = oracle_lib.knn(X, Q, 10)
    for L in (10, 11, 30):
        ids, ds, hops, ev, _ = oracle_lib.search(X, off, idx, 7, Q, 10, L)
        assert (ids == gt).all() and (ds == gd).all()
        assert (ev == 60).all()


def test_search_L_at_least_n_is_exact_on_reachable_graph(oracle_lib, small_graph):
    X, T, Q, G = small_graph
    gt, gd = oracle_lib.knn(X, Q[:30], 10)
    ids, ds, hops, ev, _ = oracle_lib.search(X, G.offsets, G.indices, G.entry, Q[:30], 10, G.n)
    assert (ids == gt).all() and (ds == gd).all()
    assert (ev == G.n).all()
    assert oracle_lib.recall(ids, gt, 10) == 1.0


def test_search_path_graph_by_hand(oracle_lib):
    # points on a line, delta = -x*q; path 0-1-2-3-4 (both directions)
    X = np.array([[1], [2], [3], [4], [5]], np.float32)
    rows = [[1], [0, 2], [1, 3], [2, 4], [3]]
    off = np.array([0, 1, 3, 5, 7, 8], np.int64)
    idx = np.array(sum(rows, []), np.uint32)
    # q = +1 prefers larger x.  L=1 from entry 0: 0 -> 1 -> 2 -> 3 -> 4.
    # Node i holds x = i + 1; the scale of a pair is |q x| = x.
    # Each expansion evicts the old entry: margins (delta_old - delta_new) /
    # (S_new + S_old) = 1/3, 1/5, 1/7, 1/9; the smallest is 1/9.
    ids, ds, hops, ev, gaps = oracle_lib.search(X, off, idx, 0, np.array([[1]], np.float32), 1, 1)
    assert ids[0, 0] == 4 and ds[0, 0] == -5.0 and hops[0] == 5 and ev[0] == 5
    assert gaps[0] == pytest.approx(1 / 9, rel=1e-15)
    # q = -1 prefers smaller x: from entry 2 with L=2: expand 2 (sees 1, 3),
    # queue [1, 2] and 3 rejected: margins (4-2)/(2+4), (4-3)/(3+4) = 1/7;
    # expand 1 (sees 0), queue [0, 1] and 2 evicted: (3-1)/4, (3-2)/5;
    # expand 0; done.  Smallest: 1/7.
    ids, ds, hops, ev, gaps = oracle_lib.search(X, off, idx, 2, np.array([[-1]], np.float32), 2, 2)
    assert list(ids[0]) == [0, 1] and list(ds[0]) == [1.0, 2.0]
    assert hops[0] == 3 and ev[0] == 4
    assert gaps[0] == pytest.approx(1 / 7, rel=1e-15)


def test_search_single_node_and_padding(oracle_lib):
    X = np.array([[2.0, 0.0]], np.float32)
    ids, ds, hops, ev, _ = oracle_lib.search(X, np.array([0, 0], np.int64), np.zeros(0, np.uint32), 0,
                                             np.array([[1.0, 1.0]], np.float32), 3, 2)
    assert ids[0, 0] == 0 and ds[0, 0] == -2.0
    assert ids[0, 1] == oracle_lib.NONE and math.isinf(ds[0, 2])
    assert hops[0] == 1 and ev[0] == 1


def test_search_margin_is_sound_under_perturbation(oracle_lib, small_graph):
    # The margin promises that distances perturbed by less than margin * S
    # (S = sum |q_i x_i|) leave every decision unchanged.  Perturb each
    # coordinate of X by a relative 0.4 * margin with random sign, which
    # moves every distance by at most 0.4 * margin * S (plus float rounding,
    # 2^-24 relative, kept far below by skipping tiny margins): the search
    # must expand the same nodes and return the same ids.
    X, T, Q, G = small_graph
    rng = np.random.default_rng(17)
    checked = 0
    for L, k in ((16, 10), (48, 10), (32, 32)):
        ids, ds, hops, ev, gaps = oracle_lib.search(X, G.offsets, G.indices, G.entry, Q[:24], k, L)
        for q in range(24):
            g = float(gaps[q])
            if not (1e-5 < g < np.inf):
                continue
            eps = 0.4 * g
            Xp = (X.astype(np.float64) * (1.0 + eps * rng.choice([-1.0, 1.0], size=X.shape))).astype(np.float32)
            i2, _, h2, e2, _ = oracle_lib.search(Xp, G.offsets, G.indices, G.entry, Q[q:q + 1], k, L)
            assert set(i2[0].tolist()) == set(ids[q].tolist()) and h2[0] == hops[q] and e2[0] == ev[q]
            checked += 1
    assert checked >= 20


def test_perturbed_search(oracle_lib, small_graph):
    # eps = 0 is the plain search; eps below a query's margin changes
    # nothing; on an exact tie a perturbation can pick either node, and only
    # those two (every other distance is far away)
    X, T, Q, G = small_graph
    a = oracle_lib.search(X, G.offsets, G.indices, G.entry, Q[:30], 10, 32)
    b = oracle_lib.search_perturbed(X, G.offsets, G.indices, G.entry, Q[:30], 10, 32, 0.0, 5)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all() and (a[2] == b[2]).all() and (a[3] == b[3]).all()
    gaps = a[4]
    for q in np.nonzero(gaps > 1e-6)[0][:10]:
        for seed in range(3):
            c = oracle_lib.search_perturbed(X, G.offsets, G.indices, G.entry, Q[q:q + 1], 10, 32,
                                            0.9 * gaps[q], seed)
            # the margin covers the first k against the rest, not the order
            # among the first k (swaps there are judged by distance)
            assert set(c[0][0].tolist()) == set(a[0][q].tolist()) and c[2][0] == a[2][q] and c[3][0] == a[3][q]
    Xt = np.array([[1, 0], [0, 1], [0, 1], [-1, 0]], np.float32)
    off, idx = _complete(4)
    got = set()
    for seed in range(24):
        ids, _, _, _ = oracle_lib.search_perturbed(Xt, off, idx, 0, np.array([[0, 1]], np.float32), 1, 1,
                                                   1e-3, seed)
        got.add(int(ids[0, 0]))
    assert got == {1, 2}


def test_search_exact_tie_has_zero_gap(oracle_lib):
    X = np.array([[1, 0], [0, 1], [0, 1]], np.float32)  # nodes 1 and 2 tie for any query
    off, idx = _complete(3)
    ids, ds, hops, ev, gaps = oracle_lib.search(X, off, idx, 0, np.array([[0, 1]], np.float32), 1, 1)
    assert ids[0, 0] == 1 and gaps[0] == 0.0


# --------------------------------------------------------------------------
# recall@k (Sec. 2.1.1)
# --------------------------------------------------------------------------
def test_recall_definition(oracle_lib):
    res = np.array([[1, 2, 3], [4, 5, 6]], np.uint32)
    gt = np.array([[3, 2, 9, 1], [7, 8, 9, 4]], np.uint32)
    assert oracle_lib.recall(res, gt, 3) == pytest.approx((2 / 3 + 0) / 2)
    assert oracle_lib.recall(res, gt, 1) == pytest.approx(0.0)


# --------------------------------------------------------------------------
# number formats of the reduced-precision form, against torch's CPU casts
# --------------------------------------------------------------------------
def test_bf16_matches_torch_rounding(oracle_lib):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    x = np.concatenate([
        rng.standard_normal(20000).astype(np.float32),
        (rng.standard_normal(2000) * 1e-30).astype(np.float32),
        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -2.5, 65504.0], np.float32),
    ])
    # exact ties: low 16 bits == 0x8000
    b = rng.integers(0, 2 ** 31, size=2000, dtype=np.uint32) & np.uint32(0x7F7F0000) | np.uint32(0x8000)
    x = np.concatenate([x, b.view(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = oracle_lib.bf16(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_e4m3_code_values_match_torch(oracle_lib):
    torch = pytest.importorskip("torch")
    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    for c in range(256):
        v = oracle_lib.e4m3_value(c)
        if math.isnan(codes[c]):
            assert math.isnan(v)
        else:
            assert v == codes[c], c
    assert oracle_lib.e4m3_value(0x7E) == 448.0


def test_e4m3_encode_matches_torch(oracle_lib):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    y = np.concatenate([rng.uniform(-448, 448, 4000), rng.standard_normal(4000) * 0.01,
                        np.array([0.0, 448.0, -448.0, 0.0009765625, 1.0625, 17.0, 0.01953125 / 2])])
    # midpoints between neighbouring codes (exact ties)
    vals = np.array([oracle_lib.e4m3_value(c) for c in range(0x7F)])
    y = np.concatenate([y, (vals[:-1] + vals[1:]) / 2, -(vals[:-1] + vals[1:]) / 2])
    ref = torch.from_numpy(y.astype(np.float32)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = np.array([oracle_lib.e4m3_encode(float(np.float32(v))) for v in y], np.uint8)
    assert np.array_equal(got, ref)


def test_fp8_scale_and_error_bound(oracle_lib):
    rng = np.random.default_rng(6)
    X = (rng.standard_normal((50, 64)) * rng.uniform(1e-3, 1e3, size=(50, 1))).astype(np.float32)
    X[3] = 0
    codes, scales, deq = oracle_lib.quant_fp8(X)
    for r in range(50):
        s = float(scales[r])
        m, e = math.frexp(s)
        assert m == 0.5                                      # a power of two
        amax = float(np.abs(X[r]).max())
        if amax == 0:
            assert s == 1.0 and (deq[r] == 0).all()
            continue
        assert amax <= 448 * s and amax > 224 * s            # smallest such power
        err = np.abs(deq[r].astype(np.float64) - X[r])
        # e4m3: relative 2^-4 for normals, absolute 2^-10 * s below 2^-6 * s
        assert (err <= np.maximum(np.abs(X[r]) * 2.0 ** -4, 2.0 ** -10 * s) + 0).all()


def test_rerank_search_with_exact_storage_equals_plain(oracle_lib, small_graph):
    X, T, Q, G = small_graph
    a = oracle_lib.search(X, G.offsets, G.indices, G.entry, Q[:40], 10, 32)
    b = oracle_lib.search_rerank(X, X, G.offsets, G.indices, G.entry, Q[:40], 10, 32)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all() and (a[2] == b[2]).all()


def test_rerank_hand_worked(oracle_lib):
    g = json.load(open(os.path.join(GOLDEN, "rerank_hand.json")))
    X = np.array(g["X"], np.float32)
    Xq = np.array(g["Xq"], np.float32)
    off, idx = _complete(len(X))
    q = np.array([g["query"]], np.float32)
    for k, e in g["expect"].items():
        ids, ds, _, _, _ = oracle_lib.search_rerank(Xq, X, off, idx, g["entry"], q, int(k), g["L"])
        assert ids[0].tolist() == e["ids"] and ds[0].tolist() == e["dists"]


def test_rerank_complete_graph_equals_brute_force_on_fp32_rows(oracle_lib):
    # with L >= n on a complete graph the final queue holds every row, so the
    # rerank must return the exact kNN on X whatever the stored rows are
    rng = np.random.default_rng(5)
    X = rng.standard_normal((50, 6)).astype(np.float32)
    Xq = rng.standard_normal((50, 6)).astype(np.float32)   # unrelated stored rows
    Q = rng.standard_normal((20, 6)).astype(np.float32)
    off, idx = _complete(50)
    gt, gd = oracle_lib.knn(X, Q, 7)
    ids, ds, _, ev, _ = oracle_lib.search_rerank(Xq, X, off, idx, 3, Q, 7, 50)
    assert (ids == gt).all() and (ds == gd).all()
    assert (ev == 50).all()
    # on the stored rows alone the answer differs
    ids_q, _ = oracle_lib.knn(Xq, Q, 7)
    assert (ids_q != gt).any()


# --------------------------------------------------------------------------
# updates: insertion through the bipartite graph, tombstones (Sec. 6)
# --------------------------------------------------------------------------
def _five_point_state(oracle_lib):
    from oracle.updates import Updatable
    g = json.load(open(os.path.join(GOLDEN, "projection_5pt.json")))
    X = np.array([unit2(a) for a in g["base_angles_deg"]], np.float32)
    T = np.array([unit2(a) for a in g["train_angles_deg"]], np.float32)
    G = oracle_lib.Graph(X, T, g["Nq"], g["M"], g["L"])
    return Updatable.from_graph(G, X, T)


def test_insert_hand_worked(oracle_lib):
    u = json.load(open(os.path.join(GOLDEN, "updates_5pt.json")))
    st = _five_point_state(oracle_lib)
    assert st.rows == u["start_rows"] and st.nout == u["start_nout"]
    for i, a in enumerate(u["inserts_deg"]):
        ids = st.insert(np.array([unit2(a)], np.float32))
        assert ids.tolist() == [5 + i]
    assert st.rows == u["final_rows"]
    assert st.nout == u["final_nout"]


def test_insert_invariants(oracle_lib, small_graph):
    from oracle.updates import Updatable
    X, T, Q, G = small_graph
    st = Updatable.from_graph(G, X, T)
    gen = datagen.Generator(1, n=1500, n_train=1500, n_test=200)
    V = np.concatenate([gen.in_distribution(60), Q[:60]])
    before = sum(len(r) for r in st.nout)
    st.insert(V[:70], L=64)
    st.insert(V[70:], L=64)
    n = st.n
    assert n == G.n + len(V)
    off, idx = st.csr()
    deg = np.diff(off)
    assert deg.max() <= G.M and (deg[G.n:] > 0).all()
    assert _bfs(off, idx, st.entry, n).all()                 # every node, old and new, reachable
    rows = [idx[off[i]:off[i + 1]] for i in range(n)]
    assert all(len(set(r.tolist())) == len(r) and i not in r for i, r in enumerate(rows))
    assert sum(len(r) for r in st.nout) - before <= len(V)    # each v joins at most one N_out
    # a row loses a neighbour only by the selection rule on a full row, and
    # such a row stays full
    old = G.rows("final")
    lost = [i for i in range(G.n) if set(old[i].tolist()) - set(rows[i].tolist())]
    assert all(len(rows[i]) == G.M for i in lost)
    assert any(len(rows[i]) > len(old[i]) for i in range(G.n))


def test_tombstones_exact_on_complete_graph(oracle_lib):
    # a complete graph with L >= n visits everything: the results are the
    # exact nearest non-deleted rows (brute force)
    from oracle.updates import Updatable
    rng = np.random.default_rng(4)
    n, d = 60, 12
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = rng.standard_normal((9, d)).astype(np.float32)
    rows = [[j for j in range(n) if j != i] for i in range(n)]
    st = Updatable(rows, 0, n, n, X, X[:1], [0], [[]])
    dead = rng.choice(n, 25, replace=False)
    st.delete(dead)
    ids, ds = st.search(Q, 10, n)
    S = -(Q.astype(np.float64) @ X.astype(np.float64).T)
    S[:, dead] = np.inf
    want = np.argsort(S, axis=1, kind="stable")[:, :10]
    assert np.array_equal(ids, want.astype(np.uint32))
    assert np.allclose(ds, np.take_along_axis(S, want, 1))
    # more deleted than the queue can skip: padding
    st.delete(range(n))
    ids, ds = st.search(Q, 10, 20)
    assert (ids == NONE).all() and np.isinf(ds).all()
