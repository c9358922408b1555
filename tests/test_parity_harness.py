"""The GPU-vs-oracle comparison itself (CPU only): what it accepts and what
it rejects, on oracle results perturbed by hand."""
import numpy as np
import pytest

import datagen
from parity import compare, gamma_search, oracle_explainer


@pytest.fixture(scope="module")
def case(oracle_lib):
    g = datagen.Generator(1, n=1500, n_train=1500, n_test=80)
    X, T, Q = g.base(), g.train(), g.test()
    G = oracle_lib.Graph(X, T, 16, 16, 120)
    oi, od, oh, oe, gaps = oracle_lib.search(X, G.offsets, G.indices, G.entry, Q, 10, 48)
    return X, Q, G, oi, od, oe, gaps


def test_identical_results_pass(oracle_lib, case):
    X, Q, G, oi, od, oe, gaps = case
    r = compare(oi, od.astype(np.float32), oi, od, gaps, Q, X, gpu_evals=oe, or_evals=oe, exact_visits=True)
    assert r["certified"] + r["swap_rule"] == len(Q) and r["certified"] > 0


def test_wrong_id_on_a_certified_query_fails(oracle_lib, case):
    X, Q, G, oi, od, oe, gaps = case
    q = int(np.argmax(gaps))
    assert gaps[q] > gamma_search(X.shape[1])
    bad = oi.copy()
    bad[q, -1] = (int(bad[q, -1]) + 1) % X.shape[0]
    d = od.astype(np.float32)
    d[q, -1] = -(X[bad[q, -1]].astype(np.float64) @ Q[q].astype(np.float64))
    with pytest.raises(AssertionError):
        compare(bad, d, oi, od, gaps, Q, X)


def test_distance_outside_tolerance_fails(oracle_lib, case):
    X, Q, G, oi, od, oe, gaps = case
    d = od.astype(np.float32)
    d[3, 2] += 1e-4 * np.linalg.norm(Q[3]) * np.linalg.norm(X[oi[3, 2]])
    with pytest.raises(AssertionError):
        compare(oi, d, oi, od, gaps, Q, X)


def test_extra_evaluation_on_exact_kernel_fails(oracle_lib, case):
    X, Q, G, oi, od, oe, gaps = case
    ev = oe.copy()
    ev[int(np.argmax(gaps))] += 1
    with pytest.raises(AssertionError):
        compare(oi, od.astype(np.float32), oi, od, gaps, Q, X, gpu_evals=ev, or_evals=oe, exact_visits=True)


def test_swap_within_tolerance_on_near_tie_passes(oracle_lib):
    # nodes 1 and 2 tie exactly; returning 2 instead of 1 is a swap of equal
    # distances and passes; returning 3 (far worse) fails
    X = np.array([[1, 0], [0, 1], [0, 1], [-1, 0]], np.float32)
    n = 4
    off = np.arange(0, n * (n - 1) + 1, n - 1, dtype=np.int64)
    idx = np.array([j for i in range(n) for j in range(n) if j != i], np.uint32)
    Q = np.array([[0, 1]], np.float32)
    oi, od, _, _, gaps = oracle_lib.search(X, off, idx, 0, Q, 1, 1)
    assert gaps[0] == 0.0 and oi[0, 0] == 1
    r = compare(np.array([[2]], np.uint32), np.array([[-1.0]], np.float32), oi, od, gaps, Q, X)
    assert r["swap_rule"] == 1
    with pytest.raises(AssertionError):
        compare(np.array([[3]], np.uint32), np.array([[0.0]], np.float32), oi, od, gaps, Q, X)


def test_divergence_explained_by_perturbation(oracle_lib):
    # A near tie at the first expansion: from entry 0, nodes 1 and 2 score
    # within 1e-8 of each other and only one fits in the queue (L = 1); each
    # leads to a different far node (3 or 4) of clearly different distance.
    # A GPU result ending at either is explained by rounding within the
    # bound; the swap rule alone accepts only the oracle's.
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [1.0, 1e-8, 0.0], [2.0, 0.0, 0.0],
                  [1.5, 0.0, 0.0]], np.float32)
    rows = [[1, 2], [3], [4], [], []]
    off = np.zeros(6, np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array(sum(rows, []), np.uint32)
    Q = np.array([[1.0, 1.0, 0.0]], np.float32)
    oi, od, _, _, gaps = oracle_lib.search(X, off, idx, 0, Q, 1, 1)
    other = 3 if oi[0, 0] == 4 else 4
    gd = np.array([[-(X[other].astype(np.float64) @ Q[0].astype(np.float64))]], np.float32)
    with pytest.raises(AssertionError):
        compare(np.array([[other]], np.uint32), gd, oi, od, gaps, Q, X)
    r = compare(np.array([[other]], np.uint32), gd, oi, od, gaps, Q, X,
                explain=oracle_explainer(oracle_lib, X, off, idx, 0, Q, 1, 1))
    assert r["explained"] == 1
