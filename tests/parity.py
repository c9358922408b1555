"""Comparison of GPU search results with the FP64 oracle.

Tolerance (stated for the search path): every returned distance is within
1e-5 * |q| * |x| of the FP64 value of the same pair (inner products have no
useful relative scale near 0, so the Cauchy-Schwarz bound of the pair sets
it).

Ids.  The GPU computes each distance as FP32 fused multiply-adds along one
lane (EPC * NCH terms) followed by a log2(G)-level shuffle tree, so its error
is at most gamma_m * S with S = sum_i |q_i x_i| and m = EPC * NCH + log2(G)
+ 1, gamma_m = m u / (1 - m u), u = 2^-24.  The oracle reports each query's
decision margin: the smallest (delta_b - delta_a) / (S_a + S_b) over the
pairs whose order decides the search (selection, what each expansion keeps
against what it drops, the first k against the rest).  Above gamma_m the GPU
takes every one of those decisions as the oracle does ("certified"): the
same k ids, the same number of rows scored with an exact visited set, and
rank by rank distances within tolerance (a differing order inside the k is a
swap of near-equal distances).

Every other query ("near tie") must satisfy the swap rule: rank by rank the
distances agree within tolerance, and any returned id outside the oracle's k
lies within tolerance of the oracle's k-th distance.  A near-tie query that
fails it is accepted only if the oracle itself returns the GPU's ids when its
distances are moved by at most gamma_m * S (the perturbed oracle search over
a few seeds): the GPU result is then what some rounding within the proven
bound produces.  Nothing else passes.
"""
import numpy as np

NONE = 0xFFFFFFFF


# (G, NCH) per dimension class (d <= 64, 128, 224, 256, 512, 1024) and storage;
# a chunk holds EPC elements (4 FP32, 8 BF16, 16 E4M3).
CLASS_MAX_D = (64, 128, 224, 256, 512, 1024)
SHAPES = {
    "fp32": (4, ((16, 1), (16, 2), (8, 7), (16, 4), (16, 8), (32, 8))),
    "bf16": (8, ((8, 1), (16, 1), (8, 4), (8, 4), (16, 4), (32, 4))),
    "fp8": (16, ((4, 2), (8, 2), (8, 2), (8, 3), (16, 3), (32, 3))),
}


def kernel_shape(d, storage="fp32"):
    """(G, NCH, EPC) the search kernel uses for dimension d and storage."""
    epc, table = SHAPES[storage]
    for lim, gn in zip(CLASS_MAX_D, table):
        if d <= lim:
            return gn[0], gn[1], epc
    raise ValueError(d)


def gamma_search(d, storage="fp32"):
    """Error bound factor (relative to S = sum |q_i x_i|) of the search's FP32
    distances; for reduced storage it also covers the FP32 rerank."""
    u = 2.0 ** -24
    worst = 0
    for st in {"fp32", storage}:
        g, c, epc = kernel_shape(d, st)
        worst = max(worst, epc * c + int(np.log2(g)) + 1)
    return worst * u / (1 - worst * u)


def _delta64(Q, X, q, ids):
    ids = np.asarray(ids, np.int64)
    return -(X[ids].astype(np.float64) @ Q[q].astype(np.float64))


def compare(gpu_ids, gpu_d, or_ids, or_d, gaps, Q, X, storage="fp32", label="", gpu_evals=None, or_evals=None,
            exact_visits=False, explain=None, tol_rel=1e-5, seeds=24):
    """Checks one batch of GPU results against the oracle's (see the module
    docstring).  explain(q, eps, seed) -> ids of the oracle's perturbed search
    for query q; without it a near-tie query must meet the swap rule."""
    gpu_ids = np.asarray(gpu_ids, np.uint32)
    gpu_d = np.asarray(gpu_d, np.float64)
    or_ids = np.asarray(or_ids, np.uint32)
    or_d = np.asarray(or_d, np.float64)
    nq, k = gpu_ids.shape
    qn = np.linalg.norm(Q.astype(np.float64), axis=1)
    xn = np.linalg.norm(X.astype(np.float64), axis=1)
    gamma = gamma_search(X.shape[1], storage)
    valid = gpu_ids != NONE
    assert (valid == (or_ids != NONE)).all(), f"{label}: padding differs"
    assert np.isinf(gpu_d[~valid]).all(), f"{label}: padded distance not +inf"
    sure = gaps > gamma
    worst = 0.0
    stats = {"certified": 0, "swap_rule": 0, "explained": 0}
    fails = []
    for q in range(nq):
        v = valid[q]
        gi = gpu_ids[q][v].astype(np.int64)
        oi = or_ids[q][v].astype(np.int64)
        # every returned distance is its own pair's FP64 value within tolerance
        exact = _delta64(Q, X, q, gi)
        err = np.abs(gpu_d[q][v] - exact)
        tol_own = tol_rel * qn[q] * xn[gi]
        if err.size:
            worst = max(worst, float((err / (qn[q] * xn[gi])).max()))
        if not (err <= tol_own).all():
            fails.append(f"query {q}: distance error {float(err.max()):.3e} above tolerance")
            continue
        # rank by rank, against the oracle's distance at the same rank
        tol_rank = tol_rel * qn[q] * np.maximum(xn[gi], xn[oi])
        rank_ok = bool((np.abs(gpu_d[q][v] - or_d[q][v]) <= tol_rank).all())
        if sure[q]:
            if set(gi.tolist()) != set(oi.tolist()) or not rank_ok:
                fails.append(f"certified query {q} (margin {gaps[q]:.3e} > {gamma:.3e}) differs")
                continue
            if exact_visits and gpu_evals is not None and int(gpu_evals[q]) != int(or_evals[q]):
                fails.append(f"certified query {q}: {int(gpu_evals[q])} rows scored, oracle {int(or_evals[q])}")
                continue
            stats["certified"] += 1
            continue
        # near tie: the swap rule
        extra = np.setdiff1d(gi, oi)
        swap_ok = rank_ok
        if swap_ok and extra.size:
            kth = or_d[q][v][-1]
            ok_x = np.abs(_delta64(Q, X, q, extra) - kth) <= tol_rel * qn[q] * np.maximum(xn[extra], xn[oi[-1]])
            swap_ok = bool(ok_x.all())
        if swap_ok:
            stats["swap_rule"] += 1
            continue
        # otherwise the oracle must produce the GPU's ids under distance
        # errors within the bound
        if explain is not None and any(set(explain(q, gamma, s)[v].tolist()) == set(gi.tolist())
                                       for s in range(seeds)):
            stats["explained"] += 1
            continue
        fails.append(f"near-tie query {q} (margin {gaps[q]:.3e}): ids {gi.tolist()} vs oracle {oi.tolist()}")
    stats.update({"near_tie": int((~sure).sum()), "queries": int(nq), "gamma": gamma, "max_err_rel": worst})
    print(f"  {label}: {stats}", flush=True)
    assert not fails, f"{label}: {len(fails)} of {nq} queries fail: " + "; ".join(fails[:5])
    return stats


def oracle_explainer(oracle_lib, X, off, idx, entry, Q, k, L, Xq=None):
    """explain(q, eps, seed) for compare(): the oracle's search of query q
    with distances moved by eps * S (sign per node from the seed)."""
    def explain(q, eps, seed):
        ids, _, _, _ = oracle_lib.search_perturbed(X, off, idx, entry, Q[q:q + 1], k, L,
                                                   eps, seed, Xq=Xq)
        return ids[0]
    return explain
