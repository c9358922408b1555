"""Comparison of GPU search results with the FP64 oracle.

Tolerance (stated for the search path): every returned distance is within
1e-5 * |q| * max|x| of the FP64 value of the same pair (inner products have
no useful relative scale near 0, so the Cauchy-Schwarz bound sets it).

Ids: the GPU computes each distance as FP32 fused multiply-adds along one
lane (EPC*NCH terms) followed by a log2(G)-level shuffle tree, so its error
is at most gamma_m * sum|q_i x_i| <= gamma_m * |q| * |x| with m = EPC*NCH +
log2(G) and gamma_m = m u / (1 - m u), u = 2^-24.  The oracle reports, per
query, the smallest margin of any comparison that decided its search.  When
that margin exceeds twice the bound, the GPU must take the same decisions:
it returns the same id set and distances within tolerance, position by
position.  Queries below the margin are near ties; they are counted, and the
fraction of them whose distances still agree rank by rank is checked.
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
    """Error bound factor of the search's FP32 distances; for reduced
    storage also covers the FP32 rerank."""
    u = 2.0 ** -24
    worst = 0
    for st in {"fp32", storage}:
        g, c, epc = kernel_shape(d, st)
        worst = max(worst, epc * c + int(np.log2(g)) + 1)
    return worst * u / (1 - worst * u)


def compare(gpu_ids, gpu_d, or_ids, or_d, gaps, Q, X, tol_rel=1e-5, max_near_tie_frac=1.0,
            min_agreement=0.99, min_near_same=0.95, label="", storage="fp32"):
    gpu_ids = np.asarray(gpu_ids, np.uint32)
    gpu_d = np.asarray(gpu_d, np.float64)
    Qd = Q.astype(np.float64)
    Xd = X.astype(np.float64)
    qn = np.linalg.norm(Qd, axis=1)
    xmax = float(np.linalg.norm(Xd, axis=1).max())
    tol = tol_rel * qn * xmax
    tau = gamma_search(X.shape[1], storage) * qn * xmax
    nq, k = gpu_ids.shape
    # every returned distance matches the FP64 value of its own pair
    valid = gpu_ids != NONE
    assert (valid == (or_ids != NONE)).all(), f"{label}: padding differs"
    rows, cols = np.nonzero(valid)
    exact = -np.einsum("ij,ij->i", Qd[rows], Xd[gpu_ids[rows, cols].astype(np.int64)])
    err = np.abs(gpu_d[rows, cols] - exact)
    assert (err <= tol[rows]).all(), f"{label}: distance error {err.max():.3e} above tolerance"
    assert np.isinf(gpu_d[~valid]).all()
    sure = gaps > 2 * tau
    # rank by rank the distances agree within tolerance, so any id that
    # differs is a swap among distances closer than the tolerance
    both = valid & (or_ids != NONE)
    rank_ok = np.where(both, np.abs(gpu_d - np.where(both, or_d, 0.0)) <= tol[:, None], valid == (or_ids != NONE))
    q_ok = rank_ok.all(axis=1)
    for q in np.nonzero(sure)[0]:
        assert set(gpu_ids[q].tolist()) == set(or_ids[q].tolist()), f"{label}: certified query {q} ids differ"
        assert q_ok[q], f"{label}: certified query {q} distances differ"
    agree = np.mean([len(set(gpu_ids[q]) & set(or_ids[q])) / k for q in range(nq)])
    near = ~sure
    near_ok = float(q_ok[near].mean()) if near.any() else 1.0
    assert near.mean() <= max_near_tie_frac, f"{label}: {near.mean():.2%} near-tie queries"
    assert near_ok >= min_near_same, f"{label}: only {near_ok:.4f} of near-tie queries match rank by rank"
    assert agree >= min_agreement, f"{label}: id agreement {agree:.4f}"
    out = {"certified": int(sure.sum()), "near_tie": int(near.sum()), "near_tie_rank_match": near_ok,
           "agreement": float(agree), "max_err": float(err.max()) if err.size else 0.0}
    print(f"  {label}: {out}", flush=True)
    return out
