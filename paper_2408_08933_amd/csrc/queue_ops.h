// Sorted-queue merge shared by the search kernels (FP32 keys) and the
// construction-time canonical search (FP64 keys).  One wavefront owns the
// queue; all arrays live in LDS.
#pragma once

#include <climits>

#include "rg_internal.h"
#include "wave_ops.h"

namespace rg {

template <typename K>
struct QueueLds {
    K *qd;          // queue keys, ascending
    uint32_t *qi;   // queue ids, top bit = expanded
    K *cd;          // candidate batch keys
    uint32_t *ci;   // candidate batch ids
    K *sd;          // survivors (scratch)
    uint32_t *si;
    int32_t *slb;
};

template <typename K>
__device__ __forceinline__ int lower_bound_q(const K *qd, const uint32_t *qi, int qn, K kd, uint32_t kid) {
    int lo = 0, hi = qn;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (kless(qd[mid], qi[mid] & ~kExpanded, kd, kid))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// #{t < S : slb[t] <= i}, slb non-decreasing
__device__ __forceinline__ int count_le(const int32_t *slb, int S, int i) {
    int lo = 0, hi = S;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (slb[mid] <= i)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Merge the candidate batch s.cd/s.ci[0..cnt) into the queue s.qd/s.qi[0..qn):
// sort the batch, keep the entries that beat the queue's last key (all, if
// the queue is not full) and are not already queued, then move queue
// entries and survivors to their merged places, truncating at Leff.  The
// result is the best Leff of queue u batch, whatever the batch order.
// When at most this many candidates survive (they beat the last key of a
// full queue and are not queued yet), they are ordered by counting the
// survivors ahead of each one instead of sorting the whole batch.
constexpr int kRankByCount = 32;

// QR = queue capacity / 64: each lane holds QR of the entries that move.
template <int E, typename K, int QR = kMaxL / 64>
__device__ __forceinline__ void merge_batch(const QueueLds<K> &s, int cnt, int Leff, int &qn, int &ptr) {
    const int lane = lane_id();
    const bool full = qn == Leff;
    const K lastd = full ? s.qd[Leff - 1] : (K)0;
    const uint32_t lasti = full ? (s.qi[Leff - 1] & ~kExpanded) : 0u;
    int total = 0;
    bool sorted = false;
    if constexpr (E == 1) {
        // one candidate per lane: find the survivors and their queue ranks
        K kc = (K)__builtin_inf();
        uint32_t ic = kNone;
        bool sv = false;
        int lbc = 0;
        if (lane < cnt) {
            kc = s.cd[lane];
            ic = s.ci[lane];
            sv = ic != kNone && (!full || kless(kc, ic, lastd, lasti));
        }
        if (sv) {
            lbc = lower_bound_q(s.qd, s.qi, qn, kc, ic);
            if (lbc < qn && (s.qi[lbc] & ~kExpanded) == ic) sv = false;  // already queued
        }
        const uint64_t m = ballot64(sv);
        total = (int)__popcll(m);
        if (total == 0) return;
        if (total <= kRankByCount) {
            // survivor order = number of survivors that precede it
            __syncthreads();
            if (sv) {
                s.sd[lanes_below(m)] = kc;
                s.si[lanes_below(m)] = ic;
            }
            __syncthreads();
            int rank = 0;
            if (sv)
                for (int t = 0; t < total; ++t) rank += kless(s.sd[t], s.si[t], kc, ic) ? 1 : 0;
            __syncthreads();
            if (sv) {
                s.sd[rank] = kc;
                s.si[rank] = ic;
                s.slb[rank] = lbc;
            }
            __syncthreads();
            sorted = true;
        }
    } else if (full) {  // nothing to do unless some candidate beats the last entry
        bool any = false;
        for (int i = lane; i < cnt; i += 64) any |= kless(s.cd[i], s.ci[i], lastd, lasti);
        if (ballot64(any) == 0) return;
    }
    if (!sorted) {
        K k[E];
        uint32_t id[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = lane * E + e;
            k[e] = i < cnt ? s.cd[i] : (K)__builtin_inf();
            id[e] = i < cnt ? s.ci[i] : kNone;
        }
        wave_sort<E, K>(k, id);
        int lb[E];
        bool sv[E];
        int mine = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            sv[e] = id[e] != kNone && (!full || kless(k[e], id[e], lastd, lasti));
            lb[e] = 0;
            if (sv[e]) {
                lb[e] = lower_bound_q(s.qd, s.qi, qn, k[e], id[e]);
                if (lb[e] < qn && (s.qi[lb[e]] & ~kExpanded) == id[e]) sv[e] = false;  // already queued
            }
            mine += sv[e] ? 1 : 0;
        }
        // order-preserving compaction: exclusive prefix of per-lane counts
        int incl = mine;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        total = __shfl(incl, 63);
        int w = incl - mine;
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (sv[e]) {
                s.sd[w] = k[e];
                s.si[w] = id[e];
                s.slb[w] = lb[e];
                ++w;
            }
        }
        __syncthreads();
        if (total == 0) return;
    }
    const int lbmin = s.slb[0];
    // entries of the queue that move, and their new places
    constexpr int R = QR;
    K md[R];
    uint32_t mi[R];
    int mp[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = lbmin + lane + 64 * r;
        mp[r] = INT_MAX;
        if (i < qn) {
            md[r] = s.qd[i];
            mi[r] = s.qi[i];
            mp[r] = i + count_le(s.slb, total, i);
        }
    }
    K pd[2];
    uint32_t pi[2];
    int pp[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int t = lane + 64 * r;
        pp[r] = INT_MAX;
        if (t < total) {
            pd[r] = s.sd[t];
            pi[r] = s.si[t];
            pp[r] = s.slb[t] + t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (mp[r] < Leff) {
            s.qd[mp[r]] = md[r];
            s.qi[mp[r]] = mi[r];
        }
#pragma unroll
    for (int r = 0; r < 2; ++r)
        if (pp[r] < Leff) {
            s.qd[pp[r]] = pd[r];
            s.qi[pp[r]] = pi[r];
        }
    qn = min(Leff, qn + total);
    ptr = min(ptr, lbmin);
    __syncthreads();
}


}  // namespace rg
