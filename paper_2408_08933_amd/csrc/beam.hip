// Batched beam search over the RoarGraph index (Sec. 4.3), one 64-lane
// wavefront (= one workgroup) per query on gfx950.
//
// Per query, in LDS:
//   * the queue: the best L_eff (delta, id) pairs seen, sorted ascending, the
//     id's top bit marking "expanded";
//   * an open-addressing visited table of node ids.  When it passes half
//     load it is cleared; a node seen again is then scored again and dropped
//     at the merge if it is already queued.  Because the queue's last key
//     only decreases once the queue is full, a forgotten node that was
//     rejected or evicted is rejected again, so clearing changes only the
//     work done, never the result;
//   * the candidate batch of the current expansion.
// Per expansion: pick the first unexpanded queue entry, read its adjacency
// row (ELL, one id per lane), filter through the visited table, gather the
// new neighbours' rows (G lanes per row, float4 loads, coalesced), reduce
// the FP32 dot products inside each G-lane group with xor shuffles, sort the
// batch in registers, and merge the entries that beat the queue's last key.
// The search stops when every queue entry is expanded.
//
// Dot products: lane j of a group accumulates, with fused multiply-adds in
// order, the coordinates 4c..4c+3 of chunks c = j, j+G, j+2G, ...; then the
// G partial sums are added by a log2(G)-level xor tree.  A distance is
// therefore a fixed function of (query, row) whichever group computes it.
#include "rg_internal.h"
#include "queue_ops.h"
#include "wave_ops.h"

#include <climits>

namespace rg {
namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int kCand = 128;  // candidate-batch capacity (>= the largest ELL width)

struct Lds {
    float *qd;
    uint32_t *qi;
    float *cd;
    uint32_t *ci;
    float *sd;
    uint32_t *si;
    int32_t *slb;
    uint32_t *htab;
};

__device__ __forceinline__ Lds carve(unsigned char *p, int Leff) {
    Lds s;
    s.qd = reinterpret_cast<float *>(p);
    s.qi = reinterpret_cast<uint32_t *>(s.qd + Leff);
    s.cd = reinterpret_cast<float *>(s.qi + Leff);
    s.ci = reinterpret_cast<uint32_t *>(s.cd + kCand);
    s.sd = reinterpret_cast<float *>(s.ci + kCand);
    s.si = reinterpret_cast<uint32_t *>(s.sd + kCand);
    s.slb = reinterpret_cast<int32_t *>(s.si + kCand);
    s.htab = reinterpret_cast<uint32_t *>(s.slb + kCand);
    return s;
}

typedef float f32x2 __attribute__((ext_vector_type(2)));


template <int G, int NCH>
__device__ __forceinline__ void load_query(const float *q, int d, float4 (&qv)[NCH]) {
    const int j = lane_id() % G;
#pragma unroll
    for (int t = 0; t < NCH; ++t) {
        const int e = 4 * (j + G * t);
        qv[t].x = e + 0 < d ? q[e + 0] : 0.f;
        qv[t].y = e + 1 < d ? q[e + 1] : 0.f;
        qv[t].z = e + 2 < d ? q[e + 2] : 0.f;
        qv[t].w = e + 3 < d ? q[e + 3] : 0.f;
    }
}

// This lane's partial dot product of the query with row u (kNone -> 0).
template <int G, int NCH, int ST>
__device__ __forceinline__ float row_partial(const SearchArgs &a, uint32_t u, const float4 (&qv)[NCH],
                                             int nch) {
    float acc = 0.f;
    if (u == kNone) return acc;
    const int j = lane_id() % G;
    if constexpr (ST == RG_STORE_FP32) {
        const float4 *row = reinterpret_cast<const float4 *>(a.base + (size_t)u * a.pitch);
        float4 x[NCH];
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
            const int c = j + G * t;
            x[t] = c < nch ? row[c] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
            acc = fmaf(qv[t].x, x[t].x, acc);
            acc = fmaf(qv[t].y, x[t].y, acc);
            acc = fmaf(qv[t].z, x[t].z, acc);
            acc = fmaf(qv[t].w, x[t].w, acc);
        }
    } else if constexpr (ST == RG_STORE_BF16) {
        const uint2 *row = reinterpret_cast<const uint2 *>(a.base_bf16 + (size_t)u * a.pitch);
        uint2 x[NCH];
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
            const int c = j + G * t;
            x[t] = c < nch ? row[c] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
            acc = fmaf(qv[t].x, __uint_as_float(x[t].x << 16), acc);
            acc = fmaf(qv[t].y, __uint_as_float(x[t].x & 0xFFFF0000u), acc);
            acc = fmaf(qv[t].z, __uint_as_float(x[t].y << 16), acc);
            acc = fmaf(qv[t].w, __uint_as_float(x[t].y & 0xFFFF0000u), acc);
        }
    } else {
        const uint32_t *row = reinterpret_cast<const uint32_t *>(a.base_fp8 + (size_t)u * a.pitch8);
        uint32_t x[NCH];
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
            const int c = j + G * t;
            x[t] = c < nch ? row[c] : 0u;
        }
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
            // gfx950 converts OCP E4M3 pairs exactly (every code is a float)
            const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)x[t], false);
            const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)x[t], true);
            acc = fmaf(qv[t].x, lo[0], acc);
            acc = fmaf(qv[t].y, lo[1], acc);
            acc = fmaf(qv[t].z, hi[0], acc);
            acc = fmaf(qv[t].w, hi[1], acc);
        }
    }
    return acc;
}

template <int G>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// delta of this group's row u (uniform within the group)
template <int G, int ST>
__device__ __forceinline__ float finish_delta(const SearchArgs &a, uint32_t u, float sum) {
    if constexpr (ST == RG_STORE_FP8E4M3) {
        const float s = u == kNone ? 1.f : a.scale_fp8[u];
        return -(s * sum);
    } else {
        return -sum;
    }
}

// Score ids[0..cnt) (LDS) into dout[0..cnt) (LDS); two rows per group in flight.
template <int G, int NCH, int ST>
__device__ __forceinline__ void score_batch(const SearchArgs &a, const float4 (&qv)[NCH], int nch,
                                            const uint32_t *ids, uint32_t idmask, float *dout, int cnt) {
    constexpr int NG = 64 / G;
    const int g = lane_id() / G, j = lane_id() % G;
    for (int p = 0; p < cnt; p += 2 * NG) {
        const int s0 = p + g, s1 = p + NG + g;
        const uint32_t u0 = s0 < cnt ? (ids[s0] & idmask) : kNone;
        const uint32_t u1 = s1 < cnt ? (ids[s1] & idmask) : kNone;
        float a0 = row_partial<G, NCH, ST>(a, u0, qv, nch);
        float a1 = row_partial<G, NCH, ST>(a, u1, qv, nch);
        a0 = group_sum<G>(a0);
        a1 = group_sum<G>(a1);
        if (j == 0) {
            if (s0 < cnt) dout[s0] = finish_delta<G, ST>(a, u0, a0);
            if (s1 < cnt) dout[s1] = finish_delta<G, ST>(a, u1, a1);
        }
    }
}

__device__ __forceinline__ uint32_t hslot(uint32_t u, int hb) { return (u * 2654435761u) >> (32 - hb); }

// Visited set kept in LDS: open addressing, cleared when it passes half load
// (clearing only costs re-scoring; see the file comment).
struct VisitLds {
    uint32_t *htab;
    int hb, H, hcount;
    __device__ __forceinline__ void clear() {
        for (int i = lane_id(); i < H; i += 64) htab[i] = kEmpty;
        hcount = 0;
    }
    __device__ __forceinline__ void mark_entry(uint32_t u) {  // lane 0, table just cleared
        htab[hslot(u, hb)] = u;
    }
    __device__ __forceinline__ void begin_hop(int ell) {
        if (hcount + ell > (H >> 1)) {
            clear();
            __syncthreads();
        }
    }
    __device__ __forceinline__ bool insert(uint32_t u) {
        const uint32_t hmask = (uint32_t)H - 1u;
        uint32_t h = hslot(u, hb);
        for (int probe = 0; probe < H; ++probe) {
            const uint32_t old = atomicCAS(&htab[h], kEmpty, u);
            if (old == kEmpty) return true;
            if (old == u) return false;
            h = (h + 1u) & hmask;
        }
        return false;
    }
    __device__ __forceinline__ void added(int k) { hcount += k; }
};

// Exact visited set: one bit per base node in device memory, owned by the
// workgroup for the query it is running; test-and-set with vector atomics.
struct VisitBitmap {
    uint32_t *bm;
    int64_t words;  // multiple of 4
    __device__ __forceinline__ void clear() {
        uint4 *b4 = reinterpret_cast<uint4 *>(bm);
        const uint4 z = make_uint4(0u, 0u, 0u, 0u);
        for (int64_t i = lane_id(); i < (words >> 2); i += 64) b4[i] = z;
        __threadfence();
    }
    __device__ __forceinline__ void mark_entry(uint32_t u) { atomicOr(&bm[u >> 5], 1u << (u & 31u)); }
    __device__ __forceinline__ void begin_hop(int) {}
    __device__ __forceinline__ bool insert(uint32_t u) {
        const uint32_t bit = 1u << (u & 31u);
        return (atomicOr(&bm[u >> 5], bit) & bit) == 0u;
    }
    __device__ __forceinline__ void added(int) {}
};

// Expansions until done or `budget` expansions were made.
template <int G, int NCH, int ST, class VIS>
__device__ __forceinline__ void run_search(const SearchArgs &a, const float4 (&qv)[NCH], const Lds &s, VIS &vis,
                                           int &qn, int &ptr, uint32_t &hops, uint32_t &evals, int budget,
                                           bool &done) {
    const int lane = lane_id();
    const int Leff = a.Leff, ell = a.ell, nch = (a.d + 3) >> 2;
    done = false;
    for (; budget > 0; --budget) {
        int sel = -1;
        for (int b = ptr; b < qn; b += 64) {
            const int i = b + lane;
            const bool un = i < qn && !(s.qi[i] & kExpanded);
            const uint64_t m = ballot64(un);
            if (m) {
                sel = b + (int)__builtin_ctzll(m);
                break;
            }
        }
        if (sel < 0) {
            done = true;
            break;
        }
        ptr = sel;
        const uint32_t v = s.qi[sel];
        __syncthreads();
        if (lane == 0) s.qi[sel] = v | kExpanded;
        ++hops;
        vis.begin_hop(ell);
        int nnew = 0;
        for (int b = 0; b < ell; b += 64) {
            const int e = b + lane;
            const uint32_t u = e < ell ? a.adj[(size_t)v * ell + e] : kNone;
            const bool fresh = u != kNone && vis.insert(u);
            const uint64_t m = ballot64(fresh);
            if (fresh) s.ci[nnew + lanes_below(m)] = u;
            nnew += (int)__popcll(m);
        }
        vis.added(nnew);
        evals += (uint32_t)nnew;
        __syncthreads();
        if (nnew == 0) continue;
        score_batch<G, NCH, ST>(a, qv, nch, s.ci, 0xFFFFFFFFu, s.cd, nnew);
        __syncthreads();
        const QueueLds<float> ql{s.qd, s.qi, s.cd, s.ci, s.sd, s.si, s.slb};
        if (nnew <= 64)
            merge_batch<1, float>(ql, nnew, Leff, qn, ptr);
        else
            merge_batch<2, float>(ql, nnew, Leff, qn, ptr);
    }
}

// Queue = [entry]; the visited set is cleared and holds the entry.
template <int G, int NCH, int ST, class VIS>
__device__ __forceinline__ void init_state(const SearchArgs &a, const float4 (&qv)[NCH], const Lds &s, VIS &vis,
                                           int &qn, int &ptr, uint32_t &hops, uint32_t &evals) {
    const int lane = lane_id();
    vis.clear();
    const uint32_t u = lane < G ? a.entry : kNone;
    float acc = row_partial<G, NCH, ST>(a, u, qv, (a.d + 3) >> 2);
    acc = group_sum<G>(acc);
    __syncthreads();
    if (lane == 0) {
        s.qd[0] = finish_delta<G, ST>(a, a.entry, acc);
        s.qi[0] = a.entry;
        vis.mark_entry(a.entry);
    }
    vis.added(1);
    qn = 1;
    ptr = 0;
    hops = 0;
    evals = 1;
    __syncthreads();
}

// Rescore the final queue against FP32 rows and sort it (reduced-precision storage).
template <int G, int NCH>
__device__ __forceinline__ void rerank_queue(const SearchArgs &a, const float4 (&qv)[NCH], const Lds &s, int qn) {
    score_batch<G, NCH, RG_STORE_FP32>(a, qv, (a.d + 3) >> 2, s.qi, ~kExpanded, s.qd, qn);
    __syncthreads();
    constexpr int E = kMaxL / 64;
    const int lane = lane_id();
    float k[E];
    uint32_t id[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = lane * E + e;
        k[e] = i < qn ? s.qd[i] : __builtin_inff();
        id[e] = i < qn ? (s.qi[i] & ~kExpanded) : kNone;
    }
    wave_sort<E>(k, id);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = lane * E + e;
        if (i < qn) {
            s.qd[i] = k[e];
            s.qi[i] = id[e];
        }
    }
    __syncthreads();
}

template <int G, int NCH, int ST>
__device__ __forceinline__ void write_result(const SearchArgs &a, const Lds &s, int64_t q, int qn, uint32_t hops,
                                             uint32_t evals) {
    const int lane = lane_id();
    for (int i = lane; i < a.k; i += 64) {
        a.out_ids[q * a.k + i] = i < qn ? (s.qi[i] & ~kExpanded) : kNone;
        a.out_d[q * a.k + i] = i < qn ? s.qd[i] : __builtin_inff();
    }
    if (lane == 0) {
        if (a.out_hops) a.out_hops[q] = hops;
        if (a.out_evals) a.out_evals[q] = evals;
    }
}

// One query per workgroup, visited set in LDS.
template <int G, int NCH, int ST>
__global__ __launch_bounds__(64) void k_search(SearchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t q = blockIdx.x;
    const Lds s = carve(smem, a.Leff);
    VisitLds vis{s.htab, a.hash_bits, 1 << a.hash_bits, 0};
    float4 qv[NCH];
    load_query<G, NCH>(a.queries + q * a.d, a.d, qv);
    int qn, ptr;
    uint32_t hops, evals;
    bool done;
    init_state<G, NCH, ST>(a, qv, s, vis, qn, ptr, hops, evals);
    run_search<G, NCH, ST>(a, qv, s, vis, qn, ptr, hops, evals, INT_MAX, done);
    if constexpr (ST != RG_STORE_FP32) rerank_queue<G, NCH>(a, qv, s, qn);
    write_result<G, NCH, ST>(a, s, q, qn, hops, evals);
}

// Persistent grid: each workgroup stays resident, takes queries from a
// device counter until none are left, and keeps an exact visited bitmap
// (one bit per base node) in device memory, so LDS holds only the queue and
// the candidate batch and many more queries are in flight per CU.
template <int G, int NCH, int ST>
__global__ __launch_bounds__(64) void k_search_persistent(SearchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Lds s = carve(smem, a.Leff);
    VisitBitmap vis{a.bitmap + (size_t)blockIdx.x * a.bm_words, a.bm_words};
    const int lane = lane_id();
    for (;;) {
        int q = 0;
        if (lane == 0) q = (int)atomicAdd(a.work, 1u);
        q = __shfl(q, 0);
        if ((int64_t)q >= a.nq) break;
        float4 qv[NCH];
        load_query<G, NCH>(a.queries + (int64_t)q * a.d, a.d, qv);
        int qn, ptr;
        uint32_t hops, evals;
        bool done;
        init_state<G, NCH, ST>(a, qv, s, vis, qn, ptr, hops, evals);
        run_search<G, NCH, ST>(a, qv, s, vis, qn, ptr, hops, evals, INT_MAX, done);
        if constexpr (ST != RG_STORE_FP32) rerank_queue<G, NCH>(a, qv, s, qn);
        write_result<G, NCH, ST>(a, s, q, qn, hops, evals);
        __syncthreads();
    }
}

// One scheduler step of the serving loop: advance each listed slot by up to
// hops_budget expansions, keeping its whole state in device memory.
template <int G, int NCH, int ST>
__global__ __launch_bounds__(64) void k_serve_step(SlotArgs sa) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int slot = sa.active[blockIdx.x];
    SearchArgs a = sa.s;
    a.k = sa.slot_k[slot];
    a.Leff = max(sa.slot_L[slot], a.k);
    const Lds s = carve(smem, a.Leff);
    const int lane = lane_id();
    const int H = 1 << a.hash_bits;
    float4 qv[NCH];
    load_query<G, NCH>(sa.slot_q + (size_t)slot * a.d, a.d, qv);
    int32_t *st = sa.slot_state + (size_t)slot * 8;
    float *gqd = sa.slot_qd + (size_t)slot * kMaxL;
    uint32_t *gqi = sa.slot_qi + (size_t)slot * kMaxL;
    uint32_t *gh = sa.slot_hash + ((size_t)slot << a.hash_bits);
    int qn, ptr;
    uint32_t hops, evals;
    VisitLds vis{s.htab, a.hash_bits, H, 0};
    if (st[0] == 0) {
        init_state<G, NCH, ST>(a, qv, s, vis, qn, ptr, hops, evals);
    } else {
        qn = st[0];
        ptr = st[1];
        vis.hcount = st[2];
        hops = (uint32_t)st[3];
        evals = (uint32_t)st[4];
        for (int i = lane; i < qn; i += 64) {
            s.qd[i] = gqd[i];
            s.qi[i] = gqi[i];
        }
        for (int i = lane; i < H; i += 64) s.htab[i] = gh[i];
        __syncthreads();
    }
    bool done;
    run_search<G, NCH, ST>(a, qv, s, vis, qn, ptr, hops, evals, sa.hops_budget, done);
    if (done) {
        if constexpr (ST != RG_STORE_FP32) rerank_queue<G, NCH>(a, qv, s, qn);
        int pos = 0;
        if (lane == 0) pos = (int)atomicAdd(sa.out_count, 1u);
        pos = __shfl(pos, 0);
        ServeRecord *r = sa.out_rec + pos;
        for (int i = lane; i < a.k; i += 64) {
            r->ids[i] = i < qn ? (s.qi[i] & ~kExpanded) : kNone;
            r->d[i] = i < qn ? s.qd[i] : __builtin_inff();
        }
        if (lane == 0) {
            r->slot = slot;
            r->qn = qn;
            r->hops = hops;
            r->evals = evals;
            st[0] = 0;
        }
    } else {
        for (int i = lane; i < qn; i += 64) {
            gqd[i] = s.qd[i];
            gqi[i] = s.qi[i];
        }
        for (int i = lane; i < H; i += 64) gh[i] = s.htab[i];
        if (lane == 0) {
            st[0] = qn;
            st[1] = ptr;
            st[2] = vis.hcount;
            st[3] = (int32_t)hops;
            st[4] = (int32_t)evals;
        }
    }
}

__global__ __launch_bounds__(64) void k_serve_admit(int32_t n, const int32_t *slots, const float *q,
                                                   const int32_t *k, const int32_t *L, int32_t d, float *slot_q,
                                                   int32_t *slot_k, int32_t *slot_L, int32_t *slot_state) {
    const int i = blockIdx.x;
    const int s = slots[i];
    for (int j = threadIdx.x; j < d; j += 64) slot_q[(size_t)s * d + j] = q[(size_t)i * d + j];
    if (threadIdx.x < 8) slot_state[(size_t)s * 8 + threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        slot_k[s] = k[i];
        slot_L[s] = L[i];
    }
}

template <int G, int NCH, int ST>
int launch_one(const SearchArgs &a, hipStream_t stream) {
    const size_t lds = search_lds_bytes(a.Leff, a.ell, a.hash_bits);
    hipLaunchKernelGGL((k_search<G, NCH, ST>), dim3((unsigned)a.nq), dim3(64), lds, stream, a);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

template <int G, int NCH, int ST>
int launch_persistent(const SearchArgs &a, hipStream_t stream) {
    const size_t lds = search_lds_bytes(a.Leff, a.ell, 0);
    hipLaunchKernelGGL((k_search_persistent<G, NCH, ST>), dim3((unsigned)a.grid), dim3(64), lds, stream, a);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

template <int G, int NCH, int ST>
int occupancy_of(int Leff, int *blocks_per_cu) {
    const size_t lds = search_lds_bytes(Leff, 0, 0);
    RG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_search_persistent<G, NCH, ST>, 64, lds));
    return RG_OK;
}

template <int G, int NCH, int ST>
int launch_step(const SlotArgs &sa, hipStream_t stream) {
    const size_t lds = search_lds_bytes(kMaxL, sa.s.ell, sa.s.hash_bits);
    hipLaunchKernelGGL((k_serve_step<G, NCH, ST>), dim3((unsigned)sa.n_active), dim3(64), lds, stream, sa);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

// (G, NCH) for a dimension: G lanes per row, NCH float4 chunks per lane.
template <template <int, int, int> class F, int ST, typename Arg>
int dispatch_dim(int d, const Arg &a, hipStream_t stream) {
    const int nch = (d + 3) / 4;
    if (nch <= 16) return F<16, 1, ST>::run(a, stream);
    if (nch <= 32) return F<16, 2, ST>::run(a, stream);
    if (nch <= 56) return F<8, 7, ST>::run(a, stream);
    if (nch <= 64) return F<16, 4, ST>::run(a, stream);
    if (nch <= 128) return F<16, 8, ST>::run(a, stream);
    if (nch <= 256) return F<32, 8, ST>::run(a, stream);
    set_error("search: d > 1024 is not supported");
    return RG_EINVAL;
}

template <int G, int NCH, int ST>
struct SearchLaunch {
    static int run(const SearchArgs &a, hipStream_t s) { return launch_one<G, NCH, ST>(a, s); }
};
template <int G, int NCH, int ST>
struct PersistentLaunch {
    static int run(const SearchArgs &a, hipStream_t s) { return launch_persistent<G, NCH, ST>(a, s); }
};
template <int G, int NCH, int ST>
struct OccLaunch {
    static int run(const SearchArgs &a, hipStream_t) { return occupancy_of<G, NCH, ST>(a.Leff, a.occ_out); }
};
template <int G, int NCH, int ST>
struct StepLaunch {
    static int run(const SlotArgs &a, hipStream_t s) { return launch_step<G, NCH, ST>(a, s); }
};

}  // namespace

size_t search_lds_bytes(int Leff, int ell, int hash_bits) {
    (void)ell;
    return (size_t)Leff * 8 + (size_t)kCand * 20 + (hash_bits > 0 ? ((size_t)4 << hash_bits) : 0);
}

int default_hash_bits(int Leff) {
    // table of about 16 entries per queue slot, 2^11 .. 2^13
    int hb = 11;
    while (hb < 13 && (1 << hb) < 16 * Leff) ++hb;
    return hb;
}

int launch_search(const SearchArgs &a, hipStream_t stream) {
    if (a.nq == 0) return RG_OK;
    switch (a.storage) {
    case RG_STORE_FP32: return dispatch_dim<SearchLaunch, RG_STORE_FP32>(a.d, a, stream);
    case RG_STORE_BF16: return dispatch_dim<SearchLaunch, RG_STORE_BF16>(a.d, a, stream);
    case RG_STORE_FP8E4M3: return dispatch_dim<SearchLaunch, RG_STORE_FP8E4M3>(a.d, a, stream);
    default: set_error("search: unknown storage"); return RG_EINVAL;
    }
}

int launch_search_persistent(const SearchArgs &a, hipStream_t stream) {
    if (a.nq == 0) return RG_OK;
    switch (a.storage) {
    case RG_STORE_FP32: return dispatch_dim<PersistentLaunch, RG_STORE_FP32>(a.d, a, stream);
    case RG_STORE_BF16: return dispatch_dim<PersistentLaunch, RG_STORE_BF16>(a.d, a, stream);
    case RG_STORE_FP8E4M3: return dispatch_dim<PersistentLaunch, RG_STORE_FP8E4M3>(a.d, a, stream);
    default: set_error("search: unknown storage"); return RG_EINVAL;
    }
}

int search_occupancy(const SearchArgs &a, int *blocks_per_cu) {
    SearchArgs b = a;
    b.occ_out = blocks_per_cu;
    switch (a.storage) {
    case RG_STORE_FP32: return dispatch_dim<OccLaunch, RG_STORE_FP32>(a.d, b, nullptr);
    case RG_STORE_BF16: return dispatch_dim<OccLaunch, RG_STORE_BF16>(a.d, b, nullptr);
    case RG_STORE_FP8E4M3: return dispatch_dim<OccLaunch, RG_STORE_FP8E4M3>(a.d, b, nullptr);
    default: set_error("search: unknown storage"); return RG_EINVAL;
    }
}

int launch_serve_admit(int32_t n, const int32_t *slots, const float *q, const int32_t *k, const int32_t *L,
                       int32_t d, float *slot_q, int32_t *slot_k, int32_t *slot_L, int32_t *slot_state,
                       hipStream_t stream) {
    if (n == 0) return RG_OK;
    hipLaunchKernelGGL(k_serve_admit, dim3((unsigned)n), dim3(64), 0, stream, n, slots, q, k, L, d, slot_q, slot_k,
                       slot_L, slot_state);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

int launch_serve_step(const SlotArgs &sa, hipStream_t stream) {
    if (sa.n_active == 0) return RG_OK;
    switch (sa.s.storage) {
    case RG_STORE_FP32: return dispatch_dim<StepLaunch, RG_STORE_FP32>(sa.s.d, sa, stream);
    case RG_STORE_BF16: return dispatch_dim<StepLaunch, RG_STORE_BF16>(sa.s.d, sa, stream);
    case RG_STORE_FP8E4M3: return dispatch_dim<StepLaunch, RG_STORE_FP8E4M3>(sa.s.d, sa, stream);
    default: set_error("serve: unknown storage"); return RG_EINVAL;
    }
}

}  // namespace rg
