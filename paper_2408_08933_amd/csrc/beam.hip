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
// row (ELL, one id per lane; or a CSR row of any length, 128 ids at a time),
// filter through the visited set, gather the
// new neighbours' rows (G lanes per row, 16-byte loads, R rows per group in
// flight), reduce the FP32 dot products inside each G-lane group (DPP lane
// moves), order the survivors, and merge the entries that beat the queue's
// last key.  The search stops when every queue entry is expanded.
//
// Rows are read in 16-byte chunks of EPC elements (4 FP32, 8 BF16 or 16
// E4M3 values).  Lane j of a group accumulates, with fused multiply-adds in
// order, the elements of chunks c = j, j+G, j+2G, ...; then the G partial
// sums are added by a log2(G)-level xor tree (times the row's scale for
// E4M3).  A distance is therefore a fixed function of (query, row)
// whichever group computes it.
#include "rg_internal.h"
#include "queue_ops.h"
#include "wave_ops.h"

#include <climits>
#include <mutex>

namespace rg {
namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int kCand = 128;  // largest candidate batch (the widest ELL row, a CSR chunk)

struct Lds {
    float *qs;      // the query, zero padded to the row pitch
    float *qd;
    uint32_t *qi;
    float *cd;
    uint32_t *ci;
    float *sd;
    uint32_t *si;
    int32_t *slb;
    uint32_t *htab;
};

// cand = the candidate-batch capacity of this launch (64 or 128)
__device__ __forceinline__ Lds carve(unsigned char *p, int Leff, int pitch, int cand) {
    Lds s;
    s.qs = reinterpret_cast<float *>(p);
    s.qd = s.qs + pitch;
    s.qi = reinterpret_cast<uint32_t *>(s.qd + Leff);
    s.cd = reinterpret_cast<float *>(s.qi + Leff);
    s.ci = reinterpret_cast<uint32_t *>(s.cd + cand);
    s.sd = reinterpret_cast<float *>(s.ci + cand);
    s.si = reinterpret_cast<uint32_t *>(s.sd + cand);
    s.slb = reinterpret_cast<int32_t *>(s.si + cand);
    s.htab = reinterpret_cast<uint32_t *>(s.slb + cand);
    return s;
}

typedef float f32x2 __attribute__((ext_vector_type(2)));


// Storage formats: 16-byte chunks of EPC elements.
template <int ST>
struct Fmt {
    static constexpr int EPC = 4;
};
template <>
struct Fmt<RG_STORE_BF16> {
    static constexpr int EPC = 8;
};
template <>
struct Fmt<RG_STORE_FP8E4M3> {
    static constexpr int EPC = 16;
};

// Lane shape per dimension class (d <= 64, 128, 224, 256, 512, 1024) and
// storage: G lanes per row and NCH chunks per lane, G * NCH * EPC >= d; R rows
// per group whose loads are in flight together.
constexpr int kClassMaxD[6] = {64, 128, 224, 256, 512, 1024};
constexpr int shape_g(int st, int cls) {
    constexpr int g32[6] = {16, 16, 8, 16, 16, 32}, g16[6] = {8, 16, 8, 8, 16, 32}, g8[6] = {4, 8, 8, 8, 16, 32};
    return st == RG_STORE_FP32 ? g32[cls] : st == RG_STORE_BF16 ? g16[cls] : g8[cls];
}
// E4M3 rows also hold their scale after the codes (up to d + 7 bytes), so
// each E4M3 shape covers the class's largest d plus 8 bytes.
constexpr int shape_nch(int st, int cls) {
    constexpr int n32[6] = {1, 2, 7, 4, 8, 8}, n16[6] = {1, 1, 4, 4, 4, 4}, n8[6] = {2, 2, 2, 3, 3, 3};
    return st == RG_STORE_FP32 ? n32[cls] : st == RG_STORE_BF16 ? n16[cls] : n8[cls];
}
constexpr int shape_r(int st, int cls) { return st == RG_STORE_FP8E4M3 && cls <= 2 ? 4 : 2; }

// Copy the query into LDS, zero padded to qpad (every element a row chunk
// can reach, so bytes past d meet a zero).
__device__ __forceinline__ void load_query(const float *q, int d, int qpad, float *qs) {
    for (int i = lane_id(); i < qpad; i += 64) qs[i] = i < d ? q[i] : 0.f;
    __syncthreads();
}

// Chunks of a stored row the search reads: the d elements, and for E4M3 rows
// the scale that follows the codes.
template <int ST>
__device__ __forceinline__ int row_chunk_count(int d) {
    if constexpr (ST == RG_STORE_FP8E4M3) return (((d + 3) & ~3) + 4 + 15) >> 4;
    return (d + Fmt<ST>::EPC - 1) / Fmt<ST>::EPC;
}

template <int ST>
__device__ __forceinline__ const uint4 *row_chunks(const SearchArgs &a, uint32_t u) {
    if constexpr (ST == RG_STORE_FP32) return reinterpret_cast<const uint4 *>(a.base + (size_t)u * a.pitch);
    if constexpr (ST == RG_STORE_BF16) return reinterpret_cast<const uint4 *>(a.base_bf16 + (size_t)u * a.pitch);
    return reinterpret_cast<const uint4 *>(a.base_fp8 + (size_t)u * a.pitch8);
}

// acc += q . chunk c, in element order; q is read from LDS
template <int ST>
__device__ __forceinline__ float fma_chunk(const float *qs, int c, uint4 x, float acc) {
    constexpr int EPC = Fmt<ST>::EPC;
    const float4 *q4 = reinterpret_cast<const float4 *>(qs + c * EPC);
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
    if constexpr (ST == RG_STORE_FP32) {
        const float4 q = q4[0];
        acc = fmaf(q.x, __uint_as_float(w[0]), acc);
        acc = fmaf(q.y, __uint_as_float(w[1]), acc);
        acc = fmaf(q.z, __uint_as_float(w[2]), acc);
        acc = fmaf(q.w, __uint_as_float(w[3]), acc);
    } else if constexpr (ST == RG_STORE_BF16) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const float4 q = q4[i];
            acc = fmaf(q.x, __uint_as_float(w[2 * i] << 16), acc);
            acc = fmaf(q.y, __uint_as_float(w[2 * i] & 0xFFFF0000u), acc);
            acc = fmaf(q.z, __uint_as_float(w[2 * i + 1] << 16), acc);
            acc = fmaf(q.w, __uint_as_float(w[2 * i + 1] & 0xFFFF0000u), acc);
        }
    } else {
        // bytes at and past d (the scale, padding) decode to finite values and
        // meet zero query elements; the scale is taken separately
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            // gfx950 converts OCP E4M3 pairs exactly (every code is a float)
            const float4 q = q4[i];
            const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);
            const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], true);
            acc = fmaf(q.x, lo[0], acc);
            acc = fmaf(q.y, lo[1], acc);
            acc = fmaf(q.z, hi[0], acc);
            acc = fmaf(q.w, hi[1], acc);
        }
    }
    return acc;
}

// This lane's partial dot products with rows u[0..R) (kNone -> 0); all loads
// are issued before the first multiply.
// sc[r] receives the E4M3 row scale in the lane whose chunk holds it (0
// elsewhere), so a group sum yields it.
template <int ST, int G, int NCH, int R>
__device__ __forceinline__ void dot_rows(const SearchArgs &a, const uint32_t (&u)[R], const float *qs, int nch,
                                         float (&acc)[R], float (&sc)[R]) {
    const int j = lane_id() % G;
    uint4 raw[R][NCH];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint4 *row = row_chunks<ST>(a, u[r] != kNone ? u[r] : 0u);
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
            const int c = j + G * t;
            raw[r][t] = (u[r] != kNone && c < nch) ? row[c] : make_uint4(0u, 0u, 0u, 0u);
        }
    }
    const int s_off = (a.d + 3) & ~3, s_chunk = s_off >> 4, s_word = (s_off & 15) >> 2;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        acc[r] = 0.f;
        sc[r] = 0.f;
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
            const int c = j + G * t;
            if (c < nch) acc[r] = fma_chunk<ST>(qs, c, raw[r][t], acc[r]);
            if constexpr (ST == RG_STORE_FP8E4M3) {
                if (c == s_chunk) {
                    const uint32_t w = s_word == 0 ? raw[r][t].x : s_word == 1 ? raw[r][t].y
                                     : s_word == 2 ? raw[r][t].z : raw[r][t].w;
                    sc[r] = __uint_as_float(w);
                }
            }
        }
    }
}

// lane l reads lane l + n of its 16-lane row (row shift left) or lane
// l ^ 2 / l ^ 1 (quad permutes); lanes past the row read 0
template <int CTRL>
__device__ __forceinline__ float dpp_read(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum of the G lanes of each group, valid in the group's first lane.  The
// steps are those of an xor butterfly with the largest offset first, as
// seen from the first lane, so the value is the butterfly's bit for bit;
// inside a 16-lane row they use DPP (no LDS round trip), across rows
// (G = 32) a shuffle.
template <int G>
__device__ __forceinline__ float group_sum(float v) {
    if constexpr (G >= 32) v += __shfl_down(v, 16);
    if constexpr (G >= 16) v += dpp_read<0x108>(v);  // row_shl:8: lane + 8
    if constexpr (G >= 8) v += dpp_read<0x104>(v);   // row_shl:4: lane + 4
    if constexpr (G >= 4) v += dpp_read<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    if constexpr (G >= 2) v += dpp_read<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    return v;
}

// delta of this group's row from its group-summed dot product (and, for
// E4M3, the row's power-of-two scale: the product is exact)
template <int ST>
__device__ __forceinline__ float finish_delta(float sum, float scale) {
    if constexpr (ST == RG_STORE_FP8E4M3) return -(scale * sum);
    return -sum;
}

// Score ids[0..cnt) (LDS) into dout[0..cnt) (LDS); R rows per group in flight.
template <int ST, int G, int NCH, int R>
__device__ __forceinline__ void score_batch(const SearchArgs &a, const float *qs, int nch, const uint32_t *ids,
                                            uint32_t idmask, float *dout, int cnt) {
    constexpr int NG = 64 / G;
    const int g = lane_id() / G, j = lane_id() % G;
    for (int p = 0; p < cnt; p += NG * R) {
        uint32_t u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int sl = p + r * NG + g;
            u[r] = sl < cnt ? (ids[sl] & idmask) : kNone;
        }
        float acc[R], sc[R];
        dot_rows<ST, G, NCH, R>(a, u, qs, nch, acc, sc);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            acc[r] = group_sum<G>(acc[r]);
            if constexpr (ST == RG_STORE_FP8E4M3) sc[r] = group_sum<G>(sc[r]);
        }
        if (j == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int sl = p + r * NG + g;
                if (sl < cnt) dout[sl] = finish_delta<ST>(acc[r], sc[r]);
            }
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

// Expansions until done or `budget` expansions were made; the queue holds
// up to 64 * QR entries.
template <int ST, int CLS, int QR, class VIS>
__device__ __forceinline__ void run_search(const SearchArgs &a, const Lds &s, VIS &vis,
                                           int &qn, int &ptr, uint32_t &hops, uint32_t &evals, int budget,
                                           bool &done) {
    constexpr int G = shape_g(ST, CLS), NCH = shape_nch(ST, CLS), R = shape_r(ST, CLS);
    const int lane = lane_id();
    const int Leff = a.Leff, ell = a.ell, nch = row_chunk_count<ST>(a.d);
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
        // ELL row (width ell), or a CSR row of any length taken a.cand ids
        // at a time; each chunk is scored and merged before the next, which
        // ends in the same queue as one merge of the whole row.
        int64_t row = (int64_t)v * ell;
        int deg = ell;
        if (a.adj_off) {
            row = a.adj_off[v];
            deg = (int)(a.adj_off[v + 1] - row);
        }
        for (int c0 = 0; c0 < deg; c0 += a.cand) {
            const int cl = min(a.cand, deg - c0);
            const uint32_t *ids = a.adj + row + c0;
            vis.begin_hop(cl);
            const uint32_t r0 = lane < cl ? ids[lane] : kNone;
            const uint32_t r1 = lane + 64 < cl ? ids[lane + 64] : kNone;
            int nnew = 0;
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                if (half == 1 && cl <= 64) break;
                const uint32_t u = half == 0 ? r0 : r1;
                const bool fresh = u != kNone && vis.insert(u);
                const uint64_t m = ballot64(fresh);
                if (fresh) s.ci[nnew + lanes_below(m)] = u;
                nnew += (int)__popcll(m);
            }
            vis.added(nnew);
            evals += (uint32_t)nnew;
            __syncthreads();
            if (nnew == 0) continue;
            score_batch<ST, G, NCH, R>(a, s.qs, nch, s.ci, 0xFFFFFFFFu, s.cd, nnew);
            __syncthreads();
            const QueueLds<float> ql{s.qd, s.qi, s.cd, s.ci, s.sd, s.si, s.slb};
            if (nnew <= 64)
                merge_batch<1, float, QR>(ql, nnew, Leff, qn, ptr);
            else
                merge_batch<2, float, QR>(ql, nnew, Leff, qn, ptr);
            __syncthreads();
        }
    }
}

// Queue = [entry]; the visited set is cleared and holds the entry.
template <int ST, int CLS, class VIS>
__device__ __forceinline__ void init_state(const SearchArgs &a, const Lds &s, VIS &vis, int &qn, int &ptr,
                                           uint32_t &hops, uint32_t &evals) {
    constexpr int G = shape_g(ST, CLS), NCH = shape_nch(ST, CLS);
    const int lane = lane_id();
    vis.clear();
    const uint32_t u[1] = {lane < G ? a.entry : kNone};
    float acc[1], sc[1];
    dot_rows<ST, G, NCH, 1>(a, u, s.qs, row_chunk_count<ST>(a.d), acc, sc);
    acc[0] = group_sum<G>(acc[0]);
    if constexpr (ST == RG_STORE_FP8E4M3) sc[0] = group_sum<G>(sc[0]);
    __syncthreads();
    if (lane == 0) {
        s.qd[0] = finish_delta<ST>(acc[0], sc[0]);
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

// Rescore the final queue (at most 64 * QR entries) against FP32 rows and
// sort it (reduced-precision storage).
template <int CLS, int QR>
__device__ __forceinline__ void rerank_queue(const SearchArgs &a, const Lds &s, int qn) {
    constexpr int G = shape_g(RG_STORE_FP32, CLS), NCH = shape_nch(RG_STORE_FP32, CLS);
    score_batch<RG_STORE_FP32, G, NCH, 2>(a, s.qs, (a.d + 3) >> 2, s.qi, ~kExpanded, s.qd, qn);
    __syncthreads();
    constexpr int E = QR;
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

// The k results: the first k entries of the final queue that are not
// deleted (a tombstoned node still routes the search but is never
// returned), padded with kNone / +inf.
__device__ __forceinline__ void emit_topk(const SearchArgs &a, const Lds &s, int qn, uint32_t *ids, float *ds) {
    const int lane = lane_id();
    if (!a.tomb) {
        for (int i = lane; i < a.k; i += 64) {
            ids[i] = i < qn ? (s.qi[i] & ~kExpanded) : kNone;
            ds[i] = i < qn ? s.qd[i] : __builtin_inff();
        }
        return;
    }
    int w = 0;
    for (int b0 = 0; b0 < qn && w < a.k; b0 += 64) {
        const int i = b0 + lane;
        uint32_t u = kNone;
        bool alive = false;
        if (i < qn) {
            u = s.qi[i] & ~kExpanded;
            alive = ((a.tomb[u >> 5] >> (u & 31u)) & 1u) == 0u;
        }
        const uint64_t m = ballot64(alive);
        const int pos = w + lanes_below(m);
        if (alive && pos < a.k) {
            ids[pos] = u;
            ds[pos] = s.qd[i];
        }
        w += (int)__popcll(m);
    }
    for (int i = min(w, a.k) + lane; i < a.k; i += 64) {
        ids[i] = kNone;
        ds[i] = __builtin_inff();
    }
}

__device__ __forceinline__ void write_result(const SearchArgs &a, const Lds &s, int64_t q, int qn, uint32_t hops,
                                             uint32_t evals) {
    const int lane = lane_id();
    emit_topk(a, s, qn, a.out_ids + q * a.k, a.out_d + q * a.k);
    if (lane == 0) {
        if (a.out_hops) a.out_hops[q] = hops;
        if (a.out_evals) a.out_evals[q] = evals;
    }
}

// One query per workgroup, visited set in LDS.  Five resident wavefronts per
// SIMD (<= 102 VGPRs) measured fastest for the BF16/FP8 searches, which wait
// on memory latency more than on bandwidth; six or more spill.  FP32 rows
// (more chunks in flight per row) take four, which keeps them out of
// scratch: 4.6% faster on a 10M-row graph.
// QR = queue capacity / 64: kMaxL / 64, or kMaxSearchL / 64 for L_eff above
// kMaxL, where twice the queue entries per lane in the merge and the rerank
// take four resident wavefronts per SIMD for every storage form.
template <int ST, int CLS, int QR>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(ST == RG_STORE_FP32 || QR > kMaxL / 64 ? 4 : 5))) void k_search(SearchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t q = blockIdx.x;
    const Lds s = carve(smem, a.Leff, a.qpad, a.cand);
    VisitLds vis{s.htab, a.hash_bits, 1 << a.hash_bits, 0};
    load_query(a.queries + q * a.d, a.d, a.qpad, s.qs);
    int qn, ptr;
    uint32_t hops, evals;
    bool done;
    init_state<ST, CLS>(a, s, vis, qn, ptr, hops, evals);
    run_search<ST, CLS, QR>(a, s, vis, qn, ptr, hops, evals, INT_MAX, done);
    if constexpr (ST != RG_STORE_FP32) rerank_queue<CLS, QR>(a, s, qn);
    write_result(a, s, q, qn, hops, evals);
}

// Persistent grid: each workgroup stays resident, takes queries from a
// device counter until none are left, and keeps an exact visited bitmap
// (one bit per base node) in device memory, so LDS holds only the queue and
// the candidate batch and many more queries are in flight per CU.
// Four resident wavefronts per SIMD (<= 128 VGPRs) measured fastest for all
// storage forms, ahead of fewer waves with more registers.
// QR as for k_search.
template <int ST, int CLS, int QR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_search_persistent(SearchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Lds s = carve(smem, a.Leff, a.qpad, a.cand);
    VisitBitmap vis{a.bitmap + (size_t)blockIdx.x * a.bm_words, a.bm_words};
    const int lane = lane_id();
    for (;;) {
        int q = 0;
        if (lane == 0) q = (int)atomicAdd(a.work, 1u);
        q = __shfl(q, 0);
        if ((int64_t)q >= a.nq) break;
        load_query(a.queries + (int64_t)q * a.d, a.d, a.qpad, s.qs);
        int qn, ptr;
        uint32_t hops, evals;
        bool done;
        init_state<ST, CLS>(a, s, vis, qn, ptr, hops, evals);
        run_search<ST, CLS, QR>(a, s, vis, qn, ptr, hops, evals, INT_MAX, done);
        if constexpr (ST != RG_STORE_FP32) rerank_queue<CLS, QR>(a, s, qn);
        write_result(a, s, q, qn, hops, evals);
        __syncthreads();
    }
}

// One scheduler step of the serving loop: advance each listed slot by up to
// hops_budget expansions, keeping its whole state in device memory.  Five
// resident wavefronts per SIMD, as for k_search: the step is latency-bound.
// Slot state word 0: 0 = admitted, not started; > 0 = queue length of a
// search in progress; -1 = finished (its record written; the slot is
// skipped until the host admits a new request into it).
template <int ST, int CLS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void k_serve_step(SlotArgs sa) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int slot = sa.active[blockIdx.x];
    if (sa.slot_state[(size_t)slot * 8] < 0) return;
    SearchArgs a = sa.s;
    a.k = sa.slot_k[slot];
    a.Leff = max(sa.slot_L[slot], a.k);
    const Lds s = carve(smem, a.Leff, a.qpad, a.cand);
    const int lane = lane_id();
    const int H = 1 << a.hash_bits;
    load_query(sa.slot_q + (size_t)slot * a.d, a.d, a.qpad, s.qs);
    int32_t *st = sa.slot_state + (size_t)slot * 8;
    float *gqd = sa.slot_qd + (size_t)slot * kMaxL;
    uint32_t *gqi = sa.slot_qi + (size_t)slot * kMaxL;
    uint32_t *gh = sa.slot_hash + ((size_t)slot << a.hash_bits);
    int qn, ptr;
    uint32_t hops, evals;
    VisitLds vis{s.htab, a.hash_bits, H, 0};
    if (st[0] == 0) {
        init_state<ST, CLS>(a, s, vis, qn, ptr, hops, evals);
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
    run_search<ST, CLS, kMaxL / 64>(a, s, vis, qn, ptr, hops, evals, sa.hops_budget, done);
    if (done) {
        if constexpr (ST != RG_STORE_FP32) rerank_queue<CLS, kMaxL / 64>(a, s, qn);
        int pos = 0;
        if (lane == 0) pos = (int)atomicAdd(sa.out_count, 1u);
        pos = __shfl(pos, 0);
        ServeRecord *r = sa.out_rec + pos;
        emit_topk(a, s, qn, r->ids, r->d);
        if (lane == 0) {
            r->slot = slot;
            r->qn = qn;
            r->hops = hops;
            r->evals = evals;
            st[0] = -1;
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

// The kernels for a queue of L_eff entries: kMaxL or fewer, or up to kMaxSearchL.
template <int ST, int CLS>
void (*table_kernel(int Leff))(SearchArgs) {
    return Leff > kMaxL ? k_search<ST, CLS, kMaxSearchL / 64> : k_search<ST, CLS, kMaxL / 64>;
}
template <int ST, int CLS>
void (*persistent_kernel(int Leff))(SearchArgs) {
    return Leff > kMaxL ? k_search_persistent<ST, CLS, kMaxSearchL / 64> : k_search_persistent<ST, CLS, kMaxL / 64>;
}

template <int ST, int CLS>
int launch_one(const SearchArgs &a, hipStream_t stream) {
    const size_t lds = search_lds_bytes(a.Leff, a.qpad, a.hash_bits, a.cand);
    if (a.Leff > kMaxL)
        hipLaunchKernelGGL((k_search<ST, CLS, kMaxSearchL / 64>), dim3((unsigned)a.nq), dim3(64), lds, stream, a);
    else
        hipLaunchKernelGGL((k_search<ST, CLS, kMaxL / 64>), dim3((unsigned)a.nq), dim3(64), lds, stream, a);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

template <int ST, int CLS>
int launch_persistent(const SearchArgs &a, hipStream_t stream) {
    const size_t lds = search_lds_bytes(a.Leff, a.qpad, 0, a.cand);
    if (a.Leff > kMaxL)
        hipLaunchKernelGGL((k_search_persistent<ST, CLS, kMaxSearchL / 64>), dim3((unsigned)a.grid), dim3(64), lds,
                           stream, a);
    else
        hipLaunchKernelGGL((k_search_persistent<ST, CLS, kMaxL / 64>), dim3((unsigned)a.grid), dim3(64), lds, stream,
                           a);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

template <int ST, int CLS>
int occupancy_of(int Leff, int pitch, int cand, int *blocks_per_cu) {
    const size_t lds = search_lds_bytes(Leff, pitch, 0, cand);
    RG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, persistent_kernel<ST, CLS>(Leff), 64, lds));
    return RG_OK;
}

template <int ST, int CLS>
int launch_step(const SlotArgs &sa, hipStream_t stream) {
    const size_t lds = search_lds_bytes(kMaxL, sa.s.qpad, sa.s.hash_bits, sa.s.cand);
    hipLaunchKernelGGL((k_serve_step<ST, CLS>), dim3((unsigned)sa.n_active), dim3(64), lds, stream, sa);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

// dimension class of d (see kClassMaxD)
template <template <int, int> class F, int ST, typename Arg>
int dispatch_dim(int d, const Arg &a, hipStream_t stream) {
    if (d <= kClassMaxD[0]) return F<ST, 0>::run(a, stream);
    if (d <= kClassMaxD[1]) return F<ST, 1>::run(a, stream);
    if (d <= kClassMaxD[2]) return F<ST, 2>::run(a, stream);
    if (d <= kClassMaxD[3]) return F<ST, 3>::run(a, stream);
    if (d <= kClassMaxD[4]) return F<ST, 4>::run(a, stream);
    if (d <= kClassMaxD[5]) return F<ST, 5>::run(a, stream);
    set_error("search: d > 1024 is not supported");
    return RG_EINVAL;
}

template <int ST, int CLS>
struct SearchLaunch {
    static int run(const SearchArgs &a, hipStream_t s) { return launch_one<ST, CLS>(a, s); }
};
template <int ST, int CLS>
struct PersistentLaunch {
    static int run(const SearchArgs &a, hipStream_t s) { return launch_persistent<ST, CLS>(a, s); }
};
template <int ST, int CLS>
struct TableOcc {
    static int run(const SearchArgs &a, hipStream_t) {
        const size_t lds = search_lds_bytes(a.Leff, a.qpad, a.hash_bits, a.cand);
        RG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(a.occ_out, table_kernel<ST, CLS>(a.Leff), 64, lds));
        return RG_OK;
    }
};
template <int ST, int CLS>
struct OccLaunch {
    static int run(const SearchArgs &a, hipStream_t) {
        return occupancy_of<ST, CLS>(a.Leff, a.qpad, a.cand, a.occ_out);
    }
};
template <int ST, int CLS>
struct StepLaunch {
    static int run(const SlotArgs &a, hipStream_t s) { return launch_step<ST, CLS>(a, s); }
};
template <int ST, int CLS>
struct StepOcc {
    static int run(const SlotArgs &a, hipStream_t) {
        const size_t lds = search_lds_bytes(kMaxL, a.s.qpad, a.s.hash_bits, a.s.cand);
        RG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(a.s.occ_out, k_serve_step<ST, CLS>, 64, lds));
        return RG_OK;
    }
};

}  // namespace

size_t search_lds_bytes(int Leff, int pitch, int hash_bits, int cand) {
    return (size_t)pitch * 4 + (size_t)Leff * 8 + (size_t)cand * 20 + (hash_bits > 0 ? ((size_t)4 << hash_bits) : 0);
}

int cand_capacity(int ell, bool csr) { return csr || ell > 64 ? kCand : 64; }

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

int table_search_occupancy(const SearchArgs &a, int *blocks_per_cu) {
    SearchArgs b = a;
    b.occ_out = blocks_per_cu;
    switch (a.storage) {
    case RG_STORE_FP32: return dispatch_dim<TableOcc, RG_STORE_FP32>(a.d, b, nullptr);
    case RG_STORE_BF16: return dispatch_dim<TableOcc, RG_STORE_BF16>(a.d, b, nullptr);
    case RG_STORE_FP8E4M3: return dispatch_dim<TableOcc, RG_STORE_FP8E4M3>(a.d, b, nullptr);
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

int serve_step_occupancy(const SlotArgs &a, int *blocks_per_cu) {
    SlotArgs b = a;
    b.s.occ_out = blocks_per_cu;
    switch (a.s.storage) {
    case RG_STORE_FP32: return dispatch_dim<StepOcc, RG_STORE_FP32>(a.s.d, b, nullptr);
    case RG_STORE_BF16: return dispatch_dim<StepOcc, RG_STORE_BF16>(a.s.d, b, nullptr);
    case RG_STORE_FP8E4M3: return dispatch_dim<StepOcc, RG_STORE_FP8E4M3>(a.s.d, b, nullptr);
    default: set_error("serve: unknown storage"); return RG_EINVAL;
    }
}

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free search (rg_search_noalloc): the
// persistent search's work counter (first 256 bytes) and one visited bitmap
// per resident workgroup.  Each device holds its own copy of this array from
// the library's first use on it until the process ends.  In host code the
// array's name is not a device address: the address comes from
// hipGetSymbolAddress, taken once per device with that device current.
// ---------------------------------------------------------------------------
namespace {

__device__ __align__(256) uint32_t scratch[kNoAllocScratchBytes / 4];

__global__ void k_zero_words(uint32_t *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

}  // namespace

int noalloc_scratch(int device, uint32_t **out) {
    static std::mutex mu;
    static uint32_t *ptr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) {
        set_error("search_noalloc: device index out of range");
        return RG_EINVAL;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[device]) {
        int cur = -1;
        RG_HIP(hipGetDevice(&cur));
        if (cur != device) {
            set_error("search_noalloc: the index's device must be the current device");
            return RG_EINVAL;
        }
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("search_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
            return RG_EDEVICE;
        }
        ptr[device] = static_cast<uint32_t *>(p);
    }
    *out = ptr[device];
    return RG_OK;
}

// a fill kernel rather than a memset, so callers may capture the search in a graph
int launch_zero_words(uint32_t *p, int n, hipStream_t stream) {
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, stream, p, n);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

}  // namespace rg
