// Construction-time beam search with the canonical FP64 distance.
//
// Connectivity enhancement (Algorithm 1; Sec. 4.2.4) searches the projected
// graph once per base vector, with the base vector as the query and a queue
// of length L, and uses the final queue as candidate neighbours.  Those
// candidates decide the graph, so they are computed with the same
// canonical distance the host uses everywhere in construction:
// delta(a, b) = -sum_i a_i b_i, accumulated in FP64 in increasing i.  On the
// GPU each lane computes one neighbour's sum as a chain of FP64 fused
// multiply-adds; the product of two floats is exact in FP64, so every step
// rounds exactly like the host's add, and the value is bit-identical.
//
// One wavefront per searched node; the queue (FP64 keys), candidate batch
// and visited table live in LDS; the expansion rule, the lossy visited table
// and the merge are those of the query-time search, so the final queue
// equals the host searcher's.
#include "queue_ops.h"
#include "rg_internal.h"
#include "wave_ops.h"

namespace rg {
namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int kCand = 128;

struct CanonArgs {
    const float *X;         // n x pitch (zero padded)
    const uint32_t *adj;    // n x ell
    uint32_t *out_ids;      // count x L
    double *out_d;          // count x L
    int32_t *out_n;         // count
    int64_t x0, count;
    int32_t d, pitch, ell, L, hash_bits;
    uint32_t entry;
};

__device__ __forceinline__ double canon_delta(const float *q, const float *row, int d) {
    double s = 0.0;
    const float4 *q4 = reinterpret_cast<const float4 *>(q);
    const float4 *r4 = reinterpret_cast<const float4 *>(row);
    const int d4 = d >> 2;
    for (int c = 0; c < d4; ++c) {
        const float4 a = q4[c], b = r4[c];
        s = fma((double)a.x, (double)b.x, s);
        s = fma((double)a.y, (double)b.y, s);
        s = fma((double)a.z, (double)b.z, s);
        s = fma((double)a.w, (double)b.w, s);
    }
    for (int i = d4 * 4; i < d; ++i) s = fma((double)q[i], (double)row[i], s);
    return -s;
}

__device__ __forceinline__ uint32_t hslot(uint32_t u, int hb) { return (u * 2654435761u) >> (32 - hb); }

__global__ __launch_bounds__(64) void k_canon_search(CanonArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = lane_id();
    const int L = a.L, ell = a.ell, d = a.d;
    const int64_t b = blockIdx.x;
    const int64_t x = a.x0 + b;
    // LDS: query row, queue, batch, survivors, visited table
    float *qrow = reinterpret_cast<float *>(smem);
    double *qd = reinterpret_cast<double *>(qrow + a.pitch);
    double *cd = qd + L;
    double *sd = cd + kCand;
    uint32_t *qi = reinterpret_cast<uint32_t *>(sd + kCand);
    uint32_t *ci = qi + L;
    uint32_t *si = ci + kCand;
    int32_t *slb = reinterpret_cast<int32_t *>(si + kCand);
    uint32_t *htab = reinterpret_cast<uint32_t *>(slb + kCand);
    const int hb = a.hash_bits;
    const int H = 1 << hb;
    const uint32_t hmask = (uint32_t)H - 1u;
    const QueueLds<double> ql{qd, qi, cd, ci, sd, si, slb};

    for (int i = lane; i < a.pitch; i += 64) qrow[i] = a.X[x * a.pitch + i];
    for (int i = lane; i < H; i += 64) htab[i] = kEmpty;
    __syncthreads();
    if (lane == 0) {
        qd[0] = canon_delta(qrow, a.X + (size_t)a.entry * a.pitch, d);
        qi[0] = a.entry;
        htab[hslot(a.entry, hb)] = a.entry;
    }
    int qn = 1, ptr = 0, hcount = 1;
    __syncthreads();
    for (;;) {
        int sel = -1;
        for (int bb = ptr; bb < qn; bb += 64) {
            const int i = bb + lane;
            const uint64_t m = ballot64(i < qn && !(qi[i] & kExpanded));
            if (m) {
                sel = bb + (int)__builtin_ctzll(m);
                break;
            }
        }
        if (sel < 0) break;
        ptr = sel;
        const uint32_t v = qi[sel];
        __syncthreads();
        if (lane == 0) qi[sel] = v | kExpanded;
        if (hcount + ell > (H >> 1)) {
            for (int i = lane; i < H; i += 64) htab[i] = kEmpty;
            hcount = 0;
            __syncthreads();
        }
        int nnew = 0;
        for (int e0 = 0; e0 < ell; e0 += 64) {
            const int e = e0 + lane;
            const uint32_t u = e < ell ? a.adj[(size_t)v * ell + e] : kNone;
            bool fresh = false;
            if (u != kNone) {
                uint32_t h = hslot(u, hb);
                for (int probe = 0; probe < H; ++probe) {
                    const uint32_t old = atomicCAS(&htab[h], kEmpty, u);
                    if (old == kEmpty) {
                        fresh = true;
                        break;
                    }
                    if (old == u) break;
                    h = (h + 1u) & hmask;
                }
            }
            const uint64_t m = ballot64(fresh);
            if (fresh) ci[nnew + lanes_below(m)] = u;
            nnew += (int)__popcll(m);
        }
        hcount += nnew;
        __syncthreads();
        if (nnew == 0) continue;
        for (int j = lane; j < nnew; j += 64) cd[j] = canon_delta(qrow, a.X + (size_t)ci[j] * a.pitch, d);
        __syncthreads();
        if (nnew <= 64)
            merge_batch<1, double>(ql, nnew, L, qn, ptr);
        else
            merge_batch<2, double>(ql, nnew, L, qn, ptr);
    }
    for (int i = lane; i < qn; i += 64) {
        a.out_ids[b * L + i] = qi[i] & ~kExpanded;
        a.out_d[b * L + i] = qd[i];
    }
    if (lane == 0) a.out_n[b] = qn;
}

// AcquireNeighbors (Algorithm 3, without the fill) for every searched node,
// on the device: the candidates are the node's final queue without the node
// itself, already ranked by (delta, id); a candidate is kept iff
// delta(x, c) < delta(c, p) for every kept p (strict), until m are kept.
// Lane r computes delta(c, kept_r) as the same sequential FP64 chain as the
// host (exact float products, one rounding per addition), so every decision
// is the host's.  The kept rows sit in LDS when they fit.
struct SelectArgs {
    const float *X;          // n x pitch
    int32_t d, pitch;
    const uint32_t *ids;     // count x L search output
    const double *dists;
    const int32_t *counts;
    int32_t L, m, head_len, kept_in_lds;
    int64_t x0;
    uint32_t *sel_ids;       // count x m
    double *sel_d;
    int32_t *sel_n;
    uint32_t *head;          // count x head_len: the first candidates
    int32_t *head_n;         // candidates per node (without the node)
};

__global__ __launch_bounds__(64) void k_canon_select(SelectArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    float *K = reinterpret_cast<float *>(smem);  // m x pitch kept rows
    const int lane = lane_id();
    const int64_t b = blockIdx.x;
    const uint32_t x = (uint32_t)(a.x0 + b);
    const uint32_t *cid = a.ids + b * a.L;
    const double *cdd = a.dists + b * a.L;
    const int qn = a.counts[b];
    int nr = 0, hn = 0;
    uint32_t mine = kNone;  // lane r < nr: kept id r
    for (int j = 0; j < qn; ++j) {
        const uint32_t c = cid[j];
        if (c == x) continue;
        if (hn < a.head_len && lane == 0) a.head[b * a.head_len + hn] = c;
        ++hn;
        if (nr >= a.m) continue;
        const double dxc = cdd[j];
        bool lane_ok = true;
        if (lane < nr) {
            const float *pr = a.kept_in_lds ? K + (size_t)lane * a.pitch : a.X + (size_t)mine * a.pitch;
            const float *cr = a.X + (size_t)c * a.pitch;
            double s = 0.0;
            for (int i = 0; i < a.d; ++i) s = fma((double)cr[i], (double)pr[i], s);
            lane_ok = dxc < -s;
        }
        if (ballot64(!lane_ok) != 0) continue;
        if (lane == nr) mine = c;
        if (a.kept_in_lds)
            for (int i = lane; i < a.pitch; i += 64) K[(size_t)nr * a.pitch + i] = a.X[(size_t)c * a.pitch + i];
        if (lane == 0) {
            a.sel_ids[b * a.m + nr] = c;
            a.sel_d[b * a.m + nr] = dxc;
        }
        ++nr;
        __syncthreads();
    }
    if (lane == 0) {
        a.sel_n[b] = nr;
        a.head_n[b] = hn;
    }
}

}  // namespace

int launch_canon_select(const float *X, int32_t d, int32_t pitch, const uint32_t *ids, const double *dists,
                        const int32_t *counts, int32_t L, int64_t x0, int64_t count, int32_t m, uint32_t *sel_ids,
                        double *sel_d, int32_t *sel_n, uint32_t *head, int32_t head_len, int32_t *head_n,
                        hipStream_t stream) {
    if (count == 0) return RG_OK;
    if (m < 1 || L < 1) {
        set_error("canon select: bad arguments");
        return RG_EINVAL;
    }
    SelectArgs a{};
    a.X = X;
    a.d = d;
    a.pitch = pitch;
    a.ids = ids;
    a.dists = dists;
    a.counts = counts;
    a.L = L;
    a.m = m;
    a.head_len = head_len;
    a.x0 = x0;
    a.sel_ids = sel_ids;
    a.sel_d = sel_d;
    a.sel_n = sel_n;
    a.head = head;
    a.head_n = head_n;
    const size_t kept_bytes = (size_t)m * pitch * sizeof(float);
    a.kept_in_lds = kept_bytes <= (48u << 10);
    hipLaunchKernelGGL(k_canon_select, dim3((unsigned)count), dim3(64), a.kept_in_lds ? kept_bytes : 0, stream, a);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

size_t canon_lds_bytes(int L, int pitch, int hash_bits) {
    return (size_t)pitch * 4 + (size_t)L * 12 + (size_t)kCand * 24 + ((size_t)4 << hash_bits);
}

int launch_canon_search(const float *X, int32_t d, int32_t pitch, const uint32_t *adj, int32_t ell,
                        uint32_t entry, int32_t L, int64_t x0, int64_t count, uint32_t *ids, double *dists,
                        int32_t *counts, hipStream_t stream) {
    if (count == 0) return RG_OK;
    if (L < 1 || L > kMaxL || ell > kCand || pitch % 4 != 0) {
        set_error("canon search: unsupported L, row width or pitch");
        return RG_EINVAL;
    }
    CanonArgs a{};
    a.X = X;
    a.adj = adj;
    a.out_ids = ids;
    a.out_d = dists;
    a.out_n = counts;
    a.x0 = x0;
    a.count = count;
    a.d = d;
    a.pitch = pitch;
    a.ell = ell;
    a.L = L;
    a.hash_bits = 13;
    a.entry = entry;
    const size_t lds = canon_lds_bytes(L, pitch, a.hash_bits);
    hipLaunchKernelGGL(k_canon_search, dim3((unsigned)count), dim3(64), lds, stream, a);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

}  // namespace rg
