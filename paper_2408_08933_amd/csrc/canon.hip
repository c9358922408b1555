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

}  // namespace

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
