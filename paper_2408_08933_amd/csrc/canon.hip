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

// delta(c, kept row r) for r in [r0, r0 + nk), nk <= KG, for this lane's
// candidate row c: one pass over c, one sequential FP64 chain per kept row
// (each pair's sum runs in increasing i, as on the host).  kr(t) gives the
// kept row r0 + t (in LDS, or in device memory when the rows do not fit).
constexpr int KG = 16;
template <class KR>
__device__ __forceinline__ void canon_against_kept(const float *crow, KR kr, int d, int nk, double (&acc)[KG]) {
    const float *kp[KG];
#pragma unroll
    for (int t = 0; t < KG; ++t) {
        acc[t] = 0.0;
        kp[t] = t < nk ? kr(t) : kr(0);
    }
    for (int i = 0; i < d; ++i) {
        const double ci = (double)crow[i];
#pragma unroll
        for (int t = 0; t < KG; ++t)
            if (t < nk) acc[t] = fma(ci, (double)kp[t][i], acc[t]);
    }
}

__global__ __launch_bounds__(64) void k_canon_select(SelectArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *kid = reinterpret_cast<uint32_t *>(smem);   // m kept ids
    float *K = reinterpret_cast<float *>(smem) + ((a.m + 3) & ~3);  // m x pitch kept rows (if they fit)
    const int lane = lane_id();
    const int64_t b = blockIdx.x;
    const uint32_t x = (uint32_t)(a.x0 + b);
    const uint32_t *cid = a.ids + b * a.L;
    const double *cdd = a.dists + b * a.L;
    const int qn = a.counts[b];
    int nr = 0, hn = 0;
    auto kept_row = [&](int r) -> const float * {
        return a.kept_in_lds ? K + (size_t)r * a.pitch : a.X + (size_t)kid[r] * a.pitch;
    };
    // 64 candidates at a time, one per lane, in rank order
    for (int j0 = 0; j0 < qn; j0 += 64) {
        const int j = j0 + lane;
        const uint32_t c = j < qn ? cid[j] : kNone;
        const bool valid = j < qn && c != x;
        const uint64_t vm = ballot64(valid);
        const int pos = hn + lanes_below(vm);
        if (valid && pos < a.head_len) a.head[b * a.head_len + pos] = c;
        hn += (int)__popcll(vm);
        if (nr >= a.m) continue;
        const double dxc = valid ? cdd[j] : 0.0;
        const float *crow = a.X + (size_t)(valid ? c : 0u) * a.pitch;
        // rejected by a row kept before this batch?
        bool alive = valid;
        for (int r0 = 0; r0 < nr && ballot64(alive) != 0; r0 += KG) {
            const int nk = min(KG, nr - r0);
            if (alive) {
                double acc[KG];
                canon_against_kept(crow, [&](int t) { return kept_row(r0 + t); }, a.d, nk, acc);
#pragma unroll
                for (int t = 0; t < KG; ++t)
                    if (t < nk && !(dxc < -acc[t])) alive = false;
            }
        }
        // in rank order: the lowest surviving candidate is kept, and the
        // later survivors are checked against it
        for (;;) {
            const uint64_t am = ballot64(alive);
            if (am == 0 || nr >= a.m) break;
            const int js = (int)__builtin_ctzll(am);
            const uint32_t cs = (uint32_t)__shfl((int)c, js);
            const double ds = __shfl(dxc, js);
            if (a.kept_in_lds)
                for (int i = lane; i < a.pitch; i += 64) K[(size_t)nr * a.pitch + i] = a.X[(size_t)cs * a.pitch + i];
            if (lane == 0) {
                kid[nr] = cs;
                a.sel_ids[b * a.m + nr] = cs;
                a.sel_d[b * a.m + nr] = ds;
            }
            ++nr;
            __syncthreads();
            if (lane == js) alive = false;
            if (alive) {
                double acc[KG];
                const int rn = nr - 1;
                canon_against_kept(crow, [&](int t) { return kept_row(rn + t); }, a.d, 1, acc);
                if (!(dxc < -acc[0])) alive = false;
            }
        }
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
    const size_t id_bytes = (size_t)((m + 3) & ~3) * sizeof(uint32_t);
    const size_t kept_bytes = (size_t)m * pitch * sizeof(float);
    a.kept_in_lds = id_bytes + kept_bytes <= (48u << 10);
    hipLaunchKernelGGL(k_canon_select, dim3((unsigned)count), dim3(64), id_bytes + (a.kept_in_lds ? kept_bytes : 0),
                       stream, a);
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
    a.hash_bits = 11;  // 8 KB of LDS: fastest at L = 500 (the table size bounds work, not results)
    a.entry = entry;
    const size_t lds = canon_lds_bytes(L, pitch, a.hash_bits);
    hipLaunchKernelGGL(k_canon_search, dim3((unsigned)count), dim3(64), lds, stream, a);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

}  // namespace rg
