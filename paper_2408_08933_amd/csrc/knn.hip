// Exact-kNN candidates on gfx950: S = Q X^T with FP32 MFMA
// (v_mfma_f32_16x16x4_f32), fused with a streaming top-K per query row, so
// the nq x n score matrix is never written.  This is the preprocessing step
// of index construction (the training queries' nearest base vectors,
// Algorithm 1 input) and the ground truth of recall@k (Def. 1).
//
// Workgroup = 4 wavefronts, a 128-query x 128-base output tile per step,
// each wavefront owning a 64 x 64 quarter as 4 x 4 MFMA blocks (64
// accumulator registers).  Operands are staged through LDS in 32-wide
// slices of the coordinate axis, row-major with a 4-float pad (16-byte
// writes and reads, conflict free for 16 lanes).  The contraction order is
// free, so in the slice's k-step t lane l supplies coordinate 8*(l/16) + t:
// each lane reads its 8 coordinates of a row with two 16-byte LDS loads.  A
// last slice shorter than 32 is stored permuted so that its data meet the
// first k-steps, and only ceil(rem / 4) k-steps run on it.
//
// Top-K: every query row of the tile keeps, in global memory, a buffer of up
// to CAP (score, id) pairs and in LDS an admission threshold (the K-th best
// score after the last compaction; -inf before).  Each score >= threshold is
// appended; a row whose buffer could overflow on the next tile is compacted
// by one wavefront (in-register bitonic sort of CAP pairs, keep K).  After a
// workgroup has swept its share of the base it sorts each row once more and
// writes the K best by (score desc, id asc).  When the base is split across
// workgroups, a merge kernel combines the per-split lists the same way.
#include "rg_internal.h"
#include "wave_ops.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>

namespace rg {
namespace {

typedef float fx4 __attribute__((ext_vector_type(4)));

constexpr int BQ = 128, BX = 128, KC = 32, KCP = KC + 4;
constexpr int CAP = 512;        // per-row candidate buffer
constexpr int CE = CAP / 64;    // pairs per lane when sorting a buffer

struct KnnArgs {
    const void *Q;  // FP32 rows (k_knn) or FP16 rows padded to whole tiles (k_knn16)
    const void *X;
    float *buf_sc;
    uint32_t *buf_id;
    float *out_sc;
    uint32_t *out_id;
    int64_t nq, n;
    int64_t q_tile0;
    int64_t xtiles, xtiles_per_split;
    int32_t ldq, ldx, d, K, splits;
    int32_t vec_q, vec_x;
};

__device__ __forceinline__ float4 ld4(const float *M, int64_t rows, int ld, int d, int64_t r, int k, bool vec) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r >= rows) return v;
    const float *p = M + r * (int64_t)ld + k;
    if (vec && k + 3 < d) return *reinterpret_cast<const float4 *>(p);
    if (k + 0 < d) v.x = p[0];
    if (k + 1 < d) v.y = p[1];
    if (k + 2 < d) v.z = p[2];
    if (k + 3 < d) v.w = p[3];
    return v;
}

// Sort the row's buffer (count c) by (score desc, id asc) and keep K.
// Returns the new count; thr receives the K-th best score when c >= K.
__device__ __forceinline__ int compact_row(float *bsc, uint32_t *bid, int c, int K, float &thr) {
    const int lane = lane_id();
    float key[CE];
    uint32_t id[CE];
#pragma unroll
    for (int e = 0; e < CE; ++e) {
        const int i = lane * CE + e;
        key[e] = i < c ? -bsc[i] : __builtin_inff();
        id[e] = i < c ? bid[i] : kNone;
    }
    wave_sort<CE>(key, id);
#pragma unroll
    for (int e = 0; e < CE; ++e) {
        const int i = lane * CE + e;
        if (i < K && i < c) {
            bsc[i] = -key[e];
            bid[i] = id[e];
        }
    }
    const int src = (K - 1) / CE, se = (K - 1) % CE;
    float kth = 0.f;
#pragma unroll
    for (int e = 0; e < CE; ++e)
        if (e == se) kth = key[e];
    kth = __shfl(kth, src);
    if (c >= K) thr = -kth;
    return c < K ? c : K;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_knn(KnnArgs a) {
    // two LDS buffers per operand: the MFMAs read one slice while the next is
    // stored into the other, one barrier per slice (73.7 KB per workgroup,
    // two workgroups per CU)
    __shared__ __align__(16) float As[2][BQ * KCP];
    __shared__ __align__(16) float Bs[2][BX * KCP];
    __shared__ float thr[BQ];
    __shared__ int cnt[BQ];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int64_t qt = a.q_tile0 + blockIdx.x;
    const int sp = blockIdx.y;
    const int64_t q0 = qt * BQ;
    const int64_t slot = (int64_t)blockIdx.x * a.splits + sp;
    float *bsc = a.buf_sc + slot * BQ * CAP;
    uint32_t *bid = a.buf_id + slot * BQ * CAP;
    const bool vq = a.vec_q != 0, vx = a.vec_x != 0;

    if (tid < BQ) {
        thr[tid] = -__builtin_inff();
        cnt[tid] = 0;
    }
    const int64_t xt0 = (int64_t)sp * a.xtiles_per_split;
    const int64_t xt1 = min(a.xtiles, xt0 + a.xtiles_per_split);
    const int lr = tid >> 3, lk = (tid & 7) * 4;
    const int kq = (lane >> 4) * 8;  // this lane's coordinates within a slice
    const int nsl = (a.d + KC - 1) / KC;
    float4 va[4], vb[4];
    // interior tiles and full slices load without bounds checks
    const float *Qf = static_cast<const float *>(a.Q), *Xf = static_cast<const float *>(a.X);
    const bool q_in = vq && q0 + BQ <= a.nq;
    const float *qrow = Qf + (q0 + lr) * (int64_t)a.ldq + lk;
    auto load_slice = [&](int64_t xt, int k0) {
        const int64_t x0 = xt * BX;
        if (q_in && vx && x0 + BX <= a.n && k0 + KC <= a.d) {
            const float *xrow = Xf + (x0 + lr) * (int64_t)a.ldx + lk + k0;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                va[p] = *reinterpret_cast<const float4 *>(qrow + (int64_t)p * 32 * a.ldq + k0);
                vb[p] = *reinterpret_cast<const float4 *>(xrow + (int64_t)p * 32 * a.ldx);
            }
            return;
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            va[p] = ld4(Qf, a.nq, a.ldq, a.d, q0 + p * 32 + lr, k0 + lk, vq);
            vb[p] = ld4(Xf, a.n, a.ldx, a.d, x0 + p * 32 + lr, k0 + lk, vx);
        }
    };
    // A partial last slice is stored permuted: coordinate c at position
    // 8 (c % 4) + c / 4, where k-step s of lane group g reads 8 g + s, so
    // step s meets coordinates 4 s .. 4 s + 3 and the steps past the data
    // can be skipped.
    auto store_slice = [&](int buf, bool tail) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int r = p * 32 + lr;
            if (!tail) {
                *reinterpret_cast<float4 *>(&As[buf][r * KCP + lk]) = va[p];
                *reinterpret_cast<float4 *>(&Bs[buf][r * KCP + lk]) = vb[p];
            } else {
                float *pa = &As[buf][r * KCP + (lk >> 2)], *pb = &Bs[buf][r * KCP + (lk >> 2)];
                pa[0] = va[p].x;
                pa[8] = va[p].y;
                pa[16] = va[p].z;
                pa[24] = va[p].w;
                pb[0] = vb[p].x;
                pb[8] = vb[p].y;
                pb[16] = vb[p].z;
                pb[24] = vb[p].w;
            }
        }
    };
    // The slices of consecutive tiles form one pipeline: the buffer parity
    // runs on across tiles, and the next tile's first slice is loaded while
    // the current tile's last slice is multiplied.
    int gsl = 0;
    if (xt0 < xt1) {
        load_slice(xt0, 0);
        store_slice(0, KC > a.d);
    }
    __syncthreads();
    for (int64_t xt = xt0; xt < xt1; ++xt) {
        const int64_t x0 = xt * BX;
        fx4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = fx4{0.f, 0.f, 0.f, 0.f};
        for (int sl = 0; sl < nsl; ++sl, ++gsl) {
            const int buf = gsl & 1;
            // the slice stored next: (xt, sl + 1), else the next tile's first
            const bool more = sl + 1 < nsl || xt + 1 < xt1;
            const bool more_tail = sl + 1 < nsl ? (sl + 2) * KC > a.d : KC > a.d;
            if (sl + 1 < nsl)
                load_slice(xt, (sl + 1) * KC);
            else if (xt + 1 < xt1)
                load_slice(xt + 1, 0);
            // k-steps of this slice: 8, or ceil(rem / 4) for a partial last one
            const int ns = (sl + 1) * KC <= a.d ? 8 : (a.d - sl * KC + 3) >> 2;
#pragma unroll 1
            for (int h = 0; h < 2 && 4 * h < ns; ++h) {
                float4 af[4], bf[4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    af[i] = *reinterpret_cast<const float4 *>(
                        &As[buf][(wr * 64 + i * 16 + (lane & 15)) * KCP + kq + 4 * h]);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    bf[j] = *reinterpret_cast<const float4 *>(
                        &Bs[buf][(wc * 64 + j * 16 + (lane & 15)) * KCP + kq + 4 * h]);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (4 * h + t >= ns) break;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][t], bf[j][t], acc[i][j], 0, 0, 0);
                }
            }
            if (more) store_slice(buf ^ 1, more_tail);
            __syncthreads();
        }
        // filter: accumulator element r of block (i, j) is row 4*(lane/16)+r, column lane%16
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wr * 64 + i * 16 + 4 * (lane >> 4) + r;
                const float t = thr[row];
                const bool rok = q0 + row < a.nq;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t gx = x0 + wc * 64 + j * 16 + (lane & 15);
                    const float s = acc[i][j][r];
                    if (rok && gx < a.n && s >= t) {
                        const int pos = atomicAdd(&cnt[row], 1);
                        bsc[(int64_t)row * CAP + pos] = s;
                        bid[(int64_t)row * CAP + pos] = (uint32_t)gx;
                    }
                }
            }
        }
        __syncthreads();
        for (int row = w; row < BQ; row += 4) {
            const int c = cnt[row];
            if (c > CAP - BX) {
                float t = thr[row];
                const int nc = compact_row(bsc + (int64_t)row * CAP, bid + (int64_t)row * CAP, c, a.K, t);
                if (lane == 0) {
                    cnt[row] = nc;
                    thr[row] = t;
                }
            }
        }
        __syncthreads();
    }
    for (int row = w; row < BQ; row += 4) {
        const int64_t gq = q0 + row;
        if (gq >= a.nq) continue;
        float t = thr[row];
        float *rs = bsc + (int64_t)row * CAP;
        uint32_t *ri = bid + (int64_t)row * CAP;
        const int c = compact_row(rs, ri, cnt[row], a.K, t);
        float *os = a.out_sc + ((int64_t)sp * a.nq + gq) * a.K;
        uint32_t *oi = a.out_id + ((int64_t)sp * a.nq + gq) * a.K;
        for (int i = lane; i < a.K; i += 64) {
            os[i] = i < c ? rs[i] : -__builtin_inff();
            oi[i] = i < c ? ri[i] : kNone;
        }
    }
}

// ---------------------------------------------------------------------------
// FP16 candidate pass (v_mfma_f32_16x16x32_f16, FP32 accumulation).
//
// The rows arrive rounded to FP16 (round to nearest even) and zero padded to
// a multiple of 32 coordinates and to whole tiles, so every load is in
// bounds and unchecked.  A workgroup owns 128 query rows and sweeps 128-row
// tiles of the base; its four wavefronts each hold a 64 x 64 quarter of the
// tile as 4 x 4 blocks of 16 x 16 (64 accumulator registers).
//
// At the FP16 matrix rate one 32-coordinate stage of a tile is only ~256
// cycles of MFMA work per wavefront, far less than a load's latency, so the
// operands go straight from global memory into a ring of NST16 LDS stages
// (global_load_lds, no registers involved): the loads of stage s + NST16 - 1
// are issued while stage s is multiplied.  One instruction moves a 16-row x
// 32-coordinate block (1 KB, 16 bytes per lane, consecutive in LDS); within
// it row j's 16-byte chunk c sits at 64 j + 16 (c ^ ((j >> 2) & 3)), so the
// 16 lanes of a quarter-wave that read one chunk of 16 rows hit distinct
// banks.  In an MFMA k-step lane l supplies, for row (or column) l % 16, the
// 8 coordinates 8 * (l / 16) .. + 7 of the stage, the same coordinates for
// both operands.  The filter and the per-row candidate buffers are those of
// k_knn above.  The scores are FP32 sums of exact products of the rounded
// inputs; how far they may be from the exact ones is bounded in the
// certification (knn_exact).
// ---------------------------------------------------------------------------
typedef _Float16 hx8 __attribute__((ext_vector_type(8)));

constexpr int BQ16 = 128, BX16 = 128, KS16 = 32, NST16 = 4;
constexpr int STAGE16 = (BQ16 + BX16) * KS16;  // halves per stage: A blocks, then B blocks

// s_waitcnt immediates: vmcnt [3:0] and [15:14], expcnt [6:4], lgkmcnt
// [11:8]; a field at its maximum does not wait.
constexpr int kWaitLgkm0 = 0xC07F;                       // LDS done, memory ops may be outstanding
__device__ __forceinline__ void wait_vm(int n) {         // at most n (0, 4 or 8) vector-memory ops outstanding
    if (n >= 8)
        __builtin_amdgcn_s_waitcnt(0x0F78);
    else if (n >= 4)
        __builtin_amdgcn_s_waitcnt(0x0F74);
    else
        __builtin_amdgcn_s_waitcnt(0x0F70);
}

// The LDS reads that follow the ring's loads are written as one asm block
// each, which waits for its own results: the compiler cannot tell which ring
// slot a global_load_lds writes and would otherwise wait for every load in
// flight before any LDS read, emptying the ring at each stage.  The stage
// loads are waited for by wait_vm above, before the barrier.
__device__ __forceinline__ void lds_frags(uint32_t a_addr, uint32_t b_addr, hx8 &a0, hx8 &a1, hx8 &a2, hx8 &a3,
                                          hx8 &b0, hx8 &b1, hx8 &b2, hx8 &b3) {
    asm volatile(
        "ds_read_b128 %0, %8\n\t"
        "ds_read_b128 %1, %8 offset:1024\n\t"
        "ds_read_b128 %2, %8 offset:2048\n\t"
        "ds_read_b128 %3, %8 offset:3072\n\t"
        "ds_read_b128 %4, %9\n\t"
        "ds_read_b128 %5, %9 offset:1024\n\t"
        "ds_read_b128 %6, %9 offset:2048\n\t"
        "ds_read_b128 %7, %9 offset:3072\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(a3), "=&v"(b0), "=&v"(b1), "=&v"(b2), "=&v"(b3)
        : "v"(a_addr), "v"(b_addr)
        : "memory");
}

__device__ __forceinline__ fx4 lds_f4(uint32_t addr) {
    fx4 v;
    asm volatile("ds_read_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=&v"(v) : "v"(addr) : "memory");
    return v;
}

__device__ __forceinline__ int lds_i32(uint32_t addr) {
    int v;
    asm volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=&v"(v) : "v"(addr) : "memory");
    return v;
}

__device__ __forceinline__ uint32_t lds_addr(const void *p) { return (uint32_t)(uintptr_t)p; }

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_knn16(KnnArgs a) {
    __shared__ __align__(1024) _Float16 ring[NST16 * STAGE16];
    __shared__ __align__(16) float thr[BQ16];
    __shared__ int cnt[BQ16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int64_t qt = a.q_tile0 + blockIdx.x;
    const int sp = blockIdx.y;
    const int64_t q0 = qt * BQ16;
    const int64_t slot = (int64_t)blockIdx.x * a.splits + sp;
    float *bsc = a.buf_sc + slot * BQ16 * CAP;
    uint32_t *bid = a.buf_id + slot * BQ16 * CAP;
    const _Float16 *Qh = static_cast<const _Float16 *>(a.Q), *Xh = static_cast<const _Float16 *>(a.X);

    if (tid < BQ16) {
        thr[tid] = -__builtin_inff();
        cnt[tid] = 0;
    }
    __syncthreads();
    const int64_t xt0 = (int64_t)sp * a.xtiles_per_split;
    const int64_t xt1 = min(a.xtiles, xt0 + a.xtiles_per_split);
    const int nks = a.d / KS16;  // d is the padded width here
    const int64_t nstage = (xt1 > xt0 ? xt1 - xt0 : 0) * nks;
    // this lane's share of a block: row j of the block, the chunk that lands
    // in its 16 bytes
    const int bj = lane >> 2, bc = ((lane & 3) ^ ((bj >> 2) & 3)) * 8;
    // wave w moves blocks 2w and 2w + 1 of both operands (rows 32 w .. 32 w + 31)
    const _Float16 *qsrc = Qh + (q0 + 32 * w + bj) * (int64_t)a.ldq + bc;
    const _Float16 *xsrc = Xh + (32 * w + bj) * (int64_t)a.ldx + bc;
    const int64_t q16 = 16 * (int64_t)a.ldq, x16 = 16 * (int64_t)a.ldx;
    // the next stage to load: coordinate offset ik of the tile at xs, ring slot islot
    int ik = 0, islot = 0;
    const _Float16 *xs = xsrc + xt0 * BX16 * (int64_t)a.ldx;
    const int64_t xtile = BX16 * (int64_t)a.ldx;
    auto issue = [&]() {
        _Float16 *dst = ring + islot * STAGE16 + 2 * w * 512;
        __builtin_amdgcn_global_load_lds(qsrc + ik, dst, 16, 0, 0);
        __builtin_amdgcn_global_load_lds(qsrc + ik + q16, dst + 512, 16, 0, 0);
        __builtin_amdgcn_global_load_lds(xs + ik, dst + BQ16 * KS16, 16, 0, 0);
        __builtin_amdgcn_global_load_lds(xs + ik + x16, dst + BQ16 * KS16 + 512, 16, 0, 0);
        islot = islot + 1 == NST16 ? 0 : islot + 1;
        ik += KS16;
        if (ik == a.d) {
            ik = 0;
            xs += xtile;
        }
    };
    for (int64_t g = 0; g < NST16 - 1 && g < nstage; ++g) issue();
    // fragment reads: block row fr of the wave's blocks, chunk fg (k-group)
    const int fr = lane & 15, fg = lane >> 4;
    const int foff = fr * 32 + ((fg ^ ((fr >> 2) & 3)) * 8);
    const uint32_t ring_a = lds_addr(ring + wr * 4 * 512 + foff);
    const uint32_t ring_b = lds_addr(ring + BQ16 * KS16 + wc * 4 * 512 + foff);
    int64_t g = 0;
    int cslot = 0;  // ring slot of stage g
    for (int64_t xt = xt0; xt < xt1; ++xt) {
        const int64_t x0 = xt * BX16;
        fx4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = fx4{0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < nks; ++ks, ++g) {
            // stage g has landed once at most the later stages' loads (4 per
            // stage) are outstanding; the barrier then also tells every wave
            // that all waves are done with slot (g - 1) % NST16
            wait_vm(4 * (int)min<int64_t>(NST16 - 2, nstage - 1 - g));
            __builtin_amdgcn_s_barrier();
            if (g + NST16 - 1 < nstage) issue();
            const uint32_t so = (uint32_t)cslot * STAGE16 * 2;
            cslot = cslot + 1 == NST16 ? 0 : cslot + 1;
            hx8 af[4], bf[4];
            lds_frags(ring_a + so, ring_b + so, af[0], af[1], af[2], af[3], bf[0], bf[1], bf[2], bf[3]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        // filter: accumulator element r of block (i, j) is query row
        // 16 i + 4 (lane / 16) + r of the wave's half, base column lane % 16
        bool stored = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rb = wr * 64 + i * 16 + 4 * (lane >> 4);
            const fx4 t4 = lds_f4(lds_addr(&thr[rb]));
            bool hit = false;
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int j = 0; j < 4; ++j) hit |= acc[i][j][r] >= t4[r];
            if (!__builtin_amdgcn_ballot_w64(hit)) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rb + r;
                const bool rok = q0 + row < a.nq;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t gx = x0 + wc * 64 + j * 16 + fr;
                    const float sc = acc[i][j][r];
                    if (rok && gx < a.n && sc >= t4[r]) {
                        const int pos = atomicAdd(&cnt[row], 1);
                        bsc[(int64_t)row * CAP + pos] = sc;
                        bid[(int64_t)row * CAP + pos] = (uint32_t)gx;
                        stored = true;
                    }
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        __builtin_amdgcn_s_barrier();
        // rows w, w + 4, ..: lane l < 32 looks at row w + 4 l; compaction of a
        // row whose buffer could overflow on the next tile (rare)
        const int myc = lane < BQ16 / 4 ? lds_i32(lds_addr(&cnt[w + 4 * lane])) : 0;
        uint64_t full = __builtin_amdgcn_ballot_w64(myc > CAP - BX16);
        while (full) {
            const int l = __builtin_ctzll(full);
            full &= full - 1;
            const int row = w + 4 * l;
            float t = thr[row];
            const int nc = compact_row(bsc + (int64_t)row * CAP, bid + (int64_t)row * CAP, cnt[row], a.K, t);
            stored = true;
            if (lane == 0) {
                cnt[row] = nc;
                thr[row] = t;
            }
        }
        // the candidate stores count in the same counter as the stage
        // loads; drain them so the waits above keep their meaning.  The
        // kernel issues no other vector-memory operation (no register
        // spills; the build checks that it uses no scratch)
        if (__builtin_amdgcn_ballot_w64(stored)) __builtin_amdgcn_s_waitcnt(0x0F70);
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        __builtin_amdgcn_s_barrier();
    }
    __syncthreads();
    for (int row = w; row < BQ16; row += 4) {
        const int64_t gq = q0 + row;
        if (gq >= a.nq) continue;
        float t = thr[row];
        float *rs = bsc + (int64_t)row * CAP;
        uint32_t *ri = bid + (int64_t)row * CAP;
        const int c = compact_row(rs, ri, cnt[row], a.K, t);
        float *os = a.out_sc + ((int64_t)sp * a.nq + gq) * a.K;
        uint32_t *oi = a.out_id + ((int64_t)sp * a.nq + gq) * a.K;
        for (int i = lane; i < a.K; i += 64) {
            os[i] = i < c ? rs[i] : -__builtin_inff();
            oi[i] = i < c ? ri[i] : kNone;
        }
    }
}

// FP32 rows -> FP16 (round to nearest even), rows_pad x dp, zeros past
// (rows, d).
__global__ void k_to_f16(const float *src, int64_t rows, int32_t d, int64_t ld, _Float16 *dst, int64_t rows_pad,
                         int32_t dp) {
    const int64_t total = rows_pad * dp;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / dp;
        const int c = (int)(i - r * dp);
        dst[i] = (r < rows && c < d) ? (_Float16)src[r * ld + c] : (_Float16)0.f;
    }
}

// Merge per-split top-K lists into one (one wavefront per query row).
__global__ __launch_bounds__(64) void k_knn_merge(const float *sc, const uint32_t *id, int64_t nq, int K,
                                                  int splits, float *out_sc, uint32_t *out_id) {
    const int64_t q = blockIdx.x;
    const int lane = lane_id();
    float key[CE];
    uint32_t v[CE];
    // running list occupies slots [0, K); the next split's list [K, 2K)
#pragma unroll
    for (int e = 0; e < CE; ++e) {
        const int i = lane * CE + e;
        key[e] = i < K ? -sc[q * K + i] : __builtin_inff();
        v[e] = i < K ? id[q * K + i] : kNone;
    }
    for (int s = 1; s < splits; ++s) {
        const float *ss = sc + ((int64_t)s * nq + q) * K;
        const uint32_t *si = id + ((int64_t)s * nq + q) * K;
#pragma unroll
        for (int e = 0; e < CE; ++e) {
            const int i = lane * CE + e;
            if (i >= K) {
                key[e] = i < 2 * K ? -ss[i - K] : __builtin_inff();
                v[e] = i < 2 * K ? si[i - K] : kNone;
            }
        }
        wave_sort<CE>(key, v);
    }
#pragma unroll
    for (int e = 0; e < CE; ++e) {
        const int i = lane * CE + e;
        if (i < K) {
            out_sc[q * K + i] = -key[e];
            out_id[q * K + i] = v[e];
        }
    }
}

// Certification of the exact k nearest rows from the FP32 candidates (one
// wavefront per query row).  Each lane rescores its candidates with the
// canonical distance delta = -sum_i q_i x_i, a chain of FP64 fused
// multiply-adds in increasing i (the products of floats are exact in FP64,
// so every step rounds like a plain FP64 add and the value equals the host's
// sum bit for bit), the wave sorts (delta, id) ascending, and the row is
// certified when the K-th candidate's FP32 score plus the error bound of
// both sums is below the k-th canonical score: no row outside the candidate
// list can then be among the k nearest.
constexpr int CERT_E = 4;  // candidates per lane (K <= 256)

struct CertArgs {
    const float *Q;
    const float *X;
    const uint32_t *cid;  // m x K, FP32 score descending
    const float *csc;
    uint32_t *out_id;  // m x k
    double *out_d;     // m x k or null
    uint8_t *ok;       // m
    int64_t m, n, ldq, ldx;
    int32_t d, K, k;
    double gsum, xmax;  // relative error bound factor of the candidate scores (and the canonical sum), max row norm
    double eta, abs0;   // absolute part of that bound: eta * (|t| + xmax) + abs0 (FP16 underflow)
};

__device__ __forceinline__ double canon_dot(const float *qs, const float *row, int d) {
    double s = 0.0;
    for (int i = 0; i < d; ++i) s = fma((double)qs[i], (double)row[i], s);
    return s;
}

__global__ __launch_bounds__(64) void k_knn_certify(CertArgs a) {
    extern __shared__ float qs[];
    const int64_t r = blockIdx.x;
    const int lane = lane_id();
    const float *q = a.Q + r * a.ldq;
    for (int i = lane; i < a.d; i += 64) qs[i] = q[i];
    __syncthreads();
    // candidate c = lane + 64 e (the sort takes any placement)
    double key[CERT_E];
    uint32_t id[CERT_E];
    int valid = 0;
#pragma unroll
    for (int e = 0; e < CERT_E; ++e) {
        const int c = lane + 64 * e;
        key[e] = __builtin_inf();
        id[e] = kNone;
        if (c < a.K) {
            const uint32_t u = a.cid[r * a.K + c];
            if (u != kNone) {
                id[e] = u;
                key[e] = -canon_dot(qs, a.X + (int64_t)u * a.ldx, a.d);
                ++valid;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) valid += __shfl_xor(valid, o);
    wave_sort<CERT_E, double>(key, id);
    bool certified = (int64_t)a.K >= a.n;
    if (!certified && valid >= a.k) {
        double tn = 0.0;
        for (int i = 0; i < a.d; ++i) tn = fma((double)qs[i], (double)qs[i], tn);
        const double tnorm = sqrt(tn) * (1.0 + 1e-12);
        const double tau = a.gsum * tnorm * a.xmax + a.eta * (tnorm + a.xmax) + a.abs0;
        const double sigma = (double)a.csc[r * a.K + a.K - 1];
        const int src = (a.k - 1) / CERT_E, se = (a.k - 1) % CERT_E;
        double kth = 0.0;
#pragma unroll
        for (int e = 0; e < CERT_E; ++e)
            if (e == se) kth = key[e];
        kth = __shfl(kth, src);
        certified = sigma + tau < -kth;
    }
    if (lane == 0) a.ok[r] = certified ? 1 : 0;
    if (!certified) return;
#pragma unroll
    for (int e = 0; e < CERT_E; ++e) {
        const int j = lane * CERT_E + e;
        if (j < a.k) {
            a.out_id[r * a.k + j] = j < valid ? id[e] : kNone;
            if (a.out_d) a.out_d[r * a.k + j] = j < valid ? key[e] : __builtin_inf();
        }
    }
}

}  // namespace

namespace {

// One kernel of the candidate pass: the kernel, its query rows per
// workgroup and base rows per tile, and the byte size of a row element.
struct KnnKernel {
    void (*fn)(KnnArgs);
    int bq, bx, threads;
    size_t elem;
};

// Candidates of query rows [0, nq) of Q (one launch series, one split policy).
int knn_range(const KnnKernel &kk, const void *Q, int64_t nq, int32_t ldq, const void *X, int64_t n, int32_t ldx,
              int32_t d, int32_t K, uint32_t *ids, float *scores, bool vec_q, bool vec_x, hipStream_t stream) {
    if (nq == 0) return RG_OK;
    const int64_t qtiles = (nq + kk.bq - 1) / kk.bq;
    const int64_t xtiles = (n + kk.bx - 1) / kk.bx;
    // split the base when there are too few query tiles to fill the chip
    int splits = (int)std::min<int64_t>(16, std::max<int64_t>(1, 1024 / qtiles));
    splits = (int)std::min<int64_t>(splits, xtiles);
    const int64_t per = (xtiles + splits - 1) / splits;
    splits = (int)((xtiles + per - 1) / per);
    const int64_t tiles_per_launch = std::max<int64_t>(1, 1024 / splits);
    const int64_t slots = std::min(qtiles, tiles_per_launch) * splits;

    float *buf_sc = nullptr, *tmp_sc = nullptr;
    uint32_t *buf_id = nullptr, *tmp_id = nullptr;
    auto cleanup = [&]() {
        if (buf_sc) (void)hipFree(buf_sc);
        if (buf_id) (void)hipFree(buf_id);
        if (tmp_sc) (void)hipFree(tmp_sc);
        if (tmp_id) (void)hipFree(tmp_id);
    };
    if (hipMalloc(&buf_sc, sizeof(float) * slots * kk.bq * CAP) != hipSuccess ||
        hipMalloc(&buf_id, sizeof(uint32_t) * slots * kk.bq * CAP) != hipSuccess) {
        cleanup();
        set_error("knn: out of device memory for candidate buffers");
        return RG_ENOMEM;
    }
    if (splits > 1) {
        if (hipMalloc(&tmp_sc, sizeof(float) * splits * nq * K) != hipSuccess ||
            hipMalloc(&tmp_id, sizeof(uint32_t) * splits * nq * K) != hipSuccess) {
            cleanup();
            set_error("knn: out of device memory for split lists");
            return RG_ENOMEM;
        }
    }
    KnnArgs a{};
    a.Q = Q;
    a.X = X;
    a.buf_sc = buf_sc;
    a.buf_id = buf_id;
    a.out_sc = splits > 1 ? tmp_sc : scores;
    a.out_id = splits > 1 ? tmp_id : ids;
    a.nq = nq;
    a.n = n;
    a.xtiles = xtiles;
    a.xtiles_per_split = per;
    a.ldq = ldq;
    a.ldx = ldx;
    a.d = d;
    a.K = K;
    a.splits = splits;
    a.vec_q = vec_q;
    a.vec_x = vec_x;
    const bool log = std::getenv("RG_LOG") != nullptr && qtiles > tiles_per_launch;
    for (int64_t t0 = 0; t0 < qtiles; t0 += tiles_per_launch) {
        a.q_tile0 = t0;
        const int64_t nt = std::min(tiles_per_launch, qtiles - t0);
        hipLaunchKernelGGL(kk.fn, dim3((unsigned)nt, (unsigned)splits), dim3(kk.threads), 0, stream, a);
        if (hipGetLastError() != hipSuccess) {
            cleanup();
            set_error("knn: kernel launch failed");
            return RG_EDEVICE;
        }
        if (log) {  // progress for long sweeps (waits for this launch)
            (void)hipStreamSynchronize(stream);
            std::fprintf(stderr, "[rg] knn tiles %lld / %lld\n", (long long)(t0 + nt), (long long)qtiles);
        }
    }
    if (splits > 1) {
        hipLaunchKernelGGL(k_knn_merge, dim3((unsigned)nq), dim3(64), 0, stream, tmp_sc, tmp_id, nq, K, splits,
                           scores, ids);
        if (hipGetLastError() != hipSuccess) {
            cleanup();
            set_error("knn: merge launch failed");
            return RG_EDEVICE;
        }
    }
    // buffers are freed only after the kernels that use them have finished
    if (hipStreamSynchronize(stream) != hipSuccess) {
        cleanup();
        set_error("knn: kernel failed");
        return RG_EDEVICE;
    }
    cleanup();
    return RG_OK;
}

// Each workgroup sweeps the base for one query tile.  When the tiles leave
// a thin last wave of workgroups (under half the device), its tiles run
// with the base split across workgroups instead, so the chip is not mostly
// idle for a whole sweep (same candidates).
int knn_series(const KnnKernel &kk, const void *Q, int64_t nq, int32_t ldq, const void *X, int64_t n, int32_t ldx,
               int32_t d, int32_t K, uint32_t *ids, float *scores, bool vec_q, bool vec_x, hipStream_t stream) {
    int per_cu = 0, cus = 0, dev = 0;
    RG_HIP(hipGetDevice(&dev));
    RG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    RG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kk.fn, kk.threads, 0));
    const int64_t resident = (int64_t)std::max(1, per_cu) * std::max(1, cus);
    const int64_t qtiles = (nq + kk.bq - 1) / kk.bq;
    const int64_t rem = qtiles % resident;
    if (qtiles > resident && rem != 0 && rem < resident / 2) {
        const int64_t nq_main = (qtiles - rem) * kk.bq;
        const int rc = knn_range(kk, Q, nq_main, ldq, X, n, ldx, d, K, ids, scores, vec_q, vec_x, stream);
        if (rc) return rc;
        const void *Qr = static_cast<const char *>(Q) + (size_t)nq_main * ldq * kk.elem;
        return knn_range(kk, Qr, nq - nq_main, ldq, X, n, ldx, d, K, ids + nq_main * K, scores + nq_main * K,
                         vec_q, vec_x, stream);
    }
    return knn_range(kk, Q, nq, ldq, X, n, ldx, d, K, ids, scores, vec_q, vec_x, stream);
}

}  // namespace

int launch_knn_candidates(const float *Q, int64_t nq, int32_t ldq, const float *X, int64_t n, int32_t ldx,
                          int32_t d, int32_t K, uint32_t *ids, float *scores, hipStream_t stream) {
    if (K < 1 || K > CAP - BX || K > CAP / 2) {
        set_error("knn: K must be in [1, 256]");
        return RG_EINVAL;
    }
    const KnnKernel kk{k_knn, BQ, BX, 256, sizeof(float)};
    const bool vq = (ldq % 4 == 0) && ((uintptr_t)Q % 16 == 0);
    const bool vx = (ldx % 4 == 0) && ((uintptr_t)X % 16 == 0);
    return knn_series(kk, Q, nq, ldq, X, n, ldx, d, K, ids, scores, vq, vx, stream);
}

int64_t knn16_rows(int64_t rows) { return (rows + BQ16 - 1) / BQ16 * BQ16; }

int32_t knn16_width(int32_t d) { return (d + KS16 - 1) / KS16 * KS16; }

int launch_to_f16(const float *src, int64_t rows, int32_t d, int64_t ld, void *dst, int64_t rows_pad, int32_t dp,
                  hipStream_t stream) {
    if (rows_pad == 0) return RG_OK;
    const int64_t total = rows_pad * dp;
    const unsigned blocks = (unsigned)std::min<int64_t>(65536, (total + 255) / 256);
    hipLaunchKernelGGL(k_to_f16, dim3(blocks), dim3(256), 0, stream, src, rows, d, ld, static_cast<_Float16 *>(dst),
                       rows_pad, dp);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

int launch_knn16_candidates(const void *Q16, int64_t nq, const void *X16, int64_t n, int32_t d, int32_t dp,
                            int32_t K, uint32_t *ids, float *scores, hipStream_t stream) {
    if (K < 1 || K > CAP - BX16 || K > CAP / 2 || dp % KS16 != 0 || d < 1 || d > dp) {
        set_error("knn16: K must be in [1, 256] and the width a multiple of 32");
        return RG_EINVAL;
    }
    const KnnKernel kk{k_knn16, BQ16, BX16, 256, sizeof(_Float16)};
    return knn_series(kk, Q16, nq, dp, X16, n, dp, dp, K, ids, scores, true, true, stream);
}

int launch_knn_certify(const float *Q, int64_t m, int64_t ldq, const float *X, int64_t n, int64_t ldx, int32_t d,
                       const uint32_t *cid, const float *csc, int32_t K, int32_t k, double gsum, double xmax,
                       double eta, double abs0, uint32_t *out_id, double *out_d, uint8_t *ok, hipStream_t stream) {
    if (K < k || K > 64 * CERT_E || k < 1 || d < 1 || d > 16384) {
        set_error("knn certify: bad candidate count or dimension");
        return RG_EINVAL;
    }
    if (m == 0) return RG_OK;
    CertArgs a{};
    a.Q = Q;
    a.X = X;
    a.cid = cid;
    a.csc = csc;
    a.out_id = out_id;
    a.out_d = out_d;
    a.ok = ok;
    a.m = m;
    a.n = n;
    a.ldq = ldq;
    a.ldx = ldx;
    a.d = d;
    a.K = K;
    a.k = k;
    a.gsum = gsum;
    a.xmax = xmax;
    a.eta = eta;
    a.abs0 = abs0;
    hipLaunchKernelGGL(k_knn_certify, dim3((unsigned)m), dim3(64), sizeof(float) * (size_t)d, stream, a);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

}  // namespace rg
