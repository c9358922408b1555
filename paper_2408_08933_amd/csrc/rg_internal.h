// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/roargraph.h"

namespace rg {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kExpanded = 0x80000000u;  // queue-entry flag (ids < 2^31)
constexpr int kMaxL = 512;                    // largest queue of the serving and construction searches
constexpr int kMaxSearchL = 1024;            // largest queue of rg_search (L_eff above kMaxL: long-queue kernels)
constexpr int kMaxEll = 128;                  // widest ELL row; wider graphs are searched as CSR

void set_error(const std::string &msg);

// status helpers
#define RG_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ::rg::set_error(std::string(#call) + ": " + hipGetErrorString(e_));       \
            return RG_EDEVICE;                                                        \
        }                                                                             \
    } while (0)

// Device-side search parameters (one struct, passed by value).
struct SearchArgs {
    const float *base;          // fp32 rows, pitch floats
    const uint16_t *base_bf16;  // bf16 rows (pitch elements) or null
    const uint8_t *base_fp8;    // e4m3 rows (pitch8 bytes: codes, the row's scale) or null
    const uint32_t *adj;        // ELL adjacency, n x ell, kNone padded; or CSR indices
    const int64_t *adj_off;     // CSR offsets (n + 1), or null for ELL
    const uint32_t *tomb;       // deleted-node bitmap (ceil(n/32) words), or null
    const float *queries;       // nq x d
    uint32_t *out_ids;          // nq x k
    float *out_d;               // nq x k
    uint32_t *out_hops;         // nq or null
    uint32_t *out_evals;        // nq or null
    int64_t nq;
    int32_t d, pitch, pitch8, ell;
    int32_t qpad;               // floats of the query kept in LDS (zero padded): every element a chunk reaches
    int32_t k, Leff;
    int32_t cand;               // candidate-batch capacity (64 or 128; cand_capacity)
    int32_t hash_bits;
    uint32_t entry;
    int32_t storage;            // RG_STORE_*
    // persistent variant: visited bitmaps (grid x bm_words) and the work counter
    uint32_t *bitmap;
    int64_t bm_words;
    uint32_t *work;
    int32_t grid;
    int *occ_out;
};

// beam.hip
int launch_search(const SearchArgs &a, hipStream_t stream);
// Scratch of the allocation-free search: a file-scope device array of this
// size per device; noalloc_scratch gives this device's address of it.
constexpr size_t kNoAllocScratchBytes = 256ull << 20;
constexpr int kMaxDevices = 64;
int noalloc_scratch(int device, uint32_t **out);
int launch_zero_words(uint32_t *p, int n, hipStream_t stream);
int launch_search_persistent(const SearchArgs &a, hipStream_t stream);
int search_occupancy(const SearchArgs &a, int *blocks_per_cu);
// workgroups of the LDS-table search (k_search) one CU holds with a.hash_bits
int table_search_occupancy(const SearchArgs &a, int *blocks_per_cu);
size_t search_lds_bytes(int Leff, int pitch, int hash_bits, int cand);
int cand_capacity(int ell, bool csr);  // candidate-batch capacity for a graph layout
// E4M3 row layout: d codes, zeros to a multiple of 4, the FP32 scale, zeros
// to a multiple of 16 bytes (the bytes a search reads), then zeros to a
// multiple of 128 bytes: rows start on a cache line and a search touches
// the fewest lines (d = 200: 208 bytes read, 2 lines per row instead of 2.5
// on average at a 208-byte pitch)
inline int32_t fp8_row_bytes(int32_t d) { return (((d + 3) & ~3) + 4 + 15) & ~15; }
inline int32_t fp8_pitch(int32_t d) { return (fp8_row_bytes(d) + 127) & ~127; }
// query floats a search of this storage form reads (the row's chunks)
inline int32_t query_pad(int32_t d, int32_t pitch, int32_t storage) {
    return storage == RG_STORE_FP8E4M3 ? std::max(pitch, fp8_row_bytes(d)) : pitch;
}
int default_hash_bits(int Leff);

// Serving step: same per-query arithmetic as launch_search, resumable.
struct SlotArgs {
    SearchArgs s;               // queries/out_* unused; per-slot arrays below
    const int32_t *active;      // list of slot indices to advance
    int32_t n_active;
    float *slot_q;              // slots x d query vectors
    int32_t *slot_k, *slot_L;
    float *slot_qd;             // slots x kMaxL queue distances
    uint32_t *slot_qi;          // slots x kMaxL queue ids (+flag)
    int32_t *slot_state;        // slots x 4: qn, ptr, hops, evals
    uint32_t *slot_hash;        // slots x (1 << hash_bits)
    int32_t *slot_hcount;       // slots
    uint32_t *slot_out_ids;     // unused
    float *slot_out_d;          // unused
    int32_t *slot_done;         // unused
    int32_t hops_budget;
    // finished requests are appended here: out_count (atomic) and records
    uint32_t *out_count;
    struct ServeRecord *out_rec;
};
// One finished request as the step kernel reports it.
struct ServeRecord {
    int32_t slot, qn;
    uint32_t hops, evals;
    uint32_t ids[kMaxL];
    float d[kMaxL];
};
int launch_serve_step(const SlotArgs &a, hipStream_t stream);
// workgroups of the serving step kernel one CU holds at once for these arguments
int serve_step_occupancy(const SlotArgs &a, int *blocks_per_cu);
// Scatter n admitted requests (compact arrays) into their slots and reset their state.
int launch_serve_admit(int32_t n, const int32_t *slots, const float *q, const int32_t *k, const int32_t *L,
                       int32_t d, float *slot_q, int32_t *slot_k, int32_t *slot_L, int32_t *slot_state,
                       hipStream_t stream);

// knn.hip: top-K candidates by FP32 score (desc), ids asc on ties.
int launch_knn_candidates(const float *Q, int64_t nq, int32_t ldq, const float *X, int64_t n,
                          int32_t ldx, int32_t d, int32_t K, uint32_t *ids, float *scores,
                          hipStream_t stream);
// peaks.hip: probes of the device's read bandwidth and matrix throughput
int launch_read_stream(const void *src, int64_t bytes, void *sink, int blocks, hipStream_t stream);
int launch_mfma_probe(int kind, int iters, void *sink, int blocks, hipStream_t stream, double *flop);

// The same from FP16 rows (round to nearest even): Q16 and X16 hold
// knn16_rows(rows) rows of knn16_width(d) halves, zero padded.
int64_t knn16_rows(int64_t rows);
int32_t knn16_width(int32_t d);
int launch_to_f16(const float *src, int64_t rows, int32_t d, int64_t ld, void *dst, int64_t rows_pad, int32_t dp,
                  hipStream_t stream);
int launch_knn16_candidates(const void *Q16, int64_t nq, const void *X16, int64_t n, int32_t d, int32_t dp,
                            int32_t K, uint32_t *ids, float *scores, hipStream_t stream);
// Canonical FP64 rescoring, sort and certification of m rows of K
// candidates (see knn.hip); ok[i] = 1 where row i's k results are exact.
// A candidate score errs by at most gsum |t| xmax + eta (|t| + xmax) + abs0.
int launch_knn_certify(const float *Q, int64_t m, int64_t ldq, const float *X, int64_t n, int64_t ldx, int32_t d,
                       const uint32_t *cid, const float *csc, int32_t K, int32_t k, double gsum, double xmax,
                       double eta, double abs0, uint32_t *out_id, double *out_d, uint8_t *ok, hipStream_t stream);

// quant.hip
int launch_pad_rows(const float *src, int64_t n, int32_t d, float *dst, int32_t pitch,
                    hipStream_t stream);
int launch_quant_bf16(const float *src, int64_t n, int32_t pitch, uint16_t *dst,
                      hipStream_t stream);
int launch_quant_fp8(const float *src, int64_t n, int32_t d, int32_t pitch, uint8_t *dst,
                     int32_t pitch8, float *scales, hipStream_t stream);

int launch_copy_probe(void *dst, const void *src, int64_t bytes, hipStream_t stream);

// host_build.cpp
// Graphs the construction passes through, kept on request: the bipartite
// graph G_bi (bridge lists B(x) of the base nodes, ascending t, and the
// out-lists N_out(t) of the training queries without their pivot), its
// base-to-base routing rows (row x = N_out(t) for each t in B(x)) with their
// entry, and the projected graph G_pj (rows sorted by neighbour id).
// canonical FP64 distance: -sum_i a_i b_i, exact products added in increasing i
double canon_dist(const float *a, const float *b, int32_t d);

// Canonical distances between pairs of base rows, remembered while one
// node's reverse insertions are replayed (the same pairs recur from one
// insertion to the next).  delta is symmetric bit for bit (the products commute, the
// sum runs in increasing i), so a pair is keyed without order.  Forgetting
// (a clear when the table fills) only costs recomputation.
class PairCache {
  public:
    explicit PairCache(int bits = 16) : mask_((1u << bits) - 1u), key_((size_t)1 << bits, kFree),
                                        val_((size_t)1 << bits, 0.0) {}
    void clear() {
        for (uint32_t h : used_) key_[h] = kFree;
        used_.clear();
    }
    double get(const float *X, int d, uint32_t a, uint32_t b) {
        const uint64_t k = a < b ? ((uint64_t)a << 32 | b) : ((uint64_t)b << 32 | a);
        uint32_t h = (uint32_t)((k * 0x9E3779B97F4A7C15ull) >> 40) & mask_;
        while (key_[h] != kFree) {
            if (key_[h] == k) return val_[h];
            h = (h + 1u) & mask_;
        }
        const double v = canon_dist(X + (int64_t)a * d, X + (int64_t)b * d, d);
        if (used_.size() * 2 > mask_) clear();  // keep the load under one half
        h = (uint32_t)((k * 0x9E3779B97F4A7C15ull) >> 40) & mask_;
        while (key_[h] != kFree) h = (h + 1u) & mask_;
        key_[h] = k;
        val_[h] = v;
        used_.push_back(h);
        return v;
    }

  private:
    static constexpr uint64_t kFree = ~0ull;
    uint32_t mask_;
    std::vector<uint64_t> key_;
    std::vector<double> val_;
    std::vector<uint32_t> used_;
};

// Insertion (updates through the saved bipartite graph) also needs the
// vectors on the host, the ids appended to each N_out(t) since the build,
// and, per base node, the queries whose N_out holds it.
struct StageGraphs {
    bool kept = false;
    int64_t nt = 0;
    int32_t q1 = 0;
    int64_t n_built = 0;
    std::vector<int64_t> b_off;  // n_built + 1
    std::vector<uint32_t> b_idx;
    std::vector<uint32_t> nout;  // nt x q1
    std::vector<int64_t> bi_off;
    std::vector<uint32_t> bi_idx;
    uint32_t entry_bi = 0;
    std::vector<int64_t> pj_off;
    std::vector<uint32_t> pj_idx;
    // updates
    std::vector<float> base;                       // n x d, grows with insertions
    std::vector<float> train;                      // nt x d (empty: no insertion)
    std::vector<std::vector<uint32_t>> nout_add;   // per query: inserted ids appended to N_out(t)
    std::vector<int64_t> inq_off;                  // per built node: queries t with x in N_out(t)
    std::vector<uint32_t> inq_idx;
    std::vector<std::vector<uint32_t>> inq_add;    // per inserted node: the query it joined
    mutable std::vector<int64_t> nout_view_off;    // full N_out(t) lists as CSR (rg_index_bipartite),
    mutable std::vector<uint32_t> nout_view_idx;   // made on request, dropped by an insertion
};

struct HostGraph {
    rg::StageGraphs stages;
    std::vector<int64_t> offsets;
    std::vector<uint32_t> indices;
    uint32_t entry = 0;
    int64_t repairs = 0;
    double t_knn = 0, t_project = 0, t_enhance = 0, t_total = 0;
    double t_enhance_search = 0;
};
// Device resources construction may use: the padded FP32 base on the device.
struct GpuCtx {
    const float *X;      // n x pitch
    int32_t pitch;
    hipStream_t stream;
};
// knn lists: nt x Nq canonical ids.  X: host n x d.  gpu == nullptr: host only.
int host_construct(const float *X, int64_t n, int32_t d, const uint32_t *knn, int64_t nt,
                   int32_t Nq, int32_t M, int32_t L, int32_t m_pj, int32_t m_ce, int threads,
                   const GpuCtx *gpu, bool keep_stages, HostGraph *out);

// Insertion (updates through the saved bipartite graph).  The nv new rows
// are already appended to sg.base (ids n0 .. n0+nv-1); queue_ids / queue_n
// hold each new row's canonical search queue (L entries per row) on the
// graph (offsets, indices) as it stood before the call.  Updates the graph
// in place to n0 + nv rows.
int host_insert(StageGraphs &sg, int32_t d, int32_t M, int32_t m_pj, int32_t L, uint32_t entry, int64_t n0,
                int64_t nv, const uint32_t *queue_ids, const int32_t *queue_n, std::vector<int64_t> &offsets,
                std::vector<uint32_t> &indices, int threads);
// Canonical searches of rows x0 .. x0+count-1 of X (host) on a host CSR
// graph, queue length L, on host threads (indexes without device data).
void host_canon_searches(const float *X, int32_t d, const int64_t *off, const uint32_t *idx, uint32_t entry,
                         int32_t L, int64_t x0, int64_t count, int threads, uint32_t *ids, int32_t *counts);

// canon.hip: AcquireNeighbors without fill over each searched node's queue
// (the enhancement's own selection), canonical FP64, on the device
int launch_canon_select(const float *X, int32_t d, int32_t pitch, const uint32_t *ids, const double *dists,
                        const int32_t *counts, int32_t L, int64_t x0, int64_t count, int32_t m, uint32_t *sel_ids,
                        double *sel_d, int32_t *sel_n, uint32_t *head, int32_t head_len, int32_t *head_n,
                        hipStream_t stream);

// canon.hip: construction-time searches with the canonical FP64 distance
int launch_canon_search(const float *X, int32_t d, int32_t pitch, const uint32_t *adj, int32_t ell,
                        uint32_t entry, int32_t L, int64_t x0, int64_t count, uint32_t *ids, double *dists,
                        int32_t *counts, hipStream_t stream);

// canonical FP64 distance helpers (host)
double canon_dist(const float *a, const float *b, int32_t d);

// exact kNN = GPU candidates + host certification (api.cpp)
int knn_exact(const float *Qdev, int64_t nq, const float *Xdev, int64_t n, int32_t d, int32_t k,
              int32_t slack, const float *Qhost, const float *Xhost, int threads,
              std::vector<uint32_t> *ids_out, std::vector<double> *d_out, hipStream_t stream);

int hw_threads(int requested);

}  // namespace rg

struct rg_index {
    int64_t n = 0;
    int32_t d = 0, pitch = 0, pitch8 = 0, ell = 0;
    int32_t metric = RG_METRIC_IP;
    int32_t storage = RG_STORE_FP32;
    uint32_t entry = 0;
    int32_t Nq = 0, M = 0, L_build = 0, m_pj = 0, m_ce = 0;
    int64_t repairs = 0;
    std::vector<int64_t> offsets;    // host CSR
    std::vector<uint32_t> indices;
    float *d_base = nullptr;          // n x pitch fp32
    uint32_t *d_adj = nullptr;        // n x ell (ELL) or nnz (CSR)
    int64_t *d_adj_off = nullptr;     // CSR offsets, null for ELL
    uint32_t *d_tomb = nullptr;       // deleted-node bitmap, null while nothing is deleted
    std::vector<uint32_t> tomb;       // host copy of the bitmap
    int64_t n_deleted = 0;
    uint16_t *d_bf16 = nullptr;       // n x pitch
    uint8_t *d_fp8 = nullptr;         // n x pitch8
    float *d_scale = nullptr;         // n
    int device = 0;
    double t_knn = 0, t_project = 0, t_enhance = 0, t_total = 0;
    rg::StageGraphs stages;
};
