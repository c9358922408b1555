/*
 * roargraph.h -- C ABI of the MI355X RoarGraph library.
 *
 * RoarGraph (Chen et al., PVLDB 17(11), 2024) is a graph index for
 * cross-modal approximate nearest-neighbour search that is built with the
 * help of a set of training queries: a query-base bipartite graph (Algorithm 1,
 * Sec. 4.2.2) is projected onto the base vectors (Algorithm 2 with the
 * neighbour-selection rule of Algorithm 3, Sec. 4.2.3), then every base
 * vector is searched on the projected graph to add supplementary edges
 * (connectivity enhancement, Algorithm 1, Sec. 4.2.4).  Queries run a beam
 * search from the medoid with a queue of length L (Sec. 4.3).
 *
 * Conventions for every call:
 *   - Return value: RG_OK (0) or a negative RG_E* code; rg_last_error()
 *     then returns a message for the calling thread.
 *   - Vectors are float32, row-major, rows of d contiguous floats.
 *   - "device" pointers are HIP device memory on the current device (e.g.
 *     torch tensors' data_ptr()); "host" pointers are ordinary memory.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream);
 *     calls that return host results synchronise that stream before return.
 *   - Distance: delta(q, x) = -<q, x> (maximum inner product, Sec. 5.1);
 *     cosine workloads pass L2-normalised rows.  Smaller delta is closer;
 *     ties are broken by the smaller id.
 *   - The caller owns every buffer it passes.  The library owns rg_index and
 *     rg_server objects (their device copies of the base, the graph and the
 *     reduced-precision copies) until rg_free / rg_server_destroy.
 *   - rg_search, rg_knn and rg_index_graph may run concurrently on one const
 *     index; rg_index_set_storage, rg_save and rg_free may not overlap any
 *     other call on the same index.
 */
#ifndef ROARGRAPH_H
#define ROARGRAPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rg_index rg_index;
typedef struct rg_server rg_server;

enum {
    RG_OK = 0,
    RG_EINVAL = -1,    /* bad argument (sizes, null pointers, unsupported mode) */
    RG_ENOMEM = -2,    /* host or device allocation failed */
    RG_EDEVICE = -3,   /* a HIP call or kernel launch failed */
    RG_EAGAIN = -4,    /* serving: no slot or memory free right now, retry */
    RG_ECORRUPT = -5,  /* index file unreadable or its checksum does not match */
    RG_EINTERNAL = -6  /* an internal invariant failed (reported, never ignored) */
};

enum { RG_METRIC_IP = 0 };

/* Storage of the base rows that the search scores against (Sec. 4.3 calls
 * compression orthogonal to the index; Sec. 7 names scalar quantisation with
 * rescoring).  BF16: round-to-nearest-even.  FP8: OCP E4M3 codes with one
 * power-of-two scale per row, s = the smallest 2^e with 448*2^e >= max|x_i|.
 * Either way the final queue is rescored exactly in FP32. */
enum { RG_STORE_FP32 = 0, RG_STORE_BF16 = 1, RG_STORE_FP8E4M3 = 2 };

/* Build options; pass NULL for the defaults. */
typedef struct {
    int32_t L_build;   /* candidate-list length in projection and queue length of the
                          enhancement searches ("L", Algorithms 1-2); default 500 (Sec. 5.1) */
    int32_t m_pj;      /* out-degree bound of the projected graph; 0 => ceil((M-1)/2) */
    int32_t m_ce;      /* out-degree bound of the enhancement lists; 0 => floor((M-1)/2) */
    int32_t threads;   /* host threads for construction; 0 => all hardware threads */
    int32_t knn_slack; /* extra GPU kNN candidates per training query before the exact
                          rerank; 0 => max(16, Nq/4) */
    int32_t keep_stages; /* nonzero: keep the bipartite and projected graphs on the host
                            (rg_index_stage_graph, rg_index_bipartite) */
} rg_build_opts;

/* Graphs the construction passes through (Algorithm 1; the ablation of
 * Sec. 5.4 searches both). */
enum { RG_STAGE_PROJECTED = 1, RG_STAGE_BIPARTITE = 2 };

/*
 * rg_build -- build the index (Algorithm 1).
 *   base   device, n x d float32: the base vectors X.
 *   train  device, nt x d float32: the training queries T (Sec. 4.2.1).
 *   Nq     number of nearest base vectors per training query (>= 2, <= n).
 *   M      bound on every node's final out-degree (>= 3); projection and
 *          enhancement use m_pj + m_ce <= M - 1 and one slot per node is left
 *          for the reachability repair.
 * The Nq-NN lists come from the GPU kNN (rg_knn semantics: FP16 or FP32 MFMA
 * candidates, exact FP64 rerank with a certified margin); the graph steps run
 * on host threads with the canonical FP64 distance (sum of exact products in
 * increasing coordinate order).  The result is deterministic and independent
 * of the thread count.  On success *out owns a device copy of the base, the
 * adjacency, and a host CSR view (rg_index_graph).
 * Errors: RG_EINVAL (n < 1, n >= 2^31, d < 1, nt < 1, Nq < 2, Nq > n, M < 3,
 * M > 128, metric != RG_METRIC_IP, null pointers), RG_ENOMEM, RG_EDEVICE,
 * RG_EINTERNAL.
 */
int rg_build(const float *base, int64_t n, int32_t d, const float *train, int64_t nt,
             int32_t Nq, int32_t M, int32_t metric, const rg_build_opts *opts, void *stream,
             rg_index **out);

/*
 * rg_build_from_knn -- the host half of rg_build, for callers that already
 * hold the preprocessing result (the Nq nearest base rows of each training
 * query, Algorithm 1 input).
 *   base_host  host, n x d float32.
 *   knn_host   host, nt x Nq uint32, each row in (delta, id) order with the
 *              canonical FP64 distance (as rg_knn returns them).
 *   train_host host, nt x d float32 training queries, or NULL; kept (with
 *              keep_stages) only for rg_insert, which needs them.
 * Runs bipartite graph, projection, enhancement, repair and CSR on host
 * threads; the index holds only the graph (rg_index_graph, rg_save need
 * no device data; rg_search returns RG_EINVAL).  No HIP call is made.
 * Errors: RG_EINVAL (as rg_build, plus ids >= n), RG_EINTERNAL.
 */
int rg_build_from_knn(const float *base_host, int64_t n, int32_t d, const uint32_t *knn_host,
                      const float *train_host, int64_t nt, int32_t Nq, int32_t M,
                      const rg_build_opts *opts, rg_index **out);

/*
 * rg_index_from_csr -- wrap an existing graph as an index.
 *   base    device, n x d float32 (copied).
 *   offsets host, n+1 int64, offsets[0] = 0, non-decreasing.
 *   indices host, offsets[n] uint32 ids < n (copied).
 *   entry   start node of every search (< n).
 * Graphs with every out-degree <= 128 are held as ELL rows on the device;
 * wider ones as CSR, searched 128 neighbours at a time.
 * Errors: RG_EINVAL, RG_ENOMEM, RG_EDEVICE.
 */
int rg_index_from_csr(const float *base, int64_t n, int32_t d, const int64_t *offsets,
                      const uint32_t *indices, uint32_t entry, int32_t metric, void *stream,
                      rg_index **out);

/*
 * rg_index_graph -- host views of the final graph: CSR with rows sorted by
 * neighbour id, int64 offsets (n+1), uint32 indices (nnz), and the entry
 * point.  Views stay valid until rg_free.  Any output pointer may be NULL.
 */
int rg_index_graph(const rg_index *idx, const int64_t **offsets, const uint32_t **indices,
                   int64_t *nnz, uint32_t *entry);

/*
 * rg_index_stage_graph -- host CSR views of a graph the build passed
 * through; needs a build with keep_stages.
 *   RG_STAGE_PROJECTED: G_pj, the output of the neighbourhood-aware
 *     projection (Algorithm 2) before connectivity enhancement, rows sorted
 *     by neighbour id; entry = the index's entry (the enhancement searches
 *     start there).
 *   RG_STAGE_BIPARTITE: greedy routing on the query-base bipartite graph
 *     G_bi (Sec. 4.2.1: from a base node through its out-neighbours, the
 *     query nodes it is the pivot of, to their base out-neighbours).  Row x
 *     lists N_out(t) for each bridge t of x in ascending t, each N_out(t) in
 *     (delta(t, .), id) order without its pivot; duplicates across bridges
 *     are kept (the search visits a node once).  A base node that is no
 *     query's pivot has an empty row.  entry = the row nearest (L2) to the
 *     mean among pivots.
 * Both can be searched through rg_index_from_csr (any out-degree).  Views
 * stay valid until rg_free.  Errors: RG_EINVAL (unknown stage, stages not
 * kept).
 */
int rg_index_stage_graph(const rg_index *idx, int32_t stage, const int64_t **offsets,
                         const uint32_t **indices, int64_t *nnz, uint32_t *entry);

/*
 * rg_index_bipartite -- host views of G_bi itself (Algorithm 1, first loop):
 * bridge_offsets (n_built+1 int64) and bridges (nt uint32) list, per base
 * node x of the build (n_built = the rows the build had; inserted rows are
 * no query's pivot), the training queries t whose nearest base row is x
 * (edge x -> t), in ascending t; nout_offsets (nt+1 int64) and nout hold
 * N_out(t), the other Nq - 1 nearest rows of t in (delta, id) order,
 * followed by the rows rg_insert has added to it.  Needs keep_stages.
 * Views stay valid until the next rg_insert or rg_free.  Errors: RG_EINVAL.
 */
int rg_index_bipartite(const rg_index *idx, const int64_t **bridge_offsets, const uint32_t **bridges,
                       int64_t *n_built, const int64_t **nout_offsets, const uint32_t **nout, int64_t *nt);

/*
 * rg_insert -- insert nv new base vectors (host, nv x d float32) through the
 * saved bipartite graph (Sec. 6, "Update"); they get ids n .. n+nv-1 in
 * input order.  Needs an index built with keep_stages (from kNN lists: with
 * train_host).  Each vector v is searched on the index as it stood when the
 * call began (canonical FP64 distance, queue length L; 0 => the build's L),
 * on the device when the index has device data, else on host threads.
 * Then, in input order:
 *   - b = the first node of v's queue joined to a query node (b is the pivot
 *     of t or b is in N_out(t)); q = the joined query nearest to v by
 *     (delta(v, t), t);
 *   - the sub-bipartite graph N_out(q) u {q, v} is projected with v as pivot
 *     (Algorithm 2 for one pivot: candidates N_out(q) by (delta(v, .), id), at
 *     most L, AcquireNeighbors with fill to m_pj); the selection is v's row;
 *   - each selected p takes v through Algorithm 2's reverse step on its whole
 *     row in the index: row(p) <- AcquireNeighbors(p, row(p) u {v}, M, with
 *     fill).  A row with room simply gains v; a full row keeps M entries by
 *     the selection rule, which may drop v or one of its old neighbours.  If
 *     no p keeps v, v gets one in-edge by the build's repair rule (the first
 *     queue node with a free slot, else the first in BFS order);
 *   - v is appended to N_out(q).  With no joined node in the queue, v's
 *     candidates are its queue and no N_out changes.
 * At the end of the call every node the entry no longer reaches (an old
 * node can lose its last in-edge to a full row's selection) gets one
 * in-edge, in ascending id, from the first node in BFS order with a free
 * slot.  Out-degrees stay <= M and every node stays reachable from the
 * entry.  The device copies (rows, adjacency, tombstones, the chosen storage
 * form) are remade.  Deterministic.  Not concurrent with other calls on the
 * index.  Every argument is checked before anything changes (non-finite
 * values are rejected); a failure after that leaves the index with its
 * previous rows, graph and storage form.
 * Errors: RG_EINVAL (no kept stages or training queries, L > 512, graph held
 * as CSR, a value that is not finite), RG_ENOMEM, RG_EDEVICE, RG_EINTERNAL.
 */
int rg_insert(rg_index *idx, const float *vectors, int64_t nv, int32_t L, void *stream);

/*
 * rg_delete -- mark nodes deleted (tombstones, Sec. 6): they stay in the
 * graph and keep routing searches, but rg_search and the server skip them
 * when taking the k results from the final queue (so fewer than k results
 * can come back, padded with 0xFFFFFFFF / +inf).  ids host, each < n;
 * deleting a node twice is harmless.  Not concurrent with other calls on
 * the index.  Errors: RG_EINVAL, RG_ENOMEM, RG_EDEVICE.
 */
int rg_delete(rg_index *idx, const uint32_t *ids, int64_t count, void *stream);

/* rg_index_tombstones -- host view of the deleted-node bitmap (bit i of word
 * i/32; NULL while nothing was deleted) and the number of deleted nodes. */
int rg_index_tombstones(const rg_index *idx, const uint32_t **bits, int64_t *count);

/* rg_index_info -- n, d, the padded row pitch in floats, the ELL row width of
 * the device adjacency (0 when the graph is held as CSR because a row is
 * wider than 128), and device bytes held.  Any output may be NULL. */
int rg_index_info(const rg_index *idx, int64_t *n, int32_t *d, int32_t *pitch,
                  int32_t *ell_width, int64_t *device_bytes);

/*
 * rg_index_set_storage -- choose the storage searched by rg_search
 * (RG_STORE_*).  BF16 / FP8 copies are made on the device from the index's
 * FP32 rows; the FP32 rows are kept for the exact rerank.
 * Errors: RG_EINVAL, RG_ENOMEM, RG_EDEVICE.
 */
int rg_index_set_storage(rg_index *idx, int32_t storage, void *stream);

/*
 * rg_search -- batched beam search (Sec. 4.3), one query per wavefront.
 *   queries device, nq x d float32.
 *   k       results per query (1..1024); L queue length (1..1024); the
 *           queue actually kept is L_eff = max(L, k).  Queues of up to 512
 *           entries and longer ones run in separate kernels (the longer
 *           holding twice the queue entries per lane), with the same rules.
 *   ids     device, nq x k uint32; dists device, nq x k float32 holding
 *           -<q, x_id> in FP32, ascending; when fewer than k nodes are
 *           reachable the tail is 0xFFFFFFFF / +inf.
 *   hops    device, nq uint32 or NULL: nodes expanded per query.
 *   evals   device, nq uint32 or NULL: distances computed per query
 *           (includes recomputations after the LDS visited table is reset).
 * The search expands the closest unexpanded queue entry until none is left;
 * a neighbour enters the queue if the queue is not full or it beats the last
 * entry.  With reduced-precision storage the final L_eff queue is rescored
 * against the FP32 rows and the best k are returned.  FP32 storage keeps an
 * exact visited bitmap per resident query in device memory while n/8 bytes
 * stay below 5% of a query's expected row bytes (40 L_eff rows of 4d
 * bytes) or the graph is held as CSR (rows over 128 ids);
 * otherwise, and for BF16 / FP8, a visited table in LDS that forgets and
 * rescores (the results are the same; evals counts the rescoring): the
 * largest of 2^10, 2^9 and 2^8 entries that lets the most workgroups share
 * a CU (2^8 only while it holds twice a row batch).
 * Asynchronous on stream.
 * Errors: RG_EINVAL, RG_EDEVICE.
 */
int rg_search(const rg_index *idx, const float *queries, int64_t nq, int32_t k, int32_t L,
              uint32_t *ids, float *dists, uint32_t *hops, uint32_t *evals, void *stream);

/*
 * rg_knn -- exact k nearest base rows of each query (Def. 1): the
 * preprocessing step of construction and the ground truth of recall@k.
 *   queries device nq x d; base device n x d; ids/dists device nq x k.
 * Candidates: when every value of both matrices is below 2^15 in magnitude,
 * the GPU first scores FP16-rounded rows with FP16 MFMA (FP32 accumulation)
 * and keeps K = min(256, n, max(2k, k + 48)) per query; every candidate is
 * rescored with the canonical FP64 distance and the row is certified when
 * the K-th candidate's score plus the score error bound (FP16 rounding of
 * both inputs and FP32 accumulation, see knn_exact) lies below the k-th
 * canonical score, so no other base row can be among the k nearest.  Rows
 * not certified are redone from FP32 MFMA scores (k + slack candidates,
 * doubling to 256) and, failing that (more than 256 rows tied), by a full
 * canonical scan on the host.  ids are in (delta, id) order and dists hold
 * the FP64 delta rounded to float.  Synchronous.
 * Errors: RG_EINVAL (k < 1, k > n, k > 224, n >= 2^31), RG_ENOMEM,
 * RG_EDEVICE.
 */
int rg_knn(const float *queries, int64_t nq, const float *base, int64_t n, int32_t d,
           int32_t k, uint32_t *ids, float *dists, void *stream);

/*
 * rg_knn_candidates -- the GPU half of rg_knn alone: for each query the K
 * best base rows by FP32 score, ordered by (score descending, id ascending).
 * ids/scores device nq x K.  Asynchronous.  Errors: RG_EINVAL, RG_EDEVICE.
 */
int rg_knn_candidates(const float *queries, int64_t nq, const float *base, int64_t n, int32_t d,
                      int32_t K, uint32_t *ids, float *scores, void *stream);

/*
 * rg_knn_candidates_f16 -- the FP16 candidate pass of rg_knn alone: the
 * rows are rounded to FP16 (nearest even) and zero padded on the device,
 * then for each query the K best base rows by the FP32 sum of the rounded
 * products, ordered by (score descending, id ascending).  ids/scores device
 * nq x K.  Values must be below 2^15 in magnitude.  Synchronous.
 * Errors: RG_EINVAL (K < 1, K > 256, K > n, values out of range), RG_ENOMEM,
 * RG_EDEVICE.
 */
int rg_knn_candidates_f16(const float *queries, int64_t nq, const float *base, int64_t n, int32_t d,
                          int32_t K, uint32_t *ids, float *scores, void *stream);

/*
 * rg_knn_last_stats -- how the calling thread's last rg_knn (or the kNN of
 * its last rg_build) certified its rows: from FP16 candidates, from FP32
 * candidates, by the host scan.  Any output may be NULL.
 */
int rg_knn_last_stats(int64_t *rows_f16, int64_t *rows_f32, int64_t *rows_host);

/*
 * rg_search_noalloc -- rg_search for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It calls no hipMalloc, hipFree or allocating library
 * routine.  It always runs the persistent search with its exact visited
 * bitmaps, kept in a file-scope device array of 256 MiB that each device
 * the library runs on holds until the process ends (the work counter, then
 * one bitmap of ceil(n / 32) words, rounded up to 64, per resident
 * workgroup); the grid shrinks to the bitmaps that fit.  Arguments, layout
 * and results are those of rg_search (the same ids and distances; hops and
 * evals are the exact counts).  The index's device must be the current
 * device.  Every call on a device shares that device's array and leaves it
 * dirty: calls that overlap on one device race and must be serialized by
 * the caller (one stream, or events).  Asynchronous, like rg_search.
 * Errors: RG_EINVAL (as rg_search; an index whose single bitmap exceeds
 * the array, n > about 2^31 rows; a device other than the index's),
 * RG_EDEVICE.
 */
int rg_search_noalloc(const rg_index *idx, const float *queries, int64_t nq, int32_t k, int32_t L,
                      uint32_t *ids, float *dists, uint32_t *hops, uint32_t *evals, void *stream);

/*
 * rg_search_hashbits -- rg_search with the LDS visited table fixed at
 * 2^hash_bits entries (8..15, and at least twice the ELL row width).  The
 * table only bounds work (a cleared table makes nodes be scored again), so
 * results are identical for every size; tests use it to show that.
 */
int rg_search_hashbits(const rg_index *idx, const float *queries, int64_t nq, int32_t k, int32_t L,
                       uint32_t *ids, float *dists, uint32_t *hops, uint32_t *evals, int32_t hash_bits,
                       void *stream);

/* rg_index_build_stats -- wall seconds of the build's kNN preprocessing
 * (Sec. 5.7 reports it as the dominant share), projection, enhancement and
 * total, and the number of repair edges.  Any output may be NULL. */
int rg_index_build_stats(const rg_index *idx, double *t_knn, double *t_project, double *t_enhance,
                         double *t_total, int64_t *repairs);

/* rg_index_storage_ptrs -- device pointers of the reduced-precision copies
 * (NULL until made by rg_index_set_storage): bf16 rows (pitch elements of
 * 2 bytes); e4m3 rows of pitch8 bytes (a multiple of 128), each holding the
 * d codes, zeros up to a multiple of 4 bytes, the row's FP32 scale and zeros
 * to the pitch (the search reads the scale with the codes); and the scales
 * again as an array of n floats.  The index keeps ownership. */
int rg_index_storage_ptrs(const rg_index *idx, const void **bf16, const void **fp8,
                          const float **scales, int32_t *pitch8);

/* rg_save / rg_load -- index file: header, parameters, entry, CSR, FP32 base
 * rows, and a 64-bit checksum over everything (rg_save needs an index with
 * device data).  Stage graphs and tombstones are not stored.  Errors: RG_EINVAL,
 * RG_ENOMEM, RG_EDEVICE, RG_ECORRUPT (bad magic, size or checksum). */
int rg_save(const rg_index *idx, const char *path);
int rg_load(const char *path, void *stream, rg_index **out);

/* rg_device_copy -- a plain streaming device-to-device copy kernel (16-byte
 * vector loads and stores).  Not part of the method: it gives a copy of
 * known size whose hardware counters calibrate the traffic measured for
 * the search kernels.  dst, src device, 16-byte aligned; bytes % 16 == 0.
 * Asynchronous.  Errors: RG_EINVAL, RG_EDEVICE. */
int rg_device_copy(void *dst, const void *src, int64_t bytes, void *stream);

/* rg_measure_peaks -- measured peaks of the current device, beside which
 * the benchmark quotes its roofline fractions (the datasheet peaks stand
 * alongside).  hbm_read_gbs: a streaming read of a 4 GiB buffer with 16-byte
 * vector loads (best of 5, GB/s).  f16_tflops / f32_tflops: independent FP16
 * 16x16x32 and FP32 16x16x4 MFMA instructions on register operands, 8 per
 * wave in flight, every SIMD busy (best of 3).  Any output may be NULL.
 * Synchronous; allocates and frees its buffers.  Errors: RG_ENOMEM,
 * RG_EDEVICE. */
int rg_measure_peaks(double *hbm_read_gbs, double *f16_tflops, double *f32_tflops, void *stream);

void rg_free(rg_index *idx);
const char *rg_last_error(void);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of search requests with mixed k and L.     */
/* Requests are admitted into device-resident slots as slots and the HBM   */
/* pool allow; every slot keeps its beam state (queue, visited table) in   */
/* device memory between scheduler steps, and each step advances every     */
/* active slot by a bounded number of expansions, so requests that arrive  */
/* while others run join the next step.  A request's result does not       */
/* depend on what else is in flight.                                       */
/* ---------------------------------------------------------------------- */
typedef struct {
    int32_t max_slots;        /* concurrent requests on the device; 0 => twice the
                                 serving-step workgroups the device holds at once */
    int64_t hbm_pool_bytes;   /* bound on slot state bytes; 0 => no bound beyond max_slots */
    int32_t hops_per_step;    /* expansions per slot per step; 0 => 32 */
    int32_t max_L;            /* largest L_eff accepted (<= 512); 0 => 512 */
    int32_t hash_bits;        /* visited table of 2^hash_bits ids per slot (8..13, and at least
                                 twice the candidate batch); it bounds work, not results;
                                 0 => 9 */
} rg_server_limits;

typedef struct {
    uint64_t tag;
    int32_t k;
    int32_t status;           /* RG_OK */
    uint32_t hops, evals;
    uint32_t ids[512];
    float dists[512];
    double t_submit, t_admit, t_done; /* seconds on the server's monotonic clock */
} rg_result;

/* rg_server_create -- start a server (and its scheduler thread) on idx.
 * lim may be NULL (every limit at its default).  idx must outlive the
 * server.  Errors: RG_EINVAL (e.g. max_slots < 0, hash_bits out of range, a
 * pool smaller than one slot), RG_ENOMEM, RG_EDEVICE. */
int rg_server_create(const rg_index *idx, const rg_server_limits *lim, rg_server **out);

/* rg_server_submit -- queue one request; query_host is d floats (copied).
 * Returns RG_EAGAIN when the pending queue is full.  Errors: RG_EINVAL. */
int rg_server_submit(rg_server *s, const float *query_host, int32_t k, int32_t L, uint64_t tag);

/* rg_server_submit_batch -- queue n requests at once (query i is
 * queries_host[i*d .. i*d+d), with k[i], L[i], tags[i]); all get the same
 * submit time.  *n_accepted = how many were queued (in order); RG_EAGAIN
 * when the pending queue filled before all n.  Errors: RG_EINVAL. */
int rg_server_submit_batch(rg_server *s, const float *queries_host, const int32_t *k, const int32_t *L,
                           const uint64_t *tags, int32_t n, int32_t *n_accepted);

/* rg_server_poll -- move up to max finished results into out; *n_out gets
 * the number written.  Never blocks. */
int rg_server_poll(rg_server *s, rg_result *out, int32_t max, int32_t *n_out);

/* rg_server_stats -- requests submitted, admitted, completed, steps run. */
int rg_server_stats(const rg_server *s, uint64_t *submitted, uint64_t *admitted,
                    uint64_t *completed, uint64_t *steps);

/* rg_server_now -- the server's clock (seconds), for request timestamps. */
double rg_server_now(const rg_server *s);

/* rg_server_slots -- slots actually allocated: min(max_slots,
 * hbm_pool_bytes / bytes of one slot's state).  A slot's state is its
 * query, k and L, a queue of 512 (key, id) pairs, 8 state words, the
 * visited table and one result record for each of the two steps in flight. */
int32_t rg_server_slots(const rg_server *s);

/* rg_server_destroy -- finish in-flight work, stop the thread, free all. */
void rg_server_destroy(rg_server *s);

#ifdef __cplusplus
}
#endif

#endif /* ROARGRAPH_H */
