// Host side of index construction: bipartite graph, neighbourhood-aware
// projection, medoid, connectivity enhancement, merge, reachability repair
// and CSR (Algorithms 1-3, Sec. 4.2).  Written for many host threads with a
// result that does not depend on the thread count.
//
// Distances are the canonical FP64 value: delta(a, b) = -sum_i a_i b_i with
// the exact products added in increasing i (a float x float product is exact
// in double, so contraction cannot change it).  All comparisons use the
// total order (delta, id).
//
// Order of updates.  Both Algorithm 2 and the enhancement loop of
// Algorithm 1 visit nodes x in ascending order, set x's own list (an
// assignment) from data that does not change during the loop (the bridges'
// kNN lists; the searches on the fixed projected graph), and then ask every
// selected p to reconsider its list with x added.  Node p's list is
// therefore touched only by (a) its own assignment at step p and (b) those
// reverse insertions, in ascending step order; the assignment discards what
// came before it.  So each p's final list is computed independently: start
// from its own assignment (or empty, for a node that is never a pivot) and
// replay, in ascending x, the reverse insertions from later steps.  This
// gives exactly the serial result with every node processed in parallel.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "rg_internal.h"

namespace rg {
namespace {

using Clock = std::chrono::steady_clock;
double secs(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

constexpr int kHead = 16;  // leading enhancement candidates kept per node for the repair

template <class F>
void parallel_for(int64_t n, int threads, int64_t grain, F &&f) {
    if (n <= 0) return;
    threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, (n + grain - 1) / grain));
    std::atomic<int64_t> next(0);
    auto work = [&](int tid) {
        for (;;) {
            const int64_t s = next.fetch_add(grain);
            if (s >= n) break;
            const int64_t e = std::min(n, s + grain);
            for (int64_t i = s; i < e; ++i) f(i, tid);
        }
    };
    if (threads == 1) {
        work(0);
        return;
    }
    std::vector<std::thread> pool;
    pool.reserve(threads);
    for (int t = 0; t < threads; ++t) pool.emplace_back(work, t);
    for (auto &th : pool) th.join();
}

// A fixed set of worker threads for many small parallel loops in a row
// (thread start-up would dominate them).  run(n, f) calls f(i, tid) for
// i < n on the workers and the caller, and returns when all are done.
class Pool {
  public:
    explicit Pool(int threads) : n_threads_(std::max(1, threads)) {
        for (int t = 1; t < n_threads_; ++t) th_.emplace_back([this, t] { worker(t); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    int size() const { return n_threads_; }
    void run(int n, const std::function<void(int, int)> &f) {
        if (n <= 0) return;
        if (n == 1 || n_threads_ == 1) {
            for (int i = 0; i < n; ++i) f(i, 0);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(m_);
            job_ = &f;
            n_ = n;
            next_.store(0);
            pending_ = n_threads_ - 1;
            ++gen_;
        }
        cv_.notify_all();
        drain(0);
        std::unique_lock<std::mutex> lk(m_);
        done_.wait(lk, [this] { return pending_ == 0; });
        job_ = nullptr;
    }

  private:
    void drain(int tid) {
        for (int i = next_.fetch_add(1); i < n_; i = next_.fetch_add(1)) (*job_)(i, tid);
    }
    void worker(int tid) {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
            }
            drain(tid);
            std::lock_guard<std::mutex> lk(m_);
            if (--pending_ == 0) done_.notify_one();
        }
    }
    int n_threads_;
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, done_;
    const std::function<void(int, int)> *job_ = nullptr;
    int n_ = 0, pending_ = 0;
    std::atomic<int> next_{0};
    uint64_t gen_ = 0;
    bool stop_ = false;
};

// Eight canonical distances at once; each chain is its own left-to-right sum.
void dist8(const float *q, const float *const r[8], int d, double out[8]) {
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0, s6 = 0, s7 = 0;
    for (int i = 0; i < d; ++i) {
        const double qi = (double)q[i];
        s0 += qi * (double)r[0][i];
        s1 += qi * (double)r[1][i];
        s2 += qi * (double)r[2][i];
        s3 += qi * (double)r[3][i];
        s4 += qi * (double)r[4][i];
        s5 += qi * (double)r[5][i];
        s6 += qi * (double)r[6][i];
        s7 += qi * (double)r[7][i];
    }
    out[0] = -s0;
    out[1] = -s1;
    out[2] = -s2;
    out[3] = -s3;
    out[4] = -s4;
    out[5] = -s5;
    out[6] = -s6;
    out[7] = -s7;
}

// out[j] = delta(q, X[ids[j]]) for j < cnt
void dist_batch(const float *X, int d, const float *q, const uint32_t *ids, int64_t cnt, double *out) {
    int64_t j = 0;
    for (; j + 8 <= cnt; j += 8) {
        const float *r[8];
        for (int t = 0; t < 8; ++t) r[t] = X + (int64_t)ids[j + t] * d;
        dist8(q, r, d, out + j);
    }
    for (; j < cnt; ++j) out[j] = canon_dist(q, X + (int64_t)ids[j] * d, d);
}

struct Cand {
    double d;
    uint32_t id;
};
inline bool cless(const Cand &a, const Cand &b) { return a.d < b.d || (a.d == b.d && a.id < b.id); }

// AcquireNeighbors (Algorithm 3) on candidates already ranked by (delta(x,c), c),
// distinct and without x.  Writes the kept candidates (with delta(x,.)) to res.
int acquire_sorted(const float *X, int d, const Cand *C, int nc, int m, bool fill, Cand *res,
                   std::vector<uint8_t> &kept) {
    if (nc <= 0 || m <= 0) return 0;
    kept.assign((size_t)nc, 0);
    int nr = 0;
    res[nr++] = C[0];
    kept[0] = 1;
    for (int j = 1; j < nc && nr < m; ++j) {
        const float *xc = X + (int64_t)C[j].id * d;
        bool ok = true;
        for (int r0 = 0; r0 < nr && ok; r0 += 8) {
            const int cnt = std::min(8, nr - r0);
            double dcp[8];
            if (cnt == 8) {
                const float *rows[8];
                for (int t = 0; t < 8; ++t) rows[t] = X + (int64_t)res[r0 + t].id * d;
                dist8(xc, rows, d, dcp);
            } else {
                for (int t = 0; t < cnt; ++t) dcp[t] = canon_dist(xc, X + (int64_t)res[r0 + t].id * d, d);
            }
            for (int t = 0; t < cnt; ++t)
                if (!(C[j].d < dcp[t])) {
                    ok = false;
                    break;
                }
        }
        if (ok) {
            res[nr++] = C[j];
            kept[j] = 1;
        }
    }
    if (fill)
        for (int j = 0; j < nc && nr < m; ++j)
            if (!kept[j]) res[nr++] = C[j];
    return nr;
}

// acquire_sorted with the candidate-to-kept distances taken from a cache.
int acquire_sorted_cached(const float *X, int d, const Cand *C, int nc, int m, bool fill, Cand *res,
                          std::vector<uint8_t> &kept, PairCache &pc) {
    if (nc <= 0 || m <= 0) return 0;
    kept.assign((size_t)nc, 0);
    int nr = 0;
    res[nr++] = C[0];
    kept[0] = 1;
    for (int j = 1; j < nc && nr < m; ++j) {
        bool ok = true;
        for (int r = 0; r < nr && ok; ++r) ok = C[j].d < pc.get(X, d, C[j].id, res[r].id);
        if (ok) {
            res[nr++] = C[j];
            kept[j] = 1;
        }
    }
    if (fill)
        for (int j = 0; j < nc && nr < m; ++j)
            if (!kept[j]) res[nr++] = C[j];
    return nr;
}

// Fixed-capacity adjacency lists with their distances to the owner.
struct Lists {
    int cap = 0;
    std::vector<Cand> a;
    std::vector<int32_t> deg;
    void init(int64_t n, int c) {
        cap = c;
        a.assign((size_t)n * c, Cand{0, 0});
        deg.assign((size_t)n, 0);
    }
    Cand *row(int64_t x) { return a.data() + x * cap; }
    const Cand *row(int64_t x) const { return a.data() + x * cap; }
};

// Events: for each target p, the ascending steps x whose selection contains p.
void build_events(const Lists &sel, int64_t n, std::vector<int64_t> &off, std::vector<uint32_t> &src) {
    off.assign((size_t)n + 1, 0);
    for (int64_t x = 0; x < n; ++x)
        for (int j = 0; j < sel.deg[x]; ++j) off[sel.row(x)[j].id + 1]++;
    for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
    src.resize((size_t)off[n]);
    std::vector<int64_t> fillp(off.begin(), off.end() - 1);
    for (int64_t x = 0; x < n; ++x)  // ascending x => each target's events ascend
        for (int j = 0; j < sel.deg[x]; ++j) src[fillp[sel.row(x)[j].id]++] = (uint32_t)x;
}

// Replay reverse insertions into p (see the file comment).
//   start: p's own assignment (is_assigned) or empty.
void replay(const float *X, int d, int64_t p, bool is_assigned, const Cand *start, int nstart,
            const uint32_t *ev, int64_t nev, int m, bool fill, Cand *out, int32_t *outdeg,
            std::vector<Cand> &cur, std::vector<Cand> &tmp, std::vector<uint8_t> &kept, PairCache &pc) {
    pc.clear();
    cur.assign(start, start + nstart);
    const float *xp = X + p * d;
    for (int64_t e = 0; e < nev; ++e) {
        const uint32_t x = ev[e];
        if (is_assigned && (int64_t)x < p) continue;  // discarded by p's own assignment
        bool present = false;
        for (const Cand &c : cur)
            if (c.id == x) {
                present = true;
                break;
            }
        if (!present) cur.push_back(Cand{canon_dist(xp, X + (int64_t)x * d, d), x});
        if (fill && (int)cur.size() <= m) continue;  // with fill, <= m candidates are all kept
        std::sort(cur.begin(), cur.end(), cless);
        tmp.resize(cur.size());
        const int nr = acquire_sorted_cached(X, d, cur.data(), (int)cur.size(), m, fill, tmp.data(), kept, pc);
        cur.assign(tmp.begin(), tmp.begin() + nr);
    }
    *outdeg = (int32_t)cur.size();
    std::copy(cur.begin(), cur.end(), out);
}

// Beam search on a fixed graph with canonical distances (Sec. 4.3 semantics).
struct Searcher {
    std::vector<uint32_t> stamp;
    uint32_t epoch = 0;
    std::vector<double> qd;
    std::vector<uint32_t> qi;
    std::vector<uint8_t> qx;
    std::vector<uint32_t> nb;
    std::vector<double> nd;
    void init(int64_t n, int Leff) {
        stamp.assign((size_t)n, 0);
        qd.resize((size_t)Leff + 1);
        qi.resize((size_t)Leff + 1);
        qx.resize((size_t)Leff + 1);
    }
    // returns the queue length; qd/qi hold the queue in (delta, id) order
    int run(const float *X, int d, const int64_t *off, const uint32_t *idx, uint32_t entry, const float *q,
            int Leff) {
        if (++epoch == 0) {
            std::fill(stamp.begin(), stamp.end(), 0);
            epoch = 1;
        }
        stamp[entry] = epoch;
        int qn = 1;
        qd[0] = canon_dist(q, X + (int64_t)entry * d, d);
        qi[0] = entry;
        qx[0] = 0;
        int ptr = 0;
        for (;;) {
            while (ptr < qn && qx[ptr]) ++ptr;
            if (ptr == qn) break;
            qx[ptr] = 1;
            const uint32_t v = qi[ptr];
            nb.clear();
            for (int64_t e = off[v]; e < off[v + 1]; ++e) {
                const uint32_t u = idx[e];
                if (stamp[u] == epoch) continue;
                stamp[u] = epoch;
                nb.push_back(u);
            }
            nd.resize(nb.size());
            dist_batch(X, d, q, nb.data(), (int64_t)nb.size(), nd.data());
            int first = qn;
            for (size_t j = 0; j < nb.size(); ++j) {
                const double du = nd[j];
                const uint32_t u = nb[j];
                if (qn == Leff && !(du < qd[Leff - 1] || (du == qd[Leff - 1] && u < qi[Leff - 1]))) continue;
                // binary search for the insertion point
                int lo = 0, hi = qn;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (qd[mid] < du || (qd[mid] == du && qi[mid] < u))
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                const int last = qn < Leff ? qn : Leff - 1;
                for (int t = last; t > lo; --t) {
                    qd[t] = qd[t - 1];
                    qi[t] = qi[t - 1];
                    qx[t] = qx[t - 1];
                }
                qd[lo] = du;
                qi[lo] = u;
                qx[lo] = 0;
                if (qn < Leff) ++qn;
                if (lo < first) first = lo;
            }
            if (first < ptr) ptr = first;
        }
        return qn;
    }
};

void lists_to_csr(const Lists &L, int64_t n, std::vector<int64_t> &off, std::vector<uint32_t> &idx) {
    off.assign((size_t)n + 1, 0);
    for (int64_t x = 0; x < n; ++x) off[x + 1] = off[x] + L.deg[x];
    idx.resize((size_t)off[n]);
    for (int64_t x = 0; x < n; ++x)
        for (int j = 0; j < L.deg[x]; ++j) idx[off[x] + j] = L.row(x)[j].id;
}

// Enhancement on the device: the searches of every node on G_pj and each
// node's own selection (AcquireNeighbors without fill), both with the
// canonical FP64 distance, so the lists are bit-identical to the host's.
// Only the selections and the first kHead candidates come back.  Double
// buffered: batch i+1 runs on the device while batch i is copied out.
int enhance_on_device(const float *X, int64_t n, int32_t d, const Lists &PJ, uint32_t entry, int32_t L, int32_t m_ce,
                      int threads, const GpuCtx &gpu, Lists &E, std::vector<uint32_t> &head,
                      std::vector<int32_t> &head_n, double *t_search) {
    (void)X;
    int32_t maxdeg = 1;
    for (int64_t x = 0; x < n; ++x) maxdeg = std::max<int32_t>(maxdeg, PJ.deg[x]);
    const int32_t ell = (maxdeg + 7) / 8 * 8;
    std::vector<uint32_t> adj((size_t)n * ell, kNone);
    for (int64_t x = 0; x < n; ++x)
        for (int j = 0; j < PJ.deg[x]; ++j) adj[x * ell + j] = PJ.row(x)[j].id;
    const int64_t B = std::min<int64_t>(n, 1 << 15);
    const int32_t m = std::max(1, m_ce);
    uint32_t *d_adj = nullptr, *d_q = nullptr;
    double *d_qd = nullptr;
    int32_t *d_qn = nullptr;
    uint32_t *d_sid[2] = {nullptr, nullptr}, *h_sid[2] = {nullptr, nullptr};
    double *d_sd[2] = {nullptr, nullptr}, *h_sd[2] = {nullptr, nullptr};
    int32_t *d_sn[2] = {nullptr, nullptr}, *h_sn[2] = {nullptr, nullptr};
    uint32_t *d_hd[2] = {nullptr, nullptr}, *h_hd[2] = {nullptr, nullptr};
    int32_t *d_hn[2] = {nullptr, nullptr}, *h_hn[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto release = [&]() {
        for (void *p : {(void *)d_adj, (void *)d_q, (void *)d_qd, (void *)d_qn})
            if (p) (void)hipFree(p);
        for (int i = 0; i < 2; ++i) {
            for (void *p : {(void *)d_sid[i], (void *)d_sd[i], (void *)d_sn[i], (void *)d_hd[i], (void *)d_hn[i]})
                if (p) (void)hipFree(p);
            for (void *p : {(void *)h_sid[i], (void *)h_sd[i], (void *)h_sn[i], (void *)h_hd[i], (void *)h_hn[i]})
                if (p) (void)hipHostFree(p);
            if (ev[i]) (void)hipEventDestroy(ev[i]);
        }
    };
    bool ok = hipMalloc(&d_adj, sizeof(uint32_t) * adj.size()) == hipSuccess &&
              hipMalloc(&d_q, sizeof(uint32_t) * B * L) == hipSuccess &&
              hipMalloc(&d_qd, sizeof(double) * B * L) == hipSuccess &&
              hipMalloc(&d_qn, sizeof(int32_t) * B) == hipSuccess;
    for (int i = 0; i < 2 && ok; ++i)
        ok = hipMalloc(&d_sid[i], sizeof(uint32_t) * B * m) == hipSuccess &&
             hipMalloc(&d_sd[i], sizeof(double) * B * m) == hipSuccess &&
             hipMalloc(&d_sn[i], sizeof(int32_t) * B) == hipSuccess &&
             hipMalloc(&d_hd[i], sizeof(uint32_t) * B * kHead) == hipSuccess &&
             hipMalloc(&d_hn[i], sizeof(int32_t) * B) == hipSuccess &&
             hipHostMalloc(&h_sid[i], sizeof(uint32_t) * B * m, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc(&h_sd[i], sizeof(double) * B * m, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc(&h_sn[i], sizeof(int32_t) * B, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc(&h_hd[i], sizeof(uint32_t) * B * kHead, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc(&h_hn[i], sizeof(int32_t) * B, hipHostMallocDefault) == hipSuccess &&
             hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        release();
        set_error("build: out of memory for enhancement searches");
        return RG_ENOMEM;
    }
    const auto tstart = Clock::now();
    double t_host = 0.0;
    int rc = RG_OK;
    // search and select batch b on the device, copy its selections into buffer b % 2
    auto issue = [&](int64_t b) -> int {
        const int64_t x0 = b * B, cnt = std::min(B, n - x0);
        const int i = (int)(b & 1);
        int r = launch_canon_search(gpu.X, d, gpu.pitch, d_adj, ell, entry, L, x0, cnt, d_q, d_qd, d_qn, gpu.stream);
        if (!r)
            r = launch_canon_select(gpu.X, d, gpu.pitch, d_q, d_qd, d_qn, L, x0, cnt, m, d_sid[i], d_sd[i], d_sn[i],
                                    d_hd[i], kHead, d_hn[i], gpu.stream);
        if (r) return r;
        if (hipMemcpyAsync(h_sid[i], d_sid[i], sizeof(uint32_t) * cnt * m, hipMemcpyDeviceToHost, gpu.stream) !=
                hipSuccess ||
            hipMemcpyAsync(h_sd[i], d_sd[i], sizeof(double) * cnt * m, hipMemcpyDeviceToHost, gpu.stream) !=
                hipSuccess ||
            hipMemcpyAsync(h_sn[i], d_sn[i], sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, gpu.stream) != hipSuccess ||
            hipMemcpyAsync(h_hd[i], d_hd[i], sizeof(uint32_t) * cnt * kHead, hipMemcpyDeviceToHost, gpu.stream) !=
                hipSuccess ||
            hipMemcpyAsync(h_hn[i], d_hn[i], sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, gpu.stream) != hipSuccess ||
            hipEventRecord(ev[i], gpu.stream) != hipSuccess) {
            set_error("build: enhancement on the device failed");
            return RG_EDEVICE;
        }
        return RG_OK;
    };
    const int64_t nb = (n + B - 1) / B;
    if (hipMemcpyAsync(d_adj, adj.data(), sizeof(uint32_t) * adj.size(), hipMemcpyHostToDevice, gpu.stream) !=
        hipSuccess)
        rc = RG_EDEVICE;
    if (!rc) rc = issue(0);
    for (int64_t b = 0; b < nb && !rc; ++b) {
        if (b + 1 < nb) rc = issue(b + 1);  // the device works on the next batch meanwhile
        if (rc) break;
        const int i = (int)(b & 1);
        if (hipEventSynchronize(ev[i]) != hipSuccess) {
            set_error("build: enhancement on the device failed");
            rc = RG_EDEVICE;
            break;
        }
        const auto th0 = Clock::now();
        const int64_t x0 = b * B, cnt = std::min(B, n - x0);
        parallel_for(cnt, threads, 256, [&](int64_t bb, int) {
            const int64_t x = x0 + bb;
            const int ns = std::min(h_sn[i][bb], m);
            for (int j = 0; j < ns; ++j) E.row(x)[j] = Cand{h_sd[i][bb * m + j], h_sid[i][bb * m + j]};
            E.deg[x] = ns;
            head_n[x] = h_hn[i][bb];
            const int nh = std::min(head_n[x], kHead);
            for (int j = 0; j < nh; ++j) head[x * kHead + j] = h_hd[i][bb * kHead + j];
        });
        t_host += secs(th0, Clock::now());
        // about ten progress lines per build
        const int64_t step = std::max<int64_t>(cnt, (n / 10 + cnt - 1) / cnt * cnt);
        if (std::getenv("RG_LOG") && ((x0 + cnt) % step == 0 || x0 + cnt == n))
            std::fprintf(stderr, "[rg] enhancement searches %lld / %lld nodes\n", (long long)(x0 + cnt), (long long)n);
        // buffer i is reused by batch b + 2, issued in the next iteration
    }
    (void)hipStreamSynchronize(gpu.stream);
    release();
    *t_search = secs(tstart, Clock::now()) - t_host;
    return rc;
}

}  // namespace

double canon_dist(const float *a, const float *b, int32_t d) {
    double s = 0.0;
    for (int32_t i = 0; i < d; ++i) s += (double)a[i] * (double)b[i];
    return -s;
}

int hw_threads(int requested) {
    if (requested > 0) return requested;
    const unsigned h = std::thread::hardware_concurrency();
    return h ? (int)h : 1;
}

int host_construct(const float *X, int64_t n, int32_t d, const uint32_t *knn, int64_t nt, int32_t Nq, int32_t M,
                   int32_t L, int32_t m_pj, int32_t m_ce, int threads, const GpuCtx *gpu, bool keep_stages,
                   HostGraph *out) {
    const auto t0 = Clock::now();
    threads = hw_threads(threads);
    const int q1 = Nq - 1;

    // --- bipartite graph (Algorithm 1): pivot of t gets t as a bridge ------
    std::vector<int64_t> boff((size_t)n + 1, 0);
    for (int64_t t = 0; t < nt; ++t) boff[knn[t * Nq] + 1]++;
    for (int64_t i = 0; i < n; ++i) boff[i + 1] += boff[i];
    std::vector<uint32_t> bidx((size_t)nt);
    {
        std::vector<int64_t> fp(boff.begin(), boff.end() - 1);
        for (int64_t t = 0; t < nt; ++t) bidx[fp[knn[t * Nq]]++] = (uint32_t)t;
    }

    // --- projection, forward selections F(x) of every pivot ---------------
    const int capl = std::max(m_pj, m_ce) + 1;
    Lists F;
    F.init(n, capl);
    {
        std::vector<std::vector<uint32_t>> stamp((size_t)threads);
        std::vector<std::vector<uint32_t>> cid((size_t)threads);
        std::vector<std::vector<double>> cdd((size_t)threads);
        std::vector<std::vector<Cand>> cc((size_t)threads);
        std::vector<std::vector<uint8_t>> kept((size_t)threads);
        parallel_for(n, threads, 64, [&](int64_t x, int tid) {
            if (boff[x] == boff[x + 1]) return;
            auto &st = stamp[tid];
            if (st.empty()) st.assign((size_t)n, 0);
            auto &ids = cid[tid];
            ids.clear();
            const uint32_t mark = (uint32_t)x + 1u;
            for (int64_t b = boff[x]; b < boff[x + 1]; ++b) {
                if ((int64_t)ids.size() >= L) break;
                const uint32_t *lst = knn + (int64_t)bidx[b] * Nq + 1;
                for (int j = 0; j < q1; ++j) {
                    const uint32_t c = lst[j];
                    if ((int64_t)c == x || st[c] == mark) continue;
                    st[c] = mark;
                    ids.push_back(c);
                }
            }
            auto &dd = cdd[tid];
            dd.resize(ids.size());
            dist_batch(X, d, X + x * d, ids.data(), (int64_t)ids.size(), dd.data());
            auto &c = cc[tid];
            c.resize(ids.size());
            for (size_t j = 0; j < ids.size(); ++j) c[j] = Cand{dd[j], ids[j]};
            std::sort(c.begin(), c.end(), cless);
            const int nk = (int)std::min<int64_t>((int64_t)c.size(), L);
            F.deg[x] = acquire_sorted(X, d, c.data(), nk, m_pj, true, F.row(x), kept[tid]);
        });
    }
    // --- projection, reverse insertions replayed per target ---------------
    Lists PJ;
    PJ.init(n, capl);
    {
        std::vector<int64_t> eoff;
        std::vector<uint32_t> esrc;
        build_events(F, n, eoff, esrc);
        std::vector<std::vector<Cand>> cur((size_t)threads), tmp((size_t)threads);
        std::vector<std::vector<uint8_t>> kept((size_t)threads);
        std::vector<PairCache> pcs((size_t)threads);
        parallel_for(n, threads, 256, [&](int64_t p, int tid) {
            const bool piv = boff[p] != boff[p + 1];
            replay(X, d, p, piv, F.row(p), piv ? F.deg[p] : 0, esrc.data() + eoff[p], eoff[p + 1] - eoff[p], m_pj,
                   true, PJ.row(p), &PJ.deg[p], cur[tid], tmp[tid], kept[tid], pcs[tid]);
        });
    }
    std::vector<int64_t> pjoff;
    std::vector<uint32_t> pjidx;
    lists_to_csr(PJ, n, pjoff, pjidx);
    const auto t1 = Clock::now();
    const bool log = std::getenv("RG_LOG") != nullptr;
    if (log) std::fprintf(stderr, "[rg] projection done in %.2f s\n", secs(t0, t1));

    // --- entry: nearest to the mean among nodes with a projected out-edge --
    std::vector<double> mu((size_t)d, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int j = 0; j < d; ++j) mu[j] += (double)X[i * d + j];
    for (int j = 0; j < d; ++j) mu[j] = mu[j] / (double)n;
    // the row nearest (L2) to the mean among rows with keep(i), or among all
    // rows when none qualifies; lower id on ties
    auto nearest_mean = [&](auto keep) -> uint32_t {
        bool any = false;
        for (int64_t i = 0; i < n && !any; ++i) any = keep(i);
        const int64_t chunk = 4096;
        const int64_t nchunk = (n + chunk - 1) / chunk;
        std::vector<double> bestd((size_t)nchunk, INFINITY);
        std::vector<int64_t> besti((size_t)nchunk, -1);
        parallel_for(nchunk, threads, 1, [&](int64_t c, int) {
            for (int64_t i = c * chunk; i < std::min(n, (c + 1) * chunk); ++i) {
                if (any && !keep(i)) continue;
                double s2 = 0.0;
                for (int j = 0; j < d; ++j) {
                    const double t = (double)X[i * d + j] - mu[j];
                    s2 += t * t;
                }
                if (s2 < bestd[c]) {
                    bestd[c] = s2;
                    besti[c] = i;
                }
            }
        });
        double b = INFINITY;
        uint32_t e = 0;
        for (int64_t c = 0; c < nchunk; ++c)
            if (besti[c] >= 0 && bestd[c] < b) {
                b = bestd[c];
                e = (uint32_t)besti[c];
            }
        return e;
    };
    const uint32_t entry = nearest_mean([&](int64_t i) { return PJ.deg[i] > 0; });

    // --- enhancement: searches on G_pj and each node's own selection E(x) --
    Lists E;
    E.init(n, capl);
    std::vector<uint32_t> head((size_t)n * kHead, kNone);
    std::vector<int32_t> head_n((size_t)n, 0);
    if (gpu) {
        const int rc = enhance_on_device(X, n, d, PJ, entry, L, m_ce, threads, *gpu, E, head, head_n,
                                         &out->t_enhance_search);
        if (rc) return rc;
    } else {
        std::vector<Searcher> sr((size_t)threads);
        std::vector<std::vector<Cand>> cc((size_t)threads);
        std::vector<std::vector<uint8_t>> kept((size_t)threads);
        parallel_for(n, threads, 16, [&](int64_t x, int tid) {
            Searcher &s = sr[tid];
            if (s.stamp.empty()) s.init(n, L);
            const int qn = s.run(X, d, pjoff.data(), pjidx.data(), entry, X + x * d, L);
            auto &c = cc[tid];
            c.clear();
            for (int j = 0; j < qn; ++j)
                if ((int64_t)s.qi[j] != x) c.push_back(Cand{s.qd[j], s.qi[j]});
            head_n[x] = (int32_t)c.size();
            for (int j = 0; j < kHead && j < (int)c.size(); ++j) head[x * kHead + j] = c[j].id;
            E.deg[x] = acquire_sorted(X, d, c.data(), (int)c.size(), m_ce, false, E.row(x), kept[tid]);
        });
    }
    const auto t1b = Clock::now();
    Lists CE;
    CE.init(n, capl);
    {
        std::vector<int64_t> eoff;
        std::vector<uint32_t> esrc;
        build_events(E, n, eoff, esrc);
        std::vector<std::vector<Cand>> cur((size_t)threads), tmp((size_t)threads);
        std::vector<std::vector<uint8_t>> kept((size_t)threads);
        std::vector<PairCache> pcs((size_t)threads);
        parallel_for(n, threads, 256, [&](int64_t p, int tid) {
            replay(X, d, p, true, E.row(p), E.deg[p], esrc.data() + eoff[p], eoff[p + 1] - eoff[p], m_ce, false,
                   CE.row(p), &CE.deg[p], cur[tid], tmp[tid], kept[tid], pcs[tid]);
        });
    }
    const auto t2 = Clock::now();
    if (log)
        std::fprintf(stderr, "[rg] enhancement done in %.2f s (searches and selections %.2f s, reverse updates %.2f s)\n",
                     secs(t1, t2), secs(t1, t1b), secs(t1b, t2));

    // --- merge: final(x) = G_pj(x) u G'(x) -------------------------------
    std::vector<std::vector<uint32_t>> fin((size_t)n);
    parallel_for(n, threads, 1024, [&](int64_t x, int) {
        auto &r = fin[x];
        r.reserve((size_t)M);
        for (int j = 0; j < PJ.deg[x]; ++j) r.push_back(PJ.row(x)[j].id);
        for (int j = 0; j < CE.deg[x]; ++j) {
            const uint32_t u = CE.row(x)[j].id;
            if (std::find(r.begin(), r.end(), u) == r.end()) r.push_back(u);
        }
        std::sort(r.begin(), r.end());  // the repair's BFS visits neighbours in ascending id
    });

    // --- reachability repair ---------------------------------------------
    int64_t repairs = 0;
    {
        std::vector<uint8_t> seen((size_t)n, 0);
        std::vector<uint32_t> order;
        order.reserve((size_t)n);
        size_t qhead = 0;
        seen[entry] = 1;
        order.push_back(entry);
        auto bfs = [&]() {
            while (qhead < order.size()) {
                const uint32_t v = order[qhead++];
                for (uint32_t w : fin[v])
                    if (!seen[w]) {
                        seen[w] = 1;
                        order.push_back(w);
                    }
            }
        };
        bfs();
        Searcher s;
        // order[0 .. first_free) are all full; rows only grow, so the first
        // node of `order` with a free slot never moves back
        size_t first_free = 0;
        int64_t searches = 0;
        for (int64_t u = 0; u < n; ++u) {
            if (seen[u]) continue;
            // first node of u's enhancement candidates (queue order) with a free
            // slot; every one of them was reached from the entry through G_pj
            int64_t r = -1;
            for (int j = 0; j < kHead && j < head_n[u] && r < 0; ++j) {
                const uint32_t c = head[u * kHead + j];
                if (seen[c] && (int)fin[c].size() < M) r = c;
            }
            if (r < 0 && head_n[u] > kHead) {  // rare: the stored head is full, search again
                if (s.stamp.empty()) s.init(n, L);
                ++searches;
                const int qn = s.run(X, d, pjoff.data(), pjidx.data(), entry, X + u * d, L);
                for (int j = 0; j < qn && r < 0; ++j) {
                    const uint32_t c = s.qi[j];
                    if ((int64_t)c != u && seen[c] && (int)fin[c].size() < M) r = c;
                }
            }
            if (r < 0) {
                while (first_free < order.size() && (int)fin[order[first_free]].size() >= M) ++first_free;
                if (first_free < order.size()) r = order[first_free];
            }
            if (r < 0) {
                set_error("build: reachability repair found no node with a free slot");
                return RG_EINTERNAL;
            }
            fin[r].push_back((uint32_t)u);
            ++repairs;
            seen[u] = 1;
            order.push_back((uint32_t)u);
            bfs();
        }
        if (log && repairs)
            std::fprintf(stderr, "[rg] repair: %lld edges, %lld nodes searched again (stored head full)\n",
                         (long long)repairs, (long long)searches);
    }

    // --- CSR, rows sorted by id ------------------------------------------
    out->offsets.assign((size_t)n + 1, 0);
    for (int64_t x = 0; x < n; ++x) out->offsets[x + 1] = out->offsets[x] + (int64_t)fin[x].size();
    out->indices.resize((size_t)out->offsets[n]);
    parallel_for(n, threads, 4096, [&](int64_t x, int) {
        std::sort(fin[x].begin(), fin[x].end());
        std::copy(fin[x].begin(), fin[x].end(), out->indices.begin() + out->offsets[x]);
    });
    out->entry = entry;
    out->repairs = repairs;
    if (keep_stages) {
        // G_bi routing: row x = N_out(t) for each bridge t of x, ascending t
        StageGraphs &sg = out->stages;
        sg.kept = true;
        sg.nt = nt;
        sg.q1 = q1;
        sg.n_built = n;
        sg.nout.resize((size_t)nt * q1);
        for (int64_t t = 0; t < nt; ++t)
            std::copy(knn + t * Nq + 1, knn + (t + 1) * Nq, sg.nout.begin() + t * q1);
        sg.bi_off.assign((size_t)n + 1, 0);
        for (int64_t x = 0; x < n; ++x) sg.bi_off[x + 1] = sg.bi_off[x] + (boff[x + 1] - boff[x]) * q1;
        sg.bi_idx.resize((size_t)sg.bi_off[n]);
        parallel_for(n, threads, 1024, [&](int64_t x, int) {
            int64_t o = sg.bi_off[x];
            for (int64_t b = boff[x]; b < boff[x + 1]; ++b, o += q1)
                std::copy(sg.nout.begin() + (int64_t)bidx[b] * q1, sg.nout.begin() + ((int64_t)bidx[b] + 1) * q1,
                          sg.bi_idx.begin() + o);
        });
        sg.entry_bi = nearest_mean([&](int64_t i) { return boff[i + 1] > boff[i]; });
        sg.b_off.swap(boff);
        sg.b_idx.swap(bidx);
        sg.pj_off.swap(pjoff);
        sg.pj_idx.swap(pjidx);
        parallel_for(n, threads, 4096, [&](int64_t x, int) {
            std::sort(sg.pj_idx.begin() + sg.pj_off[x], sg.pj_idx.begin() + sg.pj_off[x + 1]);
        });
    }
    const auto t3 = Clock::now();
    if (log) std::fprintf(stderr, "[rg] repair (%lld edges) and CSR done in %.2f s\n", (long long)repairs, secs(t2, t3));
    out->t_project = secs(t0, t1);
    out->t_enhance = secs(t1, t2);
    out->t_total = secs(t0, t3);
    return RG_OK;
}

void host_canon_searches(const float *X, int32_t d, const int64_t *off, const uint32_t *idx, uint32_t entry,
                         int32_t L, int64_t x0, int64_t count, int threads, uint32_t *ids, int32_t *counts) {
    const int64_t n = x0;  // graph nodes are the rows before x0
    threads = hw_threads(threads);
    std::vector<Searcher> sr((size_t)threads);
    parallel_for(count, threads, 8, [&](int64_t i, int tid) {
        Searcher &s = sr[tid];
        if (s.stamp.empty()) s.init(n, L);
        const int qn = s.run(X, d, off, idx, entry, X + (x0 + i) * d, L);
        counts[i] = qn;
        std::copy(s.qi.begin(), s.qi.begin() + qn, ids + i * L);
    });
}

// Insertion through the saved bipartite graph (the paper's update
// procedure), one new row v at a time in input order:
//   1. b = the first node of v's queue that is joined to a query node (b is
//      the pivot of t, or b is in N_out(t)); q = the nearest such t to v by
//      (delta(v, t), t).  Without any, v's candidates are its queue.
//   2. Project the sub-bipartite graph N_out(q) u {q, v} with v as pivot:
//      candidates N_out(q) ranked by (delta(v, c), c), cut to L,
//      AcquireNeighbors with fill to m_pj -> v's row.
//   3. Merge as Algorithm 2's reverse step: each selected p, in order, takes
//      row(p) <- AcquireNeighbors(p, row(p) u {v}, M) with fill (a row with
//      room gains v; a full row keeps M by the rule).  If no p kept v, v gets
//      one in-edge by the build's repair rule (first queue node with a free
//      slot, else the first node in BFS order from the entry).
//   4. Append v to N_out(q).
// At the end, every node the entry no longer reaches (a full row may drop an
// old neighbour) gets one in-edge, in ascending id, from the first node in
// BFS order with a free slot.
int host_insert(StageGraphs &sg, int32_t d, int32_t M, int32_t m_pj, int32_t L, uint32_t entry, int64_t n0,
                int64_t nv, const uint32_t *queue_ids, const int32_t *queue_n, std::vector<int64_t> &offsets,
                std::vector<uint32_t> &indices, int threads) {
    const float *X = sg.base.data();
    const float *T = sg.train.data();
    const int64_t nb = sg.n_built, q1 = sg.q1, N = n0 + nv;
    if (sg.inq_off.empty()) {  // queries holding each built node in N_out
        sg.inq_off.assign((size_t)nb + 1, 0);
        for (int64_t e = 0; e < sg.nt * q1; ++e) sg.inq_off[sg.nout[e] + 1]++;
        for (int64_t x = 0; x < nb; ++x) sg.inq_off[x + 1] += sg.inq_off[x];
        sg.inq_idx.resize((size_t)sg.inq_off[nb]);
        std::vector<int64_t> fp(sg.inq_off.begin(), sg.inq_off.end() - 1);
        for (int64_t t = 0; t < sg.nt; ++t)
            for (int64_t j = 0; j < q1; ++j) sg.inq_idx[fp[sg.nout[t * q1 + j]]++] = (uint32_t)t;
        sg.nout_add.assign((size_t)sg.nt, {});
    }
    sg.inq_add.resize((size_t)(N - nb));
    // rows, sorted by id, as they change
    std::vector<std::vector<uint32_t>> rows((size_t)N);
    for (int64_t x = 0; x < n0; ++x) rows[x].assign(indices.begin() + offsets[x], indices.begin() + offsets[x + 1]);
    auto joined = [&](uint32_t b, std::vector<uint32_t> &out) {
        out.clear();
        if ((int64_t)b < nb) {
            for (int64_t e = sg.b_off[b]; e < sg.b_off[b + 1]; ++e) out.push_back(sg.b_idx[e]);
            for (int64_t e = sg.inq_off[b]; e < sg.inq_off[b + 1]; ++e) out.push_back(sg.inq_idx[e]);
        } else {
            for (uint32_t t : sg.inq_add[b - nb]) out.push_back(t);
        }
    };
    // BFS from the entry over the current rows (neighbours ascending); the
    // first node with a free slot, or -1
    auto first_free_in_bfs = [&](int64_t limit) -> int64_t {
        std::vector<uint8_t> seen((size_t)limit, 0);
        std::vector<uint32_t> order{entry};
        seen[entry] = 1;
        for (size_t h = 0; h < order.size(); ++h) {
            const uint32_t x = order[h];
            if ((int64_t)rows[x].size() < M) return x;
            for (uint32_t w : rows[x])
                if (!seen[w]) {
                    seen[w] = 1;
                    order.push_back(w);
                }
        }
        return -1;
    };
    Pool pool(hw_threads(threads));
    std::vector<std::vector<Cand>> tcand((size_t)pool.size()), tres((size_t)pool.size());
    std::vector<std::vector<uint8_t>> tkept((size_t)pool.size());
    std::vector<std::vector<uint32_t>> tqs((size_t)pool.size());
    for (auto &r : tres) r.resize((size_t)std::max(M, std::max(m_pj, 1)));

    // v's bridge query q (the training query nearest v among those joined to
    // the first queue node that has any) and v's own list: AcquireNeighbors
    // over N_out(q) and the rows already linked to q, else over the queue.
    // Both read only data fixed at the call's start, except nout_add[q],
    // which grows when an earlier row of this call had the same q.
    auto bridge = [&](int64_t i, std::vector<uint32_t> &qs) -> int64_t {
        const float *xv = X + (n0 + i) * d;
        const uint32_t *queue = queue_ids + i * L;
        int64_t q = -1;
        for (int j = 0; j < queue_n[i] && q < 0; ++j) {
            joined(queue[j], qs);
            double best = INFINITY;
            for (uint32_t t : qs) {
                const double dt = canon_dist(xv, T + (int64_t)t * d, d);
                if (q < 0 || dt < best || (dt == best && t < (uint32_t)q)) {
                    best = dt;
                    q = t;
                }
            }
        }
        return q;
    };
    auto own_list = [&](int64_t i, int64_t q, std::vector<Cand> &cand, std::vector<Cand> &res,
                        std::vector<uint8_t> &kept, std::vector<uint32_t> &sel) {
        const float *xv = X + (n0 + i) * d;
        const uint32_t *queue = queue_ids + i * L;
        cand.clear();
        if (q >= 0) {
            for (int64_t j = 0; j < q1; ++j) cand.push_back(Cand{0.0, sg.nout[q * q1 + j]});
            for (uint32_t u : sg.nout_add[q]) cand.push_back(Cand{0.0, u});
        } else {
            for (int j = 0; j < queue_n[i]; ++j) cand.push_back(Cand{0.0, queue[j]});
        }
        for (Cand &c : cand) c.d = canon_dist(xv, X + (int64_t)c.id * d, d);
        std::sort(cand.begin(), cand.end(), cless);
        cand.erase(std::unique(cand.begin(), cand.end(), [](const Cand &a, const Cand &b) { return a.id == b.id; }),
                   cand.end());
        const int nc = (int)std::min<int64_t>((int64_t)cand.size(), L);
        const int ns = acquire_sorted(X, d, cand.data(), nc, m_pj, true, res.data(), kept);
        sel.resize((size_t)ns);
        for (int j = 0; j < ns; ++j) sel[j] = res[j].id;
    };
    // all rows' bridges and lists in parallel, as of the call's start
    std::vector<int64_t> qv((size_t)nv);
    std::vector<std::vector<uint32_t>> selv((size_t)nv);
    pool.run((int)nv, [&](int i, int tid) {
        qv[i] = bridge(i, tqs[tid]);
        own_list(i, qv[i], tcand[tid], tres[tid], tkept[tid], selv[i]);
    });
    std::vector<uint8_t> q_used(sg.nout_add.size(), 0);

    std::vector<uint32_t> full;
    std::vector<uint8_t> keeps_v;
    for (int64_t i = 0; i < nv; ++i) {
        const int64_t v = n0 + i;
        const float *xv = X + v * d;
        const uint32_t *queue = queue_ids + i * L;
        const int qn = queue_n[i];
        const int64_t q = qv[i];
        std::vector<uint32_t> &sel = selv[i];
        if (q >= 0 && q_used[q]) own_list(i, q, tcand[0], tres[0], tkept[0], sel);  // q gained rows in this call
        if (q >= 0) q_used[q] = 1;
        rows[v] = sel;
        std::sort(rows[v].begin(), rows[v].end());
        // each selected row is reconsidered on its own (rows are disjoint, so
        // the full ones run in parallel with the same result)
        bool took = false;
        full.clear();
        for (const uint32_t p : sel) {
            if ((int64_t)rows[p].size() < M) {
                rows[p].push_back((uint32_t)v);  // v is the largest id: the row stays sorted
                took = true;
            } else {
                full.push_back(p);
            }
        }
        keeps_v.assign(full.size(), 0);
        pool.run((int)full.size(), [&](int f, int tid) {
            const uint32_t p = full[f];
            auto &r = rows[p];
            const float *xp = X + (int64_t)p * d;
            auto &c = tcand[tid];
            c.clear();
            for (uint32_t u : r) c.push_back(Cand{canon_dist(xp, X + (int64_t)u * d, d), u});
            c.push_back(Cand{canon_dist(xp, xv, d), (uint32_t)v});
            std::sort(c.begin(), c.end(), cless);
            auto &rs = tres[tid];
            rs.resize((size_t)M);
            const int nk = acquire_sorted(X, d, c.data(), (int)c.size(), M, true, rs.data(), tkept[tid]);
            r.clear();
            for (int j = 0; j < nk; ++j) r.push_back(rs[j].id);
            std::sort(r.begin(), r.end());
            keeps_v[f] = std::binary_search(r.begin(), r.end(), (uint32_t)v);
        });
        for (uint8_t k : keeps_v) took = took || k;
        if (!took) {
            int64_t r = -1;
            for (int j = 0; j < qn && r < 0; ++j)
                if ((int64_t)rows[queue[j]].size() < M) r = queue[j];
            if (r < 0) r = first_free_in_bfs(v);
            if (r < 0) {
                set_error("insert: no node with a free slot");
                return RG_EINTERNAL;
            }
            rows[r].push_back((uint32_t)v);
        }
        if (q >= 0) {
            sg.nout_add[q].push_back((uint32_t)v);
            sg.inq_add[v - nb].push_back((uint32_t)q);
        }
    }
    // reachability after the call
    {
        std::vector<uint8_t> seen((size_t)N, 0);
        std::vector<uint32_t> order{entry};
        seen[entry] = 1;
        size_t h = 0;
        auto bfs = [&]() {
            while (h < order.size()) {
                const uint32_t x = order[h++];
                for (uint32_t w : rows[x])
                    if (!seen[w]) {
                        seen[w] = 1;
                        order.push_back(w);
                    }
            }
        };
        bfs();
        size_t first_free = 0;  // order[0 .. first_free) are full, and rows only grow
        for (int64_t u = 0; u < N; ++u) {
            if (seen[u]) continue;
            while (first_free < order.size() && (int64_t)rows[order[first_free]].size() >= M) ++first_free;
            if (first_free == order.size()) {
                set_error("insert: no node with a free slot");
                return RG_EINTERNAL;
            }
            auto &rr = rows[order[first_free]];
            rr.insert(std::upper_bound(rr.begin(), rr.end(), (uint32_t)u), (uint32_t)u);
            seen[u] = 1;
            order.push_back((uint32_t)u);
            bfs();
        }
    }
    std::vector<int64_t> off2((size_t)N + 1, 0);
    for (int64_t x = 0; x < N; ++x) off2[x + 1] = off2[x] + (int64_t)rows[x].size();
    std::vector<uint32_t> idx2((size_t)off2[N]);
    for (int64_t x = 0; x < N; ++x) std::copy(rows[x].begin(), rows[x].end(), idx2.begin() + off2[x]);
    offsets.swap(off2);
    indices.swap(idx2);
    sg.nout_view_off.clear();
    return RG_OK;
}

}  // namespace rg
