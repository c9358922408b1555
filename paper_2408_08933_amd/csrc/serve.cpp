// Serving: continuous batching of search requests with mixed (k, L).
//
// A scheduler thread owns a table of device-resident slots.  Each slot holds
// one request's whole beam-search state in device memory: query vector,
// queue (L_eff <= 512 entries), visited table, counters.  One scheduler step
// = admit pending requests into free slots (bounded by max_slots and by the
// HBM pool divided by the per-slot state size), launch one step kernel over
// all active slots, which advances each by at most hops_per_step expansions
// and saves its state, then collect the slots that finished.  Requests that
// arrive while a step runs are admitted at the next step, so new work joins
// work already on the device instead of waiting for a batch to drain.
//
// Two steps are in flight: the thread launches step s + 1 before it waits
// for step s and collects its results, so the device runs the next step
// while the host copies and hands out the last one's results and stages
// new admissions.  A slot that finished in step s is still listed in step
// s + 1 (the host has not seen it finish yet); it is marked finished in
// device memory and that step skips it.  Each step has its own staging,
// active-list, count and record buffers (two sets, used alternately).
//
// The step kernel runs the same per-query arithmetic as rg_search (same
// distance function, same merge), and a slot's state is saved and restored
// exactly, so a request returns the same ids and distances alone or in any
// mix.  The device never waits on host memory: every kernel runs to
// completion and the host waits on an event after each step.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>

#include "rg_internal.h"

using namespace rg;

namespace {

struct Pending {
    std::vector<float> q;
    int32_t k, L;
    uint64_t tag;
    double t_submit;
};

struct SlotInfo {
    bool busy = false;
    uint64_t tag = 0;
    int32_t k = 0, L = 0;
    double t_submit = 0, t_admit = 0;
};

constexpr size_t kMaxPending = 1u << 20;

// Buffers of one in-flight step.
struct StepBuf {
    int32_t *d_adm_slot = nullptr, *d_adm_k = nullptr, *d_adm_L = nullptr, *d_active = nullptr;
    float *d_adm_q = nullptr;
    uint32_t *d_count = nullptr;
    ServeRecord *d_rec = nullptr;
    int32_t *h_adm_slot = nullptr, *h_adm_k = nullptr, *h_adm_L = nullptr, *h_active = nullptr;
    float *h_adm_q = nullptr;
    uint32_t *h_count = nullptr;
    ServeRecord *h_rec = nullptr;
    hipEvent_t done = nullptr;  // the step kernel and its count copy have finished
    bool launched = false;
};

}  // namespace

struct rg_server {
    const rg_index *ix = nullptr;
    rg_server_limits lim{};
    int32_t slots = 0, hash_bits = 12;
    hipStream_t stream = nullptr;       // admissions and step kernels
    hipStream_t copy_stream = nullptr;  // result records back to the host
    // device slot arrays
    float *d_q = nullptr, *d_qd = nullptr;
    int32_t *d_k = nullptr, *d_L = nullptr, *d_state = nullptr;
    uint32_t *d_qi = nullptr, *d_hash = nullptr;
    StepBuf buf[2];
    // host side
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Pending> pending;
    std::vector<SlotInfo> info;
    std::deque<rg_result> finished;
    std::thread th;
    bool stop = false;
    uint64_t n_sub = 0, n_adm = 0, n_done = 0, n_steps = 0;
    int err = RG_OK;
    std::chrono::steady_clock::time_point t0;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
    void loop();
    bool launch(StepBuf &b, int32_t n_adm_now, int32_t n_active);
    bool collect(StepBuf &b);
    void release();
};

void rg_server::release() {
    void *ps[] = {d_q, d_qd, d_k, d_L, d_state, d_qi, d_hash};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    for (StepBuf &b : buf) {
        void *dp[] = {b.d_adm_slot, b.d_adm_k, b.d_adm_L, b.d_active, b.d_adm_q, b.d_count, b.d_rec};
        for (void *p : dp)
            if (p) (void)hipFree(p);
        void *hp[] = {b.h_adm_slot, b.h_adm_k, b.h_adm_L, b.h_active, b.h_adm_q, b.h_count, b.h_rec};
        for (void *p : hp)
            if (p) (void)hipHostFree(p);
        if (b.done) (void)hipEventDestroy(b.done);
    }
    if (stream) (void)hipStreamDestroy(stream);
    if (copy_stream) (void)hipStreamDestroy(copy_stream);
}

// Enqueue one step on the server's stream: scatter the admitted requests into
// their slots, advance the listed slots, copy the finished count back.
bool rg_server::launch(StepBuf &b, int32_t n_adm_now, int32_t n_active) {
    const int d = ix->d;
    hipStream_t st = stream;
    SlotArgs sa{};
    sa.s.base = ix->d_base;
    sa.s.base_bf16 = ix->d_bf16;
    sa.s.base_fp8 = ix->d_fp8;
    sa.s.adj = ix->d_adj;
    sa.s.adj_off = ix->d_adj_off;
    sa.s.tomb = ix->d_tomb;
    sa.s.d = d;
    sa.s.pitch = ix->pitch;
    sa.s.pitch8 = ix->pitch8;
    sa.s.qpad = query_pad(d, ix->pitch, ix->storage);
    sa.s.ell = ix->ell;
    sa.s.cand = cand_capacity(ix->ell, ix->d_adj_off != nullptr);
    sa.s.hash_bits = hash_bits;
    sa.s.entry = ix->entry;
    sa.s.storage = ix->storage;
    sa.active = b.d_active;
    sa.n_active = n_active;
    sa.slot_q = d_q;
    sa.slot_k = d_k;
    sa.slot_L = d_L;
    sa.slot_qd = d_qd;
    sa.slot_qi = d_qi;
    sa.slot_state = d_state;
    sa.slot_hash = d_hash;
    sa.hops_budget = lim.hops_per_step;
    sa.out_count = b.d_count;
    sa.out_rec = b.d_rec;
    bool ok = true;
    if (n_adm_now > 0) {
        ok = hipMemcpyAsync(b.d_adm_slot, b.h_adm_slot, 4 * n_adm_now, hipMemcpyHostToDevice, st) == hipSuccess &&
             hipMemcpyAsync(b.d_adm_k, b.h_adm_k, 4 * n_adm_now, hipMemcpyHostToDevice, st) == hipSuccess &&
             hipMemcpyAsync(b.d_adm_L, b.h_adm_L, 4 * n_adm_now, hipMemcpyHostToDevice, st) == hipSuccess &&
             hipMemcpyAsync(b.d_adm_q, b.h_adm_q, sizeof(float) * d * n_adm_now, hipMemcpyHostToDevice, st) ==
                 hipSuccess &&
             launch_serve_admit(n_adm_now, b.d_adm_slot, b.d_adm_q, b.d_adm_k, b.d_adm_L, d, d_q, d_k, d_L, d_state,
                                st) == RG_OK;
    }
    ok = ok &&
         hipMemcpyAsync(b.d_active, b.h_active, sizeof(int32_t) * n_active, hipMemcpyHostToDevice, st) ==
             hipSuccess &&
         hipMemsetAsync(b.d_count, 0, 4, st) == hipSuccess && launch_serve_step(sa, st) == RG_OK &&
         hipMemcpyAsync(b.h_count, b.d_count, 4, hipMemcpyDeviceToHost, st) == hipSuccess &&
         hipEventRecord(b.done, st) == hipSuccess;
    b.launched = ok;
    return ok;
}

// Wait for the step in b, copy its finished records back (on the copy
// stream, so the step launched after it keeps running) and hand them out.
bool rg_server::collect(StepBuf &b) {
    b.launched = false;
    if (hipEventSynchronize(b.done) != hipSuccess) return false;
    const uint32_t nf = *b.h_count;
    if (nf > 0 &&
        (hipMemcpyAsync(b.h_rec, b.d_rec, sizeof(ServeRecord) * nf, hipMemcpyDeviceToHost, copy_stream) !=
             hipSuccess ||
         hipStreamSynchronize(copy_stream) != hipSuccess))
        return false;
    const double t_done = now();
    std::lock_guard<std::mutex> lk(mu);
    ++n_steps;
    for (uint32_t i = 0; i < nf; ++i) {
        const ServeRecord &rec = b.h_rec[i];
        SlotInfo &si = info[rec.slot];
        rg_result r{};
        r.tag = si.tag;
        r.k = si.k;
        r.status = RG_OK;
        r.hops = rec.hops;
        r.evals = rec.evals;
        std::memcpy(r.ids, rec.ids, sizeof(uint32_t) * si.k);
        std::memcpy(r.dists, rec.d, sizeof(float) * si.k);
        r.t_submit = si.t_submit;
        r.t_admit = si.t_admit;
        r.t_done = t_done;
        finished.push_back(r);
        si.busy = false;
        ++n_done;
    }
    return true;
}

void rg_server::loop() {
    (void)hipSetDevice(ix->device);
    const int d = ix->d;
    int cur = 0;
    for (;;) {
        StepBuf &b = buf[cur], &prev = buf[cur ^ 1];
        int32_t n_adm_now = 0, n_active = 0;
        {
            std::unique_lock<std::mutex> lk(mu);
            bool any_busy = false;
            for (auto &s : info) any_busy |= s.busy;
            if (!any_busy && pending.empty() && !prev.launched) {
                if (stop) break;
                cv.wait_for(lk, std::chrono::milliseconds(1));
                continue;
            }
            // admission: free slots in ascending order, requests in arrival order
            const double t_adm = now();
            for (int32_t s = 0; s < slots && !pending.empty() && !stop; ++s) {
                if (info[s].busy) continue;
                Pending &p = pending.front();
                info[s] = SlotInfo{true, p.tag, p.k, p.L, p.t_submit, t_adm};
                b.h_adm_slot[n_adm_now] = s;
                b.h_adm_k[n_adm_now] = p.k;
                b.h_adm_L[n_adm_now] = p.L;
                std::memcpy(b.h_adm_q + (size_t)n_adm_now * d, p.q.data(), sizeof(float) * d);
                ++n_adm_now;
                pending.pop_front();
                ++n_adm;
            }
            // every busy slot, including those that finish in the step in
            // flight (that step marks them, and this one skips them)
            for (int32_t s = 0; s < slots; ++s)
                if (info[s].busy) b.h_active[n_active++] = s;
        }
        bool ok = n_active == 0 || launch(b, n_adm_now, n_active);
        if (ok && prev.launched) ok = collect(prev);
        if (!ok) {
            // drain what is in flight, then drop every request
            (void)hipStreamSynchronize(stream);
            (void)hipStreamSynchronize(copy_stream);
            std::lock_guard<std::mutex> lk(mu);
            err = RG_EDEVICE;
            for (auto &s : info) s.busy = false;
            pending.clear();
            for (StepBuf &x : buf) x.launched = false;
            continue;
        }
        cur ^= 1;
    }
    (void)hipStreamSynchronize(stream);
}

extern "C" {

// default visited-table size per slot: 2^9 ids for every storage form.  The
// step kernel's LDS holds a queue of 512 entries and the table, so a small
// table lets more workgroups share a CU; it costs a little rescoring.
// Measured on the 10M x 200 index with the mixed-L load and 4,096 slots:
// FP32 closed-loop capacity 297k (2^11, 11 workgroups per CU), 311k (2^10),
// 348k req/s (2^9, 19 per CU); E4M3 rows 351k at 2^9, 344k at 2^8.
static int serve_hash_bits(int32_t) { return 9; }

int rg_server_create(const rg_index *ix, const rg_server_limits *lim, rg_server **out) {
    if (!ix || !out || !ix->d_base) {
        set_error("rg_server_create: invalid argument");
        return RG_EINVAL;
    }
    *out = nullptr;
    rg_server_limits l{};
    if (lim) l = *lim;
    if (l.max_slots < 0) {
        set_error("rg_server_create: max_slots must be >= 0");
        return RG_EINVAL;
    }
    if (l.hops_per_step <= 0) l.hops_per_step = 32;
    if (l.max_L <= 0 || l.max_L > kMaxL) l.max_L = kMaxL;
    if (l.hash_bits == 0) l.hash_bits = serve_hash_bits(ix->storage);
    if (l.hash_bits < 8 || l.hash_bits > 13 ||
        (1 << l.hash_bits) < 2 * cand_capacity(ix->ell, ix->d_adj_off != nullptr) + 2) {
        set_error("rg_server_create: hash_bits out of range");
        return RG_EINVAL;
    }
    if (l.max_slots == 0) {
        // twice the step workgroups the device holds at once, so each step
        // runs whole waves of workgroups
        SlotArgs sa{};
        sa.s.d = ix->d;
        sa.s.qpad = query_pad(ix->d, ix->pitch, ix->storage);
        sa.s.cand = cand_capacity(ix->ell, ix->d_adj_off != nullptr);
        sa.s.hash_bits = l.hash_bits;
        sa.s.storage = ix->storage;
        int per_cu = 0, cus = 0;
        (void)hipSetDevice(ix->device);
        const int rc = serve_step_occupancy(sa, &per_cu);
        if (rc) return rc;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ix->device) != hipSuccess) {
            set_error("rg_server_create: device query failed");
            return RG_EDEVICE;
        }
        l.max_slots = 2 * std::max(1, per_cu) * std::max(1, cus);
    }
    rg_server *s = new rg_server();
    s->ix = ix;
    s->lim = l;
    s->hash_bits = l.hash_bits;
    // device bytes one slot keeps between steps: query, k/L, queue (keys + ids),
    // state words, visited table, a result record in each of the two steps'
    // buffers
    const int64_t per_slot = (int64_t)ix->d * 4 + 8 + (int64_t)kMaxL * 8 + 32 + ((int64_t)4 << s->hash_bits) +
                             2 * (int64_t)sizeof(ServeRecord);
    int64_t slots = l.max_slots;
    if (l.hbm_pool_bytes > 0) slots = std::min<int64_t>(slots, l.hbm_pool_bytes / per_slot);
    if (slots < 1) {
        delete s;
        set_error("rg_server_create: HBM pool smaller than one slot");
        return RG_EINVAL;
    }
    s->slots = (int32_t)slots;
    s->info.resize((size_t)slots);
    (void)hipSetDevice(ix->device);
    bool ok = hipStreamCreate(&s->stream) == hipSuccess && hipStreamCreate(&s->copy_stream) == hipSuccess;
    auto al = [&](void **p, size_t b) { ok = ok && hipMalloc(p, b) == hipSuccess; };
    auto ah = [&](void **p, size_t b) { ok = ok && hipHostMalloc(p, b, hipHostMallocDefault) == hipSuccess; };
    al((void **)&s->d_q, sizeof(float) * slots * ix->d);
    al((void **)&s->d_k, 4 * slots);
    al((void **)&s->d_L, 4 * slots);
    al((void **)&s->d_qd, sizeof(float) * slots * kMaxL);
    al((void **)&s->d_qi, sizeof(uint32_t) * slots * kMaxL);
    al((void **)&s->d_state, 32 * slots);
    al((void **)&s->d_hash, (size_t)slots << (s->hash_bits + 2));
    for (StepBuf &b : s->buf) {
        al((void **)&b.d_active, 4 * slots);
        al((void **)&b.d_count, 4);
        al((void **)&b.d_rec, sizeof(ServeRecord) * slots);
        al((void **)&b.d_adm_slot, 4 * slots);
        al((void **)&b.d_adm_k, 4 * slots);
        al((void **)&b.d_adm_L, 4 * slots);
        al((void **)&b.d_adm_q, sizeof(float) * slots * ix->d);
        ah((void **)&b.h_adm_slot, 4 * slots);
        ah((void **)&b.h_adm_k, 4 * slots);
        ah((void **)&b.h_adm_L, 4 * slots);
        ah((void **)&b.h_active, 4 * slots);
        ah((void **)&b.h_adm_q, sizeof(float) * slots * ix->d);
        ah((void **)&b.h_count, 4);
        ah((void **)&b.h_rec, sizeof(ServeRecord) * slots);
        ok = ok && hipEventCreateWithFlags(&b.done, hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
        s->release();
        delete s;
        set_error("rg_server_create: out of memory");
        return RG_ENOMEM;
    }
    s->t0 = std::chrono::steady_clock::now();
    s->th = std::thread([s]() { s->loop(); });
    *out = s;
    return RG_OK;
}

int rg_server_submit(rg_server *s, const float *q, int32_t k, int32_t L, uint64_t tag) {
    if (!s || !q || k < 1 || L < 1 || k > kMaxL || std::max(k, L) > s->lim.max_L) {
        set_error("rg_server_submit: invalid argument");
        return RG_EINVAL;
    }
    Pending p{std::vector<float>(q, q + s->ix->d), k, L, tag, s->now()};
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->err) {
            set_error("rg_server_submit: server stopped after a device error");
            return s->err;
        }
        if (s->pending.size() >= kMaxPending) return RG_EAGAIN;
        s->pending.push_back(std::move(p));
        ++s->n_sub;
    }
    s->cv.notify_one();
    return RG_OK;
}

int rg_server_submit_batch(rg_server *s, const float *queries_host, const int32_t *k, const int32_t *L,
                           const uint64_t *tags, int32_t n, int32_t *n_accepted) {
    if (!s || !n_accepted || n < 0 || (n > 0 && (!queries_host || !k || !L || !tags))) {
        set_error("rg_server_submit_batch: invalid argument");
        return RG_EINVAL;
    }
    *n_accepted = 0;
    for (int32_t i = 0; i < n; ++i)
        if (k[i] < 1 || L[i] < 1 || k[i] > kMaxL || std::max(k[i], L[i]) > s->lim.max_L) {
            set_error("rg_server_submit_batch: invalid k or L");
            return RG_EINVAL;
        }
    const int d = s->ix->d;
    const double t = s->now();
    int32_t acc = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->err) {
            set_error("rg_server_submit_batch: server stopped after a device error");
            return s->err;
        }
        for (int32_t i = 0; i < n && s->pending.size() < kMaxPending; ++i, ++acc) {
            s->pending.push_back(Pending{std::vector<float>(queries_host + (size_t)i * d, queries_host + (size_t)(i + 1) * d),
                                         k[i], L[i], tags[i], t});
            ++s->n_sub;
        }
    }
    s->cv.notify_one();
    *n_accepted = acc;
    return acc < n ? RG_EAGAIN : RG_OK;
}

int rg_server_poll(rg_server *s, rg_result *out, int32_t max, int32_t *n_out) {
    if (!s || !n_out || (max > 0 && !out)) {
        set_error("rg_server_poll: invalid argument");
        return RG_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t n = 0;
    while (n < max && !s->finished.empty()) {
        out[n++] = s->finished.front();
        s->finished.pop_front();
    }
    *n_out = n;
    return s->err;
}

int rg_server_stats(const rg_server *s, uint64_t *sub, uint64_t *adm, uint64_t *done, uint64_t *steps) {
    if (!s) return RG_EINVAL;
    std::lock_guard<std::mutex> lk(const_cast<rg_server *>(s)->mu);
    if (sub) *sub = s->n_sub;
    if (adm) *adm = s->n_adm;
    if (done) *done = s->n_done;
    if (steps) *steps = s->n_steps;
    return RG_OK;
}

double rg_server_now(const rg_server *s) { return s ? s->now() : 0.0; }

int32_t rg_server_slots(const rg_server *s) { return s ? s->slots : 0; }

void rg_server_destroy(rg_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->pending.clear();
    }
    s->cv.notify_one();
    if (s->th.joinable()) s->th.join();
    s->release();
    delete s;
}

}  // extern "C"
