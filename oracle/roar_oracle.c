/*
 * RoarGraph oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of what the RoarGraph
 * index computes (Chen et al., "RoarGraph: A Projected Bipartite Graph for
 * Efficient Cross-Modal Approximate Nearest Neighbor Search", PVLDB 17(11),
 * 2024).  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the library never does.  It shares no code, header
 * or table with the library.
 *
 * All arithmetic is IEEE double.  Build with -O2 -ffp-contract=off.
 *
 * Where the paper is silent the following readings are used (each is stated
 * again at the function that depends on it):
 *   - distance: delta(a,b) = -sum_i a_i*b_i, summed in double in increasing i
 *     (inner product, Sec. 5.1 "Datasets": MIPS; cosine workloads arrive
 *     L2-normalised).  A product of two floats is exact in double, so the
 *     value does not depend on FMA contraction.
 *   - total order: (delta, id) lexicographic, ascending, everywhere.
 *   - construction runs in ascending node order, serially, exactly as the
 *     loops of Algorithms 1 and 2 are written; "<-" in those algorithms is an
 *     assignment that replaces the list.
 *   - final out-degree bound M: projection uses m_pj and enhancement m_ce
 *     with m_pj + m_ce <= M - 1; one slot per node is kept for the
 *     reachability repair.
 *
 * Parity pins live in tests/test_oracle.py.  Projection and enhancement
 * beyond the hand-worked builds in tests/golden and the invariants
 * checked there are "parity unpinned" against the paper itself: its worked
 * examples are figures whose coordinates are not given.
 */
#define _POSIX_C_SOURCE 200809L
#include <pthread.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_NONE 0xFFFFFFFFu

/* OpenMP threads of the parallel loops (queries of a search batch, rows of */
/* the kNN, enhancement searches); 0 keeps the runtime's default.           */
void or_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Distance (Def. 1; inner product as in Sec. 5.1).                          */
/* ------------------------------------------------------------------------ */
double or_dist(const float *a, const float *b, int32_t d)
{
    double s = 0.0;
    for (int32_t i = 0; i < d; ++i)
        s += (double)a[i] * (double)b[i];
    return -s;
}

/* (delta, id) total order: a strictly before b */
static int before(double da, uint32_t ia, double db, uint32_t ib)
{
    return da < db || (da == db && ia < ib);
}

typedef struct {
    double d;
    uint32_t id;
} pair_t;

static int pair_cmp(const void *pa, const void *pb)
{
    const pair_t *a = (const pair_t *)pa, *b = (const pair_t *)pb;
    if (before(a->d, a->id, b->d, b->id))
        return -1;
    if (before(b->d, b->id, a->d, a->id))
        return 1;
    return 0;
}

static int u32_cmp(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* ------------------------------------------------------------------------ */
/* Exact k nearest neighbours (Def. 1): brute force over all n base rows.    */
/* ids/dists are nq x k; short rows are padded with OR_NONE / +inf.          */
/* ------------------------------------------------------------------------ */
void or_knn(const float *X, int64_t n, int32_t d, const float *Q, int64_t nq,
            int32_t k, uint32_t *ids, double *dists)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t q = 0; q < nq; ++q) {
        double *kd = dists + q * k;
        uint32_t *ki = ids + q * k;
        int32_t cnt = 0;
        for (int64_t i = 0; i < n; ++i) {
            double dd = or_dist(Q + q * d, X + i * d, d);
            uint32_t id = (uint32_t)i;
            if (cnt == k && !before(dd, id, kd[k - 1], ki[k - 1]))
                continue;
            int32_t pos = cnt < k ? cnt++ : k - 1;
            while (pos > 0 && before(dd, id, kd[pos - 1], ki[pos - 1])) {
                kd[pos] = kd[pos - 1];
                ki[pos] = ki[pos - 1];
                --pos;
            }
            kd[pos] = dd;
            ki[pos] = id;
        }
        for (int32_t j = cnt; j < k; ++j) {
            kd[j] = INFINITY;
            ki[j] = OR_NONE;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Entry point: "the medoid of the base data" (Sec. 4.3, Sec. 4.2.4).        */
/* Reading: the base row nearest (squared L2) to the mean of all rows, lower */
/* id on ties, chosen among the rows allowed by mask (all rows if mask is    */
/* NULL).  The index build passes the rows that have at least one           */
/* out-neighbour in the projected graph: a start node without out-edges     */
/* would make every enhancement search return the start node alone.        */
/* ------------------------------------------------------------------------ */
uint32_t or_medoid_masked(const float *X, int64_t n, int32_t d, const uint8_t *mask)
{
    double *mu = (double *)malloc(sizeof(double) * (size_t)d);
    for (int32_t j = 0; j < d; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i)
            s += (double)X[i * d + j];
        mu[j] = s / (double)n;
    }
    double best = INFINITY;
    uint32_t bi = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (mask && !mask[i])
            continue;
        double s = 0.0;
        for (int32_t j = 0; j < d; ++j) {
            double t = (double)X[i * d + j] - mu[j];
            s += t * t;
        }
        if (s < best) {
            best = s;
            bi = (uint32_t)i;
        }
    }
    free(mu);
    return bi;
}

uint32_t or_medoid(const float *X, int64_t n, int32_t d)
{
    return or_medoid_masked(X, n, d, NULL);
}

/* ------------------------------------------------------------------------ */
/* AcquireNeighbors (Algorithm 3).                                           */
/* C may hold duplicates and x itself; both are dropped.  The candidates are */
/* ranked by (delta(x,c), c).  The closest is kept; a later candidate c is   */
/* kept only if delta(x,c) < delta(c,p) for every p already kept (strict),   */
/* until m are kept.  With fill (used only while projecting), the list is    */
/* then topped up to m with skipped candidates in rank order.                */
/* Returns the number of ids written to res (capacity m).                    */
/* ------------------------------------------------------------------------ */
int32_t or_acquire(const float *X, int32_t d, uint32_t x, const uint32_t *C,
                   int32_t nc, int32_t m, int32_t fill, uint32_t *res)
{
    if (nc <= 0 || m <= 0)
        return 0;
    uint32_t *u = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nc);
    memcpy(u, C, sizeof(uint32_t) * (size_t)nc);
    qsort(u, (size_t)nc, sizeof(uint32_t), u32_cmp);
    pair_t *p = (pair_t *)malloc(sizeof(pair_t) * (size_t)nc);
    int32_t np = 0;
    for (int32_t j = 0; j < nc; ++j) {
        if (u[j] == x || (j > 0 && u[j] == u[j - 1]))
            continue;
        p[np].id = u[j];
        p[np].d = or_dist(X + (int64_t)x * d, X + (int64_t)u[j] * d, d);
        ++np;
    }
    free(u);
    qsort(p, (size_t)np, sizeof(pair_t), pair_cmp);
    int32_t nr = 0;
    if (np > 0)
        res[nr++] = p[0].id;
    for (int32_t j = 1; j < np; ++j) {
        if (nr >= m)
            break;
        int ok = 1;
        for (int32_t r = 0; r < nr; ++r) {
            double dcp = or_dist(X + (int64_t)p[j].id * d, X + (int64_t)res[r] * d, d);
            if (!(p[j].d < dcp)) {
                ok = 0;
                break;
            }
        }
        if (ok)
            res[nr++] = p[j].id;
    }
    if (fill) {
        for (int32_t j = 0; j < np && nr < m; ++j) {
            int in = 0;
            for (int32_t r = 0; r < nr; ++r)
                if (res[r] == p[j].id) {
                    in = 1;
                    break;
                }
            if (!in)
                res[nr++] = p[j].id;
        }
    }
    free(p);
    return nr;
}

/* ------------------------------------------------------------------------ */
/* Beam search (Sec. 4.3).                                                    */
/* The queue Q holds the best L_eff = max(L, k) (delta, id) seen so far.      */
/* Start from the entry; repeatedly expand the closest not-yet-expanded      */
/* entry v: every out-neighbour u of v not seen before gets its distance     */
/* computed and enters Q if Q is not full or (delta,u) beats Q's last entry. */
/* Stop when every entry of Q is expanded.  Returns Q[0..k) (padded).        */
/* (Sec. 4.3: beam search from the medoid with queue length L.)              */
/*                                                                            */
/* gap (optional) receives the decision margin of the search, for checking   */
/* an implementation whose distances carry rounding errors.  Each distance   */
/* delta(q,x) comes with its scale S(q,x) = sum_i |q_i x_i|.  For two nodes  */
/* a before b in (delta, id) order the pair's margin is                      */
/*     (delta_b - delta_a) / (S_a + S_b)                                      */
/* (+inf when both scales are 0, where both distances are exactly 0).  The   */
/* search's margin is the smallest pair margin over every comparison that    */
/* decides its course:                                                        */
/*   - selection: the expanded entry against every other unexpanded entry;   */
/*   - each expansion: every entry of the queue it leaves against every node  */
/*     it dropped (candidates rejected and entries evicted), since the new   */
/*     queue is the best L of the old queue and the new candidates;          */
/*   - the end: each of the first k entries against each later entry.        */
/* A search whose distances each err by at most g * S(q,x), with g below     */
/* the margin, orders every such pair as this one does, so it expands the    */
/* same nodes in the same order and returns the same k ids.                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *qd, *qs; /* queue: distance and its scale */
    uint32_t *qi;
    uint8_t *qx;
    double *od, *os; /* nodes dropped during one expansion */
    int32_t nout, capout;
    uint8_t *vis;
    uint32_t *touched;
    int64_t ntouched, captouched;
} search_ws;

static void ws_init(search_ws *w, int64_t n, int32_t Leff)
{
    w->qd = (double *)malloc(sizeof(double) * (size_t)(Leff + 1));
    w->qs = (double *)malloc(sizeof(double) * (size_t)(Leff + 1));
    w->qi = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(Leff + 1));
    w->qx = (uint8_t *)malloc((size_t)(Leff + 1));
    w->capout = 64;
    w->od = (double *)malloc(sizeof(double) * (size_t)w->capout);
    w->os = (double *)malloc(sizeof(double) * (size_t)w->capout);
    w->nout = 0;
    w->vis = (uint8_t *)calloc((size_t)n, 1);
    w->captouched = 1024;
    w->touched = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)w->captouched);
    w->ntouched = 0;
}

static void ws_free(search_ws *w)
{
    free(w->qd);
    free(w->qs);
    free(w->qi);
    free(w->qx);
    free(w->od);
    free(w->os);
    free(w->vis);
    free(w->touched);
}

static void ws_mark(search_ws *w, uint32_t u)
{
    w->vis[u] = 1;
    if (w->ntouched == w->captouched) {
        w->captouched *= 2;
        w->touched = (uint32_t *)realloc(w->touched, sizeof(uint32_t) * (size_t)w->captouched);
    }
    w->touched[w->ntouched++] = u;
}

static void ws_drop(search_ws *w, double d, double sc)
{
    if (w->nout == w->capout) {
        w->capout *= 2;
        w->od = (double *)realloc(w->od, sizeof(double) * (size_t)w->capout);
        w->os = (double *)realloc(w->os, sizeof(double) * (size_t)w->capout);
    }
    w->od[w->nout] = d;
    w->os[w->nout] = sc;
    w->nout++;
}

static void ws_reset(search_ws *w)
{
    for (int64_t i = 0; i < w->ntouched; ++i)
        w->vis[w->touched[i]] = 0;
    w->ntouched = 0;
}

/* delta(q,x) and its scale sum_i |q_i x_i|, both summed in increasing i */
static double dist_scale(const float *q, const float *x, int32_t d, double *scale)
{
    double s = 0.0, a = 0.0;
    for (int32_t i = 0; i < d; ++i) {
        double p = (double)q[i] * (double)x[i];
        s += p;
        a += fabs(p);
    }
    *scale = a;
    return -s;
}

/* margin of the pair (a before b) */
static double pair_margin(double da, double sa, double db, double sb)
{
    double den = sa + sb;
    if (den == 0.0)
        return INFINITY;
    return (db - da) / den;
}

/* smallest margin between every node of the sorted list (d, s)[0..na) and
 * every node of (d2, s2)[0..nb), all of which come after it; g is the
 * current minimum, returned lowered.  smax bounds the first list's scales:
 * walking it from its end, the distances fall, so once even the largest
 * scale cannot bring a pair under g the rest cannot either. */
static double cross_margin(const double *d, const double *sc, int32_t na, const double *d2,
                           const double *s2, int32_t nb, double g)
{
    double smax = 0.0;
    for (int32_t i = 0; i < na; ++i)
        if (sc[i] > smax)
            smax = sc[i];
    for (int32_t j = 0; j < nb; ++j) {
        for (int32_t i = na - 1; i >= 0; --i) {
            double t = pair_margin(d[i], sc[i], d2[j], s2[j]);
            if (t < g)
                g = t;
            double bound = smax + s2[j] > 0.0 ? (d2[j] - d[i]) / (smax + s2[j]) : INFINITY;
            if (bound >= g)
                break;
        }
    }
    return g;
}

/* Perturbation used to explain a search run with rounding errors: node x's */
/* distance is moved by eps * sign(x) * S(q,x), sign in {-1, 0, +1} drawn   */
/* from the splitmix64 mix of (seed, x).  eps = 0 leaves it unchanged.      */
static double perturb_sign(uint64_t seed, uint32_t x)
{
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + (uint64_t)x + 1;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(int)(z % 3) - 1.0;
}

static double node_dist(const float *q, const float *X, int32_t d, uint32_t x, double eps, uint64_t seed,
                        double *scale)
{
    double dd = dist_scale(q, X + (int64_t)x * d, d, scale);
    if (eps != 0.0)
        dd += eps * perturb_sign(seed, x) * *scale;
    return dd;
}

/* returns the number of queue entries (<= Leff); qd/qi hold the queue */
static int32_t search_core(search_ws *w, const float *X, int32_t d, const int64_t *off,
                           const uint32_t *idx, uint32_t entry, const float *q, int32_t Leff,
                           uint32_t *hops, uint32_t *evals, double *gap, double eps, uint64_t seed)
{
    double g = INFINITY;
    int32_t qn = 0;
    uint32_t h = 0, ev = 0;
    ws_mark(w, entry);
    w->qd[0] = node_dist(q, X, d, entry, eps, seed, &w->qs[0]);
    w->qi[0] = entry;
    w->qx[0] = 0;
    qn = 1;
    ev = 1;
    for (;;) {
        int32_t i = 0;
        while (i < qn && w->qx[i])
            ++i;
        if (i == qn)
            break;
        if (gap) { /* the selection against every other unexpanded entry */
            double smax = 0.0;
            for (int32_t j = i + 1; j < qn; ++j)
                if (w->qs[j] > smax)
                    smax = w->qs[j];
            for (int32_t j = i + 1; j < qn; ++j) {
                if (w->qx[j])
                    continue;
                double t = pair_margin(w->qd[i], w->qs[i], w->qd[j], w->qs[j]);
                if (t < g)
                    g = t;
                if (w->qs[i] + smax > 0.0 && (w->qd[j] - w->qd[i]) / (w->qs[i] + smax) >= g)
                    break;
            }
        }
        w->qx[i] = 1;
        uint32_t v = w->qi[i];
        ++h;
        w->nout = 0;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            uint32_t u = idx[e];
            if (w->vis[u])
                continue;
            ws_mark(w, u);
            double su;
            double du = node_dist(q, X, d, u, eps, seed, &su);
            ++ev;
            if (qn == Leff) {
                if (!before(du, u, w->qd[Leff - 1], w->qi[Leff - 1])) {
                    ws_drop(w, du, su); /* rejected */
                    continue;
                }
                ws_drop(w, w->qd[Leff - 1], w->qs[Leff - 1]); /* evicted */
            }
            int32_t pos = qn < Leff ? qn++ : Leff - 1;
            while (pos > 0 && before(du, u, w->qd[pos - 1], w->qi[pos - 1])) {
                w->qd[pos] = w->qd[pos - 1];
                w->qs[pos] = w->qs[pos - 1];
                w->qi[pos] = w->qi[pos - 1];
                w->qx[pos] = w->qx[pos - 1];
                --pos;
            }
            w->qd[pos] = du;
            w->qs[pos] = su;
            w->qi[pos] = u;
            w->qx[pos] = 0;
        }
        if (gap && w->nout) /* the queue kept against everything dropped */
            g = cross_margin(w->qd, w->qs, qn, w->od, w->os, w->nout, g);
    }
    if (hops)
        *hops = h;
    if (evals)
        *evals = ev;
    if (gap)
        *gap = g;
    return qn;
}

static void search_batch(const float *X, int64_t n, int32_t d, const int64_t *off, const uint32_t *idx,
                         uint32_t entry, const float *Q, int64_t nq, int32_t k, int32_t L, uint32_t *ids,
                         double *dists, uint32_t *hops, uint32_t *evals, double *gaps, double eps,
                         uint64_t seed)
{
    int32_t Leff = L > k ? L : k;
#pragma omp parallel
    {
        search_ws w;
        ws_init(&w, n, Leff);
#pragma omp for schedule(dynamic, 4)
        for (int64_t qq = 0; qq < nq; ++qq) {
            double g = INFINITY;
            int32_t qn = search_core(&w, X, d, off, idx, entry, Q + qq * d, Leff,
                                     hops ? hops + qq : NULL, evals ? evals + qq : NULL,
                                     gaps ? &g : NULL, eps, seed);
            if (gaps && qn > k) /* the first k against the rest */
                g = cross_margin(w.qd, w.qs, k, w.qd + k, w.qs + k, qn - k, g);
            if (gaps)
                gaps[qq] = g;
            for (int32_t j = 0; j < k; ++j) {
                ids[qq * k + j] = j < qn ? w.qi[j] : OR_NONE;
                dists[qq * k + j] = j < qn ? w.qd[j] : INFINITY;
            }
            ws_reset(&w);
        }
        ws_free(&w);
    }
}

void or_search(const float *X, int64_t n, int32_t d, const int64_t *off, const uint32_t *idx,
               uint32_t entry, const float *Q, int64_t nq, int32_t k, int32_t L, uint32_t *ids,
               double *dists, uint32_t *hops, uint32_t *evals, double *gaps)
{
    search_batch(X, n, d, off, idx, entry, Q, nq, k, L, ids, dists, hops, evals, gaps, 0.0, 0);
}

/* The same search with every distance moved by eps * sign * S (see        */
/* perturb_sign): used to show that a result differing from the plain one   */
/* is what some distance errors within eps * S produce.                      */
void or_search_perturbed(const float *X, int64_t n, int32_t d, const int64_t *off, const uint32_t *idx,
                         uint32_t entry, const float *Q, int64_t nq, int32_t k, int32_t L, double eps,
                         uint64_t seed, uint32_t *ids, double *dists, uint32_t *hops, uint32_t *evals)
{
    search_batch(X, n, d, off, idx, entry, Q, nq, k, L, ids, dists, hops, evals, NULL, eps, seed);
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision storage (an optimisation the paper calls orthogonal to  */
/* the index, Sec. 4.3; scalar quantisation with rescoring, Sec. 7).         */
/* ------------------------------------------------------------------------ */

/* BF16: the nearest value with 8 significant bits, ties to an even last     */
/* bit.  Written from the definition: the two bf16 neighbours of x are the   */
/* values whose low 16 float bits are zero, and the nearer one is chosen.    */
float or_bf16(float x)
{
    if (isnan(x) || isinf(x))
        return x;
    uint32_t b;
    memcpy(&b, &x, 4);
    uint32_t lo_b = b & 0xFFFF0000u; /* magnitude <= |x| */
    uint32_t hi_b = lo_b + 0x10000u; /* next magnitude up */
    float lo, hi;
    memcpy(&lo, &lo_b, 4);
    memcpy(&hi, &hi_b, 4);
    if (lo_b == b)
        return x;
    double dlo = fabs((double)x - (double)lo);
    double dhi = isinf(hi) ? ldexp(1.0, 128) - fabs((double)x) : fabs((double)hi - (double)x);
    if (dlo < dhi)
        return lo;
    if (dhi < dlo)
        return hi;
    return (lo_b & 0x10000u) ? hi : lo;
}

void or_quant_bf16(const float *x, int64_t count, float *out)
{
    for (int64_t i = 0; i < count; ++i)
        out[i] = or_bf16(x[i]);
}

/* FP8 E4M3 (OCP "FN" variant): sign, 4 exponent bits with bias 7, 3       */
/* mantissa bits; exponent field 0 is subnormal; code 0x7F is NaN; largest  */
/* finite magnitude 448.  Value of a code, straight from that definition.   */
double or_e4m3_value(uint8_t c)
{
    int s = c >> 7, e = (c >> 3) & 15, m = c & 7;
    if (e == 15 && m == 7)
        return NAN;
    double v = e == 0 ? ldexp((double)m / 8.0, -6) : ldexp(1.0 + (double)m / 8.0, e - 7);
    return s ? -v : v;
}

/* values of the non-negative finite codes 0..0x7E, filled once from the
 * definition above; they increase with the code */
static double e4m3_table[0x7F];
static pthread_once_t e4m3_once = PTHREAD_ONCE_INIT;
static void e4m3_fill(void)
{
    for (int c = 0; c < 0x7F; ++c)
        e4m3_table[c] = or_e4m3_value((uint8_t)c);
}

/* nearest finite code to y (|y| <= 448), ties to the even code.  Because the
 * table is increasing, the two candidates are the neighbours of |y| in it,
 * found by bisection. */
uint8_t or_e4m3_encode(double y)
{
    pthread_once(&e4m3_once, e4m3_fill);
    double a = fabs(y);
    int lo = 0, hi = 0x7E; /* invariant: table[lo] <= a < table[hi] */
    if (a >= e4m3_table[0x7E]) {
        lo = hi = 0x7E;
    } else {
        while (hi - lo > 1) {
            int mid = (lo + hi) / 2;
            if (e4m3_table[mid] <= a)
                lo = mid;
            else
                hi = mid;
        }
    }
    double dl = a - e4m3_table[lo], dh = e4m3_table[hi] - a;
    int best = dl < dh ? lo : (dh < dl ? hi : ((lo & 1) == 0 ? lo : hi));
    return (uint8_t)(y < 0 || (y == 0 && signbit(y)) ? (best | 0x80) : best);
}

/* Per-vector power-of-two scale s = the smallest 2^e with 448 * 2^e >= max|x_i|
 * (s = 1 for an all-zero row).  codes[i] = e4m3(x_i / s); deq[i] = s * value. */
void or_quant_fp8(const float *X, int64_t n, int32_t d, uint8_t *codes, float *scales, float *deq)
{
    pthread_once(&e4m3_once, e4m3_fill);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        const float *x = X + r * d;
        double amax = 0.0;
        for (int32_t i = 0; i < d; ++i)
            if (fabs((double)x[i]) > amax)
                amax = fabs((double)x[i]);
        int e = 0;
        if (amax > 0.0) {
            e = ilogb(amax) - 10;
            while (ldexp(448.0, e) < amax)
                ++e;
        }
        double s = ldexp(1.0, e);
        scales[r] = (float)s;
        for (int32_t i = 0; i < d; ++i) {
            uint8_t c = or_e4m3_encode((double)x[i] / s);
            codes[r * d + i] = c;
            deq[r * d + i] = (float)(s * (c & 0x80 ? -e4m3_table[c & 0x7F] : e4m3_table[c]));
        }
    }
}

/* Search over the reduced-precision rows Xq (given dequantised, exact as    */
/* float), then rescore every entry of the final queue against the FP32 rows */
/* X with the canonical distance, order by (delta, id) and keep k.  The      */
/* margin covers the search on Xq and, with scales taken on X, the first k   */
/* of the rescored queue against the rest.                                   */
typedef struct {
    double d, s;
    uint32_t id;
} rr_t;

static int rr_cmp(const void *pa, const void *pb)
{
    const rr_t *a = (const rr_t *)pa, *b = (const rr_t *)pb;
    if (a->d < b->d)
        return -1;
    if (a->d > b->d)
        return 1;
    return a->id < b->id ? -1 : (a->id > b->id ? 1 : 0);
}

static void rerank_batch(const float *Xq, const float *X, int64_t n, int32_t d, const int64_t *off,
                         const uint32_t *idx, uint32_t entry, const float *Q, int64_t nq, int32_t k,
                         int32_t L, uint32_t *ids, double *dists, uint32_t *hops, uint32_t *evals,
                         double *gaps, double eps, uint64_t seed)
{
    int32_t Leff = L > k ? L : k;
#pragma omp parallel
    {
        search_ws w;
        ws_init(&w, n, Leff);
        rr_t *pr = (rr_t *)malloc(sizeof(rr_t) * (size_t)Leff);
        double *rd = (double *)malloc(sizeof(double) * (size_t)Leff);
        double *rs = (double *)malloc(sizeof(double) * (size_t)Leff);
#pragma omp for schedule(dynamic, 4)
        for (int64_t qq = 0; qq < nq; ++qq) {
            double g = INFINITY;
            const float *q = Q + qq * d;
            int32_t qn = search_core(&w, Xq, d, off, idx, entry, q, Leff,
                                     hops ? hops + qq : NULL, evals ? evals + qq : NULL,
                                     gaps ? &g : NULL, eps, seed);
            for (int32_t j = 0; j < qn; ++j) {
                pr[j].id = w.qi[j];
                pr[j].d = node_dist(q, X, d, w.qi[j], eps, seed ^ 0x5DEECE66Dull, &pr[j].s);
            }
            qsort(pr, (size_t)qn, sizeof(rr_t), rr_cmp);
            if (gaps && qn > k) {
                for (int32_t j = 0; j < qn; ++j) {
                    rd[j] = pr[j].d;
                    rs[j] = pr[j].s;
                }
                g = cross_margin(rd, rs, k, rd + k, rs + k, qn - k, g);
            }
            if (gaps)
                gaps[qq] = g;
            for (int32_t j = 0; j < k; ++j) {
                ids[qq * k + j] = j < qn ? pr[j].id : OR_NONE;
                dists[qq * k + j] = j < qn ? pr[j].d : INFINITY;
            }
            ws_reset(&w);
        }
        free(pr);
        free(rd);
        free(rs);
        ws_free(&w);
    }
}

void or_search_rerank(const float *Xq, const float *X, int64_t n, int32_t d, const int64_t *off,
                      const uint32_t *idx, uint32_t entry, const float *Q, int64_t nq, int32_t k,
                      int32_t L, uint32_t *ids, double *dists, uint32_t *hops, uint32_t *evals,
                      double *gaps)
{
    rerank_batch(Xq, X, n, d, off, idx, entry, Q, nq, k, L, ids, dists, hops, evals, gaps, 0.0, 0);
}

void or_search_rerank_perturbed(const float *Xq, const float *X, int64_t n, int32_t d, const int64_t *off,
                                const uint32_t *idx, uint32_t entry, const float *Q, int64_t nq, int32_t k,
                                int32_t L, double eps, uint64_t seed, uint32_t *ids, double *dists,
                                uint32_t *hops, uint32_t *evals)
{
    rerank_batch(Xq, X, n, d, off, idx, entry, Q, nq, k, L, ids, dists, hops, evals, NULL, eps, seed);
}

/* ------------------------------------------------------------------------ */
/* recall@k = |S intersect KNN(q)| / k, averaged over queries (Sec. 2.1.1).  */
/* res is nq x kr (first k used), gt is nq x kg (first k used).              */
/* ------------------------------------------------------------------------ */
double or_recall(const uint32_t *res, int32_t kr, const uint32_t *gt, int32_t kg, int64_t nq, int32_t k)
{
    double tot = 0.0;
    for (int64_t q = 0; q < nq; ++q) {
        int32_t hit = 0;
        for (int32_t i = 0; i < k; ++i)
            for (int32_t j = 0; j < k; ++j)
                if (res[q * kr + i] == gt[q * kg + j] && gt[q * kg + j] != OR_NONE) {
                    ++hit;
                    break;
                }
        tot += (double)hit / (double)k;
    }
    return nq ? tot / (double)nq : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Index construction (Algorithms 1-3).                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n, nt;
    int32_t d, Nq, M, L, m_pj, m_ce;
    uint32_t entry;
    int64_t repairs;
    /* bipartite graph: pivot of each training query, the remaining Nq-1 */
    /* neighbours of each query, and the bridge lists B(x) as CSR.        */
    uint32_t *pivot;   /* nt */
    uint32_t *nout;    /* nt x (Nq-1) */
    int64_t *b_off;    /* n+1 */
    uint32_t *b_idx;   /* nt */
    /* stage graphs as CSR in stored (selection) order */
    int64_t *pj_off;
    uint32_t *pj_idx;
    int64_t *ce_off;
    uint32_t *ce_idx;
    /* final index: CSR with rows sorted by id */
    int64_t *off;
    uint32_t *idx;
    /* enhancement search results C_x (n x L, count per row) */
    uint32_t *cx;
    int32_t *cx_n;
} or_graph;

typedef struct {
    uint32_t *a; /* n x cap */
    int32_t *deg;
    int32_t cap;
} adjl;

static void adj_init(adjl *g, int64_t n, int32_t cap)
{
    g->cap = cap;
    g->a = (uint32_t *)calloc((size_t)n * (size_t)cap, sizeof(uint32_t));
    g->deg = (int32_t *)calloc((size_t)n, sizeof(int32_t));
}

static void adj_free(adjl *g)
{
    free(g->a);
    free(g->deg);
}

static void adj_to_csr(const adjl *g, int64_t n, int sorted, int64_t **off, uint32_t **idx)
{
    *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    (*off)[0] = 0;
    for (int64_t i = 0; i < n; ++i)
        (*off)[i + 1] = (*off)[i] + g->deg[i];
    *idx = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)((*off)[n] > 0 ? (*off)[n] : 1));
    for (int64_t i = 0; i < n; ++i) {
        memcpy(*idx + (*off)[i], g->a + i * g->cap, sizeof(uint32_t) * (size_t)g->deg[i]);
        if (sorted)
            qsort(*idx + (*off)[i], (size_t)g->deg[i], sizeof(uint32_t), u32_cmp);
    }
}

/* N'(p) <- AcquireNeighbors(p, N'(p) u {x}, m, fill) */
static void reverse_insert(const float *X, int32_t d, adjl *g, uint32_t p, uint32_t x, int32_t m,
                           int32_t fill, uint32_t *tmp)
{
    int32_t c = g->deg[p];
    memcpy(tmp, g->a + (int64_t)p * g->cap, sizeof(uint32_t) * (size_t)c);
    tmp[c++] = x;
    g->deg[p] = or_acquire(X, d, p, tmp, c, m, fill, g->a + (int64_t)p * g->cap);
}

/* ------------------------------------------------------------------------ */
/* Reachability repair (the paper's claim that the enhancement connects the */
/* graph, Sec. 4.2.4, is not guaranteed by Algorithm 1; this is the reading  */
/* used for it).  rows is n x M with deg[x] entries in row x.  Each row is   */
/* first sorted by id, so the breadth-first search from the entry visits a   */
/* node's neighbours in ascending id.  Then every node u still unreached, in */
/* ascending id, gets one in-edge r -> u: r is the first node of u's         */
/* enhancement candidates cx[u] (stride cx_stride, cx_n[u] entries) that is  */
/* reached and has a free slot (degree < M); failing that, the first reached */
/* node in breadth-first order with a free slot.  The search then continues  */
/* from u.  Returns the number of edges added, or -1 if no node has a free   */
/* slot.                                                                      */
/* ------------------------------------------------------------------------ */
int64_t or_repair(int64_t n, int32_t M, uint32_t entry, uint32_t *rows, int32_t *deg, const uint32_t *cx,
                  const int32_t *cx_n, int64_t cx_stride)
{
    for (int64_t x = 0; x < n; ++x)
        qsort(rows + x * M, (size_t)deg[x], sizeof(uint32_t), u32_cmp);
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    int64_t head = 0, tail = 0, repairs = 0;
    seen[entry] = 1;
    order[tail++] = entry;
    for (int64_t u = -1; u < n; ++u) {
        if (u >= 0) {
            if (seen[u])
                continue;
            uint32_t r = OR_NONE;
            for (int32_t j = 0; j < cx_n[u]; ++j) {
                uint32_t c = cx[u * cx_stride + j];
                if (seen[c] && deg[c] < M) {
                    r = c;
                    break;
                }
            }
            for (int64_t j = 0; r == OR_NONE && j < tail; ++j)
                if (deg[order[j]] < M)
                    r = order[j];
            if (r == OR_NONE) {
                free(seen);
                free(order);
                return -1;
            }
            rows[(int64_t)r * M + deg[r]++] = (uint32_t)u;
            ++repairs;
            seen[u] = 1;
            order[tail++] = (uint32_t)u;
        }
        while (head < tail) {
            uint32_t v = order[head++];
            for (int32_t j = 0; j < deg[v]; ++j) {
                uint32_t w2 = rows[(int64_t)v * M + j];
                if (!seen[w2]) {
                    seen[w2] = 1;
                    order[tail++] = w2;
                }
            }
        }
    }
    free(seen);
    free(order);
    return repairs;
}

or_graph *or_build(const float *X, int64_t n, int32_t d, const float *T, int64_t nt, int32_t Nq,
                   int32_t M, int32_t L, int32_t m_pj, int32_t m_ce)
{
    if (n < 1 || nt < 1 || d < 1 || Nq < 2 || Nq > n || M < 3 || L < 1)
        return NULL;
    if (m_pj <= 0)
        m_pj = M / 2; /* ceil((M-1)/2) */
    if (m_ce <= 0)
        m_ce = (M - 1) / 2;
    or_graph *G = (or_graph *)calloc(1, sizeof(or_graph));
    G->n = n;
    G->nt = nt;
    G->d = d;
    G->Nq = Nq;
    G->M = M;
    G->L = L;
    G->m_pj = m_pj;
    G->m_ce = m_ce;

    /* Preprocessing: exact Nq nearest base rows of every training query. */
    uint32_t *kid = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nt * Nq));
    double *kdd = (double *)malloc(sizeof(double) * (size_t)(nt * Nq));
    or_knn(X, n, d, T, nt, Nq, kid, kdd);
    free(kdd);

    /* Algorithm 1, bipartite graph: for each t in order, x = its nearest   */
    /* base row gets the edge x -> t, and t keeps the other Nq-1 as N_out.  */
    int32_t q1 = Nq - 1;
    G->pivot = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nt);
    G->nout = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nt * q1));
    int64_t *bcnt = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    for (int64_t t = 0; t < nt; ++t) {
        G->pivot[t] = kid[t * Nq];
        memcpy(G->nout + t * q1, kid + t * Nq + 1, sizeof(uint32_t) * (size_t)q1);
        bcnt[G->pivot[t] + 1]++;
    }
    free(kid);
    G->b_off = bcnt;
    for (int64_t i = 0; i < n; ++i)
        G->b_off[i + 1] += G->b_off[i];
    G->b_idx = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nt);
    {
        int64_t *fillp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        memcpy(fillp, G->b_off, sizeof(int64_t) * (size_t)n);
        for (int64_t t = 0; t < nt; ++t)
            G->b_idx[fillp[G->pivot[t]]++] = (uint32_t)t; /* ascending t */
        free(fillp);
    }

    /* Algorithm 2, neighbourhood-aware projection, pivots in ascending id. */
    int32_t cap = (m_pj > m_ce ? m_pj : m_ce) + 1;
    adjl pj;
    adj_init(&pj, n, cap);
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cap + 1));
    {
        int64_t candcap = (int64_t)L + q1 + 1;
        uint32_t *cand = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)candcap);
        pair_t *cp = (pair_t *)malloc(sizeof(pair_t) * (size_t)candcap);
        uint32_t *trunc = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)candcap);
        int64_t *stamp = (int64_t *)calloc((size_t)n, sizeof(int64_t));
        for (int64_t x = 0; x < n; ++x) {
            if (G->b_off[x] == G->b_off[x + 1])
                continue;
            /* gather bridges' out-neighbours until at least L distinct */
            int32_t nc = 0;
            for (int64_t b = G->b_off[x]; b < G->b_off[x + 1]; ++b) {
                if (nc >= L)
                    break;
                const uint32_t *lst = G->nout + (int64_t)G->b_idx[b] * q1;
                for (int32_t j = 0; j < q1; ++j) {
                    uint32_t c = lst[j];
                    if (c == (uint32_t)x || stamp[c] == x + 1)
                        continue;
                    stamp[c] = x + 1;
                    cand[nc++] = c;
                }
            }
            /* rank by distance to the pivot, keep the L closest */
            for (int32_t j = 0; j < nc; ++j) {
                cp[j].id = cand[j];
                cp[j].d = or_dist(X + x * d, X + (int64_t)cand[j] * d, d);
            }
            qsort(cp, (size_t)nc, sizeof(pair_t), pair_cmp);
            int32_t nk = nc < L ? nc : L;
            for (int32_t j = 0; j < nk; ++j)
                trunc[j] = cp[j].id;
            pj.deg[x] = or_acquire(X, d, (uint32_t)x, trunc, nk, m_pj, 1, pj.a + x * pj.cap);
            /* reverse links: each selected p reconsiders its list with x */
            int32_t nsel = pj.deg[x];
            uint32_t sel[nsel > 0 ? nsel : 1];
            memcpy(sel, pj.a + x * pj.cap, sizeof(uint32_t) * (size_t)nsel);
            for (int32_t j = 0; j < nsel; ++j)
                reverse_insert(X, d, &pj, sel[j], (uint32_t)x, m_pj, 1, tmp);
        }
        free(stamp);
        free(cand);
        free(cp);
        free(trunc);
    }
    adj_to_csr(&pj, n, 0, &G->pj_off, &G->pj_idx);

    /* Entry: medoid, among rows with an out-neighbour in G_pj if any. */
    {
        uint8_t *mask = (uint8_t *)malloc((size_t)n);
        int any = 0;
        for (int64_t x = 0; x < n; ++x) {
            mask[x] = pj.deg[x] > 0;
            any |= mask[x];
        }
        G->entry = or_medoid_masked(X, n, d, any ? mask : NULL);
        free(mask);
    }

    /* Algorithm 1, connectivity enhancement.  The searches run on the      */
    /* unchanging projected graph, so they are independent; the list        */
    /* updates then run serially in ascending node order.                   */
    G->cx = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n * L));
    G->cx_n = (int32_t *)calloc((size_t)n, sizeof(int32_t));
#pragma omp parallel
    {
        search_ws w;
        ws_init(&w, n, L);
#pragma omp for schedule(dynamic, 8)
        for (int64_t x = 0; x < n; ++x) {
            int32_t qn = search_core(&w, X, d, G->pj_off, G->pj_idx, G->entry, X + x * d, L,
                                     NULL, NULL, NULL, 0.0, 0);
            int32_t c = 0;
            for (int32_t j = 0; j < qn; ++j)
                if (w.qi[j] != (uint32_t)x)
                    G->cx[x * L + c++] = w.qi[j];
            G->cx_n[x] = c;
            ws_reset(&w);
        }
        ws_free(&w);
    }
    adjl ce;
    adj_init(&ce, n, cap);
    for (int64_t x = 0; x < n; ++x) { /* G' <- G_pj */
        ce.deg[x] = pj.deg[x];
        memcpy(ce.a + x * cap, pj.a + x * cap, sizeof(uint32_t) * (size_t)pj.deg[x]);
    }
    for (int64_t x = 0; x < n; ++x) {
        ce.deg[x] = or_acquire(X, d, (uint32_t)x, G->cx + x * L, G->cx_n[x], m_ce, 0,
                               ce.a + x * cap);
        int32_t nsel = ce.deg[x];
        uint32_t sel[nsel > 0 ? nsel : 1];
        memcpy(sel, ce.a + x * cap, sizeof(uint32_t) * (size_t)nsel);
        for (int32_t j = 0; j < nsel; ++j)
            reverse_insert(X, d, &ce, sel[j], (uint32_t)x, m_ce, 0, tmp);
    }
    adj_to_csr(&ce, n, 0, &G->ce_off, &G->ce_idx);

    /* Merge: final(x) = G_pj(x) u G'(x). */
    adjl fin;
    adj_init(&fin, n, M);
    for (int64_t x = 0; x < n; ++x) {
        int32_t c = 0;
        for (int32_t j = 0; j < pj.deg[x]; ++j)
            fin.a[x * M + c++] = pj.a[x * cap + j];
        for (int32_t j = 0; j < ce.deg[x]; ++j) {
            uint32_t u = ce.a[x * cap + j];
            int dup = 0;
            for (int32_t r = 0; r < c; ++r)
                if (fin.a[x * M + r] == u) {
                    dup = 1;
                    break;
                }
            if (!dup)
                fin.a[x * M + c++] = u;
        }
        fin.deg[x] = c;
    }
    adj_free(&pj);
    adj_free(&ce);
    free(tmp);

    /* Reachability repair (or_repair above, a function of its own so that  */
    /* it can be pinned on a hand-made graph).                               */
    G->repairs = or_repair(n, M, G->entry, fin.a, fin.deg, G->cx, G->cx_n, L);
    if (G->repairs < 0) { /* cannot happen while the degree budget holds */
        G->repairs = 0;
        adj_free(&fin);
        return G; /* off == NULL marks failure */
    }
    adj_to_csr(&fin, n, 1, &G->off, &G->idx);
    adj_free(&fin);
    return G;
}

/* accessors for the Python wrapper */
int64_t or_graph_n(const or_graph *G) { return G->n; }
uint32_t or_graph_entry(const or_graph *G) { return G->entry; }
int64_t or_graph_repairs(const or_graph *G) { return G->repairs; }
int or_graph_ok(const or_graph *G) { return G && G->off != NULL; }
const int64_t *or_graph_off(const or_graph *G, int which)
{
    return which == 0 ? G->off : which == 1 ? G->pj_off : which == 2 ? G->ce_off : G->b_off;
}
const uint32_t *or_graph_idx(const or_graph *G, int which)
{
    return which == 0 ? G->idx : which == 1 ? G->pj_idx : which == 2 ? G->ce_idx : G->b_idx;
}
const uint32_t *or_graph_pivot(const or_graph *G) { return G->pivot; }
const uint32_t *or_graph_nout(const or_graph *G) { return G->nout; }
const uint32_t *or_graph_cx(const or_graph *G) { return G->cx; }
const int32_t *or_graph_cx_n(const or_graph *G) { return G->cx_n; }

void or_graph_free(or_graph *G)
{
    if (!G)
        return;
    free(G->pivot);
    free(G->nout);
    free(G->b_off);
    free(G->b_idx);
    free(G->pj_off);
    free(G->pj_idx);
    free(G->ce_off);
    free(G->ce_idx);
    free(G->off);
    free(G->idx);
    free(G->cx);
    free(G->cx_n);
    free(G);
}
