/* The oracle built for the CPU with address and undefined-behaviour
 * sanitizers by tests/test_sanitizers.py: its build, search (with decision
 * margins and with a perturbation), rerank search, quantisers and recall on
 * a small input.
 *
 * usage: sanitize_oracle IN OUT
 *   IN:  int64 n, nt, nq; int32 d, Nq, M, L, k; float X[n*d], T[nt*d], Q[nq*d]
 *   OUT: uint32 entry; int64 repairs; int64 offsets[n+1]; uint32 indices[];
 *        uint32 ids[nq*k]; double dists[nq*k]; double margins[nq];
 *        uint32 rerank_ids[nq*k]; double recall */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct or_graph or_graph;
or_graph *or_build(const float *X, int64_t n, int32_t d, const float *T, int64_t nt, int32_t Nq, int32_t M,
                   int32_t L, int32_t m_pj, int32_t m_ce);
int or_graph_ok(const or_graph *G);
uint32_t or_graph_entry(const or_graph *G);
int64_t or_graph_repairs(const or_graph *G);
const int64_t *or_graph_off(const or_graph *G, int which);
const uint32_t *or_graph_idx(const or_graph *G, int which);
void or_graph_free(or_graph *G);
void or_search(const float *X, int64_t n, int32_t d, const int64_t *off, const uint32_t *idx, uint32_t entry,
               const float *Q, int64_t nq, int32_t k, int32_t L, uint32_t *ids, double *dists, uint32_t *hops,
               uint32_t *evals, double *gaps);
void or_search_perturbed(const float *X, int64_t n, int32_t d, const int64_t *off, const uint32_t *idx,
                         uint32_t entry, const float *Q, int64_t nq, int32_t k, int32_t L, double eps, uint64_t seed,
                         uint32_t *ids, double *dists, uint32_t *hops, uint32_t *evals);
void or_search_rerank(const float *Xq, const float *X, int64_t n, int32_t d, const int64_t *off, const uint32_t *idx,
                      uint32_t entry, const float *Q, int64_t nq, int32_t k, int32_t L, uint32_t *ids, double *dists,
                      uint32_t *hops, uint32_t *evals, double *gaps);
void or_quant_fp8(const float *X, int64_t n, int32_t d, uint8_t *codes, float *scales, float *deq);
void or_quant_bf16(const float *x, int64_t count, float *out);
void or_knn(const float *X, int64_t n, int32_t d, const float *Q, int64_t nq, int32_t k, uint32_t *ids, double *ds);
double or_recall(const uint32_t *res, int32_t kr, const uint32_t *gt, int32_t kg, int64_t nq, int32_t k);

static void rd(FILE *f, void *p, size_t sz, size_t n)
{
    if (n && fread(p, sz, n, f) != n) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
}

int main(int argc, char **argv)
{
    if (argc != 3)
        return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f)
        return 2;
    int64_t n, nt, nq;
    int32_t d, Nq, M, L, k;
    rd(f, &n, 8, 1);
    rd(f, &nt, 8, 1);
    rd(f, &nq, 8, 1);
    rd(f, &d, 4, 1);
    rd(f, &Nq, 4, 1);
    rd(f, &M, 4, 1);
    rd(f, &L, 4, 1);
    rd(f, &k, 4, 1);
    float *X = malloc(sizeof(float) * (size_t)(n * d));
    float *T = malloc(sizeof(float) * (size_t)(nt * d));
    float *Q = malloc(sizeof(float) * (size_t)(nq * d));
    rd(f, X, 4, (size_t)(n * d));
    rd(f, T, 4, (size_t)(nt * d));
    rd(f, Q, 4, (size_t)(nq * d));
    fclose(f);
    or_graph *G = or_build(X, n, d, T, nt, Nq, M, L, 0, 0);
    if (!G || !or_graph_ok(G))
        return 4;
    const int64_t *off = or_graph_off(G, 0);
    const uint32_t *idx = or_graph_idx(G, 0);
    uint32_t entry = or_graph_entry(G);
    int64_t repairs = or_graph_repairs(G);
    uint32_t *ids = malloc(sizeof(uint32_t) * (size_t)(nq * k));
    uint32_t *ids2 = malloc(sizeof(uint32_t) * (size_t)(nq * k));
    uint32_t *gt = malloc(sizeof(uint32_t) * (size_t)(nq * k));
    double *ds = malloc(sizeof(double) * (size_t)(nq * k));
    double *ds2 = malloc(sizeof(double) * (size_t)(nq * k));
    double *gaps = malloc(sizeof(double) * (size_t)nq);
    uint32_t *hops = malloc(sizeof(uint32_t) * (size_t)nq), *ev = malloc(sizeof(uint32_t) * (size_t)nq);
    or_search(X, n, d, off, idx, entry, Q, nq, k, L, ids, ds, hops, ev, gaps);
    or_search_perturbed(X, n, d, off, idx, entry, Q, nq, k, L, 1e-6, 3, ids2, ds2, hops, ev);
    uint8_t *codes = malloc((size_t)(n * d));
    float *scales = malloc(sizeof(float) * (size_t)n), *deq = malloc(sizeof(float) * (size_t)(n * d));
    float *b16 = malloc(sizeof(float) * (size_t)(n * d));
    or_quant_fp8(X, n, d, codes, scales, deq);
    or_quant_bf16(X, n * d, b16);
    or_search_rerank(deq, X, n, d, off, idx, entry, Q, nq, k, L, ids2, ds2, hops, ev, NULL);
    or_knn(X, n, d, Q, nq, k, gt, ds2);
    double rec = or_recall(ids, k, gt, k, nq, k);
    FILE *o = fopen(argv[2], "wb");
    if (!o)
        return 2;
    fwrite(&entry, 4, 1, o);
    fwrite(&repairs, 8, 1, o);
    fwrite(off, 8, (size_t)(n + 1), o);
    fwrite(idx, 4, (size_t)off[n], o);
    fwrite(ids, 4, (size_t)(nq * k), o);
    fwrite(ds, 8, (size_t)(nq * k), o);
    fwrite(gaps, 8, (size_t)nq, o);
    fwrite(ids2, 4, (size_t)(nq * k), o);
    fwrite(&rec, 8, 1, o);
    fclose(o);
    or_graph_free(G);
    free(X); free(T); free(Q); free(ids); free(ids2); free(gt); free(ds); free(ds2); free(gaps); free(hops);
    free(ev); free(codes); free(scales); free(deq); free(b16);
    return 0;
}
