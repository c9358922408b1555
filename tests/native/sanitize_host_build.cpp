// Host construction and insertion of the library, built for the CPU with
// sanitizers (address + undefined behaviour, or thread) by
// tests/test_sanitizers.py.  The device half of the library is replaced by
// stubs that report "no device", so only host code runs: the same
// host_construct / host_canon_searches / host_insert that rg_build_from_knn
// and rg_insert call.
//
// usage: sanitize_host_build IN OUT
//   IN:  int64 n, nt, nv; int32 d, Nq, M, L, threads; then float X[n*d],
//        uint32 knn[nt*Nq], float T[nt*d], float V[nv*d]
//   OUT: uint32 entry; int64 repairs; int64 offsets[n+1]; uint32 indices[];
//        then, after inserting V, int64 offsets[n+nv+1]; uint32 indices[]
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_2408_08933_amd/csrc/rg_internal.h"

namespace rg {
static std::string g_error;
void set_error(const std::string &msg) { g_error = msg; }
int launch_canon_search(const float *, int32_t, int32_t, const uint32_t *, int32_t, uint32_t, int32_t, int64_t,
                        int64_t, uint32_t *, double *, int32_t *, hipStream_t) {
    return RG_EDEVICE;
}
int launch_canon_select(const float *, int32_t, int32_t, const uint32_t *, const double *, const int32_t *, int32_t,
                        int64_t, int64_t, int32_t, uint32_t *, double *, int32_t *, uint32_t *, int32_t, int32_t *,
                        hipStream_t) {
    return RG_EDEVICE;
}
}  // namespace rg

// the HIP runtime calls of the device-enhancement path, never reached here
extern "C" {
hipError_t hipEventCreateWithFlags(hipEvent_t *, unsigned) { return hipErrorNoDevice; }
hipError_t hipEventDestroy(hipEvent_t) { return hipErrorNoDevice; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipErrorNoDevice; }
hipError_t hipFree(void *) { return hipErrorNoDevice; }
hipError_t hipHostFree(void *) { return hipErrorNoDevice; }
hipError_t hipHostMalloc(void **, size_t, unsigned) { return hipErrorNoDevice; }
hipError_t hipMalloc(void **, size_t) { return hipErrorNoDevice; }
hipError_t hipMemcpyAsync(void *, const void *, size_t, hipMemcpyKind, hipStream_t) { return hipErrorNoDevice; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipErrorNoDevice; }
}

template <class T>
static void rd(FILE *f, T *p, size_t n) {
    if (n && std::fread(p, sizeof(T), n, f) != n) {
        std::fprintf(stderr, "short input\n");
        std::exit(2);
    }
}

template <class T>
static void wr(FILE *f, const T *p, size_t n) {
    if (n && std::fwrite(p, sizeof(T), n, f) != n) std::exit(3);
}

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n, nt, nv;
    int32_t d, Nq, M, L, threads;
    rd(f, &n, 1);
    rd(f, &nt, 1);
    rd(f, &nv, 1);
    rd(f, &d, 1);
    rd(f, &Nq, 1);
    rd(f, &M, 1);
    rd(f, &L, 1);
    rd(f, &threads, 1);
    std::vector<float> X((size_t)n * d), T((size_t)nt * d), V((size_t)nv * d);
    std::vector<uint32_t> knn((size_t)nt * Nq);
    rd(f, X.data(), X.size());
    rd(f, knn.data(), knn.size());
    rd(f, T.data(), T.size());
    rd(f, V.data(), V.size());
    std::fclose(f);
    const int32_t m_pj = M / 2, m_ce = (M - 1) / 2;
    rg::HostGraph g;
    int rc = rg::host_construct(X.data(), n, d, knn.data(), nt, Nq, M, L, m_pj, m_ce, threads, nullptr, true, &g);
    if (rc) {
        std::fprintf(stderr, "host_construct: %d %s\n", rc, rg::g_error.c_str());
        return 4;
    }
    FILE *o = std::fopen(argv[2], "wb");
    if (!o) return 2;
    wr(o, &g.entry, 1);
    wr(o, &g.repairs, 1);
    wr(o, g.offsets.data(), g.offsets.size());
    wr(o, g.indices.data(), g.indices.size());
    // insertion, as rg_insert does it for an index without device data
    rg::StageGraphs &sg = g.stages;
    sg.base = X;
    sg.train = T;
    sg.base.insert(sg.base.end(), V.begin(), V.end());
    std::vector<uint32_t> qid((size_t)nv * L);
    std::vector<int32_t> qn((size_t)nv);
    rg::host_canon_searches(sg.base.data(), d, g.offsets.data(), g.indices.data(), g.entry, L, n, nv, threads,
                            qid.data(), qn.data());
    rc = rg::host_insert(sg, d, M, m_pj, L, g.entry, n, nv, qid.data(), qn.data(), g.offsets, g.indices, threads);
    if (rc) {
        std::fprintf(stderr, "host_insert: %d %s\n", rc, rg::g_error.c_str());
        return 5;
    }
    wr(o, g.offsets.data(), g.offsets.size());
    wr(o, g.indices.data(), g.indices.size());
    std::fclose(o);
    return 0;
}
