// Wavefront (64-lane) helpers for gfx950 kernels: ballot/prefix helpers and
// an in-register bitonic sort of (key, id) pairs held E per lane.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rg {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// number of set bits of m below this lane
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

// (key, id) strict order: smaller key first, then smaller id
template <typename K>
__device__ __forceinline__ bool kless(K ka, uint32_t ia, K kb, uint32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        int w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}

// One compare-exchange stage of a bitonic network over 64*E pairs held E
// per lane (element i = lane*E + e); SIZE and STRIDE are compile-time so
// every register index is static.
template <int E, int SIZE, int STRIDE, typename K>
__device__ __forceinline__ void bitonic_stage(K (&k)[E], uint32_t (&v)[E]) {
    const int lane = lane_id();
    if constexpr (STRIDE >= E) {
        constexpr int lx = STRIDE / E;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = lane * E + e;
            const K ok = __shfl_xor(k[e], lx);
            const uint32_t ov = __shfl_xor(v[e], lx);
            const bool up = (i & SIZE) == 0;
            const bool lower = (i & STRIDE) == 0;
            const bool keep_min = (lower == up);
            const bool take = keep_min ? kless(ok, ov, k[e], v[e]) : kless(k[e], v[e], ok, ov);
            if (take) {
                k[e] = ok;
                v[e] = ov;
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if ((e & STRIDE) == 0) {
                const int p = e | STRIDE;
                const int i = lane * E + e;
                const bool up = (i & SIZE) == 0;
                const bool sw = up ? kless(k[p], v[p], k[e], v[e]) : kless(k[e], v[e], k[p], v[p]);
                const K ka = k[e], kb = k[p];
                const uint32_t va = v[e], vb = v[p];
                k[e] = sw ? kb : ka;
                k[p] = sw ? ka : kb;
                v[e] = sw ? vb : va;
                v[p] = sw ? va : vb;
            }
        }
    }
}

template <int E, int SIZE, int STRIDE, typename K>
__device__ __forceinline__ void bitonic_merge_steps(K (&k)[E], uint32_t (&v)[E]) {
    bitonic_stage<E, SIZE, STRIDE, K>(k, v);
    if constexpr (STRIDE > 1) bitonic_merge_steps<E, SIZE, STRIDE / 2, K>(k, v);
}

template <int E, int SIZE, typename K>
__device__ __forceinline__ void bitonic_sizes(K (&k)[E], uint32_t (&v)[E]) {
    bitonic_merge_steps<E, SIZE, SIZE / 2, K>(k, v);
    if constexpr (SIZE < 64 * E) bitonic_sizes<E, SIZE * 2, K>(k, v);
}

// Ascending bitonic sort of 64*E (key, id) pairs; element i = lane*E + e.
template <int E, typename K>
__device__ __forceinline__ void wave_sort(K (&k)[E], uint32_t (&v)[E]) {
    bitonic_sizes<E, 2, K>(k, v);
}

}  // namespace rg
