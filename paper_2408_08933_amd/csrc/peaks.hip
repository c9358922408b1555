// Measured peaks of the device, beside the datasheet ones: a streaming read
// of a large buffer (HBM bandwidth) and long runs of independent MFMA
// instructions on register operands (matrix throughput), timed with HIP
// events on the caller's stream.  Not part of the method: the roofline
// fractions of the search and kNN kernels are quoted against both.
#include "rg_internal.h"
#include "wave_ops.h"

namespace rg {
namespace {

typedef float fx4 __attribute__((ext_vector_type(4)));
typedef float fx16 __attribute__((ext_vector_type(16)));
typedef _Float16 hx8 __attribute__((ext_vector_type(8)));

// Each thread sums 16-byte vectors of the buffer (grid-stride) and writes
// one value, so the only traffic is the read of `src` and a negligible
// write.
__global__ __launch_bounds__(256) void k_read_stream(const uint4 *src, int64_t n16, uint32_t *sink) {
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    }
    for (; i < n16; i += stride) {
        const uint4 a = src[i];
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// 8 independent accumulators per wave, `iters` rounds: FP16 16x16x32.
__global__ __launch_bounds__(256) void k_mfma_f16(int iters, float *sink) {
    hx8 a, b;
    for (int e = 0; e < 8; ++e) {
        a[e] = (_Float16)(0.001f * (threadIdx.x + e));
        b[e] = (_Float16)(0.002f * (threadIdx.x - e));
    }
    fx4 acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = fx4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[j], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// The same with the FP32 16x16x4 instruction the FP32 kNN uses.
__global__ __launch_bounds__(256) void k_mfma_f32(int iters, float *sink) {
    const float a = 0.001f * threadIdx.x, b = 0.002f * threadIdx.x;
    fx4 acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = fx4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

int launch_read_stream(const void *src, int64_t bytes, void *sink, int blocks, hipStream_t stream) {
    hipLaunchKernelGGL(k_read_stream, dim3(blocks), dim3(256), 0, stream, static_cast<const uint4 *>(src), bytes / 16,
                       static_cast<uint32_t *>(sink));
    RG_HIP(hipGetLastError());
    return RG_OK;
}

// kind 0: FP16 16x16x32 (16384 FLOP per wave instruction); kind 1: FP32
// 16x16x4 (2048).  Returns the FLOP one launch performs.
int launch_mfma_probe(int kind, int iters, void *sink, int blocks, hipStream_t stream, double *flop) {
    if (kind == 0)
        hipLaunchKernelGGL(k_mfma_f16, dim3(blocks), dim3(256), 0, stream, iters, static_cast<float *>(sink));
    else
        hipLaunchKernelGGL(k_mfma_f32, dim3(blocks), dim3(256), 0, stream, iters, static_cast<float *>(sink));
    RG_HIP(hipGetLastError());
    *flop = (double)blocks * 4 * iters * 8 * (kind == 0 ? 16384.0 : 2048.0);
    return RG_OK;
}

}  // namespace rg
