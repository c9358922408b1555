// Device copies of the base rows: padded FP32, BF16 and FP8-E4M3 with a
// per-row power-of-two scale.  Reduced precision is the storage option the
// paper leaves open as orthogonal to the index (Sec. 4.3) and that scalar
// quantisation with rescoring realises (Sec. 7); the search rescores its
// final queue against the FP32 rows.
#include "rg_internal.h"
#include "wave_ops.h"

namespace rg {
namespace {

// dst[r][c] = src[r][c] for c < d, 0 for d <= c < pitch
__global__ void k_pad_rows(const float *src, int64_t n, int32_t d, float *dst, int32_t pitch) {
    const int64_t total = n * (int64_t)pitch;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / pitch;
        const int32_t c = (int32_t)(i - r * pitch);
        dst[i] = c < d ? src[r * d + c] : 0.f;
    }
}

// round to nearest even on the upper 16 bits
__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x7FFFFFu)) return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__global__ void k_quant_bf16(const float *src, int64_t count, uint16_t *dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = f32_to_bf16(src[i]);
}

// nearest E4M3 code of |y| <= 448 (ties to even code), sign applied
__device__ __forceinline__ uint32_t f32_to_e4m3(float y) {
    const uint32_t b = __float_as_uint(y);
    const uint32_t sgn = (b >> 24) & 0x80u;
    const float a = fabsf(y);
    uint32_t code;
    if (a >= 448.f) {
        code = 0x7Eu;
    } else if (a < 0.015625f) {            // below 2^-6: subnormal step 2^-9
        code = (uint32_t)rintf(a * 512.f);  // 0..8 (8 = smallest normal, code 0x08)
    } else {
        const uint32_t ab = __float_as_uint(a);
        const int32_t E = (int32_t)(ab >> 23) - 127;  // -6 .. 8
        const uint32_t mant = ab & 0x7FFFFFu;
        uint32_t m3 = mant >> 20;
        const uint32_t rem = mant & 0xFFFFFu;
        if (rem > 0x80000u || (rem == 0x80000u && (m3 & 1u))) ++m3;
        code = ((uint32_t)(E + 7) << 3) + m3;  // m3 == 8 carries into the exponent
    }
    return sgn | code;
}

// one wavefront per row: scale = smallest 2^e with 448 * 2^e >= max|x|.
// Row layout (pitch8 bytes): the d codes, zeros up to a multiple of 4, the
// row's FP32 scale, zeros; the scale also goes to scales[r].
__global__ __launch_bounds__(64) void k_quant_fp8(const float *src, int64_t n, int32_t d, int32_t pitch,
                                                  uint8_t *dst, int32_t pitch8, float *scales) {
    const int64_t r = blockIdx.x;
    const int lane = lane_id();
    const float *x = src + r * pitch;
    float amax = 0.f;
    for (int c = lane; c < d; c += 64) amax = fmaxf(amax, fabsf(x[c]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
    int e = 0;
    if (amax > 0.f) {
        e = ilogbf(amax) - 10;
        while (ldexpf(448.f, e) < amax) ++e;
    }
    const float sc = ldexpf(1.f, e);
    const int s_off = (d + 3) & ~3;
    const uint32_t sb = __float_as_uint(sc);
    for (int c = lane; c < pitch8; c += 64) {
        uint32_t code = 0;
        if (c < d) code = f32_to_e4m3(ldexpf(x[c], -e));
        else if (c >= s_off && c < s_off + 4) code = (sb >> (8 * (c - s_off))) & 0xFFu;
        dst[r * pitch8 + c] = (uint8_t)code;
    }
    if (lane == 0) scales[r] = sc;
}

// plain streaming copy (16 bytes per lane per step)
__global__ void k_copy_probe(uint4 *dst, const uint4 *src, int64_t n16) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

unsigned grid_for(int64_t total, int threads) {
    int64_t g = (total + threads - 1) / threads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

int launch_pad_rows(const float *src, int64_t n, int32_t d, float *dst, int32_t pitch, hipStream_t stream) {
    if (n == 0) return RG_OK;
    hipLaunchKernelGGL(k_pad_rows, dim3(grid_for(n * (int64_t)pitch, 256)), dim3(256), 0, stream, src, n, d, dst,
                       pitch);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

int launch_quant_bf16(const float *src, int64_t n, int32_t pitch, uint16_t *dst, hipStream_t stream) {
    if (n == 0) return RG_OK;
    const int64_t count = n * (int64_t)pitch;
    hipLaunchKernelGGL(k_quant_bf16, dim3(grid_for(count, 256)), dim3(256), 0, stream, src, count, dst);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

int launch_quant_fp8(const float *src, int64_t n, int32_t d, int32_t pitch, uint8_t *dst, int32_t pitch8,
                     float *scales, hipStream_t stream) {
    if (n == 0) return RG_OK;
    hipLaunchKernelGGL(k_quant_fp8, dim3((unsigned)n), dim3(64), 0, stream, src, n, d, pitch, dst, pitch8,
                       scales);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

int launch_copy_probe(void *dst, const void *src, int64_t bytes, hipStream_t stream) {
    if (bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0) {
        set_error("copy probe: bytes and pointers must be 16-byte aligned");
        return RG_EINVAL;
    }
    hipLaunchKernelGGL(k_copy_probe, dim3(4096), dim3(256), 0, stream, static_cast<uint4 *>(dst),
                       static_cast<const uint4 *>(src), bytes / 16);
    RG_HIP(hipGetLastError());
    return RG_OK;
}

}  // namespace rg
