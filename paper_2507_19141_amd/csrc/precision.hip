// Precision-form helpers of the BF16 path: master-to-BF16 rounding and the
// non-finite check behind dynamic loss scaling.  Both are plain streaming kernels.
#include "h4d_device.h"

namespace h4d {

constexpr int kCastBlock = 256;

// dst[i] = RNE BF16 of src[i]; eight elements per thread (two 16-byte loads, one
// 16-byte store).
__global__ __launch_bounds__(kCastBlock) void k_cast_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst,
                                                          int64_t count) {
    const int64_t i8 = ((int64_t)blockIdx.x * kCastBlock + threadIdx.x) * 8;
    if (i8 + 7 < count && ((((uintptr_t)src) | ((uintptr_t)dst)) & 15) == 0) {
        const float4 a = *reinterpret_cast<const float4*>(src + i8);
        const float4 b = *reinterpret_cast<const float4*>(src + i8 + 4);
        uint4 o;
        o.x = f32_to_bf16(a.x) | ((uint32_t)f32_to_bf16(a.y) << 16);
        o.y = f32_to_bf16(a.z) | ((uint32_t)f32_to_bf16(a.w) << 16);
        o.z = f32_to_bf16(b.x) | ((uint32_t)f32_to_bf16(b.y) << 16);
        o.w = f32_to_bf16(b.z) | ((uint32_t)f32_to_bf16(b.w) << 16);
        *reinterpret_cast<uint4*>(dst + i8) = o;
    } else {
        for (int64_t i = i8; i < count && i < i8 + 8; ++i) dst[i] = f32_to_bf16(src[i]);
    }
}

__global__ __launch_bounds__(kCastBlock) void k_zero_words(uint32_t* __restrict__ p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * kCastBlock + threadIdx.x; i < words; i += (int64_t)gridDim.x * kCastBlock)
        p[i] = 0u;
}

// counter += number of NaN / Inf values in p[0, count).
__global__ __launch_bounds__(kCastBlock) void k_count_nonfinite(const float* __restrict__ p, int64_t count,
                                                                int32_t* __restrict__ counter) {
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * kCastBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kCastBlock)
        bad += (__float_as_uint(p[i]) & 0x7f800000u) == 0x7f800000u;
    // wavefront sum, one atomic per wavefront with a non-finite value
    for (int s = 32; s > 0; s >>= 1) bad += __shfl_xor(bad, s, 64);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(counter, bad);
}

hipError_t launch_zero_words(void* p, int64_t words, hipStream_t s) {
    if (words <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((words + kCastBlock - 1) / kCastBlock, 4096);
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(kCastBlock), 0, s, static_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

hipError_t launch_cast_bf16(const float* src, uint16_t* dst, int64_t count, hipStream_t s) {
    const int64_t threads = (count + 7) / 8;
    hipLaunchKernelGGL(k_cast_bf16, dim3((unsigned)((threads + kCastBlock - 1) / kCastBlock)), dim3(kCastBlock), 0, s,
                       src, dst, count);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float* p, int64_t count, int32_t* counter, hipStream_t s) {
    int64_t blocks = (count + kCastBlock - 1) / kCastBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)blocks), dim3(kCastBlock), 0, s, p, count, counter);
    return hipGetLastError();
}

}  // namespace h4d

namespace h4d {

// Eq. 10: x' = x + dx, r' = r + dr, s' = s + ds from the decoder output delta
// [n, out] (dx at columns 0..2, dr at 3..6, ds at 7..9).  One thread per Gaussian;
// outputs may alias inputs.
__global__ __launch_bounds__(256) void k_deform_apply(const float* __restrict__ delta, int n, int out,
                                                      const float* x, const float* r, const float* s, float* xo,
                                                      float* ro, float* so) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float* d = delta + (int64_t)i * out;
#pragma unroll
    for (int k = 0; k < 3; ++k) xo[(int64_t)i * 3 + k] = __fadd_rn(x[(int64_t)i * 3 + k], d[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) ro[(int64_t)i * 4 + k] = __fadd_rn(r[(int64_t)i * 4 + k], d[3 + k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) so[(int64_t)i * 3 + k] = __fadd_rn(s[(int64_t)i * 3 + k], d[7 + k]);
}

hipError_t launch_deform_apply(const float* delta, int n, int out, const float* x, const float* r, const float* s,
                               float* xo, float* ro, float* so, hipStream_t st) {
    hipLaunchKernelGGL(k_deform_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, delta, n, out, x, r, s,
                       xo, ro, so);
    return hipGetLastError();
}

}  // namespace h4d
