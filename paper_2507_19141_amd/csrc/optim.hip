// Fused optimiser step over an FP32 master array (tables or decoder parameters):
// Adam with bias correction on grad * grad_scale, the BF16 copy the next step's
// BF16 form reads, and the zeroing of the gradient for the next step, in one pass
// over the arrays (the three separate passes would read and write them three times).
//
// "Lazy": the arrays are rows of `row` values, and a row whose whole gradient is
// zero (an untouched table row this step) keeps its parameters and moments.
#include "h4d_device.h"

namespace h4d {

constexpr int kAdamBlock = 256;

struct AdamArgs {
    float beta1, beta2, eps, grad_scale;
    float step_size;   // lr / (1 - beta1^t)
    float inv_sqrt_bc2;  // 1 / sqrt(1 - beta2^t)
};

__device__ __forceinline__ void adam_one(float& p, float& m, float& v, float g, const AdamArgs& a) {
    g *= a.grad_scale;
    m = a.beta1 * m + (1.f - a.beta1) * g;
    v = a.beta2 * v + (1.f - a.beta2) * (g * g);
    const float denom = sqrtf(v) * a.inv_sqrt_bc2 + a.eps;
    p -= a.step_size * (m / denom);
}

// Each thread owns units of U elements (U = 4, or 8 for rows of 8), so that every
// lazy row lies inside one unit: the row test and the zeroing never race.  Full
// units use 16-byte accesses; the arrays are 16-byte aligned (checked on entry).
template <int ROW, bool LAZY, bool BF16, bool ZERO>
__global__ __launch_bounds__(kAdamBlock) void k_adam(float* __restrict__ p, float* __restrict__ g,
                                                     float* __restrict__ m, float* __restrict__ v, int64_t count,
                                                     AdamArgs a, uint16_t* __restrict__ lo) {
    constexpr int U = ROW > 4 ? ROW : 4;
    static_assert(U % ROW == 0 && U % 4 == 0, "rows must tile the unit");
    const int64_t stride = (int64_t)gridDim.x * kAdamBlock * U;
    for (int64_t i = ((int64_t)blockIdx.x * kAdamBlock + threadIdx.x) * U; i < count; i += stride) {
        const int cnt = count - i < U ? (int)(count - i) : U;
        float pe[U], ge[U], me[U], ve[U];
        if (cnt == U) {
#pragma unroll
            for (int k = 0; k < U; k += 4) {
                const float4 pp = *reinterpret_cast<const float4*>(p + i + k);
                const float4 gg = *reinterpret_cast<const float4*>(g + i + k);
                const float4 mm = *reinterpret_cast<const float4*>(m + i + k);
                const float4 vv = *reinterpret_cast<const float4*>(v + i + k);
                pe[k] = pp.x; pe[k + 1] = pp.y; pe[k + 2] = pp.z; pe[k + 3] = pp.w;
                ge[k] = gg.x; ge[k + 1] = gg.y; ge[k + 2] = gg.z; ge[k + 3] = gg.w;
                me[k] = mm.x; me[k + 1] = mm.y; me[k + 2] = mm.z; me[k + 3] = mm.w;
                ve[k] = vv.x; ve[k + 1] = vv.y; ve[k + 2] = vv.z; ve[k + 3] = vv.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const bool in = k < cnt;
                pe[k] = in ? p[i + k] : 0.f;
                ge[k] = in ? g[i + k] : 0.f;
                me[k] = in ? m[i + k] : 0.f;
                ve[k] = in ? v[i + k] : 0.f;
            }
        }
        bool live[U];
#pragma unroll
        for (int k = 0; k < U; ++k) live[k] = true;
        if constexpr (LAZY) {
#pragma unroll
            for (int r0 = 0; r0 < U; r0 += ROW) {
                bool any = false;
#pragma unroll
                for (int k = r0; k < r0 + ROW; ++k) any |= ge[k] != 0.f;
#pragma unroll
                for (int k = r0; k < r0 + ROW; ++k) live[k] = any;
            }
        }
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (live[k]) adam_one(pe[k], me[k], ve[k], ge[k], a);
        if (cnt == U) {
#pragma unroll
            for (int k = 0; k < U; k += 4) {
                *reinterpret_cast<float4*>(p + i + k) = make_float4(pe[k], pe[k + 1], pe[k + 2], pe[k + 3]);
                *reinterpret_cast<float4*>(m + i + k) = make_float4(me[k], me[k + 1], me[k + 2], me[k + 3]);
                *reinterpret_cast<float4*>(v + i + k) = make_float4(ve[k], ve[k + 1], ve[k + 2], ve[k + 3]);
                if constexpr (BF16) {
                    ushort4 o;
                    o.x = f32_to_bf16(pe[k]); o.y = f32_to_bf16(pe[k + 1]);
                    o.z = f32_to_bf16(pe[k + 2]); o.w = f32_to_bf16(pe[k + 3]);
                    *reinterpret_cast<ushort4*>(lo + i + k) = o;
                }
                if constexpr (ZERO) *reinterpret_cast<float4*>(g + i + k) = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        } else {
            for (int k = 0; k < cnt; ++k) {
                p[i + k] = pe[k];
                m[i + k] = me[k];
                v[i + k] = ve[k];
                if constexpr (BF16) lo[i + k] = f32_to_bf16(pe[k]);
                if constexpr (ZERO) g[i + k] = 0.f;
            }
        }
    }
}

hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t count, int row, double lr, double beta1,
                       double beta2, double eps, int step, double grad_scale, uint16_t* lo, bool lazy, bool zero,
                       hipStream_t s) {
    AdamArgs a;
    a.beta1 = (float)beta1;
    a.beta2 = (float)beta2;
    a.eps = (float)eps;
    a.grad_scale = (float)grad_scale;
    a.step_size = (float)(lr / (1.0 - pow(beta1, step)));
    a.inv_sqrt_bc2 = (float)(1.0 / sqrt(1.0 - pow(beta2, step)));
    const int U = row > 4 ? row : 4;
    const int64_t units = (count + U - 1) / U;
    int64_t blocks = (units + kAdamBlock - 1) / kAdamBlock;
    if (blocks > 65536) blocks = 65536;
    const dim3 grid((unsigned)blocks), block(kAdamBlock);
    const bool bf = lo != nullptr;
#define H4D_ADAM(RR, LZ)                                                                                   \
    do {                                                                                                   \
        if (bf && zero) hipLaunchKernelGGL((k_adam<RR, LZ, true, true>), grid, block, 0, s, p, g, m, v, count, a, lo);   \
        else if (bf) hipLaunchKernelGGL((k_adam<RR, LZ, true, false>), grid, block, 0, s, p, g, m, v, count, a, lo);     \
        else if (zero) hipLaunchKernelGGL((k_adam<RR, LZ, false, true>), grid, block, 0, s, p, g, m, v, count, a, lo);   \
        else hipLaunchKernelGGL((k_adam<RR, LZ, false, false>), grid, block, 0, s, p, g, m, v, count, a, lo);            \
    } while (0)
    if (!lazy) {
        H4D_ADAM(1, false);
    } else {
        switch (row) {
            case 1: H4D_ADAM(1, true); break;
            case 2: H4D_ADAM(2, true); break;
            case 4: H4D_ADAM(4, true); break;
            case 8: H4D_ADAM(8, true); break;
            default: return hipErrorInvalidValue;
        }
    }
#undef H4D_ADAM
    return hipGetLastError();
}

}  // namespace h4d
