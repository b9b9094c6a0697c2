// Spatio-temporal smoothness regulariser (DASH Section 4.3, Eq. 11), first pass:
//   L_r = lam / n * sum_q || G(x_q) - G(clamp(x_q + eps_q)) ||^2
// and, when asked, the per-(query, level) difference d = G(x) - G(x~) written
// level-major for the table-gradient pass (the tiled scatter with the pair of
// corner sets, scaled by 2 lam / n).  Both encodes are recomputed per (query,
// level); when x and x~ fall in the same hypervoxel (the coarse levels for a small
// eps) their 16 corners coincide and one gather per corner gives d with the weight
// difference w - w~.  Work items (level, 256 queries) are placed on XCDs level by
// level, and F = 2 FP32 / BF16 tables aligned to two rows read an x-pair of corners
// that shares an aligned row pair with one load, both as in the encoder.
#include "h4d_device.h"

namespace h4d {

constexpr int kSmoothBlock = 256;

template <typename TT, int F, bool PAIRS>
__global__ __launch_bounds__(kSmoothBlock) void k_smooth(DevGrid g, const TT* __restrict__ table,
                                                         const float4* __restrict__ xyzt,
                                                         const float4* __restrict__ eps, int n,
                                                         typename AccOf<TT>::type lam_over_n,
                                                         typename AccOf<TT>::type* __restrict__ loss,
                                                         typename AccOf<TT>::type* __restrict__ d_out) {
    using A = typename AccOf<TT>::type;
    __shared__ A red[kSmoothBlock / 64];
    const int chunks = (n + kSmoothBlock - 1) / kSmoothBlock;
    int l, chunk;
    if (!xcd_item(g.L * chunks, chunks, l, chunk)) return;
    const int q = chunk * kSmoothBlock + threadIdx.x;
    A part = A(0);
    if (q < n) {
        const float4 x = xyzt[q];
        const float4 e = eps[q];
        const float4 xp = make_float4(__fadd_rn(x.x, e.x), __fadd_rn(x.y, e.y), __fadd_rn(x.z, e.z), __fadd_rn(x.w, e.w));
        const Cell c0 = level_cell(g, l, x);
        const Cell c1 = level_cell(g, l, xp);
        const bool same = c0.ix == c1.ix && c0.iy == c1.iy && c0.iz == c1.iz && c0.it == c1.it;
        uint32_t r0[16], r1[16];
        level_rows(g, l, c0, r0);
        if (!same) level_rows(g, l, c1, r1);
        A w0[16], w1[16];
        level_weights<A>(c0, w0);
        level_weights<A>(c1, w1);
        A d[F];
#pragma unroll
        for (int f = 0; f < F; ++f) d[f] = A(0);
        if (same) {
            A v[16][F];
            gather_corners<TT, F, PAIRS>(g, table, r0, v);
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const A dw = w0[k] - w1[k];
#pragma unroll
                for (int f = 0; f < F; ++f) d[f] += dw * v[k][f];
            }
        } else {
            A v0[16][F], v1[16][F];
            gather_corners<TT, F, PAIRS>(g, table, r0, v0);
            gather_corners<TT, F, PAIRS>(g, table, r1, v1);
            A a0[F], a1[F];
#pragma unroll
            for (int f = 0; f < F; ++f) a0[f] = a1[f] = A(0);
#pragma unroll
            for (int k = 0; k < 16; ++k)
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    a0[f] += w0[k] * v0[k][f];
                    a1[f] += w1[k] * v1[k][f];
                }
#pragma unroll
            for (int f = 0; f < F; ++f) d[f] = a0[f] - a1[f];
        }
#pragma unroll
        for (int f = 0; f < F; ++f) part += d[f] * d[f];
        if (d_out) {
            A* o = d_out + ((int64_t)l * n + q) * F;
#pragma unroll
            for (int f = 0; f < F; ++f) o[f] = d[f];
        }
    }
    // block sum of the squared differences, one atomic per block
    for (int s = 32; s > 0; s >>= 1) part += __shfl_xor(part, s, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        A b = A(0);
        for (int w = 0; w < kSmoothBlock / 64; ++w) b += red[w];
        if (b != A(0)) atomic_add(loss, lam_over_n * b);
    }
}

template <typename TT>
static hipError_t smooth_t(const DevGrid& g, const void* table, const float* xyzt, const float* eps, int n, double lam,
                           void* loss, void* d_out, hipStream_t s) {
    using A = typename AccOf<TT>::type;
    const int chunks = (n + kSmoothBlock - 1) / kSmoothBlock;
    const dim3 grid((unsigned)(kXcds * xcd_items_per(g.L * chunks))), block(kSmoothBlock);
    const TT* t = static_cast<const TT*>(table);
    const float4* x = reinterpret_cast<const float4*>(xyzt);
    const float4* e = reinterpret_cast<const float4*>(eps);
    const A c = (A)(lam / (double)n);
    A* lo = static_cast<A*>(loss);
    A* dd = static_cast<A*>(d_out);
    constexpr bool kPairable = !std::is_same<TT, double>::value;
    const bool pairs = kPairable && ((uintptr_t)table % (2 * 2 * sizeof(TT))) == 0;
    switch (g.F) {
        case 1: hipLaunchKernelGGL((k_smooth<TT, 1, false>), grid, block, 0, s, g, t, x, e, n, c, lo, dd); break;
        case 2:
            if (pairs)
                hipLaunchKernelGGL((k_smooth<TT, 2, kPairable>), grid, block, 0, s, g, t, x, e, n, c, lo, dd);
            else
                hipLaunchKernelGGL((k_smooth<TT, 2, false>), grid, block, 0, s, g, t, x, e, n, c, lo, dd);
            break;
        case 4: hipLaunchKernelGGL((k_smooth<TT, 4, false>), grid, block, 0, s, g, t, x, e, n, c, lo, dd); break;
        case 8: hipLaunchKernelGGL((k_smooth<TT, 8, false>), grid, block, 0, s, g, t, x, e, n, c, lo, dd); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_smoothness(const DevGrid& g, h4d_dtype dt, const void* table, const float* xyzt, const float* eps,
                             int n, double lam, void* loss, void* d_out, hipStream_t s) {
    switch (dt) {
        case H4D_F32: return smooth_t<float>(g, table, xyzt, eps, n, lam, loss, d_out, s);
        case H4D_BF16: return smooth_t<bf16_t>(g, table, xyzt, eps, n, lam, loss, d_out, s);
        case H4D_F64: return smooth_t<double>(g, table, xyzt, eps, n, lam, loss, d_out, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace h4d
