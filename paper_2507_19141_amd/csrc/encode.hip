// 4D hash encoder forward and backward kernels (DASH Section 4.2, Eqs. 8-9).
//
// One thread per (query, level).  The grid is level-major (blockIdx.y = level):
// the hardware dispatches workgroups in linear order, so at any moment the chip
// works on one or two levels and each XCD's L2 holds mostly that level's slice of
// the table (4 MiB FP32 / 2 MiB BF16 for a 2^19-row, F = 2 level) instead of the
// whole table.
#include "h4d_device.h"

namespace h4d {

constexpr int kEncodeBlock = 256;

template <typename TT, int F>
__global__ __launch_bounds__(kEncodeBlock) void k_encode(DevGrid g, const TT* __restrict__ table,
                                                         const float4* __restrict__ xyzt, int n,
                                                         typename AccOf<TT>::type* __restrict__ out,
                                                         int64_t lstride, int64_t qstride) {
    using A = typename AccOf<TT>::type;
    const int l = blockIdx.y;
    const int q = blockIdx.x * kEncodeBlock + threadIdx.x;
    if (q >= n) return;
    const Cell c = level_cell(g, l, xyzt[q]);
    uint32_t row[16];
    level_rows(g, l, c, row);
    A v[16][F];
#pragma unroll
    for (int k = 0; k < 16; ++k) RowLoad<TT, F, A>::load(table, row[k], v[k]);
    A w[16];
    level_weights<A>(c, w);
    A acc[F];
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = A(0);
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int f = 0; f < F; ++f) acc[f] += w[k] * v[k][f];
    A* o = out + (int64_t)l * lstride + (int64_t)q * qstride;
    if constexpr (F == 2 && sizeof(A) == 4) {
        *reinterpret_cast<float2*>(o) = make_float2(acc[0], acc[1]);
    } else {
#pragma unroll
        for (int f = 0; f < F; ++f) o[f] = acc[f];
    }
}

template <typename G, int F>
__global__ __launch_bounds__(kEncodeBlock) void k_encode_backward(DevGrid g, const float4* __restrict__ xyzt, int n,
                                                                  const G* __restrict__ d_feat, int64_t lstride,
                                                                  int64_t qstride, G scale, G* __restrict__ d_table) {
    const int l = blockIdx.y;
    const int q = blockIdx.x * kEncodeBlock + threadIdx.x;
    if (q >= n) return;
    const G* gp = d_feat + (int64_t)l * lstride + (int64_t)q * qstride;
    G gf[F];
#pragma unroll
    for (int f = 0; f < F; ++f) gf[f] = gp[f] * scale;
    const Cell c = level_cell(g, l, xyzt[q]);
    uint32_t row[16];
    level_rows(g, l, c, row);
    G w[16];
    level_weights<G>(c, w);
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int f = 0; f < F; ++f) atomic_add(d_table + (size_t)row[k] * F + f, w[k] * gf[f]);
}

__global__ __launch_bounds__(kEncodeBlock) void k_corner_indices(DevGrid g, const float4* __restrict__ xyzt, int n,
                                                                 int32_t* __restrict__ rows, float* __restrict__ w) {
    const int l = blockIdx.y;
    const int q = blockIdx.x * kEncodeBlock + threadIdx.x;
    if (q >= n) return;
    const Cell c = level_cell(g, l, xyzt[q]);
    uint32_t row[16];
    level_rows(g, l, c, row);
    float wt[16];
    level_weights<float>(c, wt);
    const int64_t base = ((int64_t)q * g.L + l) * 16;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (rows) rows[base + k] = (int32_t)row[k];
        if (w) w[base + k] = wt[k];
    }
}

// ---------------------------------------------------------------- launchers ----
static dim3 level_major_grid(int n, int L) { return dim3((unsigned)((n + kEncodeBlock - 1) / kEncodeBlock), (unsigned)L); }

template <typename TT>
static hipError_t encode_t(const DevGrid& g, const void* table, const float* xyzt, int n, void* out,
                           int64_t ls, int64_t qs, hipStream_t s) {
    using A = typename AccOf<TT>::type;
    const dim3 grid = level_major_grid(n, g.L), block(kEncodeBlock);
    const TT* t = static_cast<const TT*>(table);
    const float4* x = reinterpret_cast<const float4*>(xyzt);
    A* o = static_cast<A*>(out);
    switch (g.F) {
        case 1: hipLaunchKernelGGL((k_encode<TT, 1>), grid, block, 0, s, g, t, x, n, o, ls, qs); break;
        case 2: hipLaunchKernelGGL((k_encode<TT, 2>), grid, block, 0, s, g, t, x, n, o, ls, qs); break;
        case 4: hipLaunchKernelGGL((k_encode<TT, 4>), grid, block, 0, s, g, t, x, n, o, ls, qs); break;
        case 8: hipLaunchKernelGGL((k_encode<TT, 8>), grid, block, 0, s, g, t, x, n, o, ls, qs); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_encode(const DevGrid& g, h4d_dtype dt, const void* table, const float* xyzt, int n, void* out,
                         int64_t ls, int64_t qs, hipStream_t s) {
    switch (dt) {
        case H4D_F32: return encode_t<float>(g, table, xyzt, n, out, ls, qs, s);
        case H4D_BF16: return encode_t<bf16_t>(g, table, xyzt, n, out, ls, qs, s);
        case H4D_F64: return encode_t<double>(g, table, xyzt, n, out, ls, qs, s);
    }
    return hipErrorInvalidValue;
}

template <typename G>
static hipError_t encode_backward_t(const DevGrid& g, const float* xyzt, int n, const void* d_feat, int64_t ls,
                                    int64_t qs, double scale, void* d_table, hipStream_t s) {
    const dim3 grid = level_major_grid(n, g.L), block(kEncodeBlock);
    const float4* x = reinterpret_cast<const float4*>(xyzt);
    const G* df = static_cast<const G*>(d_feat);
    G* dt = static_cast<G*>(d_table);
    const G sc = (G)scale;
    switch (g.F) {
        case 1: hipLaunchKernelGGL((k_encode_backward<G, 1>), grid, block, 0, s, g, x, n, df, ls, qs, sc, dt); break;
        case 2: hipLaunchKernelGGL((k_encode_backward<G, 2>), grid, block, 0, s, g, x, n, df, ls, qs, sc, dt); break;
        case 4: hipLaunchKernelGGL((k_encode_backward<G, 4>), grid, block, 0, s, g, x, n, df, ls, qs, sc, dt); break;
        case 8: hipLaunchKernelGGL((k_encode_backward<G, 8>), grid, block, 0, s, g, x, n, df, ls, qs, sc, dt); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_encode_backward(const DevGrid& g, h4d_dtype grad_dt, const float* xyzt, int n, const void* d_feat,
                                  int64_t ls, int64_t qs, double scale, void* d_table, hipStream_t s) {
    if (grad_dt == H4D_F64) return encode_backward_t<double>(g, xyzt, n, d_feat, ls, qs, scale, d_table, s);
    return encode_backward_t<float>(g, xyzt, n, d_feat, ls, qs, scale, d_table, s);
}

hipError_t launch_corner_indices(const DevGrid& g, const float* xyzt, int n, int32_t* rows, float* w, hipStream_t s) {
    hipLaunchKernelGGL(k_corner_indices, level_major_grid(n, g.L), dim3(kEncodeBlock), 0, s, g,
                       reinterpret_cast<const float4*>(xyzt), n, rows, w);
    return hipGetLastError();
}

}  // namespace h4d
