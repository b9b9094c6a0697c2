// 3D multiresolution hash encoding G_3D of the decomposition front end (DASH
// Section 4.1, Eq. 3): per position and level, the 8 corners of its voxel, dense or
// hashed rows (the spatial hash of the 4D encoder on x, y, z alone), F features per
// corner, trilinear interpolation.  One thread per (query, level); work items
// (level, 256 queries) are XCD-placed level by level like the 4D encoder's, and the
// two x-corners of a pair come from one row-pair load where they are adjacent rows.
#include "h4d_device.h"

namespace h4d {

constexpr int kEncode3Block = 256;

template <typename TT, int F, bool PAIRS, int STRIDE>
__global__ __launch_bounds__(kEncode3Block) void k_encode3(DevGrid3 g, const TT* __restrict__ table,
                                                           const float* __restrict__ xyz, int n,
                                                           typename AccOf<TT>::type* __restrict__ out,
                                                           int64_t lstride, int64_t qstride) {
    using A = typename AccOf<TT>::type;
    const int chunks = (n + kEncode3Block - 1) / kEncode3Block;
    int l, chunk;
    if (!xcd_item(g.L * chunks, chunks, l, chunk)) return;
    const int q = chunk * kEncode3Block + threadIdx.x;
    if (q >= n) return;
    float px, py, pz;
    if constexpr (STRIDE == 4) {
        const float4 p = reinterpret_cast<const float4*>(xyz)[q];
        px = p.x; py = p.y; pz = p.z;
    } else {
        const float* p = xyz + (int64_t)q * STRIDE;
        px = p[0]; py = p[1]; pz = p[2];
    }
    const int N = g.res[l];
    int ix, iy, iz;
    float fx, fy, fz;
    cell_1d(clamp_unit(px), N, ix, fx);
    cell_1d(clamp_unit(py), N, iy, fy);
    cell_1d(clamp_unit(pz), N, iz, fz);
    // rows of the 8 corners; corner k is upper along x, y, z iff bit 0, 1, 2 of k is set
    uint32_t row[8];
    const uint32_t off = g.off[l];
    if ((g.dense_bits >> l) & 1u) {
        const uint32_t S = (uint32_t)N + 1u;
        const uint32_t base = off + (uint32_t)ix + S * ((uint32_t)iy + S * (uint32_t)iz);
#pragma unroll
        for (int k = 0; k < 8; ++k) row[k] = base + (k & 1) + ((k >> 1) & 1) * S + ((k >> 2) & 1) * S * S;
    } else {
        const uint32_t hx0 = (uint32_t)ix * g.prime[0], hx1 = hx0 + g.prime[0];
        const uint32_t hy0 = (uint32_t)iy * g.prime[1], hy1 = hy0 + g.prime[1];
        const uint32_t hz0 = (uint32_t)iz * g.prime[2], hz1 = hz0 + g.prime[2];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t h = ((k & 1) ? hx1 : hx0) ^ ((k & 2) ? hy1 : hy0) ^ ((k & 4) ? hz1 : hz0);
            row[k] = off + (g.tmask ? (h & g.tmask) : h % g.T);
        }
    }
    A v[8][F];
    if constexpr (PAIRS) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const uint32_t r0 = row[2 * p], r1 = row[2 * p + 1];
            const uint32_t a = r0 & ~1u;
            if (r1 == (r0 ^ 1u) && a + 1u < g.rows) {
                A lo[2], hi[2];
                RowPairLoad<TT, A>::load(table, a, lo, hi);
                const bool odd = r0 & 1u;
#pragma unroll
                for (int f = 0; f < 2; ++f) {
                    v[2 * p][f] = odd ? hi[f] : lo[f];
                    v[2 * p + 1][f] = odd ? lo[f] : hi[f];
                }
            } else {
                RowLoad<TT, F, A>::load(table, r0, v[2 * p]);
                RowLoad<TT, F, A>::load(table, r1, v[2 * p + 1]);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) RowLoad<TT, F, A>::load(table, row[k], v[k]);
    }
    const A wx[2] = {A(1) - A(fx), A(fx)};
    const A wy[2] = {A(1) - A(fy), A(fy)};
    const A wz[2] = {A(1) - A(fz), A(fz)};
    A acc[F];
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = A(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const A w = (wx[k & 1] * wy[(k >> 1) & 1]) * wz[k >> 2];
#pragma unroll
        for (int f = 0; f < F; ++f) acc[f] += w * v[k][f];
    }
    A* o = out + (int64_t)l * lstride + (int64_t)q * qstride;
    if constexpr (F == 2 && sizeof(A) == 4) {
        *reinterpret_cast<float2*>(o) = make_float2(acc[0], acc[1]);
    } else {
#pragma unroll
        for (int f = 0; f < F; ++f) o[f] = acc[f];
    }
}

template <typename TT, int F, bool PAIRS>
static void encode3_s(const DevGrid3& g, const TT* t, const float* xyz, int stride, int n,
                      typename AccOf<TT>::type* o, int64_t ls, int64_t qs, dim3 grid, hipStream_t s) {
    if (stride == 4) hipLaunchKernelGGL((k_encode3<TT, F, PAIRS, 4>), grid, dim3(kEncode3Block), 0, s, g, t, xyz, n, o, ls, qs);
    else hipLaunchKernelGGL((k_encode3<TT, F, PAIRS, 3>), grid, dim3(kEncode3Block), 0, s, g, t, xyz, n, o, ls, qs);
}

template <typename TT>
static hipError_t encode3_t(const DevGrid3& g, const void* table, const float* xyz, int stride, int n, void* out,
                            int64_t ls, int64_t qs, hipStream_t s) {
    using A = typename AccOf<TT>::type;
    const int chunks = (n + kEncode3Block - 1) / kEncode3Block;
    const dim3 grid((unsigned)(kXcds * xcd_items_per(g.L * chunks)));
    const TT* t = static_cast<const TT*>(table);
    A* o = static_cast<A*>(out);
    constexpr bool kPairable = !std::is_same<TT, double>::value;
    const bool pairs = kPairable && g.F == 2 && ((uintptr_t)table % (2 * 2 * sizeof(TT))) == 0;
    switch (g.F) {
        case 1: encode3_s<TT, 1, false>(g, t, xyz, stride, n, o, ls, qs, grid, s); break;
        case 2:
            if (pairs) encode3_s<TT, 2, kPairable>(g, t, xyz, stride, n, o, ls, qs, grid, s);
            else encode3_s<TT, 2, false>(g, t, xyz, stride, n, o, ls, qs, grid, s);
            break;
        case 4: encode3_s<TT, 4, false>(g, t, xyz, stride, n, o, ls, qs, grid, s); break;
        case 8: encode3_s<TT, 8, false>(g, t, xyz, stride, n, o, ls, qs, grid, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_encode3(const DevGrid3& g, h4d_dtype dt, const void* table, const float* xyz, int stride, int n,
                          void* out, int64_t ls, int64_t qs, hipStream_t s) {
    if (stride != 3 && stride != 4) return hipErrorInvalidValue;
    switch (dt) {
        case H4D_F32: return encode3_t<float>(g, table, xyz, stride, n, out, ls, qs, s);
        case H4D_BF16: return encode3_t<bf16_t>(g, table, xyz, stride, n, out, ls, qs, s);
        case H4D_F64: return encode3_t<double>(g, table, xyz, stride, n, out, ls, qs, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace h4d
