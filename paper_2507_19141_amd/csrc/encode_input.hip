// Gradient of the 4D hash encoder with respect to its input positions: the
// derivative of the quadrilinear interpolation of Eq. 9 (DASH Section 4.2) in the
// hypervoxel the forward selects, chained with the clamp.
//
// One thread per query walks the L levels: per level it gathers the 16 corner rows,
// forms tg_c = sum_f theta_c,f g_f with the level's upstream gradient g, and
// contracts tg with the four partial derivatives of the corner weights,
//   d w_c / d x_d = (upper along d ? +N_d : -N_d) * prod_{e != d} (frac_e or 1 - frac_e).
// The four sums over levels stay in registers, so each output row has one writer.
#include "h4d_device.h"

namespace h4d {

constexpr int kInputGradBlock = 256;

template <typename TT, int F>
__global__ __launch_bounds__(kInputGradBlock) void k_encode_input_grad(DevGrid g, const TT* __restrict__ table,
                                                                       const float4* __restrict__ xyzt, int n,
                                                                       const typename AccOf<TT>::type* __restrict__ d_feat,
                                                                       int64_t lstride, int64_t qstride,
                                                                       typename AccOf<TT>::type scale,
                                                                       typename AccOf<TT>::type* __restrict__ d_xyzt) {
    using A = typename AccOf<TT>::type;
    const int q = blockIdx.x * kInputGradBlock + threadIdx.x;
    if (q >= n) return;
    const float4 x = xyzt[q];
    // the clamp passes the derivative on its linear piece [0, 1]; NaN and out-of-range pass none
    const bool in[4] = {x.x >= 0.f && x.x <= 1.f, x.y >= 0.f && x.y <= 1.f, x.z >= 0.f && x.z <= 1.f,
                        x.w >= 0.f && x.w <= 1.f};
    A acc[4] = {A(0), A(0), A(0), A(0)};
    auto gather = [&](int l, A (&v)[16][F], Cell& c) {
        c = level_cell(g, l, x);
        uint32_t row[16];
        level_rows(g, l, c, row);
#pragma unroll
        for (int k = 0; k < 16; ++k) RowLoad<TT, F, A>::load(table, row[k], v[k]);
    };
    auto level = [&](int l, const A (&v)[16][F], const Cell& c) {
        const A* gp = d_feat + (int64_t)l * lstride + (int64_t)q * qstride;
        A gv[F];
#pragma unroll
        for (int f = 0; f < F; ++f) gv[f] = gp[f];
        const A w[4][2] = {{A(1) - A(c.fx), A(c.fx)}, {A(1) - A(c.fy), A(c.fy)},
                           {A(1) - A(c.fz), A(c.fz)}, {A(1) - A(c.ft), A(c.ft)}};
        A s[4] = {A(0), A(0), A(0), A(0)};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            A tg = A(0);
#pragma unroll
            for (int f = 0; f < F; ++f) tg += v[k][f] * gv[f];
            const int bx = k & 1, by = (k >> 1) & 1, bz = (k >> 2) & 1, bt = k >> 3;
            const A wx = w[0][bx], wy = w[1][by], wz = w[2][bz], wt = w[3][bt];
            const A pxy = wx * wy, pzt = wz * wt;
            const A dx = (wy * pzt) * tg, dy = (wx * pzt) * tg, dz = (pxy * wt) * tg, dt = (pxy * wz) * tg;
            s[0] += bx ? dx : -dx;
            s[1] += by ? dy : -dy;
            s[2] += bz ? dz : -dz;
            s[3] += bt ? dt : -dt;
        }
        const A Ns = A(g.res_s[l]), Nt = A(g.res_t[l]);
        acc[0] += Ns * s[0];
        acc[1] += Ns * s[1];
        acc[2] += Ns * s[2];
        acc[3] += Nt * s[3];
    };
    // Two levels per step: both levels' 32 row loads are in flight before either is
    // reduced, which halves the chain of dependent gathers per thread.
    int l = 0;
    for (; l + 1 < g.L; l += 2) {
        A va[16][F], vb[16][F];
        Cell ca, cb;
        gather(l, va, ca);
        gather(l + 1, vb, cb);
        level(l, va, ca);
        level(l + 1, vb, cb);
    }
    if (l < g.L) {
        A va[16][F];
        Cell ca;
        gather(l, va, ca);
        level(l, va, ca);
    }
    A* o = d_xyzt + (int64_t)q * 4;
#pragma unroll
    for (int d = 0; d < 4; ++d) o[d] += in[d] ? scale * acc[d] : A(0);
}

template <typename TT>
static hipError_t input_grad_t(const DevGrid& g, const void* table, const float* xyzt, int n, const void* d_feat,
                               int64_t ls, int64_t qs, double scale, void* d_xyzt, hipStream_t s) {
    using A = typename AccOf<TT>::type;
    const dim3 grid((unsigned)((n + kInputGradBlock - 1) / kInputGradBlock)), block(kInputGradBlock);
    const TT* t = static_cast<const TT*>(table);
    const float4* x = reinterpret_cast<const float4*>(xyzt);
    const A* gf = static_cast<const A*>(d_feat);
    A* o = static_cast<A*>(d_xyzt);
    switch (g.F) {
        case 1: hipLaunchKernelGGL((k_encode_input_grad<TT, 1>), grid, block, 0, s, g, t, x, n, gf, ls, qs, (A)scale, o); break;
        case 2: hipLaunchKernelGGL((k_encode_input_grad<TT, 2>), grid, block, 0, s, g, t, x, n, gf, ls, qs, (A)scale, o); break;
        case 4: hipLaunchKernelGGL((k_encode_input_grad<TT, 4>), grid, block, 0, s, g, t, x, n, gf, ls, qs, (A)scale, o); break;
        case 8: hipLaunchKernelGGL((k_encode_input_grad<TT, 8>), grid, block, 0, s, g, t, x, n, gf, ls, qs, (A)scale, o); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_encode_input_grad(const DevGrid& g, h4d_dtype dt, const void* table, const float* xyzt, int n,
                                    const void* d_feat, int64_t ls, int64_t qs, double scale, void* d_xyzt,
                                    hipStream_t s) {
    switch (dt) {
        case H4D_F32: return input_grad_t<float>(g, table, xyzt, n, d_feat, ls, qs, scale, d_xyzt, s);
        case H4D_BF16: return input_grad_t<bf16_t>(g, table, xyzt, n, d_feat, ls, qs, scale, d_xyzt, s);
        case H4D_F64: return input_grad_t<double>(g, table, xyzt, n, d_feat, ls, qs, scale, d_xyzt, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace h4d
