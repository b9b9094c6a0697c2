// Gradient of the 4D hash encoder with respect to its input positions: the
// derivative of the quadrilinear interpolation of Eq. 9 (DASH Section 4.2) in the
// hypervoxel the forward selects, chained with the clamp.
//
// One thread per query walks the L levels: per level it gathers the 16 corner rows,
// forms tg_c = sum_f theta_c,f g_f with the level's upstream gradient g, and
// contracts tg with the four partial derivatives of the corner weights,
//   d w_c / d x_d = (upper along d ? +N_d : -N_d) * prod_{e != d} (frac_e or 1 - frac_e).
// The four sums over levels stay in registers, so each output row has one writer.
//
// With a workspace (FP32 and BF16 tables) the work is split in two passes instead:
// one thread per (query, level), placed on the XCDs level by level like the encoder
// (each XCD's L2 serves one level's table slice at a time, and x-pairs of corners come
// from one row-pair load), writes the level's four terms N_d s_d to a [L, n] float4
// buffer; a second pass sums them per query in level order and applies the clamp and
// the scale.
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

// Pass 1 of the two-pass form: the four terms of level l for query q.
template <typename TT, int F, bool PAIRS>
__global__ __launch_bounds__(kInputGradBlock) void k_input_grad_levels(DevGrid g, const TT* __restrict__ table,
                                                                       const float4* __restrict__ xyzt, int n,
                                                                       const float* __restrict__ d_feat,
                                                                       int64_t lstride, int64_t qstride,
                                                                       float4* __restrict__ part) {
    const int chunks = (n + kInputGradBlock - 1) / kInputGradBlock;
    int l, chunk;
    if (!xcd_item(g.L * chunks, chunks, l, chunk)) return;
    const int q = chunk * kInputGradBlock + threadIdx.x;
    if (q >= n) return;
    const Cell c = level_cell(g, l, xyzt[q]);
    uint32_t row[16];
    level_rows(g, l, c, row);
    float v[16][F];
    gather_corners<TT, F, PAIRS>(g, table, row, v);
    const float* gp = d_feat + (int64_t)l * lstride + (int64_t)q * qstride;
    float gv[F];
#pragma unroll
    for (int f = 0; f < F; ++f) gv[f] = gp[f];
    const float w[4][2] = {{1.f - c.fx, c.fx}, {1.f - c.fy, c.fy}, {1.f - c.fz, c.fz}, {1.f - c.ft, c.ft}};
    float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        float tg = 0.f;
#pragma unroll
        for (int f = 0; f < F; ++f) tg += v[k][f] * gv[f];
        const int bx = k & 1, by = (k >> 1) & 1, bz = (k >> 2) & 1, bt = k >> 3;
        const float wx = w[0][bx], wy = w[1][by], wz = w[2][bz], wt = w[3][bt];
        const float pxy = wx * wy, pzt = wz * wt;
        const float dx = (wy * pzt) * tg, dy = (wx * pzt) * tg, dz = (pxy * wt) * tg, dt = (pxy * wz) * tg;
        s[0] += bx ? dx : -dx;
        s[1] += by ? dy : -dy;
        s[2] += bz ? dz : -dz;
        s[3] += bt ? dt : -dt;
    }
    const float Ns = (float)g.res_s[l], Nt = (float)g.res_t[l];
    part[(int64_t)l * n + q] = make_float4(Ns * s[0], Ns * s[1], Ns * s[2], Nt * s[3]);
}

// Pass 2: sum the levels in order, then the clamp and the scale; one writer per row.
__global__ __launch_bounds__(kInputGradBlock) void k_input_grad_reduce(const float4* __restrict__ part, int L, int n,
                                                                       const float4* __restrict__ xyzt, float scale,
                                                                       float* __restrict__ d_xyzt) {
    const int q = blockIdx.x * kInputGradBlock + threadIdx.x;
    if (q >= n) return;
    const float4 x = xyzt[q];
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    for (int l = 0; l < L; ++l) {
        const float4 p = part[(int64_t)l * n + q];
        a0 += p.x;
        a1 += p.y;
        a2 += p.z;
        a3 += p.w;
    }
    float4* o = reinterpret_cast<float4*>(d_xyzt) + q;
    float4 r = *o;
    r.x += (x.x >= 0.f && x.x <= 1.f) ? scale * a0 : 0.f;
    r.y += (x.y >= 0.f && x.y <= 1.f) ? scale * a1 : 0.f;
    r.z += (x.z >= 0.f && x.z <= 1.f) ? scale * a2 : 0.f;
    r.w += (x.w >= 0.f && x.w <= 1.f) ? scale * a3 : 0.f;
    *o = r;
}

size_t input_grad_workspace_bytes(int L, int n) { return (size_t)L * n * sizeof(float4); }

template <typename TT>
static hipError_t input_grad_two_pass(const DevGrid& g, const void* table, const float* xyzt, int n, const void* d_feat,
                                      int64_t ls, int64_t qs, double scale, void* d_xyzt, void* ws, hipStream_t s) {
    const int chunks = (n + kInputGradBlock - 1) / kInputGradBlock;
    const dim3 grid((unsigned)(kXcds * xcd_items_per(g.L * chunks))), block(kInputGradBlock);
    const TT* t = static_cast<const TT*>(table);
    const float4* x = reinterpret_cast<const float4*>(xyzt);
    const float* gf = static_cast<const float*>(d_feat);
    float4* part = static_cast<float4*>(ws);
    const bool pairs = ((uintptr_t)table % (2 * 2 * sizeof(TT))) == 0;
    switch (g.F) {
        case 1: hipLaunchKernelGGL((k_input_grad_levels<TT, 1, false>), grid, block, 0, s, g, t, x, n, gf, ls, qs, part); break;
        case 2:
            if (pairs) hipLaunchKernelGGL((k_input_grad_levels<TT, 2, true>), grid, block, 0, s, g, t, x, n, gf, ls, qs, part);
            else hipLaunchKernelGGL((k_input_grad_levels<TT, 2, false>), grid, block, 0, s, g, t, x, n, gf, ls, qs, part);
            break;
        case 4: hipLaunchKernelGGL((k_input_grad_levels<TT, 4, false>), grid, block, 0, s, g, t, x, n, gf, ls, qs, part); break;
        case 8: hipLaunchKernelGGL((k_input_grad_levels<TT, 8, false>), grid, block, 0, s, g, t, x, n, gf, ls, qs, part); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_input_grad_reduce, dim3((unsigned)((n + kInputGradBlock - 1) / kInputGradBlock)),
                       dim3(kInputGradBlock), 0, s, part, g.L, n, x, (float)scale, static_cast<float*>(d_xyzt));
    return hipGetLastError();
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
                                    hipStream_t s, void* ws) {
    if (ws && dt == H4D_F32) return input_grad_two_pass<float>(g, table, xyzt, n, d_feat, ls, qs, scale, d_xyzt, ws, s);
    if (ws && dt == H4D_BF16) return input_grad_two_pass<bf16_t>(g, table, xyzt, n, d_feat, ls, qs, scale, d_xyzt, ws, s);
    switch (dt) {
        case H4D_F32: return input_grad_t<float>(g, table, xyzt, n, d_feat, ls, qs, scale, d_xyzt, s);
        case H4D_BF16: return input_grad_t<bf16_t>(g, table, xyzt, n, d_feat, ls, qs, scale, d_xyzt, s);
        case H4D_F64: return input_grad_t<double>(g, table, xyzt, n, d_feat, ls, qs, scale, d_xyzt, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace h4d
