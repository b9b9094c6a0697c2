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

// ------------------------------------------------- XCD-partitioned scatter ----
// The table gradient is split by 128-byte line: line i belongs to slot i % 8.  A
// workgroup reads the hardware id of the XCC (accelerator complex die) it runs on
// and applies only the updates that fall in lines of that slot, pulling work items
// (a group of levels x a tile of queries) from its slot's queue until the queue is
// exhausted.  Every line is therefore updated from one XCC only, and its atomics
// can complete in that XCC's L2.  The last workgroup to finish processes any slot
// whose queue no workgroup touched (an XCC that received no workgroup), so the
// result never depends on how the dispatcher spreads workgroups over XCCs, and
// resets the queues for the next call.
constexpr int kXcdSlots = 8;
constexpr int kScatterLevelsPerItem = 4;
struct ScatterCtl {
    int next[kXcdSlots];
    int done;
};

__device__ __forceinline__ uint32_t xcc_slot() {
    return __builtin_amdgcn_s_getreg((3 << 11) | 20) & (kXcdSlots - 1);  // HW_REG_XCC_ID bits [3:0]
}

template <typename G, int F>
__device__ __forceinline__ void scatter_item(const DevGrid& g, const float4* __restrict__ xyzt, int n,
                                             const G* __restrict__ d_feat, int64_t lstride, int64_t qstride, G scale,
                                             G* __restrict__ d_table, int item, int ntiles, uint32_t slot) {
    const int lg = item / ntiles, tile = item - lg * ntiles;
    const int q = tile * kEncodeBlock + (int)threadIdx.x;
    if (q >= n) return;
    const float4 x = xyzt[q];
    const int l0 = lg * kScatterLevelsPerItem;
    const int l1 = min(l0 + kScatterLevelsPerItem, g.L);
    constexpr int kLineShift = (F * (int)sizeof(G) == 8) ? 4 : (F * (int)sizeof(G) == 4) ? 5 : (F * (int)sizeof(G) == 16) ? 3 : (F * (int)sizeof(G) == 32) ? 2 : 1;
    for (int l = l0; l < l1; ++l) {
        const G* gp = d_feat + (int64_t)l * lstride + (int64_t)q * qstride;
        G gf[F];
#pragma unroll
        for (int f = 0; f < F; ++f) gf[f] = gp[f] * scale;
        const Cell c = level_cell(g, l, x);
        uint32_t row[16];
        level_rows(g, l, c, row);
        G w[16];
        level_weights<G>(c, w);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (((row[k] >> kLineShift) & (kXcdSlots - 1)) == slot) {
#pragma unroll
                for (int f = 0; f < F; ++f) atomic_add(d_table + (size_t)row[k] * F + f, w[k] * gf[f]);
            }
        }
    }
}

template <typename G, int F>
__global__ __launch_bounds__(kEncodeBlock) void k_encode_backward_xcd(DevGrid g, const float4* __restrict__ xyzt,
                                                                      int n, const G* __restrict__ d_feat,
                                                                      int64_t lstride, int64_t qstride, G scale,
                                                                      G* __restrict__ d_table, ScatterCtl* ctl) {
    __shared__ int s_item;
    const uint32_t slot = xcc_slot();
    const int ntiles = (n + kEncodeBlock - 1) / kEncodeBlock;
    const int groups = (g.L + kScatterLevelsPerItem - 1) / kScatterLevelsPerItem;
    const int total = groups * ntiles;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&ctl->next[slot], 1);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= total) break;
        scatter_item<G, F>(g, xyzt, n, d_feat, lstride, qstride, scale, d_table, item, ntiles, slot);
    }
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(&ctl->done, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    for (int s = 0; s < kXcdSlots; ++s) {
        const int start = __hip_atomic_load(&ctl->next[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int item = start; item < total; ++item)
            scatter_item<G, F>(g, xyzt, n, d_feat, lstride, qstride, scale, d_table, item, ntiles, (uint32_t)s);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int s = 0; s < kXcdSlots; ++s) ctl->next[s] = 0;
        ctl->done = 0;
        __threadfence();
    }
}

__global__ void k_scatter_ctl_reset(ScatterCtl* ctl) {
    if (threadIdx.x < kXcdSlots) ctl->next[threadIdx.x] = 0;
    if (threadIdx.x == 0) ctl->done = 0;
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

size_t scatter_workspace_bytes() { return 256; }

template <typename G>
static hipError_t encode_backward_xcd_t(const DevGrid& g, const float* xyzt, int n, const void* d_feat, int64_t ls,
                                        int64_t qs, double scale, void* d_table, void* ws, hipStream_t s) {
    const float4* x = reinterpret_cast<const float4*>(xyzt);
    const G* df = static_cast<const G*>(d_feat);
    G* dt = static_cast<G*>(d_table);
    const G sc = (G)scale;
    ScatterCtl* ctl = static_cast<ScatterCtl*>(ws);
    hipLaunchKernelGGL(k_scatter_ctl_reset, dim3(1), dim3(64), 0, s, ctl);
    // enough workgroups to fill every CU twice; each XCC pulls its own queue
    const dim3 grid(kXcdSlots * 64), block(kEncodeBlock);
    switch (g.F) {
        case 1: hipLaunchKernelGGL((k_encode_backward_xcd<G, 1>), grid, block, 0, s, g, x, n, df, ls, qs, sc, dt, ctl); break;
        case 2: hipLaunchKernelGGL((k_encode_backward_xcd<G, 2>), grid, block, 0, s, g, x, n, df, ls, qs, sc, dt, ctl); break;
        case 4: hipLaunchKernelGGL((k_encode_backward_xcd<G, 4>), grid, block, 0, s, g, x, n, df, ls, qs, sc, dt, ctl); break;
        case 8: hipLaunchKernelGGL((k_encode_backward_xcd<G, 8>), grid, block, 0, s, g, x, n, df, ls, qs, sc, dt, ctl); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_encode_backward_xcd(const DevGrid& g, h4d_dtype grad_dt, const float* xyzt, int n,
                                      const void* d_feat, int64_t ls, int64_t qs, double scale, void* d_table,
                                      void* ws, hipStream_t s) {
    if (grad_dt == H4D_F64) return encode_backward_xcd_t<double>(g, xyzt, n, d_feat, ls, qs, scale, d_table, ws, s);
    return encode_backward_xcd_t<float>(g, xyzt, n, d_feat, ls, qs, scale, d_table, ws, s);
}

hipError_t launch_corner_indices(const DevGrid& g, const float* xyzt, int n, int32_t* rows, float* w, hipStream_t s) {
    hipLaunchKernelGGL(k_corner_indices, level_major_grid(n, g.L), dim3(kEncodeBlock), 0, s, g,
                       reinterpret_cast<const float4*>(xyzt), n, rows, w);
    return hipGetLastError();
}

}  // namespace h4d
