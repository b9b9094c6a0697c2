// Roofline probes: the memory ceilings the encoder kernels are measured against.
//  - gather:  uniformly random row loads (4 or 8 bytes) from a table of the
//             encoder's footprint, the pattern of the corner gathers;
//  - scatter: uniformly random 8-byte rows, each receiving two FP32 atomic adds,
//             the pattern of the table-gradient scatter (F = 2);
//  - copy:    16-byte vector stream copy, the HBM ceiling.
// Row numbers come from a counter-based hash of the load index, so no index
// array is read.
#include "h4d_device.h"

namespace h4d {

constexpr int kProbeBlock = 256;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {  // a 32-bit integer finaliser (xorshift-multiply)
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <int ROW_BYTES>
__global__ __launch_bounds__(kProbeBlock) void k_probe_gather(const void* __restrict__ table, uint32_t rows,
                                                              int64_t n_loads, uint32_t seed, float* __restrict__ sink) {
    constexpr int kPer = 16;  // independent loads in flight per thread, like the 16 corners
    const int64_t base = ((int64_t)blockIdx.x * kProbeBlock + threadIdx.x) * kPer;
    float acc = 0.f;
    uint32_t r[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) r[k] = mix32((uint32_t)(base + k) ^ seed) % rows;
    if (ROW_BYTES == 8) {
        const float2* t = static_cast<const float2*>(table);
        float2 v[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) v[k] = (base + k < n_loads) ? t[r[k]] : make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < kPer; ++k) acc += v[k].x + v[k].y;
    } else {
        const float* t = static_cast<const float*>(table);
        float v[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) v[k] = (base + k < n_loads) ? t[r[k]] : 0.f;
#pragma unroll
        for (int k = 0; k < kPer; ++k) acc += v[k];
    }
    if (acc == 1.2345678f) sink[0] = acc;  // keeps the loads alive; practically never true
}

// mode 0: any random row.  mode 1: a random row of a 128-byte line this XCD owns
// (line % 8 == the hardware XCC id), so every line is updated from one XCD only.
__global__ __launch_bounds__(kProbeBlock) void k_probe_scatter(float* __restrict__ table, uint32_t rows,
                                                               int64_t n_updates, uint32_t seed, int mode) {
    constexpr int kPer = 16;
    const int64_t base = ((int64_t)blockIdx.x * kProbeBlock + threadIdx.x) * kPer;
    const uint32_t xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20) & 7u;  // HW_REG_XCC_ID bits [3:0]
    const uint32_t lines = rows / 16;                                     // 16 rows of 8 bytes per line
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (base + k < n_updates) {
            uint32_t r = mix32((uint32_t)(base + k) ^ seed) % rows;
            if (mode == 1 && lines >= 8) {
                uint32_t line = (r / 16) & ~7u;
                line = line + xcc < lines ? line + xcc : xcc;
                r = line * 16 + (r & 15);
            }
            unsafeAtomicAdd(table + 2 * (size_t)r, 1.0f);
            unsafeAtomicAdd(table + 2 * (size_t)r + 1, 1.0f);
        }
    }
}

__global__ __launch_bounds__(kProbeBlock) void k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                            int64_t n4) {
    for (int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kProbeBlock)
        dst[i] = src[i];
}

hipError_t launch_probe_gather(const void* table, uint32_t rows, int row_bytes, int64_t n_loads, uint32_t seed,
                               float* sink, hipStream_t s) {
    const int64_t threads = (n_loads + 15) / 16;
    const dim3 grid((unsigned)((threads + kProbeBlock - 1) / kProbeBlock));
    if (row_bytes == 8)
        hipLaunchKernelGGL(k_probe_gather<8>, grid, dim3(kProbeBlock), 0, s, table, rows, n_loads, seed, sink);
    else
        hipLaunchKernelGGL(k_probe_gather<4>, grid, dim3(kProbeBlock), 0, s, table, rows, n_loads, seed, sink);
    return hipGetLastError();
}

hipError_t launch_probe_scatter(float* table, uint32_t rows, int64_t n_updates, uint32_t seed, int mode,
                                hipStream_t s) {
    const int64_t threads = (n_updates + 15) / 16;
    hipLaunchKernelGGL(k_probe_scatter, dim3((unsigned)((threads + kProbeBlock - 1) / kProbeBlock)),
                       dim3(kProbeBlock), 0, s, table, rows, n_updates, seed, mode);
    return hipGetLastError();
}

hipError_t launch_probe_copy(const void* src, void* dst, int64_t bytes, hipStream_t s) {
    const int64_t n4 = bytes / 16;
    int64_t blocks = (n4 + kProbeBlock - 1) / kProbeBlock;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_probe_copy, dim3((unsigned)blocks), dim3(kProbeBlock), 0, s,
                       static_cast<const float4*>(src), static_cast<float4*>(dst), n4);
    return hipGetLastError();
}

}  // namespace h4d

namespace h4d {

// LDS atomics: each workgroup (1024 threads) owns a 128 KiB tile and adds, per
// thread, `per_thread` times to pseudo-random words of it; `active` of every 64
// lanes take part (the rest sit out each instruction), like the table scatter
// where only the lanes whose corner falls in the tile add.  MODE 0: ds_add_f32;
// 1: ds_add_u32; 2: FP32 add by compare-and-swap (lds_add).
template <int MODE>
__global__ __launch_bounds__(1024) void k_probe_lds_atomic(int per_thread, int active, uint32_t seed,
                                                           float* __restrict__ sink) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* tile = reinterpret_cast<float*>(smem);
    constexpr int kWords = 32768;
    for (int i = threadIdx.x; i < kWords; i += 1024) tile[i] = 0.f;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t id = blockIdx.x * 1024u + threadIdx.x;
    if ((int)lane < active) {
        for (int k = 0; k < per_thread; ++k) {
            const uint32_t w = mix32(id * 977u + (uint32_t)k * 0x9e3779b9u + seed) & (kWords - 1);
            if constexpr (MODE == 0) atomicAdd(tile + w, 1.0f);
            else if constexpr (MODE == 1) atomicAdd(reinterpret_cast<unsigned int*>(tile) + w, 1u);
            else lds_add(tile + w, 1.0f);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && tile[seed & (kWords - 1)] == -1.0f) sink[0] = 1.f;  // keeps the adds alive
}

hipError_t launch_probe_lds_atomic(int blocks, int per_thread, int active, uint32_t seed, int mode, float* sink,
                                   hipStream_t s) {
    const size_t lds = 128 * 1024;
    const void* k = mode == 0 ? (const void*)k_probe_lds_atomic<0>
                  : mode == 1 ? (const void*)k_probe_lds_atomic<1> : (const void*)k_probe_lds_atomic<2>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (mode == 0) hipLaunchKernelGGL(k_probe_lds_atomic<0>, dim3(blocks), dim3(1024), lds, s, per_thread, active, seed, sink);
    else if (mode == 1) hipLaunchKernelGGL(k_probe_lds_atomic<1>, dim3(blocks), dim3(1024), lds, s, per_thread, active, seed, sink);
    else hipLaunchKernelGGL(k_probe_lds_atomic<2>, dim3(blocks), dim3(1024), lds, s, per_thread, active, seed, sink);
    return hipGetLastError();
}

}  // namespace h4d
