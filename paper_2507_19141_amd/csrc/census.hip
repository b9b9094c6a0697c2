// Collision census of one level of the 4D hash table: over the 16 corners of n
// queries, the number V of distinct vertices and R of distinct table rows (on a
// hashed level V - R vertices share their row with another).  This is the measure
// behind the paper's case for hashing only the dynamic Gaussians (the "w/o dec"
// ablation of Section 5.3).
//
// Vertices go into an open-addressing set of 64-bit ids (16 bits per coordinate),
// capacity a power of two of at least twice the 16 n corners, linear probing with
// a compare-and-swap; rows into a bitmap of the level.  Both counts are exact.
#include "h4d_device.h"

namespace h4d {

constexpr int kCensusBlock = 256;
constexpr unsigned long long kEmptySlot = ~0ull;

__device__ __forceinline__ uint64_t mix64(uint64_t v) {  // splitmix64 finaliser
    v ^= v >> 30;
    v *= 0xbf58476d1ce4e5b9ull;
    v ^= v >> 27;
    v *= 0x94d049bb133111ebull;
    return v ^ (v >> 31);
}

__global__ __launch_bounds__(kCensusBlock) void k_census_clear(unsigned long long* __restrict__ slots, int64_t cap,
                                                               uint32_t* __restrict__ bitmap, int64_t words,
                                                               unsigned long long* __restrict__ counts) {
    const int64_t stride = (int64_t)gridDim.x * kCensusBlock;
    for (int64_t i = (int64_t)blockIdx.x * kCensusBlock + threadIdx.x; i < cap; i += stride) slots[i] = kEmptySlot;
    for (int64_t i = (int64_t)blockIdx.x * kCensusBlock + threadIdx.x; i < words; i += stride) bitmap[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x < 2) counts[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(kCensusBlock) void k_census(DevGrid g, int l, const float4* __restrict__ xyzt, int n,
                                                         unsigned long long* __restrict__ slots, uint64_t cap_mask,
                                                         uint32_t* __restrict__ bitmap,
                                                         unsigned long long* __restrict__ counts) {
    const int q = blockIdx.x * kCensusBlock + threadIdx.x;
    const bool live = q < n;
    Cell c{};
    uint32_t row[16];
    if (live) {
        c = level_cell(g, l, xyzt[q]);
        level_rows(g, l, c, row);
    }
    uint32_t new_v = 0, new_r = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (!live) break;
        const uint64_t id = (uint64_t)(c.ix + (k & 1)) | ((uint64_t)(c.iy + ((k >> 1) & 1)) << 16) |
                            ((uint64_t)(c.iz + ((k >> 2) & 1)) << 32) | ((uint64_t)(c.it + (k >> 3)) << 48);
        // linear probing; at most cap_mask + 1 probes, and the set is never full
        uint64_t h = mix64(id) & cap_mask;
        for (uint64_t probe = 0; probe <= cap_mask; ++probe) {
            const unsigned long long old = atomicCAS(&slots[h], kEmptySlot, (unsigned long long)id);
            if (old == kEmptySlot) {
                ++new_v;
                break;
            }
            if (old == id) break;
            h = (h + 1) & cap_mask;
        }
        const uint32_t rel = row[k] - g.off[l];
        const uint32_t bit = 1u << (rel & 31u);
        if (!(atomicOr(&bitmap[rel >> 5], bit) & bit)) ++new_r;
    }
    // one device atomic per wavefront and count
    uint32_t v = new_v, r = new_r;
    for (int o = 32; o > 0; o >>= 1) {
        v += __shfl_xor(v, o, 64);
        r += __shfl_xor(r, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (v) atomicAdd(&counts[0], (unsigned long long)v);
        if (r) atomicAdd(&counts[1], (unsigned long long)r);
    }
}

static int64_t census_capacity(int64_t n) {
    int64_t cap = 1024;
    while (cap < 32 * n) cap <<= 1;  // at least twice the 16 n corners
    return cap;
}

size_t census_workspace_bytes(int64_t n, int64_t level_rows) {
    return (size_t)census_capacity(n) * 8 + (size_t)((level_rows + 31) / 32) * 4;
}

hipError_t launch_census(const DevGrid& g, int l, int64_t level_rows, const float* xyzt, int n, int64_t* counts,
                         void* ws, hipStream_t s) {
    const int64_t cap = census_capacity(n);
    unsigned long long* slots = static_cast<unsigned long long*>(ws);
    uint32_t* bitmap = reinterpret_cast<uint32_t*>(slots + cap);
    const int64_t words = (level_rows + 31) / 32;
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(counts);
    const int64_t clear_blocks = std::min<int64_t>((cap + kCensusBlock - 1) / kCensusBlock, 4096);
    hipLaunchKernelGGL(k_census_clear, dim3((unsigned)clear_blocks), dim3(kCensusBlock), 0, s, slots, cap, bitmap,
                       words, cnt);
    hipLaunchKernelGGL(k_census, dim3((unsigned)((n + kCensusBlock - 1) / kCensusBlock)), dim3(kCensusBlock), 0, s, g,
                       l, reinterpret_cast<const float4*>(xyzt), n, slots, (uint64_t)(cap - 1), bitmap, cnt);
    return hipGetLastError();
}

}  // namespace h4d
