// Self-supervised dynamic-static split (DASH Section 4.1, Eqs. 4-5): the step that
// decides which Gaussians the 4D hash path deforms.
//
// Keys: the FP32 squared motion magnitude s = (dx^2 + dy^2) + dz^2 of each
// Gaussian's linear-motion vector dp, rounded step by step (no fused multiply-add)
// and ordered by its bit pattern (s >= 0, so the bits order like the values; NaN
// ranks above +Inf).  The threshold tau is the (n_d + 1)-th largest key, found by an
// exact radix select (four passes over 8-bit digits, most significant first); a
// Gaussian is dynamic iff its key is strictly greater than tau.  The dynamic indices
// are then written in ascending order (a stable compaction), and the static ones get
// the static constraint lam_s / N_s * sum ||dp|| and its gradient.
#include "h4d_device.h"

namespace h4d {

constexpr int kDecBlock = 256;

// (x^2 + y^2) + z^2 in FP32, each product and sum rounded on its own: contraction is
// off in this block, so no step becomes a fused multiply-add.
__device__ __forceinline__ uint32_t motion_key(const float* __restrict__ dp, int64_t i) {
#pragma clang fp contract(off)
    const float x = dp[3 * i], y = dp[3 * i + 1], z = dp[3 * i + 2];
    const float s = (x * x + y * y) + z * z;
    return __float_as_uint(s);
}

// Select state in the workspace: [0] prefix of the key found so far, [1] rank still
// sought among the keys with that prefix (ascending, 0-based), [2] 1 when there is
// no threshold (every Gaussian dynamic), [3] the number of dynamic Gaussians.
struct SelectState {
    uint32_t prefix, rank, all, n_dyn;
};

__global__ __launch_bounds__(kDecBlock) void k_select_init(SelectState* st, uint32_t* hist, int64_t n, int64_t n_d) {
    if (threadIdx.x == 0) {
        st->prefix = 0u;
        st->all = n_d >= n ? 1u : 0u;
        st->rank = n_d >= n ? 0u : (uint32_t)(n - n_d - 1);  // the (n_d + 1)-th largest, counted from below
        st->n_dyn = 0u;
    }
    hist[threadIdx.x] = 0u;
}

// Histogram of digit `shift` over the keys whose higher digits equal the prefix.
__global__ __launch_bounds__(kDecBlock) void k_select_hist(const float* __restrict__ dp, int64_t n,
                                                           const SelectState* __restrict__ st, int shift,
                                                           uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t prefix = st->prefix;
    const uint32_t hi_mask = shift == 24 ? 0u : ~((1u << (shift + 8)) - 1u);
    for (int64_t i = (int64_t)blockIdx.x * kDecBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDecBlock) {
        const uint32_t k = motion_key(dp, i);
        if ((k & hi_mask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Pick the bucket holding the sought rank, extend the prefix, clear the histogram.
__global__ __launch_bounds__(256) void k_select_pick(SelectState* st, uint32_t* hist, int shift) {
    __shared__ uint32_t c[256];
    const uint32_t v = hist[threadIdx.x];
    c[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {  // inclusive scan
        const uint32_t a = threadIdx.x >= (unsigned)d ? c[threadIdx.x - d] : 0u;
        __syncthreads();
        c[threadIdx.x] += a;
        __syncthreads();
    }
    const uint32_t rank = st->rank;
    const uint32_t below = c[threadIdx.x] - v;
    __syncthreads();
    if (below <= rank && rank < c[threadIdx.x]) {  // exactly one bucket when the rank exists
        st->prefix |= (uint32_t)threadIdx.x << shift;
        st->rank = rank - below;
    }
    hist[threadIdx.x] = 0u;
}

__device__ __forceinline__ bool is_dynamic(uint32_t key, const SelectState& s) { return s.all || key > s.prefix; }

// Per block: dynamic count and the sum of the static magnitudes (FP32 norm).
__global__ __launch_bounds__(kDecBlock) void k_split_count(const float* __restrict__ dp, int64_t n,
                                                           const SelectState* __restrict__ st,
                                                           uint32_t* __restrict__ counts, float* __restrict__ sums) {
    __shared__ uint32_t wc[kDecBlock / 64];
    __shared__ float ws[kDecBlock / 64];
    const SelectState s = *st;
    const int64_t i = (int64_t)blockIdx.x * kDecBlock + threadIdx.x;
    bool dyn = false;
    float mag = 0.f;
    if (i < n) {
        dyn = is_dynamic(motion_key(dp, i), s);
        if (!dyn) {
            const float x = dp[3 * i], y = dp[3 * i + 1], z = dp[3 * i + 2];
            mag = sqrtf(x * x + y * y + z * z);
        }
    }
    const uint32_t c = (uint32_t)__popcll(__ballot(dyn));
    for (int o = 32; o > 0; o >>= 1) mag += __shfl_xor(mag, o, 64);
    if ((threadIdx.x & 63) == 0) {
        wc[threadIdx.x >> 6] = c;
        ws[threadIdx.x >> 6] = mag;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tc = 0;
        float ts = 0.f;
        for (int w = 0; w < kDecBlock / 64; ++w) {
            tc += wc[w];
            ts += ws[w];
        }
        counts[blockIdx.x] = tc;
        sums[blockIdx.x] = ts;
    }
}

// One workgroup: block offsets (exclusive scan of the counts), the dynamic total,
// and the static constraint added to *loss with the block sums in a fixed order.
__global__ __launch_bounds__(1024) void k_split_scan(const uint32_t* __restrict__ counts,
                                                     const float* __restrict__ sums, int nb, int64_t n,
                                                     SelectState* st, uint32_t* __restrict__ offsets,
                                                     int32_t* __restrict__ n_dynamic, float lam_s,
                                                     float* __restrict__ loss) {
    __shared__ uint32_t part[1024];
    __shared__ float fpart[1024];
    const int per = (nb + 1023) / 1024;
    const int b = threadIdx.x * per, e = min(b + per, nb);
    uint32_t c = 0;
    float f = 0.f;
    for (int i = b; i < e; ++i) {
        c += counts[i];
        f += sums[i];
    }
    part[threadIdx.x] = c;
    fpart[threadIdx.x] = f;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - c;
    for (int i = b; i < e; ++i) {
        offsets[i] = run;
        run += counts[i];
    }
    if (threadIdx.x == 0) {
        float total = 0.f;
        for (int i = 0; i < 1024; ++i) total += fpart[i];
        const uint32_t n_dyn = part[1023];
        st->n_dyn = n_dyn;
        if (n_dynamic) *n_dynamic = (int32_t)n_dyn;
        const int64_t n_s = n - (int64_t)n_dyn;
        if (loss && n_s > 0) *loss += lam_s / (float)n_s * total;
    }
}

// Dynamic: index written at its ascending position.  Static: the constraint's gradient.
__global__ __launch_bounds__(kDecBlock) void k_split_write(const float* __restrict__ dp, int64_t n,
                                                           const SelectState* __restrict__ st,
                                                           const uint32_t* __restrict__ offsets, float lam_s,
                                                           int32_t* __restrict__ dyn_idx,
                                                           uint8_t* __restrict__ is_dyn, float* __restrict__ d_dp) {
    __shared__ uint32_t wc[kDecBlock / 64];
    const SelectState s = *st;
    const int64_t i = (int64_t)blockIdx.x * kDecBlock + threadIdx.x;
    const bool dyn = i < n && is_dynamic(motion_key(dp, i), s);
    const uint64_t bal = __ballot(dyn);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wc[wave] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (i >= n) return;
    if (is_dyn) is_dyn[i] = dyn ? 1 : 0;
    if (dyn) {
        uint32_t pos = offsets[blockIdx.x];
        for (int w = 0; w < wave; ++w) pos += wc[w];
        pos += (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        if (dyn_idx) dyn_idx[pos] = (int32_t)i;
    } else if (d_dp) {
        const int64_t n_s = n - (int64_t)s.n_dyn;
        const float x = dp[3 * i], y = dp[3 * i + 1], z = dp[3 * i + 2];
        const float mag = sqrtf(x * x + y * y + z * z);
        if (mag > 0.f) {
            const float c = lam_s / (float)n_s / mag;
            d_dp[3 * i] += c * x;
            d_dp[3 * i + 1] += c * y;
            d_dp[3 * i + 2] += c * z;
        }
    }
}

size_t decompose_workspace_bytes(int64_t n) {
    const int64_t nb = (n + kDecBlock - 1) / kDecBlock;
    return 256 + 256 * 4 + (size_t)nb * 4 * 3;
}

hipError_t launch_decompose(const float* dp, int64_t n, double k_percent, float lam_s, int32_t* dyn_idx,
                            int32_t* n_dynamic, uint8_t* is_dyn, float* loss, float* d_dp, void* ws, hipStream_t s) {
    char* w = static_cast<char*>(ws);
    SelectState* st = reinterpret_cast<SelectState*>(w);
    uint32_t* hist = reinterpret_cast<uint32_t*>(w + 256);
    const int64_t nb = (n + kDecBlock - 1) / kDecBlock;
    uint32_t* counts = hist + 256;
    float* sums = reinterpret_cast<float*>(counts + nb);
    uint32_t* offsets = reinterpret_cast<uint32_t*>(sums + nb);
    const int64_t n_d = (int64_t)floor(k_percent / 100.0 * (double)n);
    hipLaunchKernelGGL(k_select_init, dim3(1), dim3(256), 0, s, st, hist, n, n_d);
    const int hist_blocks = (int)std::min<int64_t>(nb, 256);  // 256 device atomics per block and pass
    for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_select_hist, dim3(hist_blocks), dim3(kDecBlock), 0, s, dp, n, st, shift, hist);
        hipLaunchKernelGGL(k_select_pick, dim3(1), dim3(256), 0, s, st, hist, shift);
    }
    hipLaunchKernelGGL(k_split_count, dim3((unsigned)nb), dim3(kDecBlock), 0, s, dp, n, st, counts, sums);
    hipLaunchKernelGGL(k_split_scan, dim3(1), dim3(1024), 0, s, counts, sums, (int)nb, n, st, offsets, n_dynamic,
                       lam_s, loss);
    hipLaunchKernelGGL(k_split_write, dim3((unsigned)nb), dim3(kDecBlock), 0, s, dp, n, st, offsets, lam_s, dyn_idx,
                       is_dyn, d_dp);
    return hipGetLastError();
}

}  // namespace h4d
