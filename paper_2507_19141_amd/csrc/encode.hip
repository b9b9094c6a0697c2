// 4D hash encoder forward and backward kernels (DASH Section 4.2, Eqs. 8-9).
//
// Forward: one thread per (query, level).  Work items (level, 256 queries) are
// placed on XCDs level by level (xcd_item), so each XCD's L2 holds mostly one
// level's slice of the table (4 MiB FP32 / 2 MiB BF16 for a 2^19-row, F = 2 level)
// instead of every XCD streaming the whole table through its L2.
#include <string.h>

#include <mutex>

#include "h4d_device.h"

namespace h4d {

constexpr int kEncodeBlock = 256;

// PAIRS: row-pair loads (gather_corners).  The loads change; the arithmetic (and its
// order) does not.
template <typename TT, int F, bool PAIRS>
__global__ __launch_bounds__(kEncodeBlock) void k_encode(DevGrid g, const TT* __restrict__ table,
                                                         const float4* __restrict__ xyzt, int n,
                                                         typename AccOf<TT>::type* __restrict__ out,
                                                         int64_t lstride, int64_t qstride) {
    using A = typename AccOf<TT>::type;
    const int chunks = (n + kEncodeBlock - 1) / kEncodeBlock;
    int l, chunk;
    if (!xcd_item(g.L * chunks, chunks, l, chunk)) return;
    const int q = chunk * kEncodeBlock + threadIdx.x;
    if (q >= n) return;
    const Cell c = level_cell(g, l, xyzt[q]);
    uint32_t row[16];
    level_rows(g, l, c, row);
    A v[16][F];
    gather_corners<TT, F, PAIRS>(g, table, row, v);
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

// ------------------------------------------------------ tiled table scatter ----
// Device-scope FP32 atomics on MI355X complete at a fixed rate of about 2e10 per
// second whatever the footprint (they are not executed in the XCD-local L2), so
// the scatter avoids them altogether.  Owner computes: one workgroup per (level,
// tile of 2^tile_shift consecutive table rows of that level; about 32 tiles per
// level) keeps the tile's gradient in LDS, adds w_c g for the corners of the
// level's queries that fall in its tile with compare-and-swap LDS adds (lds_add2),
// and finally adds the tile to d_table with plain loads and stores (no other
// workgroup owns those rows).
//
// A pre-pass records, per (query, level), a 32-bit mask of the tiles the query's
// corners touch (tile t sets bit t >> bit_shift).  A tile workgroup reads the
// masks of its level, compacts the queries whose bit is set into per-wavefront LDS
// queues and runs the corner work on full wavefronts of those queries only.  With
// pi_1 = 1 the two x-corners of a hashed level share a tile, so a query touches at
// most 8 of a hashed level's tiles.
// PAIR: each query also subtracts the same gradient at the corners of x + eps (the
// second term of Eq. 11).

template <bool PAIR>
__global__ __launch_bounds__(kEncodeBlock) void k_tile_mask(DevGrid g, TileMap tm, const float4* __restrict__ xyzt,
                                                            const float4* __restrict__ eps, int n,
                                                            uint32_t* __restrict__ mask, uint2* __restrict__ words) {
    const int l = blockIdx.y;
    const int q = blockIdx.x * kEncodeBlock + threadIdx.x;
    if (q >= n) return;
    const float4 x = xyzt[q];
    if (!PAIR && ((tm.pair_words >> l) & 1u)) {
        const uint2 b = pair_tile_bytes(g, tm, l, level_cell(g, l, x));
        const int bs = tm.bit_shift[l];
        uint32_t m = 0;
#pragma unroll
        for (int k = 0; k < 32; k += 8) m |= (1u << (((b.x >> k) & 0xffu) >> bs)) | (1u << (((b.y >> k) & 0xffu) >> bs));
        mask[(int64_t)l * mask_stride(n) + q] = m;
        words[(int64_t)l * mask_stride(n) + q] = b;
        return;
    }
    uint32_t m = corner_tile_mask(g, tm, l, x);
    if constexpr (PAIR) {
        const float4 e = eps[q];
        const float4 xp = make_float4(__fadd_rn(x.x, e.x), __fadd_rn(x.y, e.y), __fadd_rn(x.z, e.z),
                                      __fadd_rn(x.w, e.w));
        m |= corner_tile_mask(g, tm, l, xp);
    }
    mask[(int64_t)l * mask_stride(n) + q] = m;
}

// 1024 threads share each tile: the 128 KiB of LDS allows one workgroup per CU, and
// sixteen wavefronts (four per SIMD) keep the query loads in flight.
constexpr int kScatterBlock = 1024;
constexpr int kQueueCap = 2 * kScatterBlock;  // 128 entries per wavefront

// With PAIR, a second feature gradient (the decoder's) that joins the first at x's
// corners only: a training step with Eq. 11 then scatters both in one pass.
template <typename G>
struct MainGrad {
    const G* src;  // nullptr: none
    int64_t lstride, qstride;
    G scale;
};

// What the scatter loads per queued query: position, gradient (and perturbation).
template <typename G, int F, bool PAIR>
struct TileQuery {
    float4 x;
    float4 e;     // used when PAIR
    G gv[F];
    G gmain[F];   // used when PAIR with a MainGrad
};

template <typename G, int F, bool PAIR>
__device__ __forceinline__ TileQuery<G, F, PAIR> tile_load(int l, const float4* __restrict__ xyzt,
                                                           const float4* __restrict__ eps, const G* __restrict__ src,
                                                           int64_t lstride, int64_t qstride, const MainGrad<G>& mg,
                                                           int q) {
    TileQuery<G, F, PAIR> t;
    const G* gp = src + (int64_t)l * lstride + (int64_t)q * qstride;
#pragma unroll
    for (int f = 0; f < F; ++f) t.gv[f] = gp[f];
    t.x = xyzt[q];
    if constexpr (PAIR) {
        t.e = eps[q];
        if (mg.src) {
            const G* mp = mg.src + (int64_t)l * mg.lstride + (int64_t)q * mg.qstride;
#pragma unroll
            for (int f = 0; f < F; ++f) t.gmain[f] = mp[f];
        }
    }
    return t;
}

template <typename G, int F, bool PAIR>
__device__ __forceinline__ void tile_run(const DevGrid& g, const TileMap& tm, int l, const TileQuery<G, F, PAIR>& t,
                                         G scale, const MainGrad<G>& mg, uint32_t base, uint32_t cnt, G* tile) {
    G gv[F];
#pragma unroll
    for (int f = 0; f < F; ++f) gv[f] = t.gv[f] * scale;
    if constexpr (PAIR) {
        G gx[F], gm[F];
#pragma unroll
        for (int f = 0; f < F; ++f) {
            gx[f] = mg.src ? gv[f] + t.gmain[f] * mg.scale : gv[f];
            gm[f] = -gv[f];
        }
        tile_contrib<G, F>(g, tm, l, t.x, gx, base, cnt, tile);
        const float4 x = t.x, e = t.e;
        const float4 xp = make_float4(__fadd_rn(x.x, e.x), __fadd_rn(x.y, e.y), __fadd_rn(x.z, e.z),
                                      __fadd_rn(x.w, e.w));
        tile_contrib<G, F>(g, tm, l, xp, gm, base, cnt, tile);
    } else {
        tile_contrib<G, F>(g, tm, l, t.x, gv, base, cnt, tile);
    }
}

// Levels with per-pair tile bytes (tm.pair_words): a queued query usually has one
// pair in the tile, sometimes two or more.  Every lane adds the first of its pairs at
// once; a query with more goes to a per-wavefront overflow queue (query, remaining
// pairs), which is worked off a full wavefront at a time, so no lane idles through
// another lane's extra pairs.
template <typename G, int F>
struct WordQuery {
    float4 x;
    G gv[F];
    uint2 wd;
    int q;
};

constexpr int kOverflowCap = 128;  // entries per wavefront

template <typename G, int F>
__device__ __forceinline__ void scatter_pair_words(const DevGrid& g, const TileMap& tm, int l, uint32_t tau,
                                                   uint32_t bit, const float4* __restrict__ xyzt, int n,
                                                   const uint32_t* __restrict__ lmask, const uint2* __restrict__ lwords,
                                                   const G* __restrict__ src, int64_t lstride, int64_t qstride,
                                                   G scale, int* queue, int2* overflow, G* tile) {
    const int lane = threadIdx.x & 63;
    int2* ovf = overflow + (threadIdx.x >> 6) * kOverflowCap;
    const uint32_t rmask = (1u << tm.tile_shift[l]) - 1u;
    const G* gl = src + (int64_t)l * lstride;
    int ovn = 0;  // entries in this wavefront's overflow queue (wavefront-uniform)
    // whole wavefront: add the first pair of pm (none if pm = 0), queue the rest
    auto visit = [&](float4 x, const G (&gv)[F], uint32_t pm, int q) {
        const uint32_t rest = pm & (pm - 1u);
        const uint64_t bal = __ballot(rest != 0u);
        if (rest) ovf[ovn + lane_rank(bal)] = make_int2(q, (int)rest);
        ovn += (int)__popcll(bal);
        wave_sync();
        if (pm) pair_contrib<G, F>(g, l, x, __builtin_ctz(pm), gv, rmask, tile);
    };
    // work off the overflow queue while it holds more than `keep` entries
    auto drain = [&](int keep) {
        while (ovn > keep) {
            const int take = min(ovn, 64);
            const int2 e = lane < take ? ovf[lane] : make_int2(0, 0);
            const int rest = ovn - take;
            const int2 moved = lane < rest ? ovf[64 + lane] : make_int2(0, 0);
            wave_sync();
            if (lane < rest) ovf[lane] = moved;
            wave_sync();
            ovn = rest;
            float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
            G gv[F];
#pragma unroll
            for (int f = 0; f < F; ++f) gv[f] = G(0);
            if (lane < take) {
                x = xyzt[e.x];
                const G* gp = gl + (int64_t)e.x * qstride;
#pragma unroll
                for (int f = 0; f < F; ++f) gv[f] = gp[f] * scale;
            }
            visit(x, gv, lane < take ? (uint32_t)e.y : 0u, e.x);
        }
    };
    masked_queue_loop_wave<kScatterBlock>(
        n, lmask, bit, queue,
        [&](int q) {
            WordQuery<G, F> t;
            const G* gp = gl + (int64_t)q * qstride;
#pragma unroll
            for (int f = 0; f < F; ++f) t.gv[f] = gp[f];
            t.x = xyzt[q];
            t.wd = lwords[q];
            t.q = q;
            return t;
        },
        [&](const WordQuery<G, F>& t, bool active) {
            G gv[F];
#pragma unroll
            for (int f = 0; f < F; ++f) gv[f] = t.gv[f] * scale;
            visit(t.x, gv, active ? pair_hits(t.wd, tau) : 0u, t.q);
            drain(63);
        });
    drain(0);
}

template <typename G, int F, bool PAIR>
__global__ __launch_bounds__(kScatterBlock) void k_scatter_tiled(DevGrid g, TileMap tm, const float4* __restrict__ xyzt,
                                                                const float4* __restrict__ eps, int n,
                                                                const uint32_t* __restrict__ mask,
                                                                const uint2* __restrict__ words,
                                                                const G* __restrict__ src, int64_t lstride,
                                                                int64_t qstride, G scale, G* __restrict__ d_table,
                                                                int overwrite, MainGrad<G> mg) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int queue[kQueueCap];
    __shared__ int2 overflow[PAIR ? 1 : kScatterBlock / 64 * kOverflowCap];
    G* tile = reinterpret_cast<G*>(smem);
    // XCD placement: XCD x works on the contiguous run [x per, (x + 1) per) of the
    // level-ordered tile list, so its L2 holds the masks, pair bytes and gradients of
    // two or three levels instead of every XCD fetching every level's.
    const int tiles = tm.tile_start[g.L];
    const int per = xcd_items_per(tiles);
    const int tix = ((int)blockIdx.x % kXcds) * per + (int)blockIdx.x / kXcds;
    if ((int)blockIdx.x / kXcds >= per || tix >= tiles) return;
    int l = 0;
    while (l + 1 < g.L && tix >= tm.tile_start[l + 1]) ++l;
    const uint32_t t_in_level = (uint32_t)(tix - tm.tile_start[l]);
    const uint32_t first = t_in_level << tm.tile_shift[l];
    const uint32_t base = g.off[l] + first;
    const uint32_t cnt = min(1u << tm.tile_shift[l], (uint32_t)tm.level_rows[l] - first);
    const uint32_t bit = tile_bit(tm, l, first);
    for (uint32_t i = threadIdx.x; i < cnt * F; i += kScatterBlock) tile[i] = G(0);
    __syncthreads();
    if (!PAIR && ((tm.pair_words >> l) & 1u)) {
        scatter_pair_words<G, F>(g, tm, l, t_in_level, bit, xyzt, n, mask + (int64_t)l * mask_stride(n),
                                 words + (int64_t)l * mask_stride(n), src, lstride, qstride, scale, queue, overflow,
                                 tile);
    } else {
        masked_queue_loop<kScatterBlock>(
            n, mask + (int64_t)l * mask_stride(n), bit, queue,
            [&](int q) { return tile_load<G, F, PAIR>(l, xyzt, eps, src, lstride, qstride, mg, q); },
            [&](const TileQuery<G, F, PAIR>& t) { tile_run<G, F, PAIR>(g, tm, l, t, scale, mg, base, cnt, tile); });
    }
    __syncthreads();
    // the tile's rows have no other owner: add them to d_table, or with overwrite set
    // write every row (the tiles of the levels cover all E rows)
    G* out = d_table + (size_t)base * F;
    if (overwrite) {
        for (uint32_t i = threadIdx.x; i < cnt * F; i += kScatterBlock) out[i] = tile[i];
    } else {
        for (uint32_t i = threadIdx.x; i < cnt * F; i += kScatterBlock) {
            const G v = tile[i];
            if (v != G(0)) out[i] += v;
        }
    }
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
    const int chunks = (n + kEncodeBlock - 1) / kEncodeBlock;
    const dim3 grid((unsigned)(kXcds * xcd_items_per(g.L * chunks))), block(kEncodeBlock);
    const TT* t = static_cast<const TT*>(table);
    const float4* x = reinterpret_cast<const float4*>(xyzt);
    A* o = static_cast<A*>(out);
    constexpr bool kPairable = !std::is_same<TT, double>::value;
    const bool pairs = kPairable && g.F == 2 && ((uintptr_t)table % (2 * 2 * sizeof(TT))) == 0;
    switch (g.F) {
        case 1: hipLaunchKernelGGL((k_encode<TT, 1, false>), grid, block, 0, s, g, t, x, n, o, ls, qs); break;
        case 2:
            if (pairs) hipLaunchKernelGGL((k_encode<TT, 2, kPairable>), grid, block, 0, s, g, t, x, n, o, ls, qs);
            else hipLaunchKernelGGL((k_encode<TT, 2, false>), grid, block, 0, s, g, t, x, n, o, ls, qs);
            break;
        case 4: hipLaunchKernelGGL((k_encode<TT, 4, false>), grid, block, 0, s, g, t, x, n, o, ls, qs); break;
        case 8: hipLaunchKernelGGL((k_encode<TT, 8, false>), grid, block, 0, s, g, t, x, n, o, ls, qs); break;
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

// Tiles of at most 128 KiB of LDS; tile_start is the first tile of each level.
TileMap make_tile_map(const DevGrid& g, const int64_t* level_rows, int F, int gbytes, bool pair_words) {
    TileMap tm;
    memset(&tm, 0, sizeof tm);
    tm.max_rows = kTileBytes / (F * gbytes);  // a power of two: F and gbytes are
    int t = 0;
    for (int l = 0; l < g.L; ++l) {
        tm.tile_start[l] = t;
        tm.level_rows[l] = (int32_t)level_rows[l];
        const int64_t want = (level_rows[l] + kTilesPerLevel - 1) / kTilesPerLevel;
        int sh = 8;  // at least 256 rows per tile
        while ((1 << sh) < tm.max_rows && ((int64_t)1 << sh) < want) ++sh;
        tm.tile_shift[l] = sh;
        const bool hashed = !((g.dense_bits >> l) & 1u);
        if (hashed && g.tmask != 0u && g.prime[0] == 1u && level_rows[l] >= ((int64_t)1 << sh) &&
            2 * (int64_t)g.res_s[l] <= ((int64_t)1 << sh))
            tm.pair_cotiled |= 1u << l;
        const int P = (int)((level_rows[l] + (1 << sh) - 1) >> sh);
        if (pair_words && ((tm.pair_cotiled >> l) & 1u) && P <= 256) tm.pair_words |= 1u << l;
        while (((P - 1) >> tm.bit_shift[l]) >= 32) ++tm.bit_shift[l];
        t += P;
    }
    tm.tile_start[g.L] = t;
    return tm;
}

size_t scatter_mask_bytes(int n, int L) { return (size_t)mask_stride(n) * L * (sizeof(uint32_t) + sizeof(uint2)); }

template <typename G, int F, bool PAIR>
static hipError_t tiled_f(const DevGrid& g, const TileMap& tm, const float* xyzt, const float* eps, int n,
                          const uint32_t* mask, const uint2* words, const void* src, int64_t ls, int64_t qs,
                          double scale, void* d_table, bool overwrite, const MainGradArg& main, hipStream_t s) {
    auto kern = k_scatter_tiled<G, F, PAIR>;
    const size_t lds = (size_t)tm.max_rows * F * sizeof(G);
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)(kXcds * xcd_items_per(tm.tile_start[g.L]))), dim3(kScatterBlock), lds, s, g, tm,
                       reinterpret_cast<const float4*>(xyzt), reinterpret_cast<const float4*>(eps), n, mask, words,
                       static_cast<const G*>(src), ls, qs, (G)scale, static_cast<G*>(d_table), overwrite ? 1 : 0,
                       MainGrad<G>{static_cast<const G*>(main.src), main.lstride, main.qstride, (G)main.scale});
    return hipGetLastError();
}

template <typename G, bool PAIR>
static hipError_t tiled_g(const DevGrid& g, const int64_t* level_rows, const float* xyzt, const float* eps, int n,
                          const void* src, int64_t ls, int64_t qs, double scale, void* d_table, void* mask_ws,
                          bool overwrite, const MainGradArg& main, hipStream_t s) {
    const TileMap tm = make_tile_map(g, level_rows, g.F, (int)sizeof(G), !PAIR);
    uint32_t* mask = static_cast<uint32_t*>(mask_ws);
    uint2* words = reinterpret_cast<uint2*>(mask + mask_stride(n) * g.L);
    hipLaunchKernelGGL(k_tile_mask<PAIR>, dim3((unsigned)((n + kEncodeBlock - 1) / kEncodeBlock), (unsigned)g.L),
                       dim3(kEncodeBlock), 0, s, g, tm, reinterpret_cast<const float4*>(xyzt),
                       reinterpret_cast<const float4*>(eps), n, mask, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (g.F) {
        case 1:
            return tiled_f<G, 1, PAIR>(g, tm, xyzt, eps, n, mask, words, src, ls, qs, scale, d_table, overwrite, main, s);
        case 2:
            return tiled_f<G, 2, PAIR>(g, tm, xyzt, eps, n, mask, words, src, ls, qs, scale, d_table, overwrite, main, s);
        case 4:
            return tiled_f<G, 4, PAIR>(g, tm, xyzt, eps, n, mask, words, src, ls, qs, scale, d_table, overwrite, main, s);
        case 8:
            return tiled_f<G, 8, PAIR>(g, tm, xyzt, eps, n, mask, words, src, ls, qs, scale, d_table, overwrite, main, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_scatter_tiled(const DevGrid& g, const int64_t* level_rows, h4d_dtype grad_dt, const float* xyzt,
                                const float* eps, int n, const void* src, int64_t ls, int64_t qs, double scale,
                                void* d_table, void* mask_ws, hipStream_t s, bool overwrite,
                                const MainGradArg& main) {
    if (main.src && !eps) return hipErrorInvalidValue;  // the second gradient rides on the pair form only
    if (grad_dt == H4D_F64) {
        return eps ? tiled_g<double, true>(g, level_rows, xyzt, eps, n, src, ls, qs, scale, d_table, mask_ws,
                                           overwrite, main, s)
                   : tiled_g<double, false>(g, level_rows, xyzt, eps, n, src, ls, qs, scale, d_table, mask_ws,
                                            overwrite, main, s);
    }
    return eps ? tiled_g<float, true>(g, level_rows, xyzt, eps, n, src, ls, qs, scale, d_table, mask_ws, overwrite,
                                      main, s)
               : tiled_g<float, false>(g, level_rows, xyzt, eps, n, src, ls, qs, scale, d_table, mask_ws, overwrite,
                                       main, s);
}

// ------------------------------------------ static workspace (no allocation) ----
// The tile masks of hash4d_encode_backward_noalloc live in this file-scope array:
// each GPU holds its own copy from module load until the process ends, and every
// call on that GPU shares it.  On the host the array's name is only a stand-in, not
// a device address: its address on the current device is looked up once per device
// with hipGetSymbolAddress and cached, and only that address is ever passed on.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void** ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_corner_indices(const DevGrid& g, const float* xyzt, int n, int32_t* rows, float* w, hipStream_t s) {
    hipLaunchKernelGGL(k_corner_indices, level_major_grid(n, g.L), dim3(kEncodeBlock), 0, s, g,
                       reinterpret_cast<const float4*>(xyzt), n, rows, w);
    return hipGetLastError();
}

}  // namespace h4d
