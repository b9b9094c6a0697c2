// 4D hash encoder forward and backward kernels (DASH Section 4.2, Eqs. 8-9).
//
// Forward: one thread per (query, level).  Work items (level, 256 queries) are
// placed on XCDs level by level (xcd_item), so each XCD's L2 holds mostly one
// level's slice of the table (4 MiB FP32 / 2 MiB BF16 for a 2^19-row, F = 2 level)
// instead of every XCD streaming the whole table through its L2.
#include <string.h>

#include <algorithm>
#include <cmath>
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

// Load balance of the dense levels.  A dense level's tiles hold fixed runs of
// vertices, so when the queries crowd into a few cells (every query at one timestamp,
// a clustered cloud) a few of its tiles receive most of the level's updates and the
// scatter waits for them.  The mask pass therefore also counts, per dense level, the
// queries that touch each tile bit in each chunk of kMaskChunk queries; a one-workgroup
// plan (k_tile_plan) splits a heavy tile's queries into up to kMaxSplits ranges, each
// worked by its own workgroup on its own copy of the tile in LDS and written to the
// workspace as a partial tile; a last kernel (k_tile_combine) adds each split tile's
// partials in range order and writes its rows.  Hashed levels spread their rows by the
// hash and are not split.
constexpr int kMaskChunk = 1024;            // queries per counting workgroup of the mask pass
constexpr int kMaxSplits = 16;
constexpr int kPlanTiles = 4096;            // tiles the plan may split (the first ones)
constexpr int kMaxExtraRanges = 96;         // extra workgroups for split tiles, at most

// Tile mask (and pair tile bytes) of one (query, level), and the query's position.
template <bool PAIR>
__device__ __forceinline__ uint32_t query_tile_mask(const DevGrid& g, const TileMap& tm, int l, float4 x,
                                                    const float4* __restrict__ eps, int q, int n,
                                                    uint2* __restrict__ words) {
    if (!PAIR && ((tm.pair_words >> l) & 1u)) {
        const uint2 b = pair_tile_bytes(g, tm, l, level_cell(g, l, x));
        const int bs = tm.bit_shift[l];
        uint32_t m = 0u;
#pragma unroll
        for (int k = 0; k < 32; k += 8) m |= (1u << (((b.x >> k) & 0xffu) >> bs)) | (1u << (((b.y >> k) & 0xffu) >> bs));
        words[(int64_t)l * mask_stride(n) + q] = b;
        return m;
    }
    uint32_t m = corner_tile_mask(g, tm, l, x);
    if constexpr (PAIR) {
        const float4 e = eps[q];
        const float4 xp = make_float4(__fadd_rn(x.x, e.x), __fadd_rn(x.y, e.y), __fadd_rn(x.z, e.z),
                                      __fadd_rn(x.w, e.w));
        m |= corner_tile_mask(g, tm, l, xp);
    }
    return m;
}

// Grid (ceil(n / kEncodeBlock), L).  Hashed levels: one query per thread.  Dense
// levels: the first ceil(n / kMaskChunk) workgroups take kMaskChunk queries each and
// also count, per tile bit, the queries that touch it (counts[l][32][chunk]: bit-major,
// so that the plan sums a bit's chunks with contiguous loads).
template <bool PAIR>
__global__ __launch_bounds__(kEncodeBlock) void k_tile_mask(DevGrid g, TileMap tm, const float4* __restrict__ xyzt,
                                                            const float4* __restrict__ eps, int n,
                                                            uint32_t* __restrict__ mask, uint2* __restrict__ words,
                                                            uint32_t* __restrict__ counts, int nchunks) {
    const int l = blockIdx.y;
    if (!((g.dense_bits >> l) & 1u)) {
        const int q = blockIdx.x * kEncodeBlock + threadIdx.x;
        if (q >= n) return;
        mask[(int64_t)l * mask_stride(n) + q] = query_tile_mask<PAIR>(g, tm, l, xyzt[q], eps, q, n, words);
        return;
    }
    const int chunk = blockIdx.x;
    if (chunk >= nchunks) return;  // workgroup-uniform
    __shared__ uint32_t cnt[32];
    if (threadIdx.x < 32) cnt[threadIdx.x] = 0u;
    constexpr int kPerThread = kMaskChunk / kEncodeBlock;
    float4 xs[kPerThread];  // every load in flight before the first use
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
        const int q = chunk * kMaskChunk + i * kEncodeBlock + (int)threadIdx.x;
        xs[i] = q < n ? xyzt[q] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
        const int q = chunk * kMaskChunk + i * kEncodeBlock + (int)threadIdx.x;
        if (q >= n) continue;
        uint32_t m = query_tile_mask<PAIR>(g, tm, l, xs[i], eps, q, n, words);
        mask[(int64_t)l * mask_stride(n) + q] = m;
        while (m) {  // a dense level's corners touch a few neighbouring tiles
            atomicAdd(&cnt[__builtin_ctz(m)], 1u);
            m &= m - 1u;
        }
    }
    __syncthreads();
    if (threadIdx.x < 32) counts[((int64_t)l * 32 + threadIdx.x) * nchunks + chunk] = cnt[threadIdx.x];
}

// The plan.  Entry t < tiles is tile t's first (or only) query range; entries tiles
// .. tiles + extras - 1 are the other ranges of the split tiles.  An entry holds the
// tile, its range, how many ranges the tile is split into, and the tile's first
// partial-tile slot.  info = {extras, split tiles}; split[i] = the i-th split tile.
// A dense tile's cost is its query count times kDenseCost (a dense visit adds about
// four x-pairs to the tile, a hashed visit about one).  With h the expected query
// count of a hashed tile (8 pairs over P tiles), a tile costing at most 2 h stays
// whole (more workgroups would add a round and save little); a costlier one is split
// into ceil(cost / target) ranges, at most kMaxSplits, with target = 5/4 h raised
// until the extra ranges fit in `extra`.
constexpr int kDenseCost = 3;

__global__ __launch_bounds__(1024) void k_tile_plan(DevGrid g, TileMap tm, const uint32_t* __restrict__ counts,
                                                    int nchunks, float target0, int extra, int4* __restrict__ plan,
                                                    int* __restrict__ info, int* __restrict__ split) {
    __shared__ uint32_t cost[kPlanTiles];
    __shared__ uint32_t ksum[1024];
    __shared__ uint32_t ssum[1024];
    __shared__ float target_s;
    const int tiles = tm.tile_start[g.L];
    const int cand = min(tiles, kPlanTiles);
    for (int t = threadIdx.x; t < cand; t += blockDim.x) cost[t] = 0u;
    __syncthreads();
    // queries per dense tile from the (tile bit, chunk) counts of the dense levels.
    // Item i = (the (i / 32)-th dense level, bit i % 32); wavefront w sums items w,
    // w + nwaves, ... four at a time, each lane loading chunks lane, lane + 64, ... of
    // all four before adding any (contiguous in the bit-major counts: 256 bytes per
    // load instruction; with chunk-major counts every lane's load was a line of its
    // own and this phase took 21 k cycles instead of 13 k), then a butterfly; so no
    // two lanes add into one word.
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
    const float whole = target0 * (2.f / 1.25f);
    if (threadIdx.x == 0) target_s = target0;
    const int ndense = __popc(g.dense_bits & (g.L >= 32 ? 0xffffffffu : ((1u << g.L) - 1u)));
    for (int i0 = wave * 4; i0 < ndense * 32; i0 += nwaves * 4) {
        int lv[4], bit[4];
        bool ok[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = i0 + j, dl = i / 32;
            bit[j] = i % 32;
            int l = 0, seen = -1;
            for (; l < g.L; ++l)
                if (((g.dense_bits >> l) & 1u) && ++seen == dl) break;
            lv[j] = l;
            ok[j] = i < ndense * 32 && l < g.L && tm.tile_start[l] < cand &&
                    (bit[j] << tm.bit_shift[l]) < tm.tile_start[l + 1] - tm.tile_start[l];
        }
        uint32_t sum[4] = {0u, 0u, 0u, 0u};
        for (int k0 = 0; k0 < nchunks; k0 += 4 * 64) {
            uint32_t v[4][4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int k = k0 + c * 64 + lane;
                    v[j][c] = ok[j] && k < nchunks ? counts[((int64_t)lv[j] * 32 + bit[j]) * nchunks + k] : 0u;
                }
#pragma unroll
            for (int j = 0; j < 4; ++j) sum[j] += (v[j][0] + v[j][1]) + (v[j][2] + v[j][3]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) sum[j] += __shfl_xor(sum[j], d);
            if (!ok[j]) continue;
            // every tile of the bit gets its share of the bit's count, times the dense
            // weight; a tile up to twice a hashed tile's expected work stays whole (0)
            const int l = lv[j];
            const float c = (float)(sum[j] >> tm.bit_shift[l]) * kDenseCost;
            const uint32_t cv = c <= whole ? 0u : (uint32_t)fminf(c, 4.0e9f);
            const int t0 = tm.tile_start[l] + (bit[j] << tm.bit_shift[l]);
            const int t1 = min(min(tm.tile_start[l + 1], cand), t0 + (1 << tm.bit_shift[l]));
            for (int t = t0 + lane; t < t1; t += 64) cost[t] = cv;
        }
    }
    __syncthreads();
    for (int round = 0; round < 24; ++round) {  // raise the target until the extra ranges fit
        const float target = target_s;
        uint32_t mysum = 0u;
        for (int t = threadIdx.x; t < cand; t += blockDim.x)
            mysum += min((uint32_t)kMaxSplits, max(1u, (uint32_t)ceilf((float)cost[t] / target))) - 1u;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) mysum += __shfl_xor(mysum, d);
        if (lane == 0) ksum[wave] = mysum;
        __syncthreads();
        uint32_t all = 0u;
        for (int w = 0; w < nwaves; ++w) all += ksum[w];
        const bool fits = all <= (uint32_t)extra;
        __syncthreads();
        if (fits) break;
        if (threadIdx.x == 0) target_s = target * 1.5f;
        __syncthreads();
    }
    const float target = target_s;
    // exclusive positions over the candidate tiles (four per thread): extra ranges
    // (k - 1) and split tiles (1 if split)
    constexpr int kPer = kPlanTiles / 1024;
    uint32_t kk[kPer], lext = 0u, lsplit = 0u;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int t = threadIdx.x * kPer + j;
        uint32_t k = 1u;
        if (t < cand) k = min((uint32_t)kMaxSplits, max(1u, (uint32_t)ceilf((float)cost[t] / target)));
        kk[j] = k;
        lext += k - 1u;
        lsplit += k > 1u ? 1u : 0u;
    }
    // inclusive scans within the wavefront, then the wavefront totals
    uint32_t iext = lext, isplit = lsplit;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t a = __shfl_up(iext, d), b = __shfl_up(isplit, d);
        if (lane >= d) {
            iext += a;
            isplit += b;
        }
    }
    if (lane == 63) {
        ksum[wave] = iext;
        ssum[wave] = isplit;
    }
    __syncthreads();
    uint32_t before_e = 0u, before_s = 0u, total_e = 0u, total_s = 0u;
    for (int w = 0; w < nwaves; ++w) {
        if (w < wave) {
            before_e += ksum[w];
            before_s += ssum[w];
        }
        total_e += ksum[w];
        total_s += ssum[w];
    }
    const bool fits = total_e <= (uint32_t)extra;
    uint32_t ext = before_e + iext - lext;   // extra ranges before this thread's tiles
    uint32_t sp = before_s + isplit - lsplit;  // split tiles before them
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int t = threadIdx.x * kPer + j;
        if (t >= cand) break;
        const int k = fits ? (int)kk[j] : 1;
        // a split tile's K partial slots start at (split tiles before it) + (extra
        // ranges before it): K slots per split tile, in tile order
        const int slot = (int)(sp + ext);
        plan[t] = make_int4(t, 0, k, k > 1 ? slot : -1);
        for (int r = 1; r < k; ++r) plan[tiles + (int)ext + r - 1] = make_int4(t, r, k, slot);
        if (k > 1) {
            split[sp] = t;
            ext += (uint32_t)k - 1u;
            sp += 1u;
        }
    }
    for (int t = cand + (int)threadIdx.x; t < tiles; t += blockDim.x) plan[t] = make_int4(t, 0, 1, -1);
    if (threadIdx.x == 0) {
        info[0] = fits ? (int)total_e : 0;
        info[1] = fits ? (int)total_s : 0;
    }
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

// Queries [q0, q0 + n) of the level; lmask and lwords point at query q0's entries.
template <typename G, int F>
__device__ __forceinline__ void scatter_pair_words(const DevGrid& g, const TileMap& tm, int l, uint32_t tau,
                                                   uint32_t bit, const float4* __restrict__ xyzt, int q0, int n,
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
        [&](int i) {
            WordQuery<G, F> t;
            const int q = q0 + i;
            const G* gp = gl + (int64_t)q * qstride;
#pragma unroll
            for (int f = 0; f < F; ++f) t.gv[f] = gp[f];
            t.x = xyzt[q];
            t.wd = lwords[i];
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

// *counter += the non-finite values the wavefront's lanes counted (one atomic per
// wavefront that has any).  Called by every lane of the wavefront.
__device__ __forceinline__ void add_count(int* counter, int bad) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) bad += __shfl_xor(bad, d, 64);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(counter, bad);
}

template <typename G, int F, bool PAIR>
__global__ __launch_bounds__(kScatterBlock) void k_scatter_tiled(DevGrid g, TileMap tm, const float4* __restrict__ xyzt,
                                                                const float4* __restrict__ eps, int n,
                                                                const uint32_t* __restrict__ mask,
                                                                const uint2* __restrict__ words,
                                                                const int4* __restrict__ plan,
                                                                const int* __restrict__ plan_info,
                                                                G* __restrict__ partials, int slot_elems,
                                                                const G* __restrict__ src, int64_t lstride,
                                                                int64_t qstride, G scale, G* __restrict__ d_table,
                                                                int overwrite, MainGrad<G> mg,
                                                                int* __restrict__ nonfinite) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int queue[kQueueCap];
    __shared__ int2 overflow[PAIR ? 1 : kScatterBlock / 64 * kOverflowCap];
    G* tile = reinterpret_cast<G*>(smem);
    // XCD placement: XCD x works on the contiguous run [x per, (x + 1) per) of the
    // level-ordered tiles, so its L2 holds the masks, pair bytes and gradients of two or
    // three levels instead of every XCD fetching every level's; the extra ranges of split
    // tiles go round-robin to the XCDs, since they are the heavy ones.
    const int tiles = tm.tile_start[g.L];
    const int per = xcd_items_per(tiles);
    const int x = (int)blockIdx.x % kXcds, sx = (int)blockIdx.x / kXcds;
    int six;
    if (sx < per) {
        six = x * per + sx;
        if (six >= tiles) return;
    } else {  // the extra ranges, round-robin over the XCDs
        six = (sx - per) * kXcds + x;
        if (six >= plan_info[0]) return;
        six += tiles;
    }
    const int4 pe = plan[six];
    const int tix = pe.x, range = pe.y, nranges = pe.z;
    int l = 0;
    while (l + 1 < g.L && tix >= tm.tile_start[l + 1]) ++l;
    const uint32_t t_in_level = (uint32_t)(tix - tm.tile_start[l]);
    const uint32_t first = t_in_level << tm.tile_shift[l];
    const uint32_t base = g.off[l] + first;
    const uint32_t cnt = min(1u << tm.tile_shift[l], (uint32_t)tm.level_rows[l] - first);
    const uint32_t bit = tile_bit(tm, l, first);
    // this workgroup's queries: range r of nranges, boundaries on multiples of four
    const int q0 = (int)(((int64_t)n * range / nranges) & ~(int64_t)3);
    const int q1 = range + 1 == nranges ? n : (int)(((int64_t)n * (range + 1) / nranges) & ~(int64_t)3);
    for (uint32_t i = threadIdx.x; i < cnt * F; i += kScatterBlock) tile[i] = G(0);
    __syncthreads();
    const uint32_t* lmask = mask + (int64_t)l * mask_stride(n) + q0;
    if (!PAIR && ((tm.pair_words >> l) & 1u)) {
        scatter_pair_words<G, F>(g, tm, l, t_in_level, bit, xyzt, q0, q1 - q0, lmask,
                                 words + (int64_t)l * mask_stride(n) + q0, src, lstride, qstride, scale, queue,
                                 overflow, tile);
    } else {
        masked_queue_loop<kScatterBlock>(
            q1 - q0, lmask, bit, queue,
            [&](int i) { return tile_load<G, F, PAIR>(l, xyzt, eps, src, lstride, qstride, mg, q0 + i); },
            [&](const TileQuery<G, F, PAIR>& t) { tile_run<G, F, PAIR>(g, tm, l, t, scale, mg, base, cnt, tile); });
    }
    __syncthreads();
    if (nranges > 1) {  // a split tile: k_tile_combine adds the ranges' partial tiles
        G* mine = partials + (int64_t)(pe.w + range) * slot_elems;
        for (uint32_t i = threadIdx.x; i < cnt * F; i += kScatterBlock) mine[i] = tile[i];
        return;
    }
    // the tile's rows have no other owner: add them to d_table, or with overwrite set
    // write every row (the tiles of the levels cover all E rows); count the non-finite
    // values written if asked
    G* out = d_table + (size_t)base * F;
    int bad = 0;
    if (overwrite) {
        for (uint32_t i = threadIdx.x; i < cnt * F; i += kScatterBlock) {
            const G v = tile[i];
            out[i] = v;
            bad += !__builtin_isfinite(v);
        }
    } else {
        for (uint32_t i = threadIdx.x; i < cnt * F; i += kScatterBlock) {
            const G v = tile[i];
            if (v != G(0)) {
                const G r = out[i] + v;
                out[i] = r;
                bad += !__builtin_isfinite(r);
            }
        }
    }
    if (nonfinite) add_count(nonfinite, bad);
}

// Rows of the split tiles: the sum of their ranges' partial tiles, in range order.
// Workgroup (i, part) covers part `part` of kCombineParts of the i-th split tile.
constexpr int kCombineParts = 4;
template <typename G>
__global__ __launch_bounds__(256) void k_tile_combine(DevGrid g, TileMap tm, const int4* __restrict__ plan,
                                                      const int* __restrict__ plan_info,
                                                      const int* __restrict__ split,
                                                      const G* __restrict__ partials, int slot_elems,
                                                      G* __restrict__ d_table, int overwrite,
                                                      int* __restrict__ nonfinite) {
    if ((int)blockIdx.x >= plan_info[1]) return;
    const int tix = split[blockIdx.x];
    const int4 pe = plan[tix];
    int l = 0;
    while (l + 1 < g.L && tix >= tm.tile_start[l + 1]) ++l;
    const uint32_t first = (uint32_t)(tix - tm.tile_start[l]) << tm.tile_shift[l];
    const uint32_t values = min(1u << tm.tile_shift[l], (uint32_t)tm.level_rows[l] - first) * (uint32_t)g.F;
    const uint32_t chunk = (values + kCombineParts - 1) / kCombineParts;
    const uint32_t lo = blockIdx.y * chunk, hi = min(values, lo + chunk);
    G* out = d_table + (size_t)(g.off[l] + first) * g.F;
    int bad = 0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += 256) {
        G v = partials[(int64_t)pe.w * slot_elems + i];
        for (int r = 1; r < pe.z; ++r) v += partials[(int64_t)(pe.w + r) * slot_elems + i];
        if (overwrite) {
            out[i] = v;
            bad += !__builtin_isfinite(v);
        } else if (v != G(0)) {
            const G s = out[i] + v;
            out[i] = s;
            bad += !__builtin_isfinite(s);
        }
    }
    if (nonfinite) add_count(nonfinite, bad);
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

// Workspace of the tiled scatter, each part 256-byte aligned: masks [L][stride] u32 |
// pair tile bytes [L][stride] uint2 | per-chunk tile counts [L][32][chunks] u32 | plan
// [tiles + extra] int4 | plan info (2 int) | split tiles [extra] int | partial tiles
// [2 extra][slot].  One layout serves FP32 and FP64 gradients (the larger tile count
// and tile of the two).
struct ScatterWs {
    size_t words, counts, plan, info, split, partials, total, slot_bytes;
    int chunks, extra;
};

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

static ScatterWs scatter_ws(const DevGrid& g, const int64_t* level_rows, int n) {
    ScatterWs w;
    int tiles = 0;
    w.slot_bytes = 0;
    for (int gbytes = 4; gbytes <= 8; gbytes += 4) {
        const TileMap tm = make_tile_map(g, level_rows, g.F, gbytes);
        tiles = max(tiles, tm.tile_start[g.L]);
        for (int l = 0; l < g.L; ++l) {
            const int64_t rows = min((int64_t)1 << tm.tile_shift[l], level_rows[l]);
            w.slot_bytes = max(w.slot_bytes, (size_t)rows * g.F * gbytes);
        }
    }
    w.chunks = (n + kMaskChunk - 1) / kMaskChunk;
    w.extra = min(kMaxExtraRanges, max(8, tiles / 4));
    const size_t masks = align256((size_t)mask_stride(n) * g.L * sizeof(uint32_t));
    w.words = masks;
    w.counts = w.words + align256((size_t)mask_stride(n) * g.L * sizeof(uint2));
    w.plan = w.counts + align256((size_t)g.L * w.chunks * 32 * sizeof(uint32_t));
    w.info = w.plan + align256((size_t)(tiles + w.extra) * sizeof(int4));
    w.split = w.info + 256;
    w.partials = w.split + align256((size_t)w.extra * sizeof(int));
    w.total = w.partials + (size_t)2 * w.extra * w.slot_bytes;
    return w;
}

size_t scatter_ws_bytes(const DevGrid& g, const int64_t* level_rows, int n) {
    return scatter_ws(g, level_rows, n).total;
}

struct ScatterBufs {
    uint32_t* mask;
    uint2* words;
    uint32_t* counts;
    int4* plan;
    int* info;
    int* split;
    void* partials;
    int extra;
    size_t slot_bytes;
};

template <typename G, int F, bool PAIR>
static hipError_t tiled_f(const DevGrid& g, const TileMap& tm, const float* xyzt, const float* eps, int n,
                          const ScatterBufs& b, const void* src, int64_t ls, int64_t qs, double scale, void* d_table,
                          bool overwrite, const MainGradArg& main, int32_t* nonfinite, hipStream_t s) {
    auto kern = k_scatter_tiled<G, F, PAIR>;
    const size_t lds = (size_t)tm.max_rows * F * sizeof(G);
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int rounds = xcd_items_per(tm.tile_start[g.L]) + xcd_items_per(b.extra);
    hipLaunchKernelGGL(kern, dim3((unsigned)(kXcds * rounds)), dim3(kScatterBlock), lds, s, g, tm,
                       reinterpret_cast<const float4*>(xyzt), reinterpret_cast<const float4*>(eps), n, b.mask,
                       b.words, b.plan, b.info, static_cast<G*>(b.partials),
                       (int)(b.slot_bytes / sizeof(G)), static_cast<const G*>(src), ls, qs, (G)scale,
                       static_cast<G*>(d_table), overwrite ? 1 : 0,
                       MainGrad<G>{static_cast<const G*>(main.src), main.lstride, main.qstride, (G)main.scale},
                       nonfinite);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_combine<G>, dim3((unsigned)b.extra, kCombineParts), dim3(256), 0, s, g, tm, b.plan,
                       b.info, b.split, static_cast<const G*>(b.partials),
                       (int)(b.slot_bytes / sizeof(G)), static_cast<G*>(d_table), overwrite ? 1 : 0, nonfinite);
    return hipGetLastError();
}

template <typename G, bool PAIR>
static hipError_t tiled_g(const DevGrid& g, const int64_t* level_rows, const float* xyzt, const float* eps, int n,
                          const void* src, int64_t ls, int64_t qs, double scale, void* d_table, void* mask_ws,
                          bool overwrite, const MainGradArg& main, int32_t* nonfinite, hipStream_t s) {
    const TileMap tm = make_tile_map(g, level_rows, g.F, (int)sizeof(G), !PAIR);
    const ScatterWs w = scatter_ws(g, level_rows, n);
    char* ws = static_cast<char*>(mask_ws);
    ScatterBufs b;
    b.mask = reinterpret_cast<uint32_t*>(ws);
    b.words = reinterpret_cast<uint2*>(ws + w.words);
    b.counts = reinterpret_cast<uint32_t*>(ws + w.counts);
    b.plan = reinterpret_cast<int4*>(ws + w.plan);
    b.info = reinterpret_cast<int*>(ws + w.info);
    b.split = reinterpret_cast<int*>(ws + w.split);
    b.partials = ws + w.partials;
    b.extra = w.extra;
    b.slot_bytes = w.slot_bytes;
    hipLaunchKernelGGL(k_tile_mask<PAIR>, dim3((unsigned)((n + kEncodeBlock - 1) / kEncodeBlock), (unsigned)g.L),
                       dim3(kEncodeBlock), 0, s, g, tm,
                       reinterpret_cast<const float4*>(xyzt), reinterpret_cast<const float4*>(eps), n, b.mask,
                       b.words, b.counts, w.chunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // expected queries of a hashed tile, h = n (1 - (1 - 1/P)^8), the largest over the
    // hashed levels; the plan's first target is 5/4 h
    double h = 0.0;
    for (int l = 0; l < g.L; ++l)
        if (!((g.dense_bits >> l) & 1u))
            h = std::max(h, n * (1.0 - std::pow(1.0 - 1.0 / (tm.tile_start[l + 1] - tm.tile_start[l]), 8.0)));
    hipLaunchKernelGGL(k_tile_plan, dim3(1), dim3(1024), 0, s, g, tm, b.counts, w.chunks,
                       (float)std::max(1.25 * h, 1024.0), w.extra, b.plan, b.info, b.split);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    switch (g.F) {
        case 1: return tiled_f<G, 1, PAIR>(g, tm, xyzt, eps, n, b, src, ls, qs, scale, d_table, overwrite, main, nonfinite, s);
        case 2: return tiled_f<G, 2, PAIR>(g, tm, xyzt, eps, n, b, src, ls, qs, scale, d_table, overwrite, main, nonfinite, s);
        case 4: return tiled_f<G, 4, PAIR>(g, tm, xyzt, eps, n, b, src, ls, qs, scale, d_table, overwrite, main, nonfinite, s);
        case 8: return tiled_f<G, 8, PAIR>(g, tm, xyzt, eps, n, b, src, ls, qs, scale, d_table, overwrite, main, nonfinite, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_scatter_tiled(const DevGrid& g, const int64_t* level_rows, h4d_dtype grad_dt, const float* xyzt,
                                const float* eps, int n, const void* src, int64_t ls, int64_t qs, double scale,
                                void* d_table, void* mask_ws, hipStream_t s, bool overwrite,
                                const MainGradArg& main, int32_t* nonfinite) {
    if (main.src && !eps) return hipErrorInvalidValue;  // the second gradient rides on the pair form only
    if (grad_dt == H4D_F64) {
        return eps ? tiled_g<double, true>(g, level_rows, xyzt, eps, n, src, ls, qs, scale, d_table, mask_ws,
                                           overwrite, main, nonfinite, s)
                   : tiled_g<double, false>(g, level_rows, xyzt, eps, n, src, ls, qs, scale, d_table, mask_ws,
                                            overwrite, main, nonfinite, s);
    }
    return eps ? tiled_g<float, true>(g, level_rows, xyzt, eps, n, src, ls, qs, scale, d_table, mask_ws, overwrite,
                                      main, nonfinite, s)
               : tiled_g<float, false>(g, level_rows, xyzt, eps, n, src, ls, qs, scale, d_table, mask_ws, overwrite,
                                       main, nonfinite, s);
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
