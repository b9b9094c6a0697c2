// Device helpers of the 4D hash encoder: hypervoxel corners, rows, weights and
// table-row loads (DASH Section 4.2, Eqs. 8-9).  Included by the kernel sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "h4d_internal.h"

namespace h4d {

// XCD-aware placement of level-major work items (level, chunk of queries).  The
// dispatcher hands workgroups to the eight XCDs round-robin by linear id, so
// workgroup b runs on XCD b % 8.  XCD x takes the contiguous run [x per, (x+1) per)
// of the level-major item list, so its L2 serves one level's slice of the table at
// a time instead of every XCD fetching every level.  Launch kXcds * per workgroups.
constexpr int kXcds = 8;
__host__ __device__ constexpr int xcd_items_per(int items) { return (items + kXcds - 1) / kXcds; }
__device__ __forceinline__ bool xcd_item(int items, int chunks, int& level, int& chunk) {
    const int per = xcd_items_per(items);
    const int b = (int)blockIdx.x;
    const int s = b / kXcds, x = b % kXcds;
    const int item = x * per + s;
    if (s >= per || item >= items) return false;
    level = item / chunks;
    chunk = item - level * chunks;
    return true;
}

// Clamp to [0, 1], NaN to 0: the median of (x, 0, 1).  The hardware median returns
// the smaller of the other two inputs when one input is a NaN, so a NaN gives 0; the
// canonicalization first turns a signaling NaN into a quiet one.
__device__ __forceinline__ float clamp_unit(float x) {
    return __builtin_amdgcn_fmed3f(__builtin_canonicalizef(x), 0.0f, 1.0f);
}

// Rank of this lane among the lanes set in a ballot below it (lanes 0 .. lane - 1).
__device__ __forceinline__ int lane_rank(uint64_t bal) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
}

// Lower vertex and fractional offset along one dimension: pos = x * N rounded once
// in FP32, i = min(floor(pos), N - 1), frac = pos - i, which is exact in FP32.
// Contraction is off in this block: the compiler would otherwise fuse the product
// into the subtraction (frac = fma(x, N, -i)), skipping the rounding of pos that the
// floor saw, and the weights would no longer be those of the cell the indices name.
__device__ __forceinline__ void cell_1d(float x, int N, int& i, float& fr) {
#pragma clang fp contract(off)
    const float pos = x * (float)N;
    i = min((int)floorf(pos), N - 1);
    fr = pos - (float)i;
}

// Per (query, level) state: the lower vertex and fractional offsets.
struct Cell {
    int ix, iy, iz, it;
    float fx, fy, fz, ft;
};

__device__ __forceinline__ Cell level_cell(const DevGrid& g, int l, float4 x) {
    Cell c;
    const int Ns = g.res_s[l], Nt = g.res_t[l];
    cell_1d(clamp_unit(x.x), Ns, c.ix, c.fx);
    cell_1d(clamp_unit(x.y), Ns, c.iy, c.fy);
    cell_1d(clamp_unit(x.z), Ns, c.iz, c.fz);
    cell_1d(clamp_unit(x.w), Nt, c.it, c.ft);
    return c;
}

// Table rows of the 16 corners; corner k is upper along x, y, z, t iff bit 0, 1, 2, 3
// of k is set.  Dense levels: x fastest, then y, z, t.  Hashed levels: XOR of the
// 32-bit wrapped products with the primes (Eq. 8), then mod T.
__device__ __forceinline__ void level_rows(const DevGrid& g, int l, const Cell& c, uint32_t row[16]) {
    const uint32_t off = g.off[l];
    if ((g.dense_bits >> l) & 1u) {
        const uint32_t S = (uint32_t)g.res_s[l] + 1u;
        const uint32_t S2 = S * S, S3 = S2 * S;
        const uint32_t base = off + (uint32_t)c.ix + S * ((uint32_t)c.iy + S * ((uint32_t)c.iz + S * (uint32_t)c.it));
#pragma unroll
        for (int k = 0; k < 16; ++k)
            row[k] = base + (k & 1) + ((k >> 1) & 1) * S + ((k >> 2) & 1) * S2 + ((k >> 3) & 1) * S3;
    } else {
        const uint32_t hx0 = (uint32_t)c.ix * g.prime[0], hx1 = hx0 + g.prime[0];
        const uint32_t hy0 = (uint32_t)c.iy * g.prime[1], hy1 = hy0 + g.prime[1];
        const uint32_t hz0 = (uint32_t)c.iz * g.prime[2], hz1 = hz0 + g.prime[2];
        const uint32_t ht0 = (uint32_t)c.it * g.prime[3], ht1 = ht0 + g.prime[3];
        if (g.tmask) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint32_t h = ((k & 1) ? hx1 : hx0) ^ ((k & 2) ? hy1 : hy0) ^ ((k & 4) ? hz1 : hz0) ^
                                   ((k & 8) ? ht1 : ht0);
                row[k] = off + (h & g.tmask);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint32_t h = ((k & 1) ? hx1 : hx0) ^ ((k & 2) ? hy1 : hy0) ^ ((k & 4) ? hz1 : hz0) ^
                                   ((k & 8) ? ht1 : ht0);
                row[k] = off + (h % g.T);
            }
        }
    }
}

// Quadrilinear weights of the 16 corners in precision W.
template <typename W>
__device__ __forceinline__ void level_weights(const Cell& c, W w[16]) {
    const W wx[2] = {W(1) - W(c.fx), W(c.fx)};
    const W wy[2] = {W(1) - W(c.fy), W(c.fy)};
    const W wz[2] = {W(1) - W(c.fz), W(c.fz)};
    const W wt[2] = {W(1) - W(c.ft), W(c.ft)};
#pragma unroll
    for (int k = 0; k < 16; ++k) w[k] = ((wx[k & 1] * wy[(k >> 1) & 1]) * wz[(k >> 2) & 1]) * wt[k >> 3];
}

// ---- table element types ----
struct bf16_t {
    uint16_t bits;
};

__device__ __forceinline__ float bf16_to_f32(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

// Round-to-nearest-even FP32 -> BF16 bit pattern (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Load the F features of one row as type A.
template <typename TT, int F, typename A>
struct RowLoad;

template <int F, typename A>
struct RowLoad<float, F, A> {
    __device__ __forceinline__ static void load(const float* __restrict__ t, uint32_t row, A (&v)[F]) {
        const float* p = t + (size_t)row * F;
        if constexpr (F == 1) {
            v[0] = (A)p[0];
        } else if constexpr (F == 2) {
            const float2 a = *reinterpret_cast<const float2*>(p);
            v[0] = (A)a.x; v[1] = (A)a.y;
        } else {
#pragma unroll
            for (int j = 0; j < F; j += 4) {
                const float4 a = *reinterpret_cast<const float4*>(p + j);
                v[j] = (A)a.x; v[j + 1] = (A)a.y; v[j + 2] = (A)a.z; v[j + 3] = (A)a.w;
            }
        }
    }
};

template <int F, typename A>
struct RowLoad<bf16_t, F, A> {
    __device__ __forceinline__ static void load(const bf16_t* __restrict__ t, uint32_t row, A (&v)[F]) {
        const uint16_t* p = reinterpret_cast<const uint16_t*>(t) + (size_t)row * F;
        if constexpr (F == 1) {
            v[0] = (A)bf16_to_f32(p[0]);
        } else if constexpr (F == 2) {
            const uint32_t a = *reinterpret_cast<const uint32_t*>(p);
            v[0] = (A)__uint_as_float(a << 16); v[1] = (A)__uint_as_float(a & 0xffff0000u);
        } else if constexpr (F == 4) {
            const uint2 a = *reinterpret_cast<const uint2*>(p);
            v[0] = (A)__uint_as_float(a.x << 16); v[1] = (A)__uint_as_float(a.x & 0xffff0000u);
            v[2] = (A)__uint_as_float(a.y << 16); v[3] = (A)__uint_as_float(a.y & 0xffff0000u);
        } else {
            const uint4 a = *reinterpret_cast<const uint4*>(p);
            const uint32_t u[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[2 * j] = (A)__uint_as_float(u[j] << 16);
                v[2 * j + 1] = (A)__uint_as_float(u[j] & 0xffff0000u);
            }
        }
    }
};

template <int F, typename A>
struct RowLoad<double, F, A> {
    __device__ __forceinline__ static void load(const double* __restrict__ t, uint32_t row, A (&v)[F]) {
        const double* p = t + (size_t)row * F;
#pragma unroll
        for (int j = 0; j < F; ++j) v[j] = (A)p[j];
    }
};

// Two consecutive rows (r, r + 1), r even, in one aligned load (F = 2 FP32 rows:
// 16 bytes; F = 2 BF16 rows: 8 bytes).  lo receives row r, hi row r + 1.
template <typename TT, typename A>
struct RowPairLoad;

template <typename A>
struct RowPairLoad<float, A> {
    __device__ __forceinline__ static void load(const float* __restrict__ t, uint32_t r, A (&lo)[2], A (&hi)[2]) {
        const float4 a = *reinterpret_cast<const float4*>(t + (size_t)r * 2);
        lo[0] = (A)a.x; lo[1] = (A)a.y; hi[0] = (A)a.z; hi[1] = (A)a.w;
    }
};

template <typename A>
struct RowPairLoad<bf16_t, A> {
    __device__ __forceinline__ static void load(const bf16_t* __restrict__ t, uint32_t r, A (&lo)[2], A (&hi)[2]) {
        const uint2 a = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(t) + (size_t)r * 2);
        lo[0] = (A)__uint_as_float(a.x << 16); lo[1] = (A)__uint_as_float(a.x & 0xffff0000u);
        hi[0] = (A)__uint_as_float(a.y << 16); hi[1] = (A)__uint_as_float(a.y & 0xffff0000u);
    }
};

// Compute type of each table type: FP32 for F32/BF16 tables, FP64 for FP64 tables.
template <typename TT> struct AccOf { using type = float; };
template <> struct AccOf<double> { using type = double; };

// The 16 corner rows of one cell into v.  PAIRS (F = 2 FP32 / BF16 tables aligned to
// two rows): the two corners of an x-pair (same y, z, t) sit in rows r0 and r0 ^ 1
// whenever their hashes differ only in bit 0 (pi_1 = 1 and an even lower x index;
// r1 = r0 + 1 on dense levels with r0 even), and one aligned load of the row pair
// then serves both corners.
template <typename TT, int F, bool PAIRS, typename A>
__device__ __forceinline__ void gather_corners(const DevGrid& g, const TT* __restrict__ table,
                                               const uint32_t (&row)[16], A (&v)[16][F]) {
    if constexpr (PAIRS) {
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const uint32_t r0 = row[2 * p], r1 = row[2 * p + 1];
            const uint32_t a = r0 & ~1u;
            if (a + 1u < g.rows) {
                A lo[2], hi[2];
                RowPairLoad<TT, A>::load(table, a, lo, hi);
                const bool odd = r0 & 1u;
#pragma unroll
                for (int f = 0; f < 2; ++f) v[2 * p][f] = odd ? hi[f] : lo[f];
                if (r1 == (r0 ^ 1u)) {
#pragma unroll
                    for (int f = 0; f < 2; ++f) v[2 * p + 1][f] = odd ? lo[f] : hi[f];
                } else {
                    RowLoad<TT, F, A>::load(table, r1, v[2 * p + 1]);
                }
            } else {
                RowLoad<TT, F, A>::load(table, r0, v[2 * p]);
                RowLoad<TT, F, A>::load(table, r1, v[2 * p + 1]);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) RowLoad<TT, F, A>::load(table, row[k], v[k]);
    }
}


__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }

// Add v to an FP32 word of LDS.  gfx950 runs ds_add_f32 at about one active lane
// per three clocks per CU, while its integer LDS atomics run near full rate, so the
// add is a compare-and-swap on the bit pattern: read, add in FP32, swap in if the
// word is unchanged, else try again from the value the swap returned.  A lane still
// failing after kCasTries swaps (heavy contention: many queries in one cell, as when
// every query has the same timestamp) falls back to ds_add_f32, whose hardware
// serialises same-word adds, instead of going round once per contending lane.  Each
// add rounds once either way; the order of the adds is unspecified, as with any
// atomic.
constexpr int kCasTries = 3;

__device__ __forceinline__ void lds_add(float* p, float v) {
    unsigned int* u = reinterpret_cast<unsigned int*>(p);
    // A plain load: a stale value only costs one more swap (a volatile load would
    // become a flat access that waits for every outstanding global load).
    unsigned int seen = *u;
    for (int k = 0; k < kCasTries; ++k) {
        const unsigned int prev = atomicCAS(u, seen, __float_as_uint(__uint_as_float(seen) + v));
        if (prev == seen) return;
        seen = prev;
    }
    atomicAdd(p, v);
}
__device__ __forceinline__ void lds_add(double* p, double v) { atomicAdd(p, v); }

__device__ __forceinline__ unsigned long long add_pair_bits(unsigned long long seen, float v0, float v1) {
    return (unsigned long long)__float_as_uint(__uint_as_float((unsigned int)seen) + v0) |
           ((unsigned long long)__float_as_uint(__uint_as_float((unsigned int)(seen >> 32)) + v1) << 32);
}

// Further swaps after a failed first one, then the ds_add_f32 fallback (lds_add).
__device__ __forceinline__ void lds_add2_retry(float* p, float v0, float v1, unsigned long long seen) {
    unsigned long long* u = reinterpret_cast<unsigned long long*>(p);
    for (int k = 1; k < kCasTries; ++k) {
        const unsigned long long prev = atomicCAS(u, seen, add_pair_bits(seen, v0, v1));
        if (prev == seen) return;
        seen = prev;
    }
    atomicAdd(p, v0);
    atomicAdd(p + 1, v1);
}

// Add (v0, v1) to two adjacent FP32 words of LDS (8-byte aligned) with 64-bit
// compare-and-swaps, as lds_add does for one word.
__device__ __forceinline__ void lds_add2(float* p, float v0, float v1) {
    unsigned long long* u = reinterpret_cast<unsigned long long*>(p);
    const unsigned long long seen = *u;
    const unsigned long long prev = atomicCAS(u, seen, add_pair_bits(seen, v0, v1));
    if (prev != seen) lds_add2_retry(p, v0, v1, prev);
}

// Add (a0, a1) at p and (b0, b1) at q (8-byte aligned FP32 pairs in LDS, p != q) as
// lds_add2 does, with both reads and both first swaps in flight together.
__device__ __forceinline__ void lds_add2_two(float* p, float a0, float a1, float* q, float b0, float b1) {
    unsigned long long* u = reinterpret_cast<unsigned long long*>(p);
    unsigned long long* v = reinterpret_cast<unsigned long long*>(q);
    const unsigned long long su = *u, sv = *v;
    const unsigned long long ru = atomicCAS(u, su, add_pair_bits(su, a0, a1));
    const unsigned long long rv = atomicCAS(v, sv, add_pair_bits(sv, b0, b1));
    if (ru != su) lds_add2_retry(p, a0, a1, ru);
    if (rv != sv) lds_add2_retry(q, b0, b1, rv);
}

// Add F values to one tile row.
template <typename G, int F>
__device__ __forceinline__ void lds_add_row(G* p, const G (&v)[F], G w) {
    if constexpr (sizeof(G) == 4 && F % 2 == 0) {
#pragma unroll
        for (int f = 0; f < F; f += 2) lds_add2(p + f, w * v[f], w * v[f + 1]);
    } else {
#pragma unroll
        for (int f = 0; f < F; ++f) lds_add(p + f, w * v[f]);
    }
}

// Add w_c gv at the corners of x that fall in table rows [base, base + cnt) to an
// LDS tile (row r at tile[(r - base) F]).  The corners are taken in x-pairs (2p,
// 2p + 1: same y, z, t), which share a tile on hashed levels because pi_1 = 1
// keeps them within a few rows.  Each lane walks only its own pairs with a corner
// in the tile (a bit mask), rebuilding their rows and weights from the per-axis
// terms, so a wavefront issues LDS adds for as many pairs as its busiest lane has
// in the tile (typically one on a hashed level) instead of all sixteen corners.
template <typename G, int F>
__device__ __forceinline__ void tile_contrib(const DevGrid& g, const TileMap& tm, int l, float4 x,
                                             const G (&gv)[F], uint32_t base, uint32_t cnt, G* tile) {
    const Cell c = level_cell(g, l, x);
    const bool cotiled = (tm.pair_cotiled >> l) & 1u;
    uint32_t pm = 0;
    if (cotiled) {
        // both corners of a pair share the tile: test the lower-x corner only
        const uint32_t hx = (uint32_t)c.ix;  // pi_1 = 1
        const uint32_t hy0 = (uint32_t)c.iy * g.prime[1], hy1 = hy0 + g.prime[1];
        const uint32_t hz0 = (uint32_t)c.iz * g.prime[2], hz1 = hz0 + g.prime[2];
        const uint32_t ht0 = (uint32_t)c.it * g.prime[3], ht1 = ht0 + g.prime[3];
        const uint32_t rel = base - g.off[l];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const uint32_t h = hx ^ ((p & 1) ? hy1 : hy0) ^ ((p & 2) ? hz1 : hz0) ^ ((p & 4) ? ht1 : ht0);
            pm |= (uint32_t)(((h & g.tmask) - rel) < cnt) << p;
        }
    } else {
        uint32_t row[16];
        level_rows(g, l, c, row);
#pragma unroll
        for (int p = 0; p < 8; ++p)
            pm |= (uint32_t)(((row[2 * p] - base) < cnt) | ((row[2 * p + 1] - base) < cnt)) << p;
    }
    if (pm == 0u) return;
    const G wx[2] = {G(1) - G(c.fx), G(c.fx)};
    const G wy[2] = {G(1) - G(c.fy), G(c.fy)};
    const G wz[2] = {G(1) - G(c.fz), G(c.fz)};
    const G wt[2] = {G(1) - G(c.ft), G(c.ft)};
    // Per-axis terms of the lower corner; a corner adds the axis step where its bit
    // is set.  Dense rows are their sum, hashed rows their XOR (Eq. 8).
    const bool dense = (g.dense_bits >> l) & 1u;
    const uint32_t S = (uint32_t)g.res_s[l] + 1u;
    const uint32_t px = dense ? 1u : g.prime[0], py = dense ? S : g.prime[1];
    const uint32_t pz = dense ? S * S : g.prime[2], pt = dense ? S * S * S : g.prime[3];
    const uint32_t ax = (uint32_t)c.ix * px, ay = (uint32_t)c.iy * py, az = (uint32_t)c.iz * pz,
                   at = (uint32_t)c.it * pt;
    const uint32_t off = g.off[l];
    while (pm) {
        const int p = __builtin_ctz(pm);
        pm &= pm - 1u;
        const uint32_t hy = ay + ((p & 1) ? py : 0u), hz = az + ((p & 2) ? pz : 0u), ht = at + ((p & 4) ? pt : 0u);
        uint32_t r0, r1;
        if (dense) {
            r0 = off + ax + hy + hz + ht;
            r1 = r0 + 1u;
        } else {
            const uint32_t H = hy ^ hz ^ ht, h0 = ax ^ H, h1 = (ax + px) ^ H;
            if (g.tmask) {
                r0 = off + (h0 & g.tmask);
                r1 = off + (h1 & g.tmask);
            } else {
                r0 = off + h0 % g.T;
                r1 = off + h1 % g.T;
            }
        }
        r0 -= base;
        r1 -= base;
        const G vy = wy[p & 1], vz = wz[(p >> 1) & 1], vt = wt[p >> 2];
        if (cotiled || r0 < cnt) lds_add_row<G, F>(tile + r0 * F, gv, ((wx[0] * vy) * vz) * vt);
        if (cotiled || r1 < cnt) lds_add_row<G, F>(tile + r1 * F, gv, ((wx[1] * vy) * vz) * vt);
    }
}

// Bit of the tile holding level-relative row rel_row.
__device__ __forceinline__ uint32_t tile_bit(const TileMap& tm, int l, uint32_t rel_row) {
    return 1u << ((rel_row >> tm.tile_shift[l]) >> tm.bit_shift[l]);
}

__device__ __forceinline__ uint32_t corner_tile_mask(const DevGrid& g, const TileMap& tm, int l, float4 x) {
    const Cell c = level_cell(g, l, x);
    uint32_t m = 0;
    if ((tm.pair_cotiled >> l) & 1u) {  // the lower-x corner of each pair decides
        const uint32_t hx = (uint32_t)c.ix;
        const uint32_t hy0 = (uint32_t)c.iy * g.prime[1], hy1 = hy0 + g.prime[1];
        const uint32_t hz0 = (uint32_t)c.iz * g.prime[2], hz1 = hz0 + g.prime[2];
        const uint32_t ht0 = (uint32_t)c.it * g.prime[3], ht1 = ht0 + g.prime[3];
#pragma unroll
        for (int p = 0; p < 8; ++p)
            m |= tile_bit(tm, l, (hx ^ ((p & 1) ? hy1 : hy0) ^ ((p & 2) ? hz1 : hz0) ^ ((p & 4) ? ht1 : ht0)) & g.tmask);
        return m;
    }
    uint32_t row[16];
    level_rows(g, l, c, row);
#pragma unroll
    for (int k = 0; k < 16; ++k) m |= tile_bit(tm, l, row[k] - g.off[l]);
    return m;
}

// ---- per-pair tile bytes (levels whose x-pairs share a tile, tm.pair_words) ----
// On such a level the tile of pair p = (dy, dz, dt) (bits 0, 1, 2 of p) depends only
// on the y, z and t terms of Eq. 8: the x term is below the tile's row bits.  The
// mask pass stores each pair's tile index (at most 255) in byte p of a 64-bit word
// (pairs 0-3 in .x, 4-7 in .y), so that a tile workgroup finds a query's pairs in
// its tile without hashing them again.
__device__ __forceinline__ uint2 pair_tile_bytes(const DevGrid& g, const TileMap& tm, int l, const Cell& c) {
    const uint32_t hy0 = (uint32_t)c.iy * g.prime[1], hy1 = hy0 + g.prime[1];
    const uint32_t hz0 = (uint32_t)c.iz * g.prime[2], hz1 = hz0 + g.prime[2];
    const uint32_t ht0 = (uint32_t)c.it * g.prime[3], ht1 = ht0 + g.prime[3];
    const uint32_t sh = (uint32_t)tm.tile_shift[l];
    uint32_t b[8];
#pragma unroll
    for (int p = 0; p < 8; ++p)
        b[p] = ((((p & 1) ? hy1 : hy0) ^ ((p & 2) ? hz1 : hz0) ^ ((p & 4) ? ht1 : ht0)) & g.tmask) >> sh;
    return make_uint2(b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24), b[4] | (b[5] << 8) | (b[6] << 16) | (b[7] << 24));
}

// Bit p set iff byte p of wd equals tau (tau < 256): the query's pairs in tile tau.
__device__ __forceinline__ uint32_t pair_hits(uint2 wd, uint32_t tau) {
    const uint32_t rep = tau * 0x01010101u;
    const uint32_t lo = wd.x ^ rep, hi = wd.y ^ rep;
    // exact zero-byte test: bit 7 of a byte ends up set iff the byte is zero
    const uint32_t zl = ~(((lo & 0x7f7f7f7fu) + 0x7f7f7f7fu) | lo) & 0x80808080u;
    const uint32_t zh = ~(((hi & 0x7f7f7f7fu) + 0x7f7f7f7fu) | hi) & 0x80808080u;
    // gather bits 7, 15, 23, 31 into bits 24..27 (the partial products cannot carry there)
    return (((zl >> 7) * 0x01020408u) >> 24) | ((((zh >> 7) * 0x01020408u) >> 24) << 4);
}

// Add w_c gv at both corners of x-pair p of x (same y, z, t; lower and upper x) on a
// level whose pairs share a tile; rmask = tile rows - 1 (tiles are aligned powers of
// two, so a row's place in its tile is its low bits).
template <typename G, int F>
__device__ __forceinline__ void pair_contrib(const DevGrid& g, int l, float4 x, int p, const G (&gv)[F], uint32_t rmask,
                                             G* tile) {
    const Cell c = level_cell(g, l, x);
    const uint32_t dy = (uint32_t)p & 1u, dz = ((uint32_t)p >> 1) & 1u, dt = ((uint32_t)p >> 2) & 1u;
    const uint32_t H = (((uint32_t)c.iy + dy) * g.prime[1]) ^ (((uint32_t)c.iz + dz) * g.prime[2]) ^
                       (((uint32_t)c.it + dt) * g.prime[3]);
    const uint32_t r0 = ((uint32_t)c.ix ^ H) & rmask;  // pi_1 = 1
    const uint32_t r1 = (((uint32_t)c.ix + 1u) ^ H) & rmask;
    const G wy = dy ? G(c.fy) : G(1) - G(c.fy);
    const G wz = dz ? G(c.fz) : G(1) - G(c.fz);
    const G wt = dt ? G(c.ft) : G(1) - G(c.ft);
    const G w = (wy * wz) * wt;
    const G w0 = (G(1) - G(c.fx)) * w, w1 = G(c.fx) * w;
    if constexpr (sizeof(G) == 4 && F == 2) {
        lds_add2_two(tile + r0 * 2, w0 * gv[0], w0 * gv[1], tile + r1 * 2, w1 * gv[0], w1 * gv[1]);
    } else {
        lds_add_row<G, F>(tile + r0 * F, gv, w0);
        lds_add_row<G, F>(tile + r1 * F, gv, w1);
    }
}

// Orders one wavefront's LDS queue writes before its reads by other lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Run run(load(q)) for every q < n whose tile mask lmask[q] has `bit` set.
// lmask is 16-byte aligned and readable up to mask_stride(n) entries.  Each
// wavefront scans its own interleaved slice of the masks, four per lane per step
// with one 16-byte load (the next step's already in flight), and compacts the hits
// into a private LDS queue of 128 entries.  Full 64-lane batches are software
// pipelined: the loads of a batch (load) are issued before the previous batch is
// processed (run), so their latency hides behind its LDS work.  No workgroup-wide
// barrier is involved, so the wavefronts of a workgroup overlap freely.
template <int BLOCK, typename Load, typename Run>
__device__ __forceinline__ void masked_queue_loop(int n, const uint32_t* __restrict__ lmask, uint32_t bit,
                                                  int* wqueue, Load load, Run run) {
    static_assert(BLOCK % 64 == 0, "whole wavefronts");
    using S = decltype(load(0));
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int* queue = wqueue + wave * 128;
    const uint4* __restrict__ m4 = reinterpret_cast<const uint4*>(lmask);
    const int groups = (n + 3) >> 2;
    const uint64_t below = (1ull << lane) - 1ull;
    int qn = 0;
    bool have = false;  // a loaded batch waits in `pend` (wave-uniform)
    S pend{};
    int gi = wave * 64 + lane;
    uint4 cur = gi < groups ? m4[gi] : make_uint4(0u, 0u, 0u, 0u);
    for (int g0 = wave * 64; g0 < groups; g0 += BLOCK) {
        const int gn = gi + BLOCK;
        const uint4 nxt = gn < groups ? m4[gn] : make_uint4(0u, 0u, 0u, 0u);
        const uint32_t mm[4] = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = 4 * gi + j;
            const bool hit = (mm[j] & bit) != 0u && q < n;
            const uint64_t bal = __ballot(hit);
            if (hit) queue[qn + __popcll(bal & below)] = q;
            qn += (int)__popcll(bal);
            wave_sync();
            if (qn >= 64) {
                const S fresh = load(queue[lane]);
                const int rest = qn - 64;
                const int moved = lane < rest ? queue[64 + lane] : 0;
                wave_sync();
                if (lane < rest) queue[lane] = moved;
                wave_sync();
                qn = rest;
                if (have) run(pend);
                pend = fresh;
                have = true;
            }
        }
        gi = gn;
        cur = nxt;
    }
    const bool tail = lane < qn;
    S last{};
    if (tail) last = load(queue[lane]);
    if (have) run(pend);
    if (tail) run(last);
}

// As masked_queue_loop, but run(s, active) is always called by the whole wavefront
// (active is false for the lanes of a partial last batch), so that run may use
// wavefront-wide operations.  Each step loads kScanLoads 16-byte groups of masks per
// lane (1024 queries per wavefront) with their loads issued together, so a step waits
// for its masks once; the batch loads issued while scanning are then waited for only
// by the run of that batch, one batch later.
constexpr int kScanLoads = 4;
template <int BLOCK, typename Load, typename Run>
__device__ __forceinline__ void masked_queue_loop_wave(int n, const uint32_t* __restrict__ lmask, uint32_t bit,
                                                       int* wqueue, Load load, Run run) {
    static_assert(BLOCK % 64 == 0, "whole wavefronts");
    using S = decltype(load(0));
    constexpr int kWaves = BLOCK / 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int* queue = wqueue + wave * 128;
    const uint4* __restrict__ m4 = reinterpret_cast<const uint4*>(lmask);
    const int groups = (n + 3) >> 2;
    int qn = 0;
    bool have = false;  // a loaded batch waits in `pend` (wave-uniform)
    S pend{};
    for (int g0 = wave * 64 * kScanLoads; g0 < groups; g0 += kWaves * 64 * kScanLoads) {
        uint4 m[kScanLoads];
#pragma unroll
        for (int k = 0; k < kScanLoads; ++k) {
            const int gi = g0 + k * 64 + lane;
            m[k] = gi < groups ? m4[gi] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int k = 0; k < kScanLoads; ++k) {
            const uint32_t mm[4] = {m[k].x, m[k].y, m[k].z, m[k].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int q = 4 * (g0 + k * 64 + lane) + j;
                const bool hit = (mm[j] & bit) != 0u && q < n;
                const uint64_t bal = __ballot(hit);
                if (hit) queue[qn + lane_rank(bal)] = q;
                qn += (int)__popcll(bal);
                wave_sync();
                if (qn >= 64) {
                    const S fresh = load(queue[lane]);
                    const int rest = qn - 64;
                    const int moved = lane < rest ? queue[64 + lane] : 0;
                    wave_sync();
                    if (lane < rest) queue[lane] = moved;
                    wave_sync();
                    qn = rest;
                    if (have) run(pend, true);
                    pend = fresh;
                    have = true;
                }
            }
        }
    }
    const bool tail = lane < qn;
    S last{};
    if (tail) last = load(queue[lane]);
    if (have) run(pend, true);
    if (qn > 0) run(last, tail);
}

}  // namespace h4d
