// Multi-head deformation decoder on MFMA (DASH Section 4.2: the trunk phi_d of
// Eq. 9 and the position / rotation / scale heads feeding Eq. 10), forward and
// backward.
//
// Shapes: trunk in -> 64 (ReLU) -> 64 (ReLU); heads fused into one 64 -> out layer
// (out <= 16).  Parameters are one flat array W1[64,in] b1 W2[64,64] b2 W3[out,64] b3.
//
// Formulation.  A wavefront owns a tile of 16 queries and computes every layer
// transposed, Z^T = W X^T, on 16x16 MFMA tiles: hidden (or feature, or output)
// units are the M rows and the 16 queries are the N columns.  The accumulator
// layout (lane l holds rows 4(l/16)+r, column l%16) is then directly the B
// operand of the next layer, because a contraction may take its K index in any
// order as long as A and B agree: lane group kb = l/16 contributes the rows
// hid(idx, kb) = 16(idx/4) + 4 kb + idx%4 it already holds, and the weight
// fragments are laid out in that same order.  Weight gradients contract over
// queries instead; for those the activations are transposed through a small
// per-wavefront LDS buffer.
//
// Precision policies: FP32 (v_mfma_f32_16x16x4_f32), BF16 (v_mfma_f32_16x16x32_bf16
// for the layer chain, v_mfma_f32_16x16x16_bf16 for weight gradients, FP32
// accumulation everywhere), and FP64 (the same 16x16x4 tile contraction done with
// cross-lane reads, for finite-difference gradient checks only).
#include <string.h>

#include <type_traits>

#include "h4d_device.h"

namespace h4d {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushortx8 __attribute__((ext_vector_type(8)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

constexpr int HID = H4D_HIDDEN;
constexpr int OUTP = H4D_MAX_OUT;

__device__ __forceinline__ int hid(int idx, int kb) { return 16 * (idx >> 2) + 4 * kb + (idx & 3); }

// Wait for every vector memory operation of this wavefront (s_waitcnt vmcnt(0)).
// Called before a tile loop whose first tile's inputs were loaded ahead, so that the
// compiler sees no load of the loop's entry still in flight at the loop head and does
// not make the first products of every iteration wait on that iteration's prefetch.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0f70); }

struct dacc {
    double v[4];
};

// ------------------------------------------------------------ policies ----
struct PolF32 {
    using S = float;       // parameter storage
    using V = float;       // activations / feature values
    using G = float;       // gradient accumulation
    using FE = float;      // fragment element
    using Op = float;      // operand of one MFMA per lane
    using Acc = floatx4;
    static constexpr int KC = 4, E = 1;
    __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static float get(const Acc& a, int r) { return a[r]; }
    __device__ static Op pack(const V* v) { return v[0]; }
    __device__ static Op frag(const FE* p) { return p[0]; }
    __device__ static FE to_frag(S s) { return s; }
    __device__ static float bias(S s) { return s; }
    __device__ static Acc mma(Op a, Op b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

struct PolBF16 {
    using S = uint16_t;    // BF16 bit patterns
    using V = float;
    using G = float;
    using FE = uint16_t;
    using Op = bf16x8;
    using Acc = floatx4;
    static constexpr int KC = 32, E = 8;
    __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static float get(const Acc& a, int r) { return a[r]; }
    // activations to BF16 operands with gfx950's packed conversion (round to nearest
    // even, as f32_to_bf16 does for every finite value)
    __device__ static Op pack(const V* v) {
        bf16x8 r;
#pragma unroll
        for (int e = 0; e < 8; ++e) r[e] = (__bf16)v[e];
        return r;
    }
    __device__ static Op frag(const FE* p) {
        return __builtin_bit_cast(bf16x8, *reinterpret_cast<const ushortx8*>(p));
    }
    __device__ static FE to_frag(S s) { return s; }
    __device__ static float bias(S s) { return bf16_to_f32(s); }
    __device__ static Acc mma(Op a, Op b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

struct PolF64 {
    using S = double;
    using V = double;
    using G = double;
    using FE = double;
    using Op = double;
    using Acc = dacc;
    static constexpr int KC = 4, E = 1;
    __device__ static Acc zero() { return Acc{{0.0, 0.0, 0.0, 0.0}}; }
    __device__ static double get(const Acc& a, int r) { return a.v[r]; }
    __device__ static Op pack(const V* v) { return v[0]; }
    __device__ static Op frag(const FE* p) { return p[0]; }
    __device__ static FE to_frag(S s) { return s; }
    __device__ static double bias(S s) { return s; }
    // D[i][j] += sum_k A[i][k] B[k][j] with the 16x16x4 operand layout: lane (i, k)
    // holds A[i][k], lane (j, k) holds B[k][j]; lane (j, kb) owns rows 4 kb + r.
    __device__ static Acc mma(Op a, Op b, Acc c) {
        const int lane = threadIdx.x & 63, j = lane & 15, kb = lane >> 4;
        double bk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) bk[k] = __shfl(b, j + 16 * k, 64);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * kb + r;
#pragma unroll
            for (int k = 0; k < 4; ++k) c.v[r] += __shfl(a, i + 16 * k, 64) * bk[k];
        }
        return c;
    }
};

// ------------------------------------------------------------- shapes ----
template <class Pol, int IN>
struct Shape {
    static constexpr int KC = Pol::KC, E = Pol::E;
    static constexpr int KIN = ((IN + KC - 1) / KC) * KC;  // input K padded to the chunk
    static constexpr int NC1 = KIN / KC;                    // chunks of layer 1
    static constexpr int NI = KIN / 4;                      // input features held per lane
    static constexpr int NCH = HID / KC;                    // chunks over the hidden width
    static constexpr int KO = ((OUTP + KC - 1) / KC) * KC;  // output K padded to the chunk
    static constexpr int NCO = KO / KC;
    static constexpr int NO = KO / 4;                       // upstream gradients held per lane
    static constexpr int MF = (IN + 15) / 16;               // 16-row tiles of d_feat
};

// Parameter offsets in the flat array.
struct ParamOff {
    int W1, b1, W2, b2, W3, b3, P;
    __device__ __host__ ParamOff(int in, int out) {
        W1 = 0;
        b1 = W1 + HID * in;
        W2 = b1 + HID;
        b2 = W2 + HID * HID;
        W3 = b2 + HID;
        b3 = W3 + out * HID;
        P = b3 + out;
    }
};

// Fragment tables, one per matrix operand of the layer chain: A1, A2, A3 (forward:
// W1, W2, W3) and B3, B2, B1 (backward: W3^T, W2^T, W1^T).  Matrix m has tiles(m)
// 16-row tiles and nc(m) K chunks of E elements per lane.  A table is cut into units
// of grp(m) consecutive chunks of one tile; inside a unit lane l's grp(m) E elements
// lie together, so that one LDS read (16 bytes for FP32, whose units hold four
// chunks, and for BF16) fetches the operands of grp(m) products.
enum { kA1 = 0, kA2, kA3, kB3, kB2, kB1, kMats };

template <class Pol, int IN>
struct Tab {
    using Sh = Shape<Pol, IN>;
    static constexpr int E = Pol::E;
    __host__ __device__ static constexpr int nc(int m) { return m == kA1 ? Sh::NC1 : m == kB3 ? Sh::NCO : Sh::NCH; }
    __host__ __device__ static constexpr int tiles(int m) { return m == kA3 ? 1 : m == kB1 ? Sh::MF : 4; }
    __host__ __device__ static constexpr int grp(int m) {
        return E > 1 ? 1 : nc(m) % 4 == 0 ? 4 : nc(m) % 2 == 0 ? 2 : 1;
    }
    __host__ __device__ static constexpr int size(int m) { return tiles(m) * nc(m) * 64 * E; }
    __host__ __device__ static constexpr int off(int m) { return m == 0 ? 0 : off(m - 1) + size(m - 1); }
    // table position of element e of chunk c of tile mt, lane `lane`
    __host__ __device__ static constexpr int at(int m, int mt, int c, int lane, int e) {
        return off(m) + ((mt * (nc(m) / grp(m)) + c / grp(m)) * 64 + lane) * grp(m) * E + (c % grp(m)) * E + e;
    }
    static constexpr int FWD = off(kB3);   // forward tables: A1 A2 A3
    static constexpr int ALL = off(kMats);
};

// Flat parameter index of element e of chunk c of tile mt of matrix m for lane
// (i, kb) (-1 = zero padding).
template <class Pol, int IN>
__device__ __forceinline__ int frag_param(int m, int mt, int c, int lane, int e, int out, const ParamOff& po) {
    using Sh = Shape<Pol, IN>;
    constexpr int E = Sh::E;
    const int i = lane & 15, kb = lane >> 4;
    switch (m) {
        case kA1: {  // W1[16 mt + i][kb NI + c E + e]
            const int k = kb * Sh::NI + c * E + e;
            return k < IN ? po.W1 + (16 * mt + i) * IN + k : -1;
        }
        case kA2:  // W2[16 mt + i][hid(c E + e, kb)]
            return po.W2 + (16 * mt + i) * HID + hid(c * E + e, kb);
        case kA3:  // W3[i][hid(c E + e, kb)]
            return i < out ? po.W3 + i * HID + hid(c * E + e, kb) : -1;
        case kB3: {  // W3^T: W3[kb NO + c E + e][16 mt + i]
            const int o = kb * Sh::NO + c * E + e;
            return o < out ? po.W3 + o * HID + 16 * mt + i : -1;
        }
        case kB2:  // W2^T: W2[hid(c E + e, kb)][16 mt + i]
            return po.W2 + hid(c * E + e, kb) * HID + 16 * mt + i;
        default: {  // W1^T: W1[hid(c E + e, kb)][16 mt + i]
            const int f = 16 * mt + i;
            return f < IN ? po.W1 + hid(c * E + e, kb) * IN + f : -1;
        }
    }
}

// Fragment operands: from the LDS tables for FP32 / BF16; straight from the
// parameter array for FP64 (its tables would not fit next to its other buffers).
template <class Pol, int IN, bool LDS>
struct Frags {
    using FE = typename Pol::FE;
    using TB = Tab<Pol, IN>;
    const FE* lds;                         // LDS tables (LDS == true)
    const typename Pol::S* params;         // global parameters (LDS == false)
    int out;
    ParamOff po;

    __device__ typename Pol::Op get(int m, int mt, int c) const {
        const int lane = threadIdx.x & 63;
        if constexpr (LDS) {
            return Pol::frag(lds + TB::at(m, mt, c, lane, 0));
        } else {
            FE v[Pol::E];
#pragma unroll
            for (int e = 0; e < Pol::E; ++e) {
                const int s = frag_param<Pol, IN>(m, mt, c, lane, e, out, po);
                v[e] = s >= 0 ? Pol::to_frag(params[s]) : FE(0);
            }
            return Pol::frag(v);
        }
    }
};

// Builds the LDS table of matrix M: wavefront-strided over its units, each lane
// gathering its grp E (L2-resident) parameters and storing them together.
template <class Pol, int IN, int M, int NW>
__device__ __forceinline__ void fill_table(typename Pol::FE* lds, const typename Pol::S* __restrict__ params, int out,
                                           const ParamOff& po) {
    using TB = Tab<Pol, IN>;
    using FE = typename Pol::FE;
    constexpr int G = TB::grp(M), GE = G * Pol::E, NCG = TB::nc(M) / G, UNITS = TB::tiles(M) * NCG;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int u = (int)(threadIdx.x >> 6); u < UNITS; u += NW) {
        const int mt = u / NCG, c0 = (u % NCG) * G;
        FE v[GE];
#pragma unroll
        for (int cc = 0; cc < G; ++cc)
#pragma unroll
            for (int e = 0; e < Pol::E; ++e) {
                const int s = frag_param<Pol, IN>(M, mt, c0 + cc, lane, e, out, po);
                v[cc * Pol::E + e] = s >= 0 ? Pol::to_frag(params[s]) : FE(0);
            }
        FE* dst = lds + TB::at(M, mt, c0, lane, 0);
        if constexpr (sizeof(v) == 16) {
            *reinterpret_cast<uint4*>(dst) = __builtin_bit_cast(uint4, v);
        } else if constexpr (sizeof(v) == 8) {
            *reinterpret_cast<uint2*>(dst) = __builtin_bit_cast(uint2, v);
        } else {
#pragma unroll
            for (int k = 0; k < GE; ++k) dst[k] = v[k];
        }
    }
}

template <class Pol, int IN, int NW>
__device__ void fill_forward_tables(typename Pol::FE* lds, const typename Pol::S* __restrict__ params, int out,
                                    const ParamOff& po) {
    fill_table<Pol, IN, kA1, NW>(lds, params, out, po);
    fill_table<Pol, IN, kA2, NW>(lds, params, out, po);
    fill_table<Pol, IN, kA3, NW>(lds, params, out, po);
}

template <class Pol, int IN, int NW>
__device__ void fill_all_tables(typename Pol::FE* lds, const typename Pol::S* __restrict__ params, int out,
                                const ParamOff& po) {
    fill_forward_tables<Pol, IN, NW>(lds, params, out, po);
    fill_table<Pol, IN, kB3, NW>(lds, params, out, po);
    fill_table<Pol, IN, kB2, NW>(lds, params, out, po);
    fill_table<Pol, IN, kB1, NW>(lds, params, out, po);
}

__device__ __forceinline__ int span_of_block(const MlpBatch& b) {
    int si = 0;
    for (int i = 1; i < b.count; ++i)
        if ((int)blockIdx.x >= b.s[i].block0) si = i;
    return si;
}

// Per-lane biases in accumulator order.
template <class Pol>
struct Bias {
    float v1[16], v2[16], v3[4];  // unused for FP64
    double d1[16], d2[16], d3[4];
};

// Accumulator tile mt of hidden layer 1 or 2 initialised to the layer's biases
// (lane (j, kb) holds rows 16 mt + 4 kb + r), from per-lane registers ...
template <class Pol>
struct RegBias {
    const typename Pol::V (&b1)[16];
    const typename Pol::V (&b2)[16];
    __device__ typename Pol::Acc init(int layer, int mt) const {
        const typename Pol::V* b = layer == 1 ? b1 : b2;
        typename Pol::Acc a;
        if constexpr (std::is_same<Pol, PolF64>::value) {
#pragma unroll
            for (int r = 0; r < 4; ++r) a.v[r] = b[mt * 4 + r];
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = b[mt * 4 + r];
        }
        return a;
    }
};

// ... or from LDS: b1 at lds[0, 64), b2 at lds[64, 128).
template <class Pol>
struct LdsBias {
    const typename Pol::V* lds;
    __device__ typename Pol::Acc init(int layer, int mt) const {
        const typename Pol::V* p = lds + 64 * (layer - 1) + 16 * mt + 4 * ((threadIdx.x & 63) >> 4);
        if constexpr (std::is_same<Pol, PolF64>::value) return dacc{{p[0], p[1], p[2], p[3]}};
        else return *reinterpret_cast<const floatx4*>(p);
    }
};

// Forward through the trunk for one tile: returns H1, H2 in accumulator order.
template <class Pol, int IN, class FR, class BS>
__device__ __forceinline__ void trunk_forward(const FR& fr, const typename Pol::V (&fv)[Shape<Pol, IN>::NI],
                                              const BS& bs, typename Pol::V (&h1)[16], typename Pol::V (&h2)[16]) {
    using Sh = Shape<Pol, IN>;
    using V = typename Pol::V;
    typename Pol::Acc a[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) a[mt] = bs.init(1, mt);
#pragma unroll
    for (int c = 0; c < Sh::NC1; ++c) {
        const typename Pol::Op b = Pol::pack(&fv[c * Sh::E]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::mma(fr.get(kA1, mt, c), b, a[mt]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const V z = (V)Pol::get(a[mt], r);
            h1[mt * 4 + r] = z > V(0) ? z : V(0);
        }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) a[mt] = bs.init(2, mt);
#pragma unroll
    for (int c = 0; c < Sh::NCH; ++c) {
        const typename Pol::Op b = Pol::pack(&h1[c * Sh::E]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::mma(fr.get(kA2, mt, c), b, a[mt]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const V z = (V)Pol::get(a[mt], r);
            h2[mt * 4 + r] = z > V(0) ? z : V(0);
        }
}

template <class Pol, int IN>
__device__ __forceinline__ void load_features(const typename Pol::V* __restrict__ feat, const FeatView& fvw, int q,
                                              bool valid, typename Pol::V (&fv)[Shape<Pol, IN>::NI]) {
    using Sh = Shape<Pol, IN>;
    const int kb = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int idx = 0; idx < Sh::NI; ++idx) {
        const int k = kb * Sh::NI + idx;
        fv[idx] = (valid && k < IN) ? feat[fvw.at(q, k)] : typename Pol::V(0);
    }
}

template <class Pol>
__device__ __forceinline__ void load_biases(const typename Pol::S* __restrict__ params, const ParamOff& po, int out,
                                            typename Pol::V (&b1)[16], typename Pol::V (&b2)[16],
                                            typename Pol::V (&b3)[4]) {
    const int kb = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int idx = 0; idx < 16; ++idx) {
        b1[idx] = (typename Pol::V)Pol::bias(params[po.b1 + hid(idx, kb)]);
        b2[idx] = (typename Pol::V)Pol::bias(params[po.b2 + hid(idx, kb)]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = 4 * kb + r;
        b3[r] = o < out ? (typename Pol::V)Pol::bias(params[po.b3 + o]) : typename Pol::V(0);
    }
}

// ---------------------------------------------------------------- forward ----
// Workgroups of 4 wavefronts; four wavefronts per SIMD (128 VGPRs) where the layer
// chain fits without spilling.  (Workgroups of 16 wavefronts, which build the
// fragment tables once per CU, measured slower in FP32: 40.4 against 37.5 us.)
template <class Pol, int IN>
constexpr int fwd_threads() { return 256; }
template <class Pol, int IN>
constexpr int fwd_waves_per_eu() { return (std::is_same<Pol, PolF64>::value || IN > 32) ? 1 : 4; }

template <class Pol, int IN>
__global__ __launch_bounds__((fwd_threads<Pol, IN>())) __attribute__((amdgpu_waves_per_eu(fwd_waves_per_eu<Pol, IN>())))
void k_mlp_forward(MlpBatch batch, int out) {
    constexpr int kWaves = fwd_threads<Pol, IN>() / 64;
    using Sh = Shape<Pol, IN>;
    using V = typename Pol::V;
    constexpr bool kLds = !std::is_same<Pol, PolF64>::value;
    extern __shared__ __align__(16) unsigned char smem[];
    const MlpSpan& sp = batch.s[span_of_block(batch)];
    const typename Pol::S* __restrict__ params = static_cast<const typename Pol::S*>(sp.params);
    const ParamOff po(IN, out);
    Frags<Pol, IN, kLds> fr{reinterpret_cast<const typename Pol::FE*>(smem), params, out, po};
    if constexpr (kLds)  // no staging buffer: the forward keeps its LDS small for occupancy
        fill_forward_tables<Pol, IN, kWaves>(reinterpret_cast<typename Pol::FE*>(smem), params, out, po);
    __syncthreads();
    V b1[16], b2[16], b3[4];
    load_biases<Pol>(params, po, out, b1, b2, b3);
    const int lane = threadIdx.x & 63, j = lane & 15, kb = lane >> 4;
    const int n = sp.n;
    const int tps = (n + 15) / 16;
    const int ntiles = tps * sp.segs;
    const int stride = (sp.block1 - sp.block0) * kWaves;
    // the features of the wavefront's next tile are loaded while it computes this one
    auto load_tile = [&](int tile, V (&fv)[Sh::NI]) {
        const int seg = tile / tps;
        const int q = (tile - seg * tps) * 16 + j;
        const V* __restrict__ feat = static_cast<const V*>(sp.feat) + (int64_t)seg * sp.feat_seg;
        load_features<Pol, IN>(feat, sp.fv, q, tile < ntiles && q < n, fv);
    };
    int tile = ((int)blockIdx.x - sp.block0) * kWaves + (int)(threadIdx.x >> 6);
    V next[Sh::NI];
    load_tile(tile, next);
    wait_vmem();
    for (; tile < ntiles; tile += stride) {
        // Weight fragments are read from LDS at each use rather than held in registers
        // across the loop: the smaller register footprint fits four wavefronts per SIMD.
        asm volatile("" ::: "memory");
        const int seg = tile / tps;
        const int q = (tile - seg * tps) * 16 + j;
        const bool valid = q < n;
        V* __restrict__ delta = static_cast<V*>(sp.delta) + (int64_t)seg * sp.out_seg;
        V fv[Sh::NI];
#pragma unroll
        for (int i = 0; i < Sh::NI; ++i) fv[i] = next[i];
        V h1[16], h2[16];
        trunk_forward<Pol, IN>(fr, fv, RegBias<Pol>{b1, b2}, h1, h2);
        load_tile(tile + stride, next);
        typename Pol::Acc a3 = Pol::zero();
#pragma unroll
        for (int c = 0; c < Sh::NCH; ++c) a3 = Pol::mma(fr.get(kA3, 0, c), Pol::pack(&h2[c * Sh::E]), a3);
        if (valid) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = 4 * kb + r;
                if (o < out) delta[(int64_t)q * out + o] = (V)Pol::get(a3, r) + b3[r];
            }
        }
    }
}

// --------------------------------------------------------------- backward ----
// A workgroup of NW wavefronts takes NW tiles (Q = 16 NW queries) per iteration.
// Each wavefront runs the layer chain of its own tile: the trunk recomputed, then
// the transposed backward through W3, W2 and W1, which gives d_feat.  The weight
// gradients contract over queries instead.  For those the chain values of the NW
// tiles are written transposed into a shared staging buffer (one row per unit, one
// column per query), and every 16x16 block of dW3, dW2 and dW1 has one owner
// wavefront, which contracts it over all Q queries and keeps it in registers
// across iterations.  A wavefront so holds 1/NW of the weight gradient, and every
// parameter's sum is formed by one wavefront in a fixed order.
//
// Staging: a row holds Q queries (padded), so that a lane reads one operand group
// (4 queries for the 16x16x4 products, 8 for the 16x16x32 BF16 product) with one
// 16-byte LDS read.  Query q of group m goes to K slot kb when q = QG m + (QG/4) kb
// + e; any assignment works as long as both operands use it.
template <class Pol>
struct Stage;

template <>
struct Stage<PolF32> {
    using T = float;
    static constexpr int QG = 16, PAD = 4;
    struct Grp {
        floatx4 v;
    };
    __device__ static void put(T* p, float v) { *p = v; }
    __device__ static Grp load(const T* row, int m) {
        return Grp{*reinterpret_cast<const floatx4*>(row + QG * m + 4 * ((threadIdx.x & 63) >> 4))};
    }
    __device__ static void mma(floatx4& acc, const Grp& a, const Grp& b) {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[e], b.v[e], acc, 0, 0, 0);
    }
};

template <>
struct Stage<PolBF16> {
    using T = uint16_t;  // BF16 bit patterns, rounded to nearest even once (put_tile)
    static constexpr int QG = 32, PAD = 8;
    struct Grp {
        bf16x8 v;
    };
    __device__ static Grp load(const T* row, int m) {
        return Grp{__builtin_bit_cast(
            bf16x8, *reinterpret_cast<const ushortx8*>(row + QG * m + 8 * ((threadIdx.x & 63) >> 4)))};
    }
    __device__ static void mma(floatx4& acc, const Grp& a, const Grp& b) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc, 0, 0, 0);
    }
};

template <>
struct Stage<PolF64> {
    using T = double;
    static constexpr int QG = 16, PAD = 2;
    struct Grp {
        double v[4];
    };
    __device__ static void put(T* p, double v) { *p = v; }
    __device__ static Grp load(const T* row, int m) {
        const T* p = row + QG * m + 4 * ((threadIdx.x & 63) >> 4);
        return Grp{{p[0], p[1], p[2], p[3]}};
    }
    __device__ static void mma(dacc& acc, const Grp& a, const Grp& b) {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = PolF64::mma(a.v[e], b.v[e], acc);
    }
};

// BF16 staging through the matrix pipe.  A product with a 0/1 selection matrix
// turns one chunk of chain values (lane (q, kb) holding, at query q, the rows
// hid(8 c + e, kb) or kb stride + 8 c + e, e < 8) into one 16-row tile of the staged
// layout: lane (n, kb) then holds row n at queries 4 kb .. 4 kb + 3, which it stores
// with one 8-byte write.  Each output is one product with 1, so it is exact.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ bf16x8 select_at(int target) {
    bf16x8 r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = e == target ? (__bf16)1.0f : (__bf16)0.0f;
    return r;
}
// rows hid(8 c + e, kb) of chunk c = nt / 2 onto tile nt (half = nt % 2)
__device__ __forceinline__ bf16x8 select_hid(int half) {
    const int lane = threadIdx.x & 63, n = lane & 15, kb = lane >> 4;
    const int d = n - 4 * kb;
    return select_at(d >= 0 && d < 4 ? 4 * half + d : -1);
}
// rows kb stride + 8 c + e of chunk c onto tile nt
__device__ __forceinline__ bf16x8 select_lin(int stride, int c, int nt) {
    const int lane = threadIdx.x & 63, n = lane & 15, kb = lane >> 4;
    const int e = 16 * nt + n - kb * stride - 8 * c;
    return select_at(e >= 0 && e < 8 ? e : -1);
}
__device__ __forceinline__ floatx4 select_mma(const bf16x8& a, const bf16x8& sel, floatx4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, sel, acc, 0, 0, 0);
}
// stores the tile (row n at this lane's four queries) into staging rows row0 ..
__device__ __forceinline__ void put_tile(uint16_t* tb, int S, int row0, int wave, const floatx4& d) {
    const int lane = threadIdx.x & 63, n = lane & 15, kb = lane >> 4;
    const bf16x2 lo = {(__bf16)d[0], (__bf16)d[1]}, hi = {(__bf16)d[2], (__bf16)d[3]};
    *reinterpret_cast<uint2*>(tb + (row0 + n) * S + 16 * wave + 4 * kb) =
        uint2{__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi)};
}

// Sums over queries of the rows of a staged 16-row block (the bias gradients).
// FP32 / FP64: lane (j, kb) adds up row j over its K slots; the four lane groups are
// added at the end.  BF16: one more product per operand group, with a vector of
// ones (the matrix pipe is idle there); lane (j, kb) then holds rows 4 kb + r.
template <class Pol>
struct RowSum {
    typename Pol::V s = 0;
    __device__ void add(const typename Stage<Pol>::Grp& g) { s += (g.v[0] + g.v[1]) + (g.v[2] + g.v[3]); }
    template <class F>
    __device__ void emit(F&& f) {
        typename Pol::V t = s + __shfl_xor(s, 16, 64);
        t += __shfl_xor(t, 32, 64);
        if ((threadIdx.x & 63) < 16) f(threadIdx.x & 15, t);
    }
};

template <>
struct RowSum<PolBF16> {
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    __device__ void add(const Stage<PolBF16>::Grp& g) {
        bf16x8 ones;
#pragma unroll
        for (int e = 0; e < 8; ++e) ones[e] = (__bf16)1.0f;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(g.v, ones, acc, 0, 0, 0);
    }
    template <class F>
    __device__ void emit(F&& f) {
        const int lane = threadIdx.x & 63;
        if ((lane & 15) == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) f(4 * (lane >> 4) + r, acc[r]);
        }
    }
};

constexpr size_t kLdsBudget = 160 * 1024;

template <class Pol, int IN>
struct Bwd {
    using Sh = Shape<Pol, IN>;
    using St = Stage<Pol>;
    static constexpr bool kLds = !std::is_same<Pol, PolF64>::value;
    static constexpr int MF = Sh::MF;
    // stage 1 rows: G3^T | H2^T | G1^T | F^T; stage 2 rows: G2^T | H1^T
    static constexpr int R_G3 = 0, R_H2 = 16, R_G1 = 80, R_F = 144, ROWS = 144 + 16 * MF;
    static constexpr int R_G2 = 0, R_H1 = 64;
    static constexpr size_t kFragBytes =
        kLds ? ((size_t)Tab<Pol, IN>::ALL * sizeof(typename Pol::FE) + 15) / 16 * 16 : 0;
    static constexpr size_t kBiasBytes = 128 * sizeof(typename Pol::V);  // b1 | b2
    static constexpr size_t stage_bytes(int nw) { return (size_t)ROWS * (16 * nw + St::PAD) * sizeof(typename St::T); }
    static constexpr int NW = kFragBytes + kBiasBytes + stage_bytes(8) <= kLdsBudget ? 8 : 4;
    static constexpr int Q = 16 * NW;
    static constexpr int S = Q + St::PAD;            // staging row stride, elements
    static constexpr int NG = Q / St::QG;            // operand groups per contraction
    static constexpr size_t kLdsBytes = kFragBytes + kBiasBytes + stage_bytes(NW);
    static constexpr int B2 = 16 / NW;               // dW2 blocks per wavefront (one row tile)
    static constexpr int B1 = (4 * MF + NW - 1) / NW;  // dW1 blocks per wavefront (strided)
    static_assert(kLdsBytes <= kLdsBudget, "backward LDS");
    static_assert((S * sizeof(typename St::T)) % 16 == 0, "16-byte aligned staging rows");
};

template <class Pol, int IN>
constexpr int bwd_threads() { return 64 * Bwd<Pol, IN>::NW; }

template <class Pol, int IN>
__global__ __launch_bounds__((bwd_threads<Pol, IN>())) void k_mlp_backward(MlpBatch batch, int out,
                                                                          typename Pol::V in_scale,
                                                                          typename Pol::V feat_scale,
                                                                          typename Pol::G* __restrict__ partial) {
    using C = Bwd<Pol, IN>;
    using Sh = Shape<Pol, IN>;
    using St = Stage<Pol>;
    using T = typename St::T;
    using V = typename Pol::V;
    using G = typename Pol::G;
    using Acc = typename Pol::Acc;
    constexpr int NW = C::NW, S = C::S;
    constexpr bool kLds = C::kLds;
    extern __shared__ __align__(16) unsigned char smem[];
    const int span = span_of_block(batch);
    const MlpSpan& sp = batch.s[span];
    const typename Pol::S* __restrict__ params = static_cast<const typename Pol::S*>(sp.params);
    const ParamOff po(IN, out);
    // LDS: [fragment tables (FP32/BF16 only)][b1 | b2][staging buffer]
    typename Pol::FE* frag_lds = reinterpret_cast<typename Pol::FE*>(smem);
    V* bias_lds = reinterpret_cast<V*>(smem + C::kFragBytes);
    T* tb = reinterpret_cast<T*>(smem + C::kFragBytes + C::kBiasBytes);

    Frags<Pol, IN, kLds> fr{frag_lds, params, out, po};
    if constexpr (kLds) fill_all_tables<Pol, IN, NW>(frag_lds, params, out, po);
    for (int t = threadIdx.x; t < 128; t += blockDim.x)
        bias_lds[t] = (V)Pol::bias(params[t < 64 ? po.b1 + t : po.b2 + t - 64]);
    __syncthreads();
    const LdsBias<Pol> bias{bias_lds};
    const int lane = threadIdx.x & 63, j = lane & 15, kb = lane >> 4;
    const int wave = threadIdx.x >> 6;

    // Owned gradient blocks: dW3 column tile `wave` (wave < 4); dW2 blocks
    // (mo2, nt2 + b); dW1 blocks wave + NW b of the (mo, nf) list.  The owner of a
    // row tile's first block also sums its gradient rows: db3 (wave 0), db2 (nt2 = 0),
    // db1 (nf = 0).
    const bool own3 = wave < 4;
    const int mo2 = (wave * C::B2) >> 2, nt2 = (wave * C::B2) & 3;
    Acc w3 = Pol::zero(), w2[C::B2], w1[C::B1];
    RowSum<Pol> s3, s2, s1[C::B1];
#pragma unroll
    for (int b = 0; b < C::B2; ++b) w2[b] = Pol::zero();
#pragma unroll
    for (int b = 0; b < C::B1; ++b) w1[b] = Pol::zero();

    const int n = sp.n;
    const int tps = (n + 15) / 16;
    const int ntiles = tps * sp.segs;
    // the span's tiles in contiguous, near-equal ranges per workgroup
    const int nblk = sp.block1 - sp.block0, bi = (int)blockIdx.x - sp.block0;
    const int t0 = (int)((int64_t)ntiles * bi / nblk), t1 = (int)((int64_t)ntiles * (bi + 1) / nblk);
    auto load_tile = [&](int tile, V (&fv)[Sh::NI], V (&go)[Sh::NO]) {
        const int seg = tile / tps;
        const int q = (tile - seg * tps) * 16 + j;
        const bool ok = tile < t1 && q < n;
        const V* __restrict__ feat = static_cast<const V*>(sp.feat) + (int64_t)seg * sp.feat_seg;
        const V* __restrict__ d_out = static_cast<const V*>(sp.d_out) + (int64_t)seg * sp.out_seg;
        load_features<Pol, IN>(feat, sp.fv, q, ok, fv);
#pragma unroll
        for (int idx = 0; idx < Sh::NO; ++idx) {
            const int o = kb * Sh::NO + idx;
            go[idx] = (ok && o < out) ? d_out[(int64_t)q * out + o] : V(0);
        }
    };
    V next_f[Sh::NI], next_g[Sh::NO];
    load_tile(t0 + wave, next_f, next_g);
    wait_vmem();
    T* col = tb + 16 * wave + j;  // this lane's staging column
    for (int base = t0; base < t1; base += NW) {  // uniform over the workgroup
        const int tile = base + wave;
        const bool active = tile < t1;
        // operand groups that hold queries of active tiles (the last iteration of a
        // range may have fewer than NW)
        const int ng = (16 * min(NW, t1 - base) + St::QG - 1) / St::QG;
        V fv[Sh::NI], g3[Sh::NO], h1[16], h2[16], g2[16], g1[16];
#pragma unroll
        for (int i = 0; i < Sh::NI; ++i) fv[i] = next_f[i];
        // upstream gradient of the fused heads, scaled on load
#pragma unroll
        for (int idx = 0; idx < Sh::NO; ++idx) g3[idx] = next_g[idx] * in_scale;
        if (active) {
            const int seg = tile / tps;
            const int q = (tile - seg * tps) * 16 + j;
            trunk_forward<Pol, IN>(fr, fv, bias, h1, h2);
            // prefetch after the first products, so that they wait on no load of this iteration
            load_tile(tile + NW, next_f, next_g);
            // dH2^T = W3^T G3^T, masked by ReLU'(z2)
            Acc a[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::zero();
#pragma unroll
            for (int c = 0; c < Sh::NCO; ++c) {
                const typename Pol::Op b = Pol::pack(&g3[c * Sh::E]);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::mma(fr.get(kB3, mt, c), b, a[mt]);
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) g2[mt * 4 + r] = h2[mt * 4 + r] > V(0) ? (V)Pol::get(a[mt], r) : V(0);
            // dH1^T = W2^T G2^T, masked by ReLU'(z1)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::zero();
#pragma unroll
            for (int c = 0; c < Sh::NCH; ++c) {
                const typename Pol::Op b = Pol::pack(&g2[c * Sh::E]);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::mma(fr.get(kB2, mt, c), b, a[mt]);
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) g1[mt * 4 + r] = h1[mt * 4 + r] > V(0) ? (V)Pol::get(a[mt], r) : V(0);
            // dF^T = W1^T G1^T
            Acc af[Sh::MF];
#pragma unroll
            for (int mf = 0; mf < Sh::MF; ++mf) af[mf] = Pol::zero();
#pragma unroll
            for (int c = 0; c < Sh::NCH; ++c) {
                const typename Pol::Op b = Pol::pack(&g1[c * Sh::E]);
#pragma unroll
                for (int mf = 0; mf < Sh::MF; ++mf)
                    af[mf] = Pol::mma(fr.get(kB1, mf, c), b, af[mf]);
            }
            if (q < n) {
                V* __restrict__ d_feat = static_cast<V*>(sp.d_feat) + (int64_t)seg * sp.feat_seg;
#pragma unroll
                for (int mf = 0; mf < Sh::MF; ++mf)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int f = 16 * mf + 4 * kb + r;
                        if (f < IN) d_feat[sp.fv.at(q, f)] = (V)Pol::get(af[mf], r) * feat_scale;
                    }
            }
        } else {
            // a tile past the range stages zeros (its gradients are zero)
#pragma unroll
            for (int idx = 0; idx < 16; ++idx) h1[idx] = h2[idx] = g1[idx] = g2[idx] = V(0);
        }
        // Stage 1: G3^T, H2^T, G1^T, F^T -> dW3, dW1, db3, db1.
        __syncthreads();  // the previous iteration's dW2 reads are done
        if constexpr (std::is_same<Pol, PolBF16>::value) {
            const floatx4 z = Pol::zero();
            put_tile(tb, S, C::R_G3, wave, select_mma(Pol::pack(&g3[0]), select_lin(Sh::NO, 0, 0), z));
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const bf16x8 sel = select_hid(nt & 1);
                put_tile(tb, S, C::R_H2 + 16 * nt, wave, select_mma(Pol::pack(&h2[8 * (nt >> 1)]), sel, z));
                put_tile(tb, S, C::R_G1 + 16 * nt, wave, select_mma(Pol::pack(&g1[8 * (nt >> 1)]), sel, z));
            }
#pragma unroll
            for (int nf = 0; nf < Sh::MF; ++nf) {
                floatx4 d = z;
#pragma unroll
                for (int c = 0; c < Sh::NC1; ++c) d = select_mma(Pol::pack(&fv[8 * c]), select_lin(Sh::NI, c, nf), d);
                put_tile(tb, S, C::R_F + 16 * nf, wave, d);
            }
        } else {
#pragma unroll
            for (int idx = 0; idx < Sh::NO; ++idx) {
                const int o = kb * Sh::NO + idx;
                if (o < 16) St::put(col + (C::R_G3 + o) * S, g3[idx]);
            }
#pragma unroll
            for (int idx = 0; idx < 16; ++idx) {
                St::put(col + (C::R_H2 + hid(idx, kb)) * S, h2[idx]);
                St::put(col + (C::R_G1 + hid(idx, kb)) * S, g1[idx]);
            }
#pragma unroll
            for (int idx = 0; idx < Sh::NI; ++idx) {
                const int k = kb * Sh::NI + idx;
                if (k < 16 * Sh::MF) St::put(col + (C::R_F + k) * S, fv[idx]);
            }
        }
        __syncthreads();
        // The contractions run over the operand groups that hold active queries: all
        // NG of them (straight-line code) except in a range's last, partial iteration.
        // Each contraction first reads all its operand groups, then issues its products,
        // so that the LDS latency is paid once per block rather than once per group.
        auto block = [&](auto full, Acc& acc, RowSum<Pol>& rsum, bool with_sum, const T* ra, const T* rb) {
            constexpr bool kFull = decltype(full)::value;
            typename St::Grp ga[C::NG], gb[C::NG];
#pragma unroll
            for (int m = 0; m < C::NG; ++m)
                if (kFull || m < ng) {
                    ga[m] = St::load(ra, m);
                    gb[m] = St::load(rb, m);
                }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < C::NG; ++m)
                if (kFull || m < ng) St::mma(acc, ga[m], gb[m]);
            if (with_sum) {
#pragma unroll
                for (int m = 0; m < C::NG; ++m)
                    if (kFull || m < ng) rsum.add(ga[m]);
            }
        };
        auto stage1 = [&](auto full) {
            if (own3) block(full, w3, s3, wave == 0, tb + (C::R_G3 + j) * S, tb + (C::R_H2 + 16 * wave + j) * S);
#pragma unroll
            for (int b = 0; b < C::B1; ++b) {
                const int id = wave + NW * b;
                if (id < 4 * Sh::MF)
                    block(full, w1[b], s1[b], id % Sh::MF == 0, tb + (C::R_G1 + 16 * (id / Sh::MF) + j) * S,
                          tb + (C::R_F + 16 * (id % Sh::MF) + j) * S);
            }
        };
        auto stage2 = [&](auto full) {
            constexpr bool kFull = decltype(full)::value;
            const T* ra = tb + (C::R_G2 + 16 * mo2 + j) * S;
            typename St::Grp ga[C::NG], gb[C::NG][C::B2];
#pragma unroll
            for (int m = 0; m < C::NG; ++m)
                if (kFull || m < ng) {
                    ga[m] = St::load(ra, m);
#pragma unroll
                    for (int b = 0; b < C::B2; ++b) gb[m][b] = St::load(tb + (C::R_H1 + 16 * (nt2 + b) + j) * S, m);
                }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < C::NG; ++m)
                if (kFull || m < ng) {
#pragma unroll
                    for (int b = 0; b < C::B2; ++b) St::mma(w2[b], ga[m], gb[m][b]);
                }
            if (nt2 == 0) {
#pragma unroll
                for (int m = 0; m < C::NG; ++m)
                    if (kFull || m < ng) s2.add(ga[m]);
            }
        };
        if (ng == C::NG) stage1(std::true_type{});
        else stage1(std::false_type{});
        __syncthreads();
        // Stage 2: G2^T, H1^T -> dW2, db2.
        if constexpr (std::is_same<Pol, PolBF16>::value) {
            const floatx4 z = Pol::zero();
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const bf16x8 sel = select_hid(nt & 1);
                put_tile(tb, S, C::R_G2 + 16 * nt, wave, select_mma(Pol::pack(&g2[8 * (nt >> 1)]), sel, z));
                put_tile(tb, S, C::R_H1 + 16 * nt, wave, select_mma(Pol::pack(&h1[8 * (nt >> 1)]), sel, z));
            }
        } else {
#pragma unroll
            for (int idx = 0; idx < 16; ++idx) {
                St::put(col + (C::R_G2 + hid(idx, kb)) * S, g2[idx]);
                St::put(col + (C::R_H1 + hid(idx, kb)) * S, h1[idx]);
            }
        }
        __syncthreads();
        if (ng == C::NG) stage2(std::true_type{});
        else stage2(std::false_type{});
    }

    // Every parameter of the block's partial row is written exactly once.
    G* row = partial + (size_t)blockIdx.x * po.P;
    if (wave == 0) s3.emit([&](int r, V v) { if (r < out) row[po.b3 + r] = (G)v; });
    if (nt2 == 0) s2.emit([&](int r, V v) { row[po.b2 + 16 * mo2 + r] = (G)v; });
#pragma unroll
    for (int b = 0; b < C::B1; ++b) {
        const int id = wave + NW * b;
        if (id < 4 * Sh::MF && id % Sh::MF == 0)
            s1[b].emit([&](int r, V v) { row[po.b1 + 16 * (id / Sh::MF) + r] = (G)v; });
    }
    if (own3) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 4 * kb + r;
            if (o < out) row[po.W3 + o * HID + 16 * wave + j] = (G)Pol::get(w3, r);
        }
    }
#pragma unroll
    for (int b = 0; b < C::B2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            row[po.W2 + (16 * mo2 + 4 * kb + r) * HID + 16 * (nt2 + b) + j] = (G)Pol::get(w2[b], r);
#pragma unroll
    for (int b = 0; b < C::B1; ++b) {
        const int id = wave + NW * b;
        if (id < 4 * Sh::MF) {
            const int mo = id / Sh::MF, f = 16 * (id % Sh::MF) + j;
            if (f < IN) {
#pragma unroll
                for (int r = 0; r < 4; ++r) row[po.W1 + (16 * mo + 4 * kb + r) * IN + f] = (G)Pol::get(w1[b], r);
            }
        }
    }
}

// d_params[p] += scale * sum over rows of partial[row][p].  A block owns 32
// parameters; its 8 row groups each sum every 8th row (32 coalesced 128-byte reads
// in flight per wavefront pair), then the groups are added in a fixed order, so
// the result does not depend on scheduling.
constexpr int kRedParams = 32, kRedGroups = 8;

template <typename G>
__global__ __launch_bounds__(kRedParams * kRedGroups) void k_mlp_reduce(MlpBatch batch, const G* __restrict__ partial,
                                                                        int rows_per_block, int P, G scale) {
    __shared__ G part[kRedGroups][kRedParams];
    const MlpSpan& sp = batch.s[blockIdx.y];
    const int r0 = sp.block0 * rows_per_block, r1 = sp.block1 * rows_per_block;
    const int pl = threadIdx.x % kRedParams, grp = threadIdx.x / kRedParams;
    const int p = blockIdx.x * kRedParams + pl;
    G s = G(0);
    if (p < P) {
#pragma unroll 8
        for (int r = r0 + grp; r < r1; r += kRedGroups) s += partial[(size_t)r * P + p];
    }
    part[grp][pl] = s;
    __syncthreads();
    int bad = 0;
    if (grp == 0 && p < P) {
        G t = G(0);
#pragma unroll
        for (int g = 0; g < kRedGroups; ++g) t += part[g][pl];
        G* dp = static_cast<G*>(sp.d_params) + p;
        const G v = batch.overwrite ? scale * t : *dp + scale * t;
        *dp = v;
        bad = !__builtin_isfinite(v);
    }
    if (batch.nonfinite) {  // one atomic per wavefront that wrote a non-finite value
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) bad += __shfl_xor(bad, d, 64);
        if ((threadIdx.x & 63) == 0 && bad) atomicAdd(batch.nonfinite, bad);
    }
}

// ------------------------------------------------------------------ host ----
// Persistent grids: the forward kernel fits several blocks per CU; the backward
// kernel one of 8 wavefronts (two per SIMD: its registers; for FP32 also its LDS,
// the fragment tables and a 128-query staging buffer).
constexpr int kMlpFwdMaxBlocks = 1024;
constexpr int kMlpBwdMaxBlocks = 256;
constexpr int kMlpF64MaxBlocks = 64;   // the FP64 check path spills to scratch: keep its grid small

// One workgroup per `waves` tiles of 16 queries, at most `cap`.
static int mlp_blocks(int n, int waves, int cap) {
    const int ntiles = (n + 15) / 16;
    const int want = (ntiles + waves - 1) / waves;
    return want < cap ? (want > 0 ? want : 1) : cap;
}

template <class Pol, int IN>
static size_t lds_forward(int out) {
    if (std::is_same<Pol, PolF64>::value) return 0;
    return ((size_t)Tab<Pol, IN>::FWD * sizeof(typename Pol::FE) + 15) / 16 * 16;
}

size_t mlp_workspace_bytes(h4d_dtype dt, int in, int out, int n) {
    return mlp_partial_bytes(dt, in, out, mlp_blocks_for(dt, true, n), 1);
}

template <class Pol, int IN>
static hipError_t forward_t(const MlpBatch& b, int blocks, int out, hipStream_t s) {
    const size_t lds = lds_forward<Pol, IN>(out);
    auto kern = k_mlp_forward<Pol, IN>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(fwd_threads<Pol, IN>()), lds, s, b, out);
    return hipGetLastError();
}

static size_t align_up(size_t b) { return (b + 255) / 256 * 256; }

template <class Pol>
static size_t partial_rows_bytes(int in, int out, int blocks) {
    const ParamOff po(in, out);
    return (size_t)blocks * po.P * sizeof(typename Pol::G);
}

template <class Pol, int IN>
static hipError_t backward_t(const MlpBatch& b, int blocks, int out, double in_scale, double feat_scale,
                             double param_scale, void* ws, hipStream_t s) {
    const size_t lds = Bwd<Pol, IN>::kLdsBytes;
    auto kern = k_mlp_backward<Pol, IN>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    using V = typename Pol::V;
    using G = typename Pol::G;
    // workspace: the per-block partial rows
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * Bwd<Pol, IN>::NW), lds, s, b, out, (V)in_scale,
                       (V)feat_scale, static_cast<G*>(ws));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const ParamOff po(IN, out);
    hipLaunchKernelGGL(k_mlp_reduce<G>, dim3((po.P + kRedParams - 1) / kRedParams, b.count),
                       dim3(kRedParams * kRedGroups), 0, s, b, static_cast<const G*>(ws), 1, po.P, (G)param_scale);
    return hipGetLastError();
}

template <class Pol>
static hipError_t forward_p(int in, const MlpBatch& b, int blocks, int out, hipStream_t s) {
    switch (in) {
        case 8: return forward_t<Pol, 8>(b, blocks, out, s);
        case 16: return forward_t<Pol, 16>(b, blocks, out, s);
        case 32: return forward_t<Pol, 32>(b, blocks, out, s);
        case 64: return forward_t<Pol, 64>(b, blocks, out, s);
    }
    return hipErrorInvalidValue;
}

template <class Pol>
static hipError_t backward_p(int in, const MlpBatch& b, int blocks, int out, double in_scale, double feat_scale,
                             double param_scale, void* ws, hipStream_t s) {
    switch (in) {
        case 8: return backward_t<Pol, 8>(b, blocks, out, in_scale, feat_scale, param_scale, ws, s);
        case 16: return backward_t<Pol, 16>(b, blocks, out, in_scale, feat_scale, param_scale, ws, s);
        case 32: return backward_t<Pol, 32>(b, blocks, out, in_scale, feat_scale, param_scale, ws, s);
        case 64: return backward_t<Pol, 64>(b, blocks, out, in_scale, feat_scale, param_scale, ws, s);
    }
    return hipErrorInvalidValue;
}

static int log2i(int F) { return F == 1 ? 0 : F == 2 ? 1 : F == 4 ? 2 : 3; }

int mlp_blocks_for(h4d_dtype dt, bool backward, int64_t queries) {
    const int cap = dt == H4D_F64 ? kMlpF64MaxBlocks : backward ? kMlpBwdMaxBlocks : kMlpFwdMaxBlocks;
    return mlp_blocks((int)(queries < 2147483647 ? queries : 2147483647), backward ? 8 : 4, cap);
}

size_t mlp_partial_bytes(h4d_dtype dt, int in, int out, int blocks, int) {
    switch (dt) {
        case H4D_F32: return align_up(partial_rows_bytes<PolF32>(in, out, blocks));
        case H4D_BF16: return align_up(partial_rows_bytes<PolBF16>(in, out, blocks));
        default: return align_up(partial_rows_bytes<PolF64>(in, out, blocks));
    }
}

static MlpBatch single(const void* params, const void* feat, void* delta, const void* d_out, void* d_feat,
                       void* d_params, int F, int64_t lstride, int64_t qstride, int n, int blocks) {
    MlpBatch b;
    memset(&b, 0, sizeof b);
    b.count = 1;
    MlpSpan& sp = b.s[0];
    sp.params = params;
    sp.feat = feat;
    sp.delta = delta;
    sp.d_out = d_out;
    sp.d_feat = d_feat;
    sp.d_params = d_params;
    sp.fv = FeatView{lstride, qstride, log2i(F)};
    sp.n = n;
    sp.segs = 1;
    sp.block0 = 0;
    sp.block1 = blocks;
    return b;
}

hipError_t launch_mlp_forward(h4d_dtype dt, int in, int out, const void* params, const void* feat, int F,
                              int64_t lstride, int64_t qstride, int n, void* delta, hipStream_t s) {
    const int blocks = mlp_blocks_for(dt, false, n);
    const MlpBatch b = single(params, feat, delta, nullptr, nullptr, nullptr, F, lstride, qstride, n, blocks);
    return launch_mlp_forward_batch(dt, in, out, b, blocks, s);
}

hipError_t launch_mlp_backward(h4d_dtype dt, int in, int out, const void* params, const void* feat, int F,
                               int64_t lstride, int64_t qstride, int n, const void* d_out, double in_scale,
                               double feat_scale, double param_scale, void* d_feat, int64_t dlstride, int64_t dqstride,
                               void* d_params, void* ws, hipStream_t s, bool overwrite, int32_t* nonfinite) {
    if (dlstride != lstride || dqstride != qstride) return hipErrorInvalidValue;  // d_feat shares feat's layout
    const int blocks = mlp_blocks_for(dt, true, n);
    MlpBatch b = single(params, feat, nullptr, d_out, d_feat, d_params, F, lstride, qstride, n, blocks);
    b.overwrite = overwrite ? 1 : 0;
    b.nonfinite = nonfinite;
    return launch_mlp_backward_batch(dt, in, out, b, blocks, in_scale, feat_scale, param_scale, ws, s);
}

hipError_t launch_mlp_forward_batch(h4d_dtype dt, int in, int out, const MlpBatch& b, int blocks, hipStream_t s) {
    switch (dt) {
        case H4D_F32: return forward_p<PolF32>(in, b, blocks, out, s);
        case H4D_BF16: return forward_p<PolBF16>(in, b, blocks, out, s);
        case H4D_F64: return forward_p<PolF64>(in, b, blocks, out, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_mlp_backward_batch(h4d_dtype dt, int in, int out, const MlpBatch& b, int blocks, double in_scale,
                                     double feat_scale, double param_scale, void* ws, hipStream_t s) {
    switch (dt) {
        case H4D_F32: return backward_p<PolF32>(in, b, blocks, out, in_scale, feat_scale, param_scale, ws, s);
        case H4D_BF16: return backward_p<PolBF16>(in, b, blocks, out, in_scale, feat_scale, param_scale, ws, s);
        case H4D_F64: return backward_p<PolF64>(in, b, blocks, out, in_scale, feat_scale, param_scale, ws, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace h4d
