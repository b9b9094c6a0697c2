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
constexpr int kMlpBlock = 256;
constexpr int kWaves = kMlpBlock / 64;
constexpr int kTbStride = 17;  // LDS transpose buffer row stride (2-cycle wave64 access)
constexpr int kTbRows = 128;

__device__ __forceinline__ int hid(int idx, int kb) { return 16 * (idx >> 2) + 4 * kb + (idx & 3); }

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
    // fragment tables, in elements: [tiles][chunks][64 lanes][E]
    static constexpr int A1 = 4 * NC1 * 64 * E;   // W1      (layer 1, forward)
    static constexpr int A2 = 4 * NCH * 64 * E;   // W2
    static constexpr int A3 = 1 * NCH * 64 * E;   // W3
    static constexpr int B3 = 4 * NCO * 64 * E;   // W3^T    (backward)
    static constexpr int B2 = 4 * NCH * 64 * E;   // W2^T
    static constexpr int B1 = MF * NCH * 64 * E;  // W1^T
    static constexpr int OFF_A1 = 0, OFF_A2 = OFF_A1 + A1, OFF_A3 = OFF_A2 + A2, OFF_B3 = OFF_A3 + A3,
                         OFF_B2 = OFF_B3 + B3, OFF_B1 = OFF_B2 + B2;
    static constexpr int FWD_FRAGS = OFF_B3;
    static constexpr int ALL_FRAGS = OFF_B1 + B1;
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

// Flat parameter index of fragment element t of the tables (-1 = zero padding).
template <class Pol, int IN>
__device__ int frag_source(int t, int out, const ParamOff& po) {
    using Sh = Shape<Pol, IN>;
    constexpr int E = Sh::E;
    int mat, rel;
    if (t < Sh::OFF_A2) { mat = 0; rel = t - Sh::OFF_A1; }
    else if (t < Sh::OFF_A3) { mat = 1; rel = t - Sh::OFF_A2; }
    else if (t < Sh::OFF_B3) { mat = 2; rel = t - Sh::OFF_A3; }
    else if (t < Sh::OFF_B2) { mat = 3; rel = t - Sh::OFF_B3; }
    else if (t < Sh::OFF_B1) { mat = 4; rel = t - Sh::OFF_B2; }
    else { mat = 5; rel = t - Sh::OFF_B1; }
    const int e = rel % E;
    const int lane = (rel / E) % 64;
    const int tc = rel / (E * 64);  // tile * chunks + chunk
    const int i = lane & 15, kb = lane >> 4;
    switch (mat) {
        case 0: {  // A1[mt][c]: W1[16 mt + i][kb NI + c E + e]
            const int mt = tc / Sh::NC1, c = tc % Sh::NC1;
            const int k = kb * Sh::NI + c * E + e;
            return k < IN ? po.W1 + (16 * mt + i) * IN + k : -1;
        }
        case 1: {  // A2[mt][c]: W2[16 mt + i][hid(c E + e, kb)]
            const int mt = tc / Sh::NCH, c = tc % Sh::NCH;
            return po.W2 + (16 * mt + i) * HID + hid(c * E + e, kb);
        }
        case 2: {  // A3[c]: W3[i][hid(c E + e, kb)]
            const int c = tc;
            return i < out ? po.W3 + i * HID + hid(c * E + e, kb) : -1;
        }
        case 3: {  // B3[mt][c]: W3^T -> W3[kb NO + c E + e][16 mt + i]
            const int mt = tc / Sh::NCO, c = tc % Sh::NCO;
            const int o = kb * Sh::NO + c * E + e;
            return o < out ? po.W3 + o * HID + 16 * mt + i : -1;
        }
        case 4: {  // B2[mt][c]: W2^T -> W2[hid(c E + e, kb)][16 mt + i]
            const int mt = tc / Sh::NCH, c = tc % Sh::NCH;
            return po.W2 + hid(c * E + e, kb) * HID + 16 * mt + i;
        }
        default: {  // B1[mf][c]: W1^T -> W1[hid(c E + e, kb)][16 mf + i]
            const int mf = tc / Sh::NCH, c = tc % Sh::NCH;
            const int f = 16 * mf + i;
            return f < IN ? po.W1 + hid(c * E + e, kb) * IN + f : -1;
        }
    }
}

// Fragment tables: built in LDS for FP32 / BF16; read straight from the
// parameter array for FP64 (its tables would not fit next to its other buffers).
template <class Pol, int IN, bool LDS>
struct Frags {
    using FE = typename Pol::FE;
    const FE* lds;                         // LDS tables (LDS == true)
    const typename Pol::S* params;         // global parameters (LDS == false)
    int out;
    ParamOff po;

    __device__ typename Pol::Op get(int off, int tc) const {
        const int lane = threadIdx.x & 63;
        if constexpr (LDS) {
            return Pol::frag(lds + ((size_t)(off / Pol::E + tc * 64 + lane)) * Pol::E);
        } else {
            FE v[Pol::E];
#pragma unroll
            for (int e = 0; e < Pol::E; ++e) {
                const int t = off + (tc * 64 + lane) * Pol::E + e;
                const int s = frag_source<Pol, IN>(t, out, po);
                v[e] = s >= 0 ? Pol::to_frag(params[s]) : FE(0);
            }
            return Pol::frag(v);
        }
    }
};

template <class Pol, int IN>
__device__ void fill_frags(typename Pol::FE* lds, int count, const typename Pol::S* __restrict__ params, int out,
                           const ParamOff& po) {
    // The permutation reads the (L2-resident) parameters directly, eight independent
    // loads in flight per thread before their LDS stores.
    constexpr int B = 8;
    for (int t0 = threadIdx.x; t0 < count; t0 += B * blockDim.x) {
        typename Pol::FE v[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int t = t0 + k * (int)blockDim.x;
            const int s = t < count ? frag_source<Pol, IN>(t, out, po) : -1;
            v[k] = s >= 0 ? Pol::to_frag(params[s]) : typename Pol::FE(0);
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int t = t0 + k * (int)blockDim.x;
            if (t < count) lds[t] = v[k];
        }
    }
}

// The backward's fragment tables of every span, built once per call into the
// workspace (a workgroup per 256 elements and span); each backward workgroup then
// copies its span's tables into LDS instead of rebuilding them.
template <class Pol, int IN>
__global__ __launch_bounds__(256) void k_mlp_frags(MlpBatch b, int out, typename Pol::FE* __restrict__ frags,
                                                   int64_t stride) {
    using Sh = Shape<Pol, IN>;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= Sh::ALL_FRAGS) return;
    const typename Pol::S* __restrict__ params = static_cast<const typename Pol::S*>(b.s[blockIdx.y].params);
    const ParamOff po(IN, out);
    const int s = frag_source<Pol, IN>(t, out, po);
    frags[(int64_t)blockIdx.y * stride + t] = s >= 0 ? Pol::to_frag(params[s]) : typename Pol::FE(0);
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

// Forward through the trunk for one tile: returns H1, H2 in accumulator order.
template <class Pol, int IN, class FR>
__device__ __forceinline__ void trunk_forward(const FR& fr, const typename Pol::V (&fv)[Shape<Pol, IN>::NI],
                                              const typename Pol::V (&b1)[16], const typename Pol::V (&b2)[16],
                                              typename Pol::V (&h1)[16], typename Pol::V (&h2)[16]) {
    using Sh = Shape<Pol, IN>;
    using V = typename Pol::V;
    typename Pol::Acc a[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::zero();
#pragma unroll
    for (int c = 0; c < Sh::NC1; ++c) {
        const typename Pol::Op b = Pol::pack(&fv[c * Sh::E]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::mma(fr.get(Sh::OFF_A1, mt * Sh::NC1 + c), b, a[mt]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const V z = (V)Pol::get(a[mt], r) + b1[mt * 4 + r];
            h1[mt * 4 + r] = z > V(0) ? z : V(0);
        }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::zero();
#pragma unroll
    for (int c = 0; c < Sh::NCH; ++c) {
        const typename Pol::Op b = Pol::pack(&h1[c * Sh::E]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::mma(fr.get(Sh::OFF_A2, mt * Sh::NCH + c), b, a[mt]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const V z = (V)Pol::get(a[mt], r) + b2[mt * 4 + r];
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
// Four wavefronts per SIMD (128 VGPRs) where the layer chain fits without spilling.
template <class Pol, int IN>
constexpr int fwd_waves_per_eu() { return (std::is_same<Pol, PolF64>::value || IN > 32) ? 1 : 4; }

template <class Pol, int IN>
__global__ __launch_bounds__(kMlpBlock) __attribute__((amdgpu_waves_per_eu(fwd_waves_per_eu<Pol, IN>())))
void k_mlp_forward(MlpBatch batch, int out) {
    using Sh = Shape<Pol, IN>;
    using V = typename Pol::V;
    constexpr bool kLds = !std::is_same<Pol, PolF64>::value;
    extern __shared__ __align__(16) unsigned char smem[];
    const MlpSpan& sp = batch.s[span_of_block(batch)];
    const typename Pol::S* __restrict__ params = static_cast<const typename Pol::S*>(sp.params);
    const ParamOff po(IN, out);
    Frags<Pol, IN, kLds> fr{reinterpret_cast<const typename Pol::FE*>(smem), params, out, po};
    if constexpr (kLds)  // no staging buffer: the forward keeps its LDS small for occupancy
        fill_frags<Pol, IN>(reinterpret_cast<typename Pol::FE*>(smem), Sh::FWD_FRAGS, params, out, po);
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
        load_tile(tile + stride, next);
        V h1[16], h2[16];
        trunk_forward<Pol, IN>(fr, fv, b1, b2, h1, h2);
        typename Pol::Acc a3 = Pol::zero();
#pragma unroll
        for (int c = 0; c < Sh::NCH; ++c) a3 = Pol::mma(fr.get(Sh::OFF_A3, c), Pol::pack(&h2[c * Sh::E]), a3);
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
// Weight-gradient operands over the 16 queries of a tile.  For the 16x16 block
// whose rows start at row r0 of the transpose buffer, lane (i, kb) holds the
// values of row r0 + i at the queries it contributes: q = 4c + kb for chunk c
// (FP32 / FP64, four 16x16x4 products) or q = 4kb + e (BF16, one 16x16x16 product).
template <class Pol>
struct WOp {
    typename Pol::V v[4];
};

template <class Pol>
__device__ __forceinline__ WOp<Pol> wload(const typename Pol::V* tb, int r0) {
    const int lane = threadIdx.x & 63, i = lane & 15, kb = lane >> 4;
    WOp<Pol> o;
#pragma unroll
    for (int c = 0; c < 4; ++c)
        o.v[c] = std::is_same<Pol, PolBF16>::value ? tb[(r0 + i) * kTbStride + 4 * kb + c]
                                                   : tb[(r0 + i) * kTbStride + 4 * c + kb];
    return o;
}

// acc[i][j] += sum_q A[q][i] B[q][j] over the tile's 16 queries.
template <class Pol>
__device__ __forceinline__ void wmma(typename Pol::Acc& acc, const WOp<Pol>& a, const WOp<Pol>& b) {
    if constexpr (std::is_same<Pol, PolBF16>::value) {
        shortx4 x, y;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            x[e] = __builtin_bit_cast(short, (__bf16)a.v[e]);
            y[e] = __builtin_bit_cast(short, (__bf16)b.v[e]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, y, acc, 0, 0, 0);
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) acc = Pol::mma(a.v[c], b.v[c], acc);
    }
}

template <class Pol, int IN>
__global__ __launch_bounds__(kMlpBlock) void k_mlp_backward(MlpBatch batch, int out, typename Pol::V in_scale,
                                                            typename Pol::V feat_scale,
                                                            typename Pol::G* __restrict__ partial,
                                                            const typename Pol::FE* __restrict__ frags,
                                                            int64_t frag_stride) {
    using Sh = Shape<Pol, IN>;
    using V = typename Pol::V;
    using G = typename Pol::G;
    using Acc = typename Pol::Acc;
    constexpr bool kLds = !std::is_same<Pol, PolF64>::value;
    extern __shared__ __align__(16) unsigned char smem[];
    const int span = span_of_block(batch);
    const MlpSpan& sp = batch.s[span];
    const typename Pol::S* __restrict__ params = static_cast<const typename Pol::S*>(sp.params);
    const ParamOff po(IN, out);
    // LDS: [fragment tables (FP32/BF16 only)][block gradient accumulator (FP32/BF16 only)][transpose buffers]
    typename Pol::FE* frag_lds = reinterpret_cast<typename Pol::FE*>(smem);
    size_t off = kLds ? ((size_t)Sh::ALL_FRAGS * sizeof(typename Pol::FE) + 15) / 16 * 16 : 0;
    G* wacc = reinterpret_cast<G*>(smem + off);
    if (kLds) off += ((size_t)po.P * sizeof(G) + 15) / 16 * 16;
    V* tb = reinterpret_cast<V*>(smem + off) + (threadIdx.x >> 6) * kTbRows * kTbStride;

    Frags<Pol, IN, kLds> fr{frag_lds, params, out, po};
    if constexpr (kLds) {
        // the span's tables, prepared by k_mlp_frags, copied 16 bytes per lane
        const uint4* src = reinterpret_cast<const uint4*>(frags + (int64_t)span * frag_stride);
        uint4* dst = reinterpret_cast<uint4*>(frag_lds);
        constexpr int kVec = (int)(Sh::ALL_FRAGS * sizeof(typename Pol::FE) / 16);
        static_assert(Sh::ALL_FRAGS * sizeof(typename Pol::FE) % 16 == 0, "tables are whole 16-byte vectors");
        for (int t = threadIdx.x; t < kVec; t += blockDim.x) dst[t] = src[t];
        for (int t = threadIdx.x; t < po.P; t += blockDim.x) wacc[t] = G(0);
    }
    __syncthreads();
    V b1[16], b2[16], b3[4];
    load_biases<Pol>(params, po, out, b1, b2, b3);
    const int lane = threadIdx.x & 63, j = lane & 15, kb = lane >> 4;

    Acc w3[4], w2[4][4], w1[4][Sh::MF];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        w3[a] = Pol::zero();
#pragma unroll
        for (int b = 0; b < 4; ++b) w2[a][b] = Pol::zero();
#pragma unroll
        for (int b = 0; b < Sh::MF; ++b) w1[a][b] = Pol::zero();
    }
    V sb1[16], sb2[16], sb3[Sh::NO];
#pragma unroll
    for (int idx = 0; idx < 16; ++idx) sb1[idx] = sb2[idx] = V(0);
#pragma unroll
    for (int idx = 0; idx < Sh::NO; ++idx) sb3[idx] = V(0);

    const int n = sp.n;
    const int tps = (n + 15) / 16;
    const int ntiles = tps * sp.segs;
    const int stride = (sp.block1 - sp.block0) * kWaves;
    // the inputs of the wavefront's next tile are loaded while it computes this one
    auto load_tile = [&](int tile, V (&fv)[Sh::NI], V (&go)[Sh::NO]) {
        const int seg = tile / tps;
        const int q = (tile - seg * tps) * 16 + j;
        const bool ok = tile < ntiles && q < n;
        const V* __restrict__ feat = static_cast<const V*>(sp.feat) + (int64_t)seg * sp.feat_seg;
        const V* __restrict__ d_out = static_cast<const V*>(sp.d_out) + (int64_t)seg * sp.out_seg;
        load_features<Pol, IN>(feat, sp.fv, q, ok, fv);
#pragma unroll
        for (int idx = 0; idx < Sh::NO; ++idx) {
            const int o = kb * Sh::NO + idx;
            go[idx] = (ok && o < out) ? d_out[(int64_t)q * out + o] : V(0);
        }
    };
    int tile = ((int)blockIdx.x - sp.block0) * kWaves + (int)(threadIdx.x >> 6);
    V next_f[Sh::NI], next_g[Sh::NO];
    load_tile(tile, next_f, next_g);
    for (; tile < ntiles; tile += stride) {
        const int seg = tile / tps;
        const int q = (tile - seg * tps) * 16 + j;
        const bool valid = q < n;
        V* __restrict__ d_feat = static_cast<V*>(sp.d_feat) + (int64_t)seg * sp.feat_seg;
        V fv[Sh::NI];
        // upstream gradient of the fused heads, scaled on load
        V g3[Sh::NO];
#pragma unroll
        for (int i = 0; i < Sh::NI; ++i) fv[i] = next_f[i];
#pragma unroll
        for (int idx = 0; idx < Sh::NO; ++idx) {
            g3[idx] = next_g[idx] * in_scale;
            sb3[idx] += g3[idx];
        }
        load_tile(tile + stride, next_f, next_g);
        V h1[16], h2[16];
        trunk_forward<Pol, IN>(fr, fv, b1, b2, h1, h2);
        // dH2^T = W3^T G3^T, masked by ReLU'(z2)
        Acc a[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::zero();
#pragma unroll
        for (int c = 0; c < Sh::NCO; ++c) {
            const typename Pol::Op b = Pol::pack(&g3[c * Sh::E]);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::mma(fr.get(Sh::OFF_B3, mt * Sh::NCO + c), b, a[mt]);
        }
        V g2[16];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int idx = mt * 4 + r;
                g2[idx] = h2[idx] > V(0) ? (V)Pol::get(a[mt], r) : V(0);
                sb2[idx] += g2[idx];
            }
        // dH1^T = W2^T G2^T, masked by ReLU'(z1)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::zero();
#pragma unroll
        for (int c = 0; c < Sh::NCH; ++c) {
            const typename Pol::Op b = Pol::pack(&g2[c * Sh::E]);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) a[mt] = Pol::mma(fr.get(Sh::OFF_B2, mt * Sh::NCH + c), b, a[mt]);
        }
        V g1[16];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int idx = mt * 4 + r;
                g1[idx] = h1[idx] > V(0) ? (V)Pol::get(a[mt], r) : V(0);
                sb1[idx] += g1[idx];
            }
        // dF^T = W1^T G1^T
        Acc af[Sh::MF];
#pragma unroll
        for (int mf = 0; mf < Sh::MF; ++mf) af[mf] = Pol::zero();
#pragma unroll
        for (int c = 0; c < Sh::NCH; ++c) {
            const typename Pol::Op b = Pol::pack(&g1[c * Sh::E]);
#pragma unroll
            for (int mf = 0; mf < Sh::MF; ++mf) af[mf] = Pol::mma(fr.get(Sh::OFF_B1, mf * Sh::NCH + c), b, af[mf]);
        }
        if (valid) {
#pragma unroll
            for (int mf = 0; mf < Sh::MF; ++mf)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int f = 16 * mf + 4 * kb + r;
                    if (f < IN) d_feat[sp.fv.at(q, f)] = (V)Pol::get(af[mf], r) * feat_scale;
                }
        }
        // Weight gradients: stage G^T and H^T rows through this wavefront's LDS buffer.
        // Stage 1: G3^T rows 0..15, H2^T rows 16..79 -> dW3.
#pragma unroll
        for (int idx = 0; idx < Sh::NO; ++idx) {
            const int o = kb * Sh::NO + idx;
            if (o < 16) tb[o * kTbStride + j] = g3[idx];
        }
#pragma unroll
        for (int idx = 0; idx < 16; ++idx) tb[(16 + hid(idx, kb)) * kTbStride + j] = h2[idx];
        __builtin_amdgcn_wave_barrier();
        {
            const WOp<Pol> ga = wload<Pol>(tb, 0);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) wmma<Pol>(w3[nt], ga, wload<Pol>(tb, 16 + 16 * nt));
        }
        __builtin_amdgcn_wave_barrier();
        // Stage 2: G2^T rows 0..63, H1^T rows 64..127 -> dW2.
#pragma unroll
        for (int idx = 0; idx < 16; ++idx) {
            tb[hid(idx, kb) * kTbStride + j] = g2[idx];
            tb[(64 + hid(idx, kb)) * kTbStride + j] = h1[idx];
        }
        __builtin_amdgcn_wave_barrier();
        {
            WOp<Pol> hb[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) hb[nt] = wload<Pol>(tb, 64 + 16 * nt);
#pragma unroll
            for (int mo = 0; mo < 4; ++mo) {
                const WOp<Pol> ga = wload<Pol>(tb, 16 * mo);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) wmma<Pol>(w2[mo][nt], ga, hb[nt]);
            }
        }
        __builtin_amdgcn_wave_barrier();
        // Stage 3: G1^T rows 0..63, F^T rows 64..(64 + 16 MF) -> dW1.
#pragma unroll
        for (int idx = 0; idx < 16; ++idx) tb[hid(idx, kb) * kTbStride + j] = g1[idx];
#pragma unroll
        for (int idx = 0; idx < Sh::NI; ++idx) {
            const int k = kb * Sh::NI + idx;
            if (k < 16 * Sh::MF) tb[(64 + k) * kTbStride + j] = fv[idx];
        }
        __builtin_amdgcn_wave_barrier();
        {
            WOp<Pol> fb[Sh::MF];
#pragma unroll
            for (int nf = 0; nf < Sh::MF; ++nf) fb[nf] = wload<Pol>(tb, 64 + 16 * nf);
#pragma unroll
            for (int mo = 0; mo < 4; ++mo) {
                const WOp<Pol> ga = wload<Pol>(tb, 16 * mo);
#pragma unroll
                for (int nf = 0; nf < Sh::MF; ++nf) wmma<Pol>(w1[mo][nf], ga, fb[nf]);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }

    // Reduce the bias sums over the 16 query lanes of each lane group.
#pragma unroll
    for (int s = 1; s < 16; s <<= 1) {
#pragma unroll
        for (int idx = 0; idx < 16; ++idx) {
            sb1[idx] += __shfl_xor(sb1[idx], s, 64);
            sb2[idx] += __shfl_xor(sb2[idx], s, 64);
        }
#pragma unroll
        for (int idx = 0; idx < Sh::NO; ++idx) sb3[idx] += __shfl_xor(sb3[idx], s, 64);
    }

    // Emit the wavefront partial gradients.  FP32/BF16: the parameters fall into four
    // blocks (row tiles mo of W1 and W2, column tiles nt of W3, quarters of b1 and b2;
    // b3 joins block 0), and in round r wavefront w adds its block (w + r) mod 4 to
    // the block accumulator in LDS with plain read-modify-writes.  The four
    // wavefronts work on disjoint blocks at once, and every parameter receives the
    // wavefronts' sums in a fixed order.  FP64: each wavefront writes its own row.
    static_assert(!kLds || kWaves == 4, "one parameter block per wavefront");
    const int wave = threadIdx.x >> 6;
    G* dst = kLds ? wacc : partial + (size_t)(blockIdx.x * kWaves + wave) * po.P;
    auto emit = [&](int p, G v) {
        if constexpr (kLds) dst[p] += v;
        else dst[p] = v;
    };
    for (int round = 0; round < (kLds ? kWaves : 1); ++round) {
        const int blk = (wave + round) & 3;
        auto mine = [&](int b) { return !kLds || b == blk; };
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            if (mine(nt)) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int o = 4 * kb + r;
                    if (o < out) emit(po.W3 + o * HID + 16 * nt + j, (G)Pol::get(w3[nt], r));
                }
            }
#pragma unroll
        for (int mo = 0; mo < 4; ++mo)
            if (mine(mo)) {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        emit(po.W2 + (16 * mo + 4 * kb + r) * HID + 16 * nt + j, (G)Pol::get(w2[mo][nt], r));
#pragma unroll
                for (int nf = 0; nf < Sh::MF; ++nf)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int f = 16 * nf + j;
                        if (f < IN) emit(po.W1 + (16 * mo + 4 * kb + r) * IN + f, (G)Pol::get(w1[mo][nf], r));
                    }
            }
        if (j == 0) {
#pragma unroll
            for (int idx = 0; idx < 16; ++idx)
                if (mine(idx >> 2)) {
                    emit(po.b1 + hid(idx, kb), (G)sb1[idx]);
                    emit(po.b2 + hid(idx, kb), (G)sb2[idx]);
                }
            if (mine(0)) {
#pragma unroll
                for (int idx = 0; idx < Sh::NO; ++idx) {
                    const int o = kb * Sh::NO + idx;
                    if (o < out) emit(po.b3 + o, (G)sb3[idx]);
                }
            }
        }
        if constexpr (kLds) __syncthreads();
    }
    if constexpr (kLds) {
        G* row = partial + (size_t)blockIdx.x * po.P;
        for (int t = threadIdx.x; t < po.P; t += blockDim.x) row[t] = wacc[t];
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
    if (grp == 0 && p < P) {
        G t = G(0);
#pragma unroll
        for (int g = 0; g < kRedGroups; ++g) t += part[g][pl];
        G* dp = static_cast<G*>(sp.d_params) + p;
        if (batch.overwrite) *dp = scale * t;
        else *dp += scale * t;
    }
}

// ------------------------------------------------------------------ host ----
// Persistent grids: the forward kernel fits several blocks per CU, the backward
// kernel's LDS (fragment tables, gradient accumulator, transpose buffers) one.
constexpr int kMlpFwdMaxBlocks = 1024;
constexpr int kMlpBwdMaxBlocks = 256;
constexpr int kMlpF64MaxBlocks = 64;   // the FP64 check path spills to scratch: keep its grid small

static int mlp_blocks(int n, int cap) {
    const int ntiles = (n + 15) / 16;
    const int want = (ntiles + kWaves - 1) / kWaves;
    return want < cap ? (want > 0 ? want : 1) : cap;
}

template <class Pol, int IN>
static size_t lds_forward(int out) {
    if (std::is_same<Pol, PolF64>::value) return 0;
    return ((size_t)Shape<Pol, IN>::FWD_FRAGS * sizeof(typename Pol::FE) + 15) / 16 * 16;
}

template <class Pol, int IN>
static size_t lds_backward(int out) {
    const ParamOff po(IN, out);
    size_t s = 0;
    if (!std::is_same<Pol, PolF64>::value) {
        s += ((size_t)Shape<Pol, IN>::ALL_FRAGS * sizeof(typename Pol::FE) + 15) / 16 * 16;
        s += ((size_t)po.P * sizeof(typename Pol::G) + 15) / 16 * 16;
    }
    s += (size_t)kWaves * kTbRows * kTbStride * sizeof(typename Pol::V);
    return s;
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
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kMlpBlock), lds, s, b, out);
    return hipGetLastError();
}

static size_t align_up(size_t b) { return (b + 255) / 256 * 256; }

template <class Pol>
static size_t partial_rows_bytes(int in, int out, int blocks) {
    const ParamOff po(in, out);
    return (size_t)blocks * (std::is_same<Pol, PolF64>::value ? kWaves : 1) * po.P * sizeof(typename Pol::G);
}

template <class Pol, int IN>
static size_t frag_table_bytes() {
    return align_up((size_t)Shape<Pol, IN>::ALL_FRAGS * sizeof(typename Pol::FE));
}

template <class Pol>
static size_t frag_table_bytes_for(int in) {
    switch (in) {
        case 8: return frag_table_bytes<Pol, 8>();
        case 16: return frag_table_bytes<Pol, 16>();
        case 32: return frag_table_bytes<Pol, 32>();
        default: return frag_table_bytes<Pol, 64>();
    }
}

template <class Pol, int IN>
static hipError_t backward_t(const MlpBatch& b, int blocks, int out, double in_scale, double feat_scale,
                             double param_scale, void* ws, hipStream_t s) {
    const size_t lds = lds_backward<Pol, IN>(out);
    auto kern = k_mlp_backward<Pol, IN>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    using V = typename Pol::V;
    using G = typename Pol::G;
    using FE = typename Pol::FE;
    using Sh = Shape<Pol, IN>;
    // workspace: [per-block partial rows | per-span fragment tables (FP32/BF16)]
    FE* frags = nullptr;
    const int64_t stride = (int64_t)(frag_table_bytes<Pol, IN>() / sizeof(FE));
    if constexpr (!std::is_same<Pol, PolF64>::value) {
        frags = reinterpret_cast<FE*>(static_cast<char*>(ws) + align_up(partial_rows_bytes<Pol>(IN, out, blocks)));
        hipLaunchKernelGGL((k_mlp_frags<Pol, IN>), dim3((Sh::ALL_FRAGS + 255) / 256, b.count), dim3(256), 0, s, b,
                           out, frags, stride);
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kMlpBlock), lds, s, b, out, (V)in_scale, (V)feat_scale,
                       static_cast<G*>(ws), frags, stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const ParamOff po(IN, out);
    const int rows_per_block = std::is_same<Pol, PolF64>::value ? kWaves : 1;
    hipLaunchKernelGGL(k_mlp_reduce<G>, dim3((po.P + kRedParams - 1) / kRedParams, b.count),
                       dim3(kRedParams * kRedGroups), 0, s, b, static_cast<const G*>(ws), rows_per_block, po.P,
                       (G)param_scale);
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
    return mlp_blocks((int)(queries < 2147483647 ? queries : 2147483647), cap);
}

size_t mlp_partial_bytes(h4d_dtype dt, int in, int out, int blocks, int spans) {
    switch (dt) {
        case H4D_F32: return align_up(partial_rows_bytes<PolF32>(in, out, blocks)) + spans * frag_table_bytes_for<PolF32>(in);
        case H4D_BF16: return align_up(partial_rows_bytes<PolBF16>(in, out, blocks)) + spans * frag_table_bytes_for<PolBF16>(in);
        default: return partial_rows_bytes<PolF64>(in, out, blocks);
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
                               void* d_params, void* ws, hipStream_t s, bool overwrite) {
    if (dlstride != lstride || dqstride != qstride) return hipErrorInvalidValue;  // d_feat shares feat's layout
    const int blocks = mlp_blocks_for(dt, true, n);
    MlpBatch b = single(params, feat, nullptr, d_out, d_feat, d_params, F, lstride, qstride, n, blocks);
    b.overwrite = overwrite ? 1 : 0;
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
