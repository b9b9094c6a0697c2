// Internal declarations shared by the host API and the HIP kernels of libhash4d.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hash4d.h"

namespace h4d {

// Grid description as the kernels see it: passed by value as a kernel argument,
// so every per-level field is a uniform (scalar) load from the kernarg segment.
struct DevGrid {
    int32_t L;
    int32_t F;
    uint32_t T;          // rows of a hashed level
    uint32_t tmask;      // T - 1 when T is a power of two, else 0
    uint32_t dense_bits; // bit l set: level l is dense
    uint32_t prime[4];
    int32_t res_s[H4D_MAX_LEVELS];
    int32_t res_t[H4D_MAX_LEVELS];
    uint32_t off[H4D_MAX_LEVELS]; // first row of level l (E F < 2^31, so rows fit 32 bits)
    uint32_t rows;                // E, rows of the whole table
};

// The 3D grid of G_3D as its kernel sees it (passed by value).
struct DevGrid3 {
    int32_t L;
    int32_t F;
    uint32_t T;
    uint32_t tmask;      // T - 1 when T is a power of two, else 0
    uint32_t dense_bits; // bit l set: level l is dense
    uint32_t prime[3];
    int32_t res[H4D_MAX_LEVELS];
    uint32_t off[H4D_MAX_LEVELS];
    uint32_t rows;       // E
};
// G_3D forward (encode3.hip): xyz rows of `stride` (3 or 4) floats, x y z first;
// out[l lstride + q qstride + f].
hipError_t launch_encode3(const DevGrid3& g, h4d_dtype dt, const void* table, const float* xyz, int stride, int n,
                          void* out, int64_t lstride, int64_t qstride, hipStream_t s);

// Host-side conversion of a validated h4d_grid.
DevGrid to_device(const h4d_grid& g);
// Full validation of a caller-provided grid (sets the thread's last error).
h4d_status validate_grid(const h4d_grid* g);
// The thread's last-error text (api.cpp owns it).
h4d_status set_error(h4d_status st, const char* msg);
void clear_error();

// ---- encoder launchers (encode.hip) ----
// out[l * lstride + q * qstride + f]; level-major grid (blockIdx.y = level).
hipError_t launch_encode(const DevGrid& g, h4d_dtype table_dt, const void* table, const float* xyzt, int n,
                         void* out, int64_t lstride, int64_t qstride, hipStream_t s);
// Tiled (owner-computes) table scatter: one workgroup per (level, tile of
// consecutive table rows), accumulating in LDS.  level_rows[l] = rows of level l.
// eps != NULL: each query also subtracts its gradient at the corners of x + eps.
constexpr int kTileBytes = 128 * 1024;
// Level l is cut into tiles of 2^tile_shift[l] rows, sized so that the level has
// about kTilesPerLevel tiles (a tile's work is the level's updates over its tile
// count, so every level's tiles weigh about the same), at most max_rows rows
// (kTileBytes of gradient).  Tile t of level l sets bit t >> bit_shift[l] of a
// query's mask (bit_shift[l] = 0 while the level has at most 32 tiles).
constexpr int kTilesPerLevel = 32;
struct TileMap {
    int32_t max_rows;
    int32_t tile_start[H4D_MAX_LEVELS + 1];
    int32_t level_rows[H4D_MAX_LEVELS];
    int32_t tile_shift[H4D_MAX_LEVELS];
    int32_t bit_shift[H4D_MAX_LEVELS];
    // Bit l set: on level l both corners of every x-pair lie in the same full tile
    // (hashed, T a power of two of at least one tile, pi_1 = 1 and 2 N_s <= tile
    // rows: the pair's hashes differ only in bits below log2(2 N_s)).
    uint32_t pair_cotiled;
    // Bit l set: the mask pass also stores, per (query, level), the tile of each of
    // the eight x-pairs (one byte each), and the scatter visits a query's pairs in
    // its tile from those bytes.  Levels with pair_cotiled and at most 256 tiles,
    // when make_tile_map is asked for them.
    uint32_t pair_words;
};
TileMap make_tile_map(const DevGrid& g, const int64_t* level_rows, int F, int gbytes, bool pair_words = false);
// The scatter's tile masks: one 32-bit mask per (query, level), level-major with the
// query count padded to a multiple of four so that every level starts on a 16-byte
// boundary (the scan reads four masks per load); the per-pair tile bytes follow, 8
// bytes per (query, level) in the same order, then the load-balance plan.
constexpr int64_t mask_stride(int64_t n) { return (n + 3) & ~(int64_t)3; }
size_t scatter_ws_bytes(const DevGrid& g, const int64_t* level_rows, int n);
// A second feature gradient for the pair form (eps set): added, times scale, at x's
// corners only.  src == nullptr: none.
struct MainGradArg {
    const void* src = nullptr;
    int64_t lstride = 0, qstride = 0;
    double scale = 0.0;
};
hipError_t launch_scatter_tiled(const DevGrid& g, const int64_t* level_rows, h4d_dtype grad_dt, const float* xyzt,
                                const float* eps, int n, const void* src, int64_t lstride, int64_t qstride,
                                double scale, void* d_table, void* mask_ws, hipStream_t s, bool overwrite = false,
                                const MainGradArg& main = MainGradArg{}, int32_t* nonfinite = nullptr);
// The static workspace of hash4d_encode_backward_noalloc: kStaticScratchBytes of
// device memory per GPU (a file-scope array), its address on the current device.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
hipError_t static_scratch(void** ptr);
hipError_t launch_corner_indices(const DevGrid& g, const float* xyzt, int n, int32_t* rows, float* w,
                                 hipStream_t s);
// Fused Adam step + optional BF16 copy + gradient zeroing (optim.hip); row in {1,2,4,8}.
hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t count, int row, double lr, double beta1,
                       double beta2, double eps, int step, double grad_scale, uint16_t* lo, bool lazy, bool zero,
                       hipStream_t s);
// Collision census of one level (census.hip).
size_t census_workspace_bytes(int64_t n, int64_t level_rows);
hipError_t launch_census(const DevGrid& g, int l, int64_t level_rows, const float* xyzt, int n, int64_t* counts,
                         void* ws, hipStream_t s);
// Dynamic-static split and static constraint (decompose.hip).
size_t decompose_workspace_bytes(int64_t n);
hipError_t launch_decompose(const float* dp, int64_t n, double k_percent, float lam_s, int32_t* dyn_idx,
                            int32_t* n_dynamic, uint8_t* is_dyn, float* loss, float* d_dp, void* ws, hipStream_t s);
// d_xyzt[q] += scale * d<f_h, d_feat>/dx (encode_input.hip).
// ws (FP32 / BF16 tables; at least input_grad_workspace_bytes, 16-byte aligned):
// the two-pass, level-placed form; nullptr (or FP64): one pass, one thread per query.
hipError_t launch_encode_input_grad(const DevGrid& g, h4d_dtype dt, const void* table, const float* xyzt, int n,
                                    const void* d_feat, int64_t lstride, int64_t qstride, double scale, void* d_xyzt,
                                    hipStream_t s, void* ws = nullptr);
size_t input_grad_workspace_bytes(int L, int n);

// ---- decoder launchers (mlp.hip) ----
constexpr int kMaxMlpSpans = 16;

// Feature k of query q: feat[(k / F) lstride + q qstride + k % F].
struct FeatView {
    int64_t lstride, qstride;
    int logF;
    __device__ int64_t at(int q, int k) const {
        return (int64_t)(k >> logF) * lstride + (int64_t)q * qstride + (k & ((1 << logF) - 1));
    }
};

// One scene of a decoder launch.  Its `segs` segments (for instance its timestamps)
// lie back to back: segment s of feat / d_feat starts feat_seg * s elements in, of
// delta / d_out out_seg * s elements in; fv addresses features inside a segment.
// Workgroups [block0, block1) of the persistent grid work on this scene only, so
// each builds its parameter fragments once.
struct MlpSpan {
    const void* params;
    const void* feat;
    void* delta;
    const void* d_out;
    void* d_feat;
    void* d_params;
    int64_t feat_seg, out_seg;
    FeatView fv;
    int n, segs, block0, block1;
};

struct MlpBatch {
    MlpSpan s[kMaxMlpSpans];
    int count;
    int overwrite;  // 1: d_params is written (=) instead of accumulated (+=)
    int* nonfinite; // non-NULL: += the non-finite d_params values written
};

// Persistent-grid size of the decoder kernels for a total of `queries` queries.
int mlp_blocks_for(h4d_dtype dt, bool backward, int64_t queries);
// Workspace of the decoder backward for a grid of `blocks` workgroups: one partial
// row of the parameter gradient per workgroup (`spans` does not change it).
size_t mlp_partial_bytes(h4d_dtype dt, int in, int out, int blocks, int spans);
hipError_t launch_mlp_forward_batch(h4d_dtype dt, int in, int out, const MlpBatch& b, int blocks, hipStream_t s);
hipError_t launch_mlp_backward_batch(h4d_dtype dt, int in, int out, const MlpBatch& b, int blocks, double in_scale,
                                     double feat_scale, double param_scale, void* ws, hipStream_t s);
// Features / feature gradients are addressed as feat[(k / F) lstride + q qstride + k % F].
size_t mlp_workspace_bytes(h4d_dtype dt, int in, int out, int n);
hipError_t launch_mlp_forward(h4d_dtype dt, int in, int out, const void* params, const void* feat, int F,
                              int64_t lstride, int64_t qstride, int n, void* delta, hipStream_t s);
// d_out is multiplied by in_scale on load; d_feat is written times feat_scale;
// d_params += (or, with overwrite, =) param_scale * sum of the per-block partial gradients.
hipError_t launch_mlp_backward(h4d_dtype dt, int in, int out, const void* params, const void* feat, int F,
                               int64_t lstride, int64_t qstride, int n, const void* d_out, double in_scale,
                               double feat_scale, double param_scale, void* d_feat, int64_t dlstride,
                               int64_t dqstride, void* d_params, void* ws, hipStream_t s, bool overwrite = false,
                               int32_t* nonfinite = nullptr);

// ---- precision helpers (precision.hip) ----
hipError_t launch_cast_bf16(const float* src, uint16_t* dst, int64_t count, hipStream_t s);
// p[0, words) = 0 (32-bit words) with a kernel, so that it may be captured in a graph.
hipError_t launch_zero_words(void* p, int64_t words, hipStream_t s);
hipError_t launch_count_nonfinite(const float* p, int64_t count, int32_t* counter, hipStream_t s);
hipError_t launch_deform_apply(const float* delta, int n, int out, const float* x, const float* r, const float* s,
                               float* xo, float* ro, float* so, hipStream_t st);

// ---- smoothness regulariser (smooth.hip) ----
// Loss (+=) and, if d_out != NULL, the level-major difference G(x) - G(x + eps).
hipError_t launch_smoothness(const DevGrid& g, h4d_dtype dt, const void* table, const float* xyzt, const float* eps,
                             int n, double lam, void* loss, void* d_out, hipStream_t s);

// ---- roofline probes (probe.hip) ----
hipError_t launch_probe_gather(const void* table, uint32_t rows, int row_bytes, int64_t n_loads, uint32_t seed,
                               float* sink, hipStream_t s);
hipError_t launch_probe_scatter(float* table, uint32_t rows, int64_t n_updates, uint32_t seed, int mode,
                                hipStream_t s);
hipError_t launch_probe_copy(const void* src, void* dst, int64_t bytes, hipStream_t s);
hipError_t launch_probe_lds_atomic(int blocks, int per_thread, int active, uint32_t seed, int mode, float* sink,
                                   hipStream_t s);

}  // namespace h4d
