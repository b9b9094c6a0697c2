/*
 * hash4d.h -- C ABI of libhash4d.so, the MI355X (gfx950) implementation of the
 * DASH 4D hash deformation path (arXiv 2507.19141, Section 4.2 and Section 4.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers marked (host) are host memory; every other data pointer is device
 *    memory allocated and owned by the caller.  The library never frees or keeps
 *    a caller pointer after the call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *    enqueued asynchronously on it; arguments are validated synchronously first.
 *  - Every call returns an h4d_status.  On a negative status nothing has been
 *    enqueued and h4d_last_error() (thread-local, static storage) says why.
 *  - n == 0 is valid and enqueues nothing.  n must not exceed 2^31 - 2^16 (query
 *    counts padded to whole workgroups stay inside 32-bit kernel arithmetic).
 *  - Gradient outputs ACCUMULATE (+=) unless stated otherwise, so the caller
 *    zeroes them first.
 *  - Tables [E, F] are aligned to their row size, at most 16 bytes (H4D_EINVAL
 *    otherwise).
 *  - Positions `xyzt` are FP32 [n, 4] (x, y, z, t), 16-byte aligned.  Values are
 *    clamped to [0, 1] (NaN counts as 0); normalising scene coordinates into the
 *    unit cube is the caller's job.
 *  - No entry point allocates device memory.  Scratch space, where needed, is a
 *    caller-provided workspace whose size a *_workspace_bytes call reports; it
 *    must be 16-byte aligned (H4D_EINVAL otherwise).
 */
#ifndef HASH4D_H
#define HASH4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define H4D_MAX_LEVELS 32
#define H4D_HIDDEN 64     /* decoder trunk width */
#define H4D_MAX_OUT 16    /* decoder output rows, padded */

typedef enum {
    H4D_OK = 0,
    H4D_EINVAL = -1,        /* invalid argument (null pointer, bad size, bad grid, misalignment) */
    H4D_EUNSUPPORTED = -2,  /* valid but not built (e.g. an unsupported width or dtype) */
    H4D_EHIP = -3,          /* the HIP runtime reported an error; its text is in h4d_last_error() */
    H4D_ENOPLAN = -4        /* a batched plan handle is null or was destroyed */
} h4d_status;

typedef enum {
    H4D_F32 = 0,    /* plain FP32 path */
    H4D_BF16 = 1,   /* BF16 tables / BF16 MFMA decoder with FP32 accumulation */
    H4D_F64 = 2     /* FP64 instantiation, meant for finite-difference gradient checks */
} h4d_dtype;

typedef enum {
    H4D_QUERY_MAJOR = 0,  /* features [n, L F]: feature l F + f of query q at q L F + l F + f */
    H4D_LEVEL_MAJOR = 1   /* features [L, n, F]: at l n F + q F + f (coalesced per level) */
} h4d_layout;

/* Or-ed into the layout argument of hash4d_encode_backward and deform_mlp_backward:
 * the gradient output (d_table, d_params) is WRITTEN, every element, instead of
 * accumulated, so the caller need not zero it first (n = 0 writes zeros). */
#define H4D_GRAD_OVERWRITE 0x100

typedef enum {
    H4D_SCHEDULE_GEOMETRIC = 0, /* Eq. 7: N_l = floor(N_min b^l), b = (N_max/N_min)^(1/(L-1)) */
    H4D_SCHEDULE_DOUBLING = 1   /* N_l = min(N_min 2^l, N_max) */
} h4d_schedule;

/* Multiresolution 4D grid (Section 4.2).  Host struct, filled by h4d_grid_init.
 * Level l has spatial resolution res_s[l] along x, y, z and temporal resolution
 * res_t[l] along t, so (res_s+1)^3 (res_t+1) vertices.  A level whose vertices fit
 * in T rows is stored densely (collision-free, x fastest, then y, z, t) in exactly
 * that many rows; every other level is hashed (Eq. 8) into T rows.  The table is
 * one [E, F] row-major array, E = offset[L]; level l owns rows
 * [offset[l], offset[l+1]). */
typedef struct {
    int32_t L;                          /* levels, 1..32 */
    int32_t F;                          /* features per row: 1, 2, 4 or 8 */
    int64_t T;                          /* rows of a hashed level, 1..2^30 */
    int32_t res_s[H4D_MAX_LEVELS];      /* 1..2^24 */
    int32_t res_t[H4D_MAX_LEVELS];      /* 1..2^24 */
    int64_t offset[H4D_MAX_LEVELS + 1]; /* first row of each level; offset[L] = E */
    uint8_t dense[H4D_MAX_LEVELS];      /* 1 = dense level */
    uint32_t prime[4];                  /* hash multipliers for x, y, z, t */
} h4d_grid;

/* Multiresolution 3D grid of G_3D (Section 4.1, Eq. 3): the hash encoding of the
 * canonical positions that feeds the motion decoder of the dynamic-static split.
 * Host struct, filled by h4d_grid3_init.  Level l has resolution res[l] along x,
 * y and z, so (res+1)^3 vertices; a level whose vertices fit in T rows is stored
 * densely (x fastest, then y, z), every other level is hashed into T rows with the
 * first three primes of the 4D grid.  Table [E, F], E = offset[L]. */
typedef struct {
    int32_t L;                          /* levels, 1..32 */
    int32_t F;                          /* features per row: 1, 2, 4 or 8 */
    int64_t T;                          /* rows of a hashed level, 1..2^30 */
    int32_t res[H4D_MAX_LEVELS];        /* 1..2^24 */
    int64_t offset[H4D_MAX_LEVELS + 1]; /* first row of each level; offset[L] = E */
    uint8_t dense[H4D_MAX_LEVELS];      /* 1 = dense level */
    uint32_t prime[3];                  /* hash multipliers for x, y, z */
} h4d_grid3;

/* Decoder shape (Section 4.2, Eq. 9 and the multi-head decoder).  in = L F,
 * hidden = 64, out = 10 (dx 3 | drot 4 | dscale 3).  Parameters are one flat
 * array in the order W1[hidden, in], b1[hidden], W2[hidden, hidden], b2[hidden],
 * W3[out, hidden], b3[out], weights row-major [out, in]. */
typedef struct {
    int32_t in;       /* 8, 16, 32 or 64 */
    int32_t hidden;   /* must be 64 */
    int32_t out;      /* 1..16 */
} h4d_mlp;

/* Text of the last error on this thread ("" if none).  Never NULL. */
const char* h4d_last_error(void);

/* Library version string. */
const char* h4d_version(void);

/* ---------------------------------------------------------------- grid ---- */

/* Level resolutions of one dimension (Section 4.2, Eq. 7).  Geometric: the
 * progression of Eq. 7 with its level exponent, evaluated in FP64 with a 1e-9
 * relative guard before the floor, last level pinned to n_max.  Doubling:
 * min(n_min 2^l, n_max).  res_out (host) receives L values.
 * EINVAL: L not in 1..32, n_min < 1, n_max < n_min, n_max > 2^24, res_out NULL. */
h4d_status h4d_grid_schedule(int32_t L, int32_t n_min, int32_t n_max, int32_t rule, int32_t* res_out);

/* Fill *g (host) from explicit per-level resolutions (host arrays of L values):
 * dense flags, offsets and the default primes (1, 2654435761, 805459861,
 * 3266489917).  EINVAL on any out-of-range field or if E F >= 2^31. */
h4d_status h4d_grid_init(h4d_grid* g, int32_t L, int32_t F, const int32_t* res_s, const int32_t* res_t, int64_t T);

/* Rows E of the table described by *g (host), or -1 if *g is invalid. */
int64_t h4d_grid_rows(const h4d_grid* g);

/* ------------------------------------------------------------- encoder ---- */

/* Forward encoder G_4D (Section 4.2, Eqs. 8-9).  For each query and level: scale
 * x by the level resolution in FP32 (round to nearest, no fused multiply-add),
 * take the 16 corners of the hypervoxel, index them (dense or hashed), gather F
 * features per corner and interpolate quadrilinearly.
 *   table   [E, F] of table_dt (F32, BF16 bit patterns, or F64)
 *   feat    n L F values in `layout`; FP32 for F32/BF16 tables, FP64 for F64.
 * Written, not accumulated.  Deterministic (no atomics). */
h4d_status hash4d_encode(const h4d_grid* g, h4d_dtype table_dt, const void* table,
                         const float* xyzt, int64_t n, h4d_layout layout, void* feat, void* stream);

/* Fill *g (host) for G_3D from explicit per-level resolutions (host array of L
 * values): dense iff (res+1)^3 <= T, offsets, primes (1, 2654435761, 805459861).
 * EINVAL on any out-of-range field or if E F >= 2^31. */
h4d_status h4d_grid3_init(h4d_grid3* g, int32_t L, int32_t F, const int32_t* res, int64_t T);

/* The 3D encoder G_3D of Section 4.1 (Eq. 3): per position and level, scale by the
 * level resolution in FP32 (as hash4d_encode does), take the 8 corners of the
 * voxel, gather F features per corner and interpolate trilinearly; positions are
 * clamped to [0, 1] (NaN to 0).
 *   table  [E, F] of table_dt (F32, BF16 bit patterns, or F64)
 *   xyz    n rows of `stride` FP32 values (3: [n, 3]; 4: [n, 4] with the fourth
 *          ignored, 16-byte aligned), x, y, z first
 *   feat   n L F values in `layout`; FP32 for F32/BF16 tables, FP64 for F64.
 * Written, not accumulated.  Deterministic (no atomics). */
h4d_status hash3d_encode(const h4d_grid3* g, h4d_dtype table_dt, const void* table, const float* xyz,
                         int32_t stride, int64_t n, h4d_layout layout, void* feat, void* stream);

/* Backward of hash4d_encode with respect to the table (the exact transpose of the
 * interpolation in Eq. 9): d_table[row_c, f] += grad_scale * w_c * d_feat[q, l F + f]
 * over every query, level and corner.  Corners and weights are recomputed from
 * xyzt.  grad_dt F32: d_feat and d_table are FP32; F64: both FP64.
 *   d_feat  n L F values in `layout`     d_table [E, F] (+=; = with H4D_GRAD_OVERWRITE
 *           in layout, which writes every row, zeros where no corner lands)
 * Owner-computes scatter: one workgroup per (level, tile of consecutive table rows)
 * sums its rows' updates in LDS and adds them to d_table; no device-wide atomics.
 * A pre-pass writes a per-(query, level) mask of touched tiles (and, on hashed
 * levels, each x-pair's tile) into `workspace` (device, 16-byte aligned, at least
 * hash4d_encode_backward_workspace_bytes) so that each tile only works on the
 * queries that reach it; it also counts the queries per tile of the dense levels,
 * and a tile that many queries reach is split over several workgroups whose partial
 * tiles the workspace holds.  The LDS adds (one FP32 rounding each) make the
 * summation order, hence the last bits, vary run to run. */
size_t hash4d_encode_backward_workspace_bytes(const h4d_grid* g, int64_t n);
h4d_status hash4d_encode_backward(const h4d_grid* g, h4d_dtype grad_dt, const float* xyzt, int64_t n,
                                  h4d_layout layout, const void* d_feat, float grad_scale, void* d_table,
                                  void* workspace, size_t ws_bytes, void* stream);
/* hash4d_encode_backward that also checks its output for the loss-scaled (BF16) form
 * (the overflow test of mixed-precision training: a non-finite gradient skips the
 * step and lowers the loss scale): *nonfinite (device int32) += the number of NaN or
 * infinite values among the d_table values the call writes; with H4D_GRAD_OVERWRITE
 * that is every value of d_table, so the count replaces a separate pass over it.
 * Otherwise as hash4d_encode_backward.  nonfinite: non-NULL, 4-byte aligned. */
h4d_status hash4d_encode_backward_checked(const h4d_grid* g, h4d_dtype grad_dt, const float* xyzt, int64_t n,
                                          h4d_layout layout, const void* d_feat, float grad_scale, void* d_table,
                                          void* workspace, size_t ws_bytes, int32_t* nonfinite, void* stream);

/* hash4d_encode_backward without a workspace argument and without any device
 * allocation, for callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments (minus
 * workspace / ws_bytes), kernels and results as hash4d_encode_backward.  The tile
 * masks go to a static workspace of 64 MiB (67108864 bytes) per GPU, a file-scope
 * device array that each GPU holds from the library's load until the process ends;
 * a call whose hash4d_encode_backward_workspace_bytes(g, n) exceeds it returns
 * H4D_EINVAL and launches nothing.  No call reads what an earlier call left there.
 * Every call on one GPU shares that array: calls that overlap on one GPU (two
 * streams, or two host threads, without ordering between them) race and give wrong
 * gradients, so the caller orders them. */
h4d_status hash4d_encode_backward_noalloc(const h4d_grid* g, h4d_dtype grad_dt, const float* xyzt, int64_t n,
                                          h4d_layout layout, const void* d_feat, float grad_scale, void* d_table,
                                          void* stream);

/* Gradient of the encoder with respect to its input positions, for callers that
 * learn the canonical positions through the encoder (the derivative of Eq. 9):
 *   d_xyzt[q, d] += grad_scale * sum_l sum_f d_feat[q, l F + f] * d f_h[l F + f] / d x_d
 * with d w_c / d x_d = +-N_d times the other three factors of w_c, in the cell the
 * forward selects (lower corner min(floor(x N), N - 1)); zero along d where the
 * clamp is active (x_d < 0, x_d > 1 or NaN), the inner one-sided derivative at 0
 * and 1.  table_dt F32 / BF16: d_feat and d_xyzt FP32; F64: both FP64.
 *   table [E, F]   d_feat n L F values in `layout`   d_xyzt [n, 4] (+=)
 * workspace NULL (or table_dt F64): one thread per query walks the levels.
 * Otherwise `workspace` (device, 16-byte aligned, at least
 * hash4d_encode_backward_input_workspace_bytes, i.e. L n 16 bytes) holds each
 * level's four terms: one pass per (query, level), placed on the XCDs level by
 * level, then a pass that sums the levels in order.  Either way every (q, d) output
 * has one writer. */
size_t hash4d_encode_backward_input_workspace_bytes(const h4d_grid* g, h4d_dtype table_dt, int64_t n);
h4d_status hash4d_encode_backward_input(const h4d_grid* g, h4d_dtype table_dt, const void* table,
                                        const float* xyzt, int64_t n, h4d_layout layout, const void* d_feat,
                                        float grad_scale, void* d_xyzt, void* workspace, size_t ws_bytes,
                                        void* stream);

/* Test hook: the table row (level offset included) and FP32 weight of the 16
 * corners of every query and level.  Corner c is upper along x, y, z, t iff bit
 * 0, 1, 2, 3 of c is set.
 *   rows [n, L, 16] int32      w [n, L, 16] FP32 (either may be NULL) */
h4d_status hash4d_corner_indices(const h4d_grid* g, const float* xyzt, int64_t n,
                                 int32_t* rows, float* w, void* stream);

/* Deformation of Eq. 10 from the decoder output: xyz' = xyz + delta[:, 0:3],
 * rot' = rot + delta[:, 3:7] (the rotation increment added as is), scale' =
 * scale + delta[:, 7:10], each one FP32 add.  xyz [n, 3], rot [n, 4], scale [n, 3],
 * delta [n, out] with out >= 10; outputs may alias the inputs.  The gradient of
 * this step is the identity, so it has no backward entry point. */
h4d_status hash4d_deform_apply(const float* delta, int64_t n, int32_t out, const float* xyz, const float* rot,
                               const float* scale, float* xyz_out, float* rot_out, float* scale_out, void* stream);

/* ---------------------------------------------------------- smoothness ---- */

/* Smoothness regulariser of Section 4.3 (Eq. 11) and its table gradient:
 * x~ = clamp(x + eps) (FP32 add), d = G(x) - G(x~) over all L F features,
 *   *loss   += lambda / n * sum_q ||d_q||^2
 *   d_table += (2 lambda / n) (d w at x's corners - d w~ at x~'s corners)
 * Both encodes are recomputed per query and level, nothing is kept between calls.
 * d_table may be NULL (loss only, no workspace needed).  Otherwise `workspace`
 * (device, smoothness_workspace_bytes) receives d and the scatter's tile masks, and
 * the gradient is added by the tiled scatter.  table_dt as hash4d_encode; loss and d_table are FP32 (FP64
 * for F64).  eps: FP32 [n, 4], 16-byte aligned. */
size_t smoothness_workspace_bytes(const h4d_grid* g, h4d_dtype table_dt, int64_t n);
h4d_status smoothness_reg(const h4d_grid* g, h4d_dtype table_dt, const void* table, const float* xyzt,
                          const float* eps, int64_t n, float lambda, void* loss, void* d_table, void* workspace,
                          size_t ws_bytes, void* stream);

/* The table gradient of a training step with the smoothness term, in one scatter:
 * hash4d_encode_backward of d_feat (Eq. 9's transpose) plus smoothness_reg's
 * gradient (Eq. 11), that is
 *   *loss   += lambda / n * sum_q ||d_q||^2
 *   d_table += grad_scale A^T d_feat + (2 lambda / n) (d w at x's corners - d w~ at x~'s)
 * The sum is exact up to rounding order: every update of x's corners carries
 * (2 lambda / n) d + grad_scale d_feat, every update of x~'s corners -(2 lambda / n) d.
 * One scatter over the two corner sets replaces the plain scatter plus the pair
 * scatter of the two separate calls.  d_feat: n L F values in `layout` (FP32; FP64
 * for F64); layout may carry H4D_GRAD_OVERWRITE (d_table written; n = 0 writes
 * zeros).  Other arguments as smoothness_reg; here d_table, d_feat and the
 * workspace (smoothness_workspace_bytes) are required. */
h4d_status hash4d_encode_backward_smooth(const h4d_grid* g, h4d_dtype table_dt, const void* table, const float* xyzt,
                                         const float* eps, int64_t n, h4d_layout layout, const void* d_feat,
                                         float grad_scale, float lambda, void* loss, void* d_table, void* workspace,
                                         size_t ws_bytes, void* stream);

/* ----------------------------------------------------- precision form ---- */

/* dst[i] = BF16 (round to nearest even, NaN kept quiet) of the FP32 master src[i],
 * as uint16 bit patterns: the per-step copy of tables or decoder parameters the
 * BF16 form reads.  count elements; dst may not overlap src. */
h4d_status h4d_cast_bf16(const float* src, uint16_t* dst, int64_t count, void* stream);

/* ----------------------------------------------- collision census ---- */

/* Collision census of level `level` for n queries: counts[0] = V, the distinct
 * corner vertices, counts[1] = R, the distinct table rows they map to (device int64
 * [2], written).  On a dense level R = V; on a hashed level V - R vertices share
 * their row with another: the cost of hashing more points that the paper's "w/o dec"
 * ablation shows (Section 5.3).  Vertex ids take 16 bits per coordinate, so the
 * level needs N_s, N_t < 65535 (H4D_EUNSUPPORTED otherwise).  workspace: device,
 * 16-byte aligned, hash4d_collision_workspace_bytes(g, level, n) (a set of at least
 * 32 n slots of 8 bytes and a bitmap of the level's rows).  Exact and deterministic
 * counts; uses device atomics (instrumentation, not the training path). */
size_t hash4d_collision_workspace_bytes(const h4d_grid* g, int32_t level, int64_t n);
h4d_status hash4d_collision_census(const h4d_grid* g, int32_t level, const float* xyzt, int64_t n, int64_t* counts,
                                   void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------- dynamic-static split ---- */

/* Self-supervised split of Section 4.1 (the step before the 4D path: it decides
 * which Gaussians the path deforms) and the static constraint of Eq. 5.
 *   dp [n, 3] FP32: each Gaussian's linear-motion vector (Eq. 4, p(t) = p + t dp),
 *   e.g. deform_mlp_forward with out = 3 on a 3D hash encoding of the positions.
 * Keys are the FP32 squares s = (dx^2 + dy^2) + dz^2 (no fused multiply-add),
 * ordered by bit pattern (NaN above +Inf).  n_d = floor(k_percent / 100 * n);
 * the threshold is the (n_d + 1)-th largest key (none if n_d >= n) and a Gaussian
 * is dynamic iff its key is strictly greater (ties stay static).  Outputs (each may
 * be NULL): dynamic_idx [n] int32 gets the dynamic indices in ascending order;
 * *n_dynamic (device int32) their count; is_dynamic [n] uint8 0/1;
 * *loss (device FP32) += lambda_s / N_s * sum over static ||dp|| (nothing if N_s = 0);
 * d_dp [n, 3] += its gradient lambda_s / N_s * dp / ||dp|| on static rows (0 where
 * dp = 0).  workspace: device, 16-byte aligned, hash4d_decompose_workspace_bytes(n).
 * The selection and the indices are exact and deterministic; the loss sums in a
 * fixed order. */
size_t hash4d_decompose_workspace_bytes(int64_t n);
h4d_status hash4d_decompose(const float* dp, int64_t n, float k_percent, float lambda_s, int32_t* dynamic_idx,
                            int32_t* n_dynamic, uint8_t* is_dynamic, float* loss, float* d_dp, void* workspace,
                            size_t ws_bytes, void* stream);

/* ------------------------------------------------------ optimiser step ---- */

/* Hyper-parameters of one Adam step (host struct). */
typedef struct {
    float lr, beta1, beta2, eps;
    int32_t step;        /* t >= 1: the bias corrections use beta^t */
    float grad_scale;    /* the gradient is multiplied by this first (1 / loss scale) */
} h4d_adam;

#define H4D_ADAM_LAZY 1       /* rows whose whole gradient is zero keep parameters and moments */
#define H4D_ADAM_ZERO_GRAD 2  /* grad[] is set to 0 after use, ready for the next step */

/* One Adam step over an FP32 master array (a table [E, F] or a decoder parameter
 * vector), fused with the BF16 copy the next step's BF16 form reads and with the
 * zeroing of the gradient: the step after the table and decoder gradients of
 * training under Eq. 12 (the paper leaves the optimiser to its 3DGS base).
 *   g = grad * grad_scale;  m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *   p -= lr / (1 - b1^t) * m / (sqrt(v) / sqrt(1 - b2^t) + eps)
 * params, grad, m, v: `count` FP32 values each, 16-byte aligned, not overlapping;
 * bf16_out: NULL or `count` uint16 (8-byte aligned) receiving RNE BF16 of the new
 * params.  row: the row length for H4D_ADAM_LAZY (1, 2, 4 or 8; count a multiple of
 * it), ignored otherwise.  H4D_EINVAL on bad sizes, alignment or hyper-parameters. */
h4d_status h4d_adam_step(float* params, float* grad, float* m, float* v, int64_t count, int32_t row,
                         const h4d_adam* hp, uint16_t* bf16_out, int32_t flags, void* stream);

/* *counter += number of NaN or Inf values in p[0, count) (the overflow check of
 * dynamic loss scaling).  The caller zeroes *counter (device int32). */
h4d_status h4d_count_nonfinite(const float* p, int64_t count, int32_t* counter, void* stream);

/* ------------------------------------------------------------- decoder ---- */

/* Bytes of workspace deform_mlp_backward needs for n queries (split-N partial
 * weight gradients: one row of P parameters per persistent block).  0 if *m is
 * invalid. */
size_t deform_mlp_workspace_bytes(const h4d_mlp* m, h4d_dtype dt, int64_t n);

/* Decoder forward (Section 4.2: the trunk phi_d of Eq. 9, then the position,
 * rotation and scale heads): h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2),
 * delta = W3 h2 + b3, computed on MFMA tiles of 16 queries.
 *   dt      F32: params/feat/out FP32.  BF16: params BF16 bit patterns, feat and out
 *           FP32, activations rounded to BF16 for the MFMA, FP32 accumulation.
 *           F64: everything FP64.
 *   feat    [n, in] (H4D_QUERY_MAJOR) or [in / F, n, F] (H4D_LEVEL_MAJOR, F in {1,2,4,8}
 *           dividing in; F is ignored for query-major)
 *   out     [n, out] (written) */
h4d_status deform_mlp_forward(const h4d_mlp* m, h4d_dtype dt, const void* params, const void* feat, int64_t n,
                              h4d_layout layout, int32_t F, void* out, void* stream);

/* Decoder backward: gradients of <delta, loss_scale * d_out> (ReLU passes gradient
 * where its input is > 0).  d_feat [n, in] is WRITTEN as grad_scale times the
 * feature gradient; d_params (FP32, FP64 for F64) ACCUMULATES (with H4D_GRAD_OVERWRITE
 * in layout: is written with) grad_scale times the
 * parameter gradient.  The forward is recomputed from feat; weight gradients are
 * reduced over queries per persistent block into `workspace` (device, at least
 * deform_mlp_workspace_bytes) and then summed by a second kernel, so the result is
 * deterministic for a given n.
 *   d_out [n, out] (FP32, FP64 for F64); feat and d_feat in (layout, F) as in
 *   deform_mlp_forward. */
h4d_status deform_mlp_backward(const h4d_mlp* m, h4d_dtype dt, const void* params, const void* feat, int64_t n,
                               h4d_layout layout, int32_t F, const void* d_out, float loss_scale, float grad_scale,
                               void* d_feat, void* d_params, void* workspace, size_t ws_bytes, void* stream);
/* deform_mlp_backward that also checks its parameter gradient for the loss-scaled
 * (BF16) form's overflow test: *nonfinite (device int32) += the number of NaN or
 * infinite values among the d_params values it writes (all of them with
 * H4D_GRAD_OVERWRITE; n = 0 writes zeros and counts nothing).  Otherwise as
 * deform_mlp_backward.  nonfinite: non-NULL, 4-byte aligned. */
h4d_status deform_mlp_backward_checked(const h4d_mlp* m, h4d_dtype dt, const void* params, const void* feat,
                                       int64_t n, h4d_layout layout, int32_t F, const void* d_out, float loss_scale,
                                       float grad_scale, void* d_feat, void* d_params, void* workspace,
                                       size_t ws_bytes, int32_t* nonfinite, void* stream);

/* -------------------------------------------------- deformation path ---- */

/* Workspace of hash4d_deform_backward: decoder partials, the [L, n, F] feature
 * gradient and the scatter's tile masks.  0 if the arguments are invalid. */
size_t hash4d_deform_workspace_bytes(const h4d_grid* g, const h4d_mlp* m, h4d_dtype dt, int64_t n);

/* Whole forward of the deformation field for n dynamic Gaussians at their
 * timestamps: the encoder G_4D (Eqs. 8-9) followed by the decoder (delta of
 * position, rotation and scale, the increments of Eq. 10).
 *   dt      F32: FP32 table and params.  BF16: BF16 table and params (bit patterns),
 *           FP32 features.  F64: FP64 everything.
 *   feat    [L, n, F] level-major (FP32; FP64 for F64), WRITTEN: the encoder output,
 *           kept for the backward.  m->in must equal L F.
 *   delta   [n, m->out] (FP32; FP64 for F64), WRITTEN. */
h4d_status hash4d_deform_forward(const h4d_grid* g, const h4d_mlp* m, h4d_dtype dt, const void* table,
                                 const void* params, const float* xyzt, int64_t n, void* feat, void* delta,
                                 void* stream);

/* Whole backward of the deformation field: decoder backward from d_delta (scaled
 * by loss_scale on load), then the table scatter of Eq. 9's transpose.  d_table
 * [E, F] and d_params ACCUMULATE grad_scale times their gradients (FP32; FP64 for
 * F64).  feat is the buffer hash4d_deform_forward wrote.  workspace: device, at
 * least hash4d_deform_workspace_bytes. */
h4d_status hash4d_deform_backward(const h4d_grid* g, const h4d_mlp* m, h4d_dtype dt, const void* params,
                                  const float* xyzt, int64_t n, const void* feat, const void* d_delta,
                                  float loss_scale, float grad_scale, void* d_table, void* d_params,
                                  void* workspace, size_t ws_bytes, void* stream);

/* -------------------------------------------------------- batched form ---- */

#define H4D_MAX_SCENES 16
#define H4D_MAX_TIMES 8
#define H4D_MAX_TUNED 64

/* One scene of a batched plan: its own grid, table and decoder, queried at
 * n_times timestamps per step.  All pointers are device memory owned by the
 * caller and must stay valid for the plan's lifetime. */
typedef struct {
    h4d_grid grid;              /* (host) layout of this scene's table */
    int64_t n;                  /* dynamic Gaussians */
    const float* xyz;           /* [n, 4] FP32, 16-byte aligned; the 4th value is ignored */
    int32_t n_times;            /* 1..8 timestamps per step */
    float times[H4D_MAX_TIMES]; /* (host) the timestamps, in [0, 1] */
    void* table;                /* [E, F] in the plan dtype (BF16 bit patterns for BF16) */
    const float* table_master;  /* BF16 plans: optional FP32 master, rounded into `table` each step */
    void* params;               /* decoder parameters in the plan dtype */
    const float* params_master; /* BF16 plans: optional FP32 master, rounded into `params` each step */
    float* feat;                /* [n_times, L, n, F] FP32, written by the forward */
    float* delta;               /* [n_times, n, out] FP32, written by the forward */
    const float* d_delta;       /* [n_times, n, out] FP32 upstream gradient */
    float* d_table;             /* [E, F] FP32, += grad */
    float* d_params;            /* [P] FP32, += grad */
} h4d_scene_desc;

typedef struct h4d_batched_plan h4d_batched_plan;

typedef enum {
    H4D_PLAN_AUTOTUNE = 1,   /* time candidate schedules at creation and keep the fastest */
    H4D_PLAN_ZERO_GRADS = 2, /* the backward zeroes d_table / d_params first (a training step) */
    H4D_PLAN_GRAPH = 4       /* capture forward + backward into one HIP graph for hash4d_batched_run */
} h4d_plan_flags;

typedef struct {
    int32_t kernel;          /* 0 = batched encode */
    int32_t qpt, lpb, grid;  /* queries per thread, levels per work item, persistent workgroups */
    float ms;                /* measured milliseconds per launch */
} h4d_tune_result;

typedef struct {
    int64_t queries;         /* sum over scenes of n * n_times */
    int32_t segments;        /* (scene, timestamp) pairs */
    int32_t encode_qpt, encode_lpb, encode_grid;
    int32_t scatter_tiles, scatter_rows_per_tile; /* owner-computes scatter: one workgroup per tile; rows of the largest tile */
    int32_t graph;           /* 1 if a HIP graph was captured */
    int32_t n_tuned;
    h4d_tune_result tuned[H4D_MAX_TUNED];
} h4d_batched_info;

/* Build a plan for n_scenes (1..16) scenes sharing F and the decoder shape m, in
 * dt F32 or BF16.  The plan owns device memory of its own (work lists, per-segment
 * feature gradients, decoder partials; freed by destroy).  With AUTOTUNE the
 * candidate schedules (queries per thread x levels per item x grid size) of the
 * batched encode kernel are timed on `stream` with the scenes' own data (they
 * write `feat`).  The scatter runs one workgroup per (scene, level, tile of table
 * rows), accumulating in LDS over all the scene's timestamps.  With GRAPH the
 * whole step (BF16 rounding of the masters, encode, decode, decoder backward,
 * scatter, and zeroing with ZERO_GRADS) is captured into one HIP graph.
 * Backward scaling: d_delta is multiplied by loss_scale inside the kernels and the
 * gradients by 1/loss_scale (the BF16 form's loss scaling). */
h4d_status hash4d_batched_plan_create(h4d_batched_plan** plan, const h4d_scene_desc* scenes, int32_t n_scenes,
                                      const h4d_mlp* m, h4d_dtype dt, float loss_scale, int32_t flags,
                                      void* stream);
/* Forward of every (scene, timestamp): encode then decode (feat, delta). */
h4d_status hash4d_batched_forward(h4d_batched_plan* plan, void* stream);
/* Backward of every (scene, timestamp): decoder backward then table scatter. */
h4d_status hash4d_batched_backward(h4d_batched_plan* plan, void* stream);
/* One whole step: the captured graph if the plan has one, else forward + backward. */
h4d_status hash4d_batched_run(h4d_batched_plan* plan, void* stream);
/* The chosen schedule and the autotuner's measurements. */
h4d_status hash4d_batched_plan_info(const h4d_batched_plan* plan, h4d_batched_info* info);
void hash4d_batched_plan_destroy(h4d_batched_plan* plan);

/* ---------------------------------------------------- roofline probes ---- */

/* Measurement kernels for the ceilings the encoder is compared against (not part
 * of the method).  Row numbers are uniform pseudo-random, from a counter-based
 * hash of the load index and `seed`.
 * gather:  n_loads loads of one row_bytes (4 or 8) row from table[rows]; 16 loads
 *          in flight per thread.  sink: device float, written only in a case that
 *          practically never occurs (it keeps the loads alive).
 * scatter: n_updates updates, each adding 1.0f with a device atomic to both FP32
 *          values of one random 8-byte row of table[rows][2].  mode 0: any row;
 *          mode 1: a row of a 128-byte line whose index is congruent mod 8 to the
 *          XCC (accelerator complex die) the workgroup runs on, so that each line
 *          is updated from a single XCC.
 * copy:    bytes (multiple of 16) copied src -> dst with 16-byte vector accesses. */
h4d_status h4d_probe_gather(const void* table, int64_t rows, int32_t row_bytes, int64_t n_loads, uint32_t seed,
                            float* sink, void* stream);
h4d_status h4d_probe_scatter(float* table, int64_t rows, int64_t n_updates, uint32_t seed, int32_t mode,
                             void* stream);
h4d_status h4d_probe_copy(const void* src, void* dst, int64_t bytes, void* stream);
/* lds atomic: `blocks` workgroups of 1024 threads, each with a 128 KiB LDS tile;
 *          `active` of every 64 lanes each add to `per_thread` random words.
 *          mode 0: FP32 atomic add (ds_add_f32); mode 1: 32-bit integer atomic add
 *          (ds_add_u32); mode 2: FP32 add by compare-and-swap loop (the library's
 *          tile accumulation).  Returns H4D_EINVAL for any other mode. */
h4d_status h4d_probe_lds_atomic(int32_t blocks, int32_t per_thread, int32_t active, uint32_t seed, int32_t mode,
                                float* sink, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* HASH4D_H */
