// Host side of libhash4d: argument validation, the level schedule (DASH Section
// 4.2, Eq. 7), table layout, error reporting and dispatch to the HIP kernels.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "h4d_internal.h"

namespace h4d {

static thread_local std::string g_last_error;

static h4d_status fail(h4d_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

static h4d_status hip_status(hipError_t e, const char* where) {
    if (e == hipSuccess) return H4D_OK;
    return fail(H4D_EHIP, "%s: %s", where, hipGetErrorString(e));
}

static const uint32_t kPrimes[4] = {1u, 2654435761u, 805459861u, 3266489917u};
static const int64_t kMaxRes = (int64_t)1 << 24;
static const int64_t kMaxT = (int64_t)1 << 30;
static const int64_t kMaxN = 2147483647;  // element counts (features, outputs) per call
// Queries per call: 2^31 - 2^16, so that query counts padded to whole workgroups or
// MFMA tiles (n + 255, n + 15, ...) stay inside the kernels' 32-bit arithmetic.
static const int64_t kMaxQ = kMaxN - 65535;

static bool valid_F(int F) { return F == 1 || F == 2 || F == 4 || F == 8; }

// Rows of level l and whether it is dense: (N_s+1)^3 (N_t+1) <= T (evaluated in
// 128-bit integers, so no resolution up to 2^24 can overflow).
static void level_size(int64_t Ns, int64_t Nt, int64_t T, int64_t* rows, bool* dense) {
    const unsigned __int128 S = (unsigned __int128)(Ns + 1);
    const unsigned __int128 v = S * S * S * (unsigned __int128)(Nt + 1);
    *dense = v <= (unsigned __int128)T;
    *rows = *dense ? (int64_t)v : T;
}

// Full validation of a caller-provided grid struct: every field in range and the
// derived fields consistent with the resolutions.
static h4d_status check_grid(const h4d_grid* g) {
    if (!g) return fail(H4D_EINVAL, "grid pointer is NULL");
    if (g->L < 1 || g->L > H4D_MAX_LEVELS) return fail(H4D_EINVAL, "grid: L=%d outside 1..%d", g->L, H4D_MAX_LEVELS);
    if (!valid_F(g->F)) return fail(H4D_EINVAL, "grid: F=%d not in {1,2,4,8}", g->F);
    if (g->T < 1 || g->T > kMaxT) return fail(H4D_EINVAL, "grid: T=%lld outside 1..2^30", (long long)g->T);
    if (g->offset[0] != 0) return fail(H4D_EINVAL, "grid: offset[0] != 0 (struct not initialised?)");
    for (int l = 0; l < g->L; ++l) {
        if (g->res_s[l] < 1 || g->res_s[l] > kMaxRes || g->res_t[l] < 1 || g->res_t[l] > kMaxRes)
            return fail(H4D_EINVAL, "grid: level %d resolution (%d, %d) outside 1..2^24", l, g->res_s[l], g->res_t[l]);
        int64_t rows;
        bool dense;
        level_size(g->res_s[l], g->res_t[l], g->T, &rows, &dense);
        if ((g->dense[l] != 0) != dense || g->offset[l + 1] - g->offset[l] != rows)
            return fail(H4D_EINVAL, "grid: level %d layout inconsistent with its resolutions (re-run h4d_grid_init)", l);
    }
    if (g->offset[g->L] * g->F >= ((int64_t)1 << 31))
        return fail(H4D_EINVAL, "grid: table of %lld rows x %d features exceeds 2^31 elements",
                    (long long)g->offset[g->L], g->F);
    return H4D_OK;
}

// The 3D grid of G_3D: every field in range and the derived fields consistent.
static h4d_status check_grid3(const h4d_grid3* g) {
    if (!g) return fail(H4D_EINVAL, "grid3 pointer is NULL");
    if (g->L < 1 || g->L > H4D_MAX_LEVELS) return fail(H4D_EINVAL, "grid3: L=%d outside 1..%d", g->L, H4D_MAX_LEVELS);
    if (!valid_F(g->F)) return fail(H4D_EINVAL, "grid3: F=%d not in {1,2,4,8}", g->F);
    if (g->T < 1 || g->T > kMaxT) return fail(H4D_EINVAL, "grid3: T=%lld outside 1..2^30", (long long)g->T);
    if (g->offset[0] != 0) return fail(H4D_EINVAL, "grid3: offset[0] != 0 (struct not initialised?)");
    for (int l = 0; l < g->L; ++l) {
        if (g->res[l] < 1 || g->res[l] > kMaxRes)
            return fail(H4D_EINVAL, "grid3: level %d resolution %d outside 1..2^24", l, g->res[l]);
        const int64_t S = (int64_t)g->res[l] + 1;
        const unsigned __int128 v = (unsigned __int128)S * S * S;
        const bool dense = v <= (unsigned __int128)g->T;
        if ((g->dense[l] != 0) != dense || g->offset[l + 1] - g->offset[l] != (dense ? (int64_t)v : g->T))
            return fail(H4D_EINVAL, "grid3: level %d layout inconsistent with its resolution (re-run h4d_grid3_init)", l);
    }
    if (g->offset[g->L] * g->F >= ((int64_t)1 << 31))
        return fail(H4D_EINVAL, "grid3: table of %lld rows x %d features exceeds 2^31 elements",
                    (long long)g->offset[g->L], g->F);
    return H4D_OK;
}

static DevGrid3 to_device3(const h4d_grid3& g) {
    DevGrid3 d;
    memset(&d, 0, sizeof d);
    d.L = g.L;
    d.F = g.F;
    d.T = (uint32_t)g.T;
    d.tmask = ((g.T & (g.T - 1)) == 0 && g.T > 1) ? (uint32_t)(g.T - 1) : 0u;
    for (int k = 0; k < 3; ++k) d.prime[k] = g.prime[k];
    for (int l = 0; l < g.L; ++l) {
        d.res[l] = g.res[l];
        d.off[l] = (uint32_t)g.offset[l];
        if (g.dense[l]) d.dense_bits |= 1u << l;
    }
    d.rows = (uint32_t)g.offset[g.L];
    return d;
}

// Rows of each level of a validated grid.
static void rows_of(const h4d_grid& g, int64_t* rows) {
    for (int l = 0; l < g.L; ++l) rows[l] = g.offset[l + 1] - g.offset[l];
}

DevGrid to_device(const h4d_grid& g) {
    DevGrid d;
    memset(&d, 0, sizeof d);
    d.L = g.L;
    d.F = g.F;
    d.T = (uint32_t)g.T;
    d.tmask = ((g.T & (g.T - 1)) == 0) ? (uint32_t)(g.T - 1) : 0u;
    if (g.T == 1) d.tmask = 0;  // T = 1: the generic modulo path (h % 1 = 0)
    for (int k = 0; k < 4; ++k) d.prime[k] = g.prime[k];
    for (int l = 0; l < g.L; ++l) {
        d.res_s[l] = g.res_s[l];
        d.res_t[l] = g.res_t[l];
        d.off[l] = (uint32_t)g.offset[l];
        if (g.dense[l]) d.dense_bits |= 1u << l;
    }
    d.rows = (uint32_t)g.offset[g.L];
    return d;
}

static h4d_status check_xyzt(const float* xyzt, int64_t n) {
    if (n < 0 || n > kMaxQ) return fail(H4D_EINVAL, "n=%lld outside 0..2^31-2^16", (long long)n);
    if (n > 0 && !xyzt) return fail(H4D_EINVAL, "xyzt is NULL");
    if (((uintptr_t)xyzt) & 15u) return fail(H4D_EINVAL, "xyzt is not 16-byte aligned");
    return H4D_OK;
}

// Tables are read a row at a time (up to 16-byte vector loads): align them to their
// row size, capped at 16 bytes.
static h4d_status check_table_alignment(const void* table, h4d_dtype dt, int F) {
    const size_t el = dt == H4D_F64 ? 8 : dt == H4D_BF16 ? 2 : 4;
    size_t a = el * (size_t)F;
    if (a > 16) a = 16;
    if (((uintptr_t)table) % a) return fail(H4D_EINVAL, "table is not aligned to its row size (%zu bytes)", a);
    return H4D_OK;
}

static h4d_status check_dtype(h4d_dtype dt) {
    if (dt != H4D_F32 && dt != H4D_BF16 && dt != H4D_F64) return fail(H4D_EINVAL, "unknown dtype %d", (int)dt);
    return H4D_OK;
}

static h4d_status check_mlp(const h4d_mlp* m, h4d_dtype dt) {
    if (!m) return fail(H4D_EINVAL, "mlp pointer is NULL");
    if (m->hidden != H4D_HIDDEN) return fail(H4D_EINVAL, "mlp: hidden=%d, only %d is built", m->hidden, H4D_HIDDEN);
    if (m->out < 1 || m->out > H4D_MAX_OUT) return fail(H4D_EINVAL, "mlp: out=%d outside 1..%d", m->out, H4D_MAX_OUT);
    if (m->in != 8 && m->in != 16 && m->in != 32 && m->in != 64)
        return fail(H4D_EUNSUPPORTED, "mlp: in=%d, built widths are 8, 16, 32, 64", m->in);
    return check_dtype(dt);
}

// Workspace of the tiled scatter for grid g and n queries.
static size_t scatter_ws(const h4d_grid* g, int64_t n) {
    int64_t rows[H4D_MAX_LEVELS];
    rows_of(*g, rows);
    return scatter_ws_bytes(to_device(*g), rows, (int)n);
}

// Deformation backward workspace: [decoder partials | d_feat [L, n, F] | tile masks].
static size_t deform_ws(const h4d_grid* g, const h4d_mlp* m, h4d_dtype dt, int64_t n) {
    const size_t el = dt == H4D_F64 ? sizeof(double) : sizeof(float);
    const size_t a = (mlp_workspace_bytes(dt, m->in, m->out, (int)n) + 255) / 256 * 256;
    const size_t b = ((size_t)n * g->L * g->F * el + 255) / 256 * 256;
    return a + b + scatter_ws(g, n);
}

h4d_status validate_grid(const h4d_grid* g) { return check_grid(g); }
h4d_status set_error(h4d_status st, const char* msg) {
    g_last_error = msg;
    return st;
}
void clear_error() { g_last_error.clear(); }

}  // namespace h4d

using namespace h4d;

extern "C" {

const char* h4d_last_error(void) { return g_last_error.c_str(); }

const char* h4d_version(void) { return "hash4d 0.1 gfx950"; }

h4d_status h4d_grid_schedule(int32_t L, int32_t n_min, int32_t n_max, int32_t rule, int32_t* res_out) {
    g_last_error.clear();
    if (!res_out) return fail(H4D_EINVAL, "res_out is NULL");
    if (L < 1 || L > H4D_MAX_LEVELS) return fail(H4D_EINVAL, "L=%d outside 1..%d", L, H4D_MAX_LEVELS);
    if (n_min < 1 || n_max < n_min || n_max > kMaxRes)
        return fail(H4D_EINVAL, "need 1 <= n_min <= n_max <= 2^24 (got %d, %d)", n_min, n_max);
    if (rule == H4D_SCHEDULE_DOUBLING) {
        int64_t v = n_min;
        for (int l = 0; l < L; ++l) {
            res_out[l] = (int32_t)(v < n_max ? v : n_max);
            if (v < n_max) v *= 2;
        }
        return H4D_OK;
    }
    if (rule != H4D_SCHEDULE_GEOMETRIC) return fail(H4D_EINVAL, "unknown schedule rule %d", rule);
    if (L == 1) {
        res_out[0] = n_min;
        return H4D_OK;
    }
    // Eq. 7 with its level exponent: b = exp((ln N_max - ln N_min) / (L - 1)), N_l = floor(N_min b^l).
    const double b = exp((log((double)n_max) - log((double)n_min)) / (double)(L - 1));
    for (int l = 0; l < L; ++l) {
        const double v = (double)n_min * pow(b, (double)l);
        res_out[l] = (int32_t)floor(v * (1.0 + 1e-9));
    }
    res_out[L - 1] = n_max;
    return H4D_OK;
}

h4d_status h4d_grid_init(h4d_grid* g, int32_t L, int32_t F, const int32_t* res_s, const int32_t* res_t, int64_t T) {
    g_last_error.clear();
    if (!g || !res_s || !res_t) return fail(H4D_EINVAL, "NULL argument");
    memset(g, 0, sizeof *g);
    if (L < 1 || L > H4D_MAX_LEVELS) return fail(H4D_EINVAL, "L=%d outside 1..%d", L, H4D_MAX_LEVELS);
    if (!valid_F(F)) return fail(H4D_EINVAL, "F=%d not in {1,2,4,8}", F);
    if (T < 1 || T > kMaxT) return fail(H4D_EINVAL, "T=%lld outside 1..2^30", (long long)T);
    g->L = L;
    g->F = F;
    g->T = T;
    for (int k = 0; k < 4; ++k) g->prime[k] = kPrimes[k];
    int64_t off = 0;
    for (int l = 0; l < L; ++l) {
        if (res_s[l] < 1 || res_s[l] > kMaxRes || res_t[l] < 1 || res_t[l] > kMaxRes) {
            memset(g, 0, sizeof *g);
            return fail(H4D_EINVAL, "level %d resolution (%d, %d) outside 1..2^24", l, res_s[l], res_t[l]);
        }
        g->res_s[l] = res_s[l];
        g->res_t[l] = res_t[l];
        int64_t rows;
        bool dense;
        level_size(res_s[l], res_t[l], T, &rows, &dense);
        g->dense[l] = dense ? 1 : 0;
        g->offset[l] = off;
        off += rows;
    }
    g->offset[L] = off;
    if (off * F >= ((int64_t)1 << 31)) {
        memset(g, 0, sizeof *g);
        return fail(H4D_EINVAL, "table of %lld rows x %d features exceeds 2^31 elements", (long long)off, F);
    }
    return H4D_OK;
}

h4d_status h4d_grid3_init(h4d_grid3* g, int32_t L, int32_t F, const int32_t* res, int64_t T) {
    g_last_error.clear();
    if (!g || !res) return fail(H4D_EINVAL, "NULL argument");
    memset(g, 0, sizeof *g);
    if (L < 1 || L > H4D_MAX_LEVELS) return fail(H4D_EINVAL, "L=%d outside 1..%d", L, H4D_MAX_LEVELS);
    if (!valid_F(F)) return fail(H4D_EINVAL, "F=%d not in {1,2,4,8}", F);
    if (T < 1 || T > kMaxT) return fail(H4D_EINVAL, "T=%lld outside 1..2^30", (long long)T);
    g->L = L;
    g->F = F;
    g->T = T;
    for (int k = 0; k < 3; ++k) g->prime[k] = kPrimes[k];
    int64_t off = 0;
    for (int l = 0; l < L; ++l) {
        if (res[l] < 1 || res[l] > kMaxRes) {
            memset(g, 0, sizeof *g);
            return fail(H4D_EINVAL, "level %d resolution %d outside 1..2^24", l, res[l]);
        }
        g->res[l] = res[l];
        const int64_t S = (int64_t)res[l] + 1;
        const unsigned __int128 v = (unsigned __int128)S * S * S;
        const bool dense = v <= (unsigned __int128)T;
        g->dense[l] = dense ? 1 : 0;
        g->offset[l] = off;
        off += dense ? (int64_t)v : T;
    }
    g->offset[L] = off;
    if (off * F >= ((int64_t)1 << 31)) {
        memset(g, 0, sizeof *g);
        return fail(H4D_EINVAL, "table of %lld rows x %d features exceeds 2^31 elements", (long long)off, F);
    }
    return H4D_OK;
}

int64_t h4d_grid_rows(const h4d_grid* g) {
    if (check_grid(g) != H4D_OK) return -1;
    return g->offset[g->L];
}

// Strides of feature (level l, query q): [n, L F] or [L, n, F].
static h4d_status feat_strides(h4d_layout layout, int64_t n, int L, int F, int64_t* ls, int64_t* qs) {
    if (layout == H4D_QUERY_MAJOR) {
        *ls = F;
        *qs = (int64_t)L * F;
    } else if (layout == H4D_LEVEL_MAJOR) {
        *ls = n * F;
        *qs = F;
    } else {
        return fail(H4D_EINVAL, "unknown layout %d", (int)layout);
    }
    if (n * (int64_t)L * F > kMaxN) return fail(H4D_EINVAL, "n L F exceeds 2^31-1 features");
    return H4D_OK;
}

h4d_status hash4d_encode(const h4d_grid* g, h4d_dtype table_dt, const void* table, const float* xyzt, int64_t n,
                         h4d_layout layout, void* feat, void* stream) {
    g_last_error.clear();
    h4d_status st;
    int64_t ls, qs;
    if ((st = check_grid(g)) || (st = check_dtype(table_dt)) || (st = check_xyzt(xyzt, n))) return st;
    if ((st = feat_strides(layout, n, g->L, g->F, &ls, &qs))) return st;
    if (n == 0) return H4D_OK;
    if (!table || !feat) return fail(H4D_EINVAL, "table or feat is NULL");
    if ((st = check_table_alignment(table, table_dt, g->F))) return st;
    const DevGrid d = to_device(*g);
    return hip_status(launch_encode(d, table_dt, table, xyzt, (int)n, feat, ls, qs, (hipStream_t)stream),
                      "hash4d_encode");
}

h4d_status hash3d_encode(const h4d_grid3* g, h4d_dtype table_dt, const void* table, const float* xyz,
                         int32_t stride, int64_t n, h4d_layout layout, void* feat, void* stream) {
    g_last_error.clear();
    h4d_status st;
    int64_t ls, qs;
    if ((st = check_grid3(g)) || (st = check_dtype(table_dt))) return st;
    if (stride != 3 && stride != 4) return fail(H4D_EINVAL, "stride=%d, must be 3 or 4", stride);
    if (n < 0 || n > kMaxQ) return fail(H4D_EINVAL, "n=%lld outside 0..2^31-2^16", (long long)n);
    if ((st = feat_strides(layout, n, g->L, g->F, &ls, &qs))) return st;
    if (n == 0) return H4D_OK;
    if (!table || !xyz || !feat) return fail(H4D_EINVAL, "table, xyz or feat is NULL");
    if (((uintptr_t)xyz) & (stride == 4 ? 15u : 3u))
        return fail(H4D_EINVAL, "xyz is not aligned to %d bytes", stride == 4 ? 16 : 4);
    if ((st = check_table_alignment(table, table_dt, g->F))) return st;
    return hip_status(launch_encode3(to_device3(*g), table_dt, table, xyz, stride, (int)n, feat, ls, qs,
                                     (hipStream_t)stream),
                      "hash3d_encode");
}

size_t hash4d_encode_backward_workspace_bytes(const h4d_grid* g, int64_t n) {
    if (check_grid(g) != H4D_OK || n < 0 || n > kMaxQ || n * (int64_t)g->L > kMaxN) return 0;
    return scatter_ws(g, n);
}

// Validation and launch shared by hash4d_encode_backward and its static-workspace
// form.  static_ws: the masks go to the library's static array (static_scratch)
// instead of `workspace`.
static h4d_status encode_backward_call(const h4d_grid* g, h4d_dtype grad_dt, const float* xyzt, int64_t n,
                                       h4d_layout layout, const void* d_feat, float grad_scale, void* d_table,
                                       void* workspace, size_t ws_bytes, bool static_ws, void* stream,
                                       const char* where, int32_t* nonfinite = nullptr) {
    g_last_error.clear();
    h4d_status st;
    int64_t ls, qs;
    const bool overwrite = (layout & H4D_GRAD_OVERWRITE) != 0;
    layout = (h4d_layout)(layout & ~H4D_GRAD_OVERWRITE);
    if ((st = check_grid(g)) || (st = check_xyzt(xyzt, n))) return st;
    if (grad_dt != H4D_F32 && grad_dt != H4D_F64) return fail(H4D_EINVAL, "grad dtype must be F32 or F64");
    if ((st = feat_strides(layout, n, g->L, g->F, &ls, &qs))) return st;
    if (n == 0 && !overwrite) return H4D_OK;
    if (n == 0) {  // no query: the written gradient is zero
        if (!d_table) return fail(H4D_EINVAL, "d_table is NULL");
        const int64_t words = g->offset[g->L] * g->F * (grad_dt == H4D_F64 ? 2 : 1);
        return hip_status(launch_zero_words(d_table, words, (hipStream_t)stream), where);
    }
    if (!d_feat || !d_table) return fail(H4D_EINVAL, "d_feat or d_table is NULL");
    const size_t need = scatter_ws(g, n);
    if (static_ws) {
        if (need > kStaticScratchBytes)
            return fail(H4D_EINVAL, "n=%lld, L=%d need %zu bytes of workspace; the static workspace holds %zu",
                        (long long)n, g->L, need, kStaticScratchBytes);
        if ((st = hip_status(static_scratch(&workspace), where))) return st;
    } else {
        if (!workspace || ws_bytes < need)
            return fail(H4D_EINVAL, "workspace of %zu bytes, %zu needed", workspace ? ws_bytes : (size_t)0, need);
        if (((uintptr_t)workspace) & 15u) return fail(H4D_EINVAL, "workspace is not 16-byte aligned");
    }
    const DevGrid d = to_device(*g);
    int64_t rows[H4D_MAX_LEVELS];
    rows_of(*g, rows);
    return hip_status(launch_scatter_tiled(d, rows, grad_dt, xyzt, nullptr, (int)n, d_feat, ls, qs,
                                           (double)grad_scale, d_table, workspace, (hipStream_t)stream, overwrite,
                                           MainGradArg{}, nonfinite),
                      where);
}

h4d_status hash4d_encode_backward(const h4d_grid* g, h4d_dtype grad_dt, const float* xyzt, int64_t n,
                                  h4d_layout layout, const void* d_feat, float grad_scale, void* d_table,
                                  void* workspace, size_t ws_bytes, void* stream) {
    return encode_backward_call(g, grad_dt, xyzt, n, layout, d_feat, grad_scale, d_table, workspace, ws_bytes,
                                false, stream, "hash4d_encode_backward");
}

h4d_status hash4d_encode_backward_checked(const h4d_grid* g, h4d_dtype grad_dt, const float* xyzt, int64_t n,
                                          h4d_layout layout, const void* d_feat, float grad_scale, void* d_table,
                                          void* workspace, size_t ws_bytes, int32_t* nonfinite, void* stream) {
    g_last_error.clear();
    if (!nonfinite || (((uintptr_t)nonfinite) & 3u)) return fail(H4D_EINVAL, "nonfinite is NULL or not 4-byte aligned");
    return encode_backward_call(g, grad_dt, xyzt, n, layout, d_feat, grad_scale, d_table, workspace, ws_bytes,
                                false, stream, "hash4d_encode_backward_checked", nonfinite);
}

h4d_status hash4d_encode_backward_noalloc(const h4d_grid* g, h4d_dtype grad_dt, const float* xyzt, int64_t n,
                                          h4d_layout layout, const void* d_feat, float grad_scale, void* d_table,
                                          void* stream) {
    return encode_backward_call(g, grad_dt, xyzt, n, layout, d_feat, grad_scale, d_table, nullptr, 0, true, stream,
                                "hash4d_encode_backward_noalloc");
}

size_t hash4d_encode_backward_input_workspace_bytes(const h4d_grid* g, h4d_dtype table_dt, int64_t n) {
    if (check_grid(g) != H4D_OK || check_dtype(table_dt) != H4D_OK || n < 0 || n > kMaxQ) return 0;
    if (table_dt == H4D_F64) return 0;  // the FP64 form runs in one pass
    return input_grad_workspace_bytes(g->L, (int)n);
}

h4d_status hash4d_encode_backward_input(const h4d_grid* g, h4d_dtype table_dt, const void* table,
                                        const float* xyzt, int64_t n, h4d_layout layout, const void* d_feat,
                                        float grad_scale, void* d_xyzt, void* workspace, size_t ws_bytes,
                                        void* stream) {
    g_last_error.clear();
    h4d_status st;
    int64_t ls, qs;
    if ((st = check_grid(g)) || (st = check_dtype(table_dt)) || (st = check_xyzt(xyzt, n))) return st;
    if ((st = feat_strides(layout, n, g->L, g->F, &ls, &qs))) return st;
    if (n == 0) return H4D_OK;
    if (!table || !d_feat || !d_xyzt) return fail(H4D_EINVAL, "table, d_feat or d_xyzt is NULL");
    if ((st = check_table_alignment(table, table_dt, g->F))) return st;
    if (((uintptr_t)d_xyzt) & (table_dt == H4D_F64 ? 31u : 15u))
        return fail(H4D_EINVAL, "d_xyzt is not aligned to its row (%d bytes)", table_dt == H4D_F64 ? 32 : 16);
    void* ws = nullptr;
    if (workspace && table_dt != H4D_F64) {
        const size_t need = input_grad_workspace_bytes(g->L, (int)n);
        if (ws_bytes < need) return fail(H4D_EINVAL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
        if (((uintptr_t)workspace) & 15u) return fail(H4D_EINVAL, "workspace is not 16-byte aligned");
        if (n * (int64_t)g->L > kMaxN) return fail(H4D_EINVAL, "n L exceeds 2^31-1 level terms");
        ws = workspace;
    }
    const DevGrid d = to_device(*g);
    return hip_status(launch_encode_input_grad(d, table_dt, table, xyzt, (int)n, d_feat, ls, qs, (double)grad_scale,
                                               d_xyzt, (hipStream_t)stream, ws),
                      "hash4d_encode_backward_input");
}

h4d_status hash4d_corner_indices(const h4d_grid* g, const float* xyzt, int64_t n, int32_t* rows, float* w,
                                 void* stream) {
    g_last_error.clear();
    h4d_status st;
    if ((st = check_grid(g)) || (st = check_xyzt(xyzt, n))) return st;
    if (n == 0) return H4D_OK;
    if (!rows && !w) return fail(H4D_EINVAL, "rows and w are both NULL");
    if (n * (int64_t)g->L * 16 > kMaxN) return fail(H4D_EINVAL, "n L 16 exceeds 2^31-1 outputs");
    const DevGrid d = to_device(*g);
    return hip_status(launch_corner_indices(d, xyzt, (int)n, rows, w, (hipStream_t)stream), "hash4d_corner_indices");
}

// Smoothness workspace: [d = G(x) - G(x + eps), level-major | tile masks].
static size_t smooth_ws(const h4d_grid* g, h4d_dtype table_dt, int64_t n) {
    const size_t d = ((size_t)n * g->L * g->F * (table_dt == H4D_F64 ? sizeof(double) : sizeof(float)) + 255) / 256 * 256;
    return d + scatter_ws(g, n);
}

size_t smoothness_workspace_bytes(const h4d_grid* g, h4d_dtype table_dt, int64_t n) {
    if (check_grid(g) != H4D_OK || check_dtype(table_dt) != H4D_OK || n < 0 || n > kMaxQ) return 0;
    if (n * (int64_t)g->L * g->F > kMaxN) return 0;
    return smooth_ws(g, table_dt, n);
}

h4d_status smoothness_reg(const h4d_grid* g, h4d_dtype table_dt, const void* table, const float* xyzt,
                          const float* eps, int64_t n, float lambda, void* loss, void* d_table, void* workspace,
                          size_t ws_bytes, void* stream) {
    g_last_error.clear();
    h4d_status st;
    if ((st = check_grid(g)) || (st = check_dtype(table_dt)) || (st = check_xyzt(xyzt, n))) return st;
    if (n == 0) return H4D_OK;
    if (!table || !eps || !loss) return fail(H4D_EINVAL, "table, eps or loss is NULL");
    if ((st = check_table_alignment(table, table_dt, g->F))) return st;
    if (((uintptr_t)eps) & 15u) return fail(H4D_EINVAL, "eps is not 16-byte aligned");
    if (n * (int64_t)g->L * g->F > kMaxN) return fail(H4D_EINVAL, "n L F exceeds 2^31-1 features");
    const size_t need = smooth_ws(g, table_dt, n);
    if (d_table && (!workspace || ws_bytes < need))
        return fail(H4D_EINVAL, "workspace of %zu bytes, %zu needed", workspace ? ws_bytes : (size_t)0, need);
    if (workspace && (((uintptr_t)workspace) & 15u)) return fail(H4D_EINVAL, "workspace is not 16-byte aligned");
    const DevGrid d = to_device(*g);
    const hipStream_t s = (hipStream_t)stream;
    // pass 1: loss and the feature difference d = G(x) - G(x + eps), level-major [L, n, F]
    if ((st = hip_status(launch_smoothness(d, table_dt, table, xyzt, eps, (int)n, (double)lambda, loss,
                                           d_table ? workspace : nullptr, s),
                         "smoothness_reg/diff")))
        return st;
    if (!d_table) return H4D_OK;
    // pass 2: d_table += (2 lambda / n) (d at x's corners - d at x~'s corners)
    int64_t rows[H4D_MAX_LEVELS];
    rows_of(*g, rows);
    const size_t dbytes =
        ((size_t)n * g->L * g->F * (table_dt == H4D_F64 ? sizeof(double) : sizeof(float)) + 255) / 256 * 256;
    return hip_status(launch_scatter_tiled(d, rows, table_dt == H4D_F64 ? H4D_F64 : H4D_F32, xyzt, eps, (int)n,
                                           workspace, n * g->F, g->F, 2.0 * (double)lambda / (double)n, d_table,
                                           static_cast<char*>(workspace) + dbytes, s),
                      "smoothness_reg/scatter");
}

h4d_status hash4d_encode_backward_smooth(const h4d_grid* g, h4d_dtype table_dt, const void* table, const float* xyzt,
                                         const float* eps, int64_t n, h4d_layout layout, const void* d_feat,
                                         float grad_scale, float lambda, void* loss, void* d_table, void* workspace,
                                         size_t ws_bytes, void* stream) {
    g_last_error.clear();
    h4d_status st;
    int64_t ls, qs;
    const bool overwrite = (layout & H4D_GRAD_OVERWRITE) != 0;
    layout = (h4d_layout)(layout & ~H4D_GRAD_OVERWRITE);
    if ((st = check_grid(g)) || (st = check_dtype(table_dt)) || (st = check_xyzt(xyzt, n))) return st;
    if ((st = feat_strides(layout, n, g->L, g->F, &ls, &qs))) return st;
    if (!d_table) return fail(H4D_EINVAL, "d_table is NULL");
    const hipStream_t s = (hipStream_t)stream;
    if (n == 0) {  // no query: nothing to add; a written gradient is zero
        if (!overwrite) return H4D_OK;
        const int64_t words = g->offset[g->L] * g->F * (table_dt == H4D_F64 ? 2 : 1);
        return hip_status(launch_zero_words(d_table, words, s), "hash4d_encode_backward_smooth");
    }
    if (!table || !eps || !loss || !d_feat) return fail(H4D_EINVAL, "table, eps, loss or d_feat is NULL");
    if ((st = check_table_alignment(table, table_dt, g->F))) return st;
    if (((uintptr_t)eps) & 15u) return fail(H4D_EINVAL, "eps is not 16-byte aligned");
    if (n * (int64_t)g->L * g->F > kMaxN) return fail(H4D_EINVAL, "n L F exceeds 2^31-1 features");
    const size_t need = smooth_ws(g, table_dt, n);
    if (!workspace || ws_bytes < need)
        return fail(H4D_EINVAL, "workspace of %zu bytes, %zu needed", workspace ? ws_bytes : (size_t)0, need);
    if (((uintptr_t)workspace) & 15u) return fail(H4D_EINVAL, "workspace is not 16-byte aligned");
    const DevGrid d = to_device(*g);
    // pass 1: loss and d = G(x) - G(x + eps), level-major [L, n, F]
    if ((st = hip_status(launch_smoothness(d, table_dt, table, xyzt, eps, (int)n, (double)lambda, loss, workspace, s),
                         "hash4d_encode_backward_smooth/diff")))
        return st;
    // pass 2: one scatter over both corner sets: x's corners get (2 lambda / n) d +
    // grad_scale d_feat, x~'s corners get -(2 lambda / n) d
    int64_t rows[H4D_MAX_LEVELS];
    rows_of(*g, rows);
    const size_t dbytes =
        ((size_t)n * g->L * g->F * (table_dt == H4D_F64 ? sizeof(double) : sizeof(float)) + 255) / 256 * 256;
    MainGradArg main;
    main.src = d_feat;
    main.lstride = ls;
    main.qstride = qs;
    main.scale = (double)grad_scale;
    return hip_status(launch_scatter_tiled(d, rows, table_dt == H4D_F64 ? H4D_F64 : H4D_F32, xyzt, eps, (int)n,
                                           workspace, n * g->F, g->F, 2.0 * (double)lambda / (double)n, d_table,
                                           static_cast<char*>(workspace) + dbytes, s, overwrite, main),
                      "hash4d_encode_backward_smooth/scatter");
}

size_t hash4d_collision_workspace_bytes(const h4d_grid* g, int32_t level, int64_t n) {
    if (check_grid(g) != H4D_OK || level < 0 || level >= g->L || n < 0 || n > kMaxQ) return 0;
    return census_workspace_bytes(n, g->offset[level + 1] - g->offset[level]);
}

h4d_status hash4d_collision_census(const h4d_grid* g, int32_t level, const float* xyzt, int64_t n, int64_t* counts,
                                   void* workspace, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    h4d_status st;
    if ((st = check_grid(g)) || (st = check_xyzt(xyzt, n))) return st;
    if (level < 0 || level >= g->L) return fail(H4D_EINVAL, "level %d outside 0..%d", level, g->L - 1);
    if (g->res_s[level] >= 65535 || g->res_t[level] >= 65535)
        return fail(H4D_EUNSUPPORTED, "vertex ids take 16 bits per coordinate: N_s, N_t must stay below 65535");
    if (!counts) return fail(H4D_EINVAL, "counts is NULL");
    if (((uintptr_t)counts) & 7u) return fail(H4D_EINVAL, "counts is not 8-byte aligned");
    const int64_t rows = g->offset[level + 1] - g->offset[level];
    const size_t need = census_workspace_bytes(n, rows);
    if (!workspace || ws_bytes < need)
        return fail(H4D_EINVAL, "workspace of %zu bytes, %zu needed", workspace ? ws_bytes : (size_t)0, need);
    if (((uintptr_t)workspace) & 15u) return fail(H4D_EINVAL, "workspace is not 16-byte aligned");
    const DevGrid d = to_device(*g);
    return hip_status(launch_census(d, level, rows, xyzt, (int)n, counts, workspace, (hipStream_t)stream),
                      "hash4d_collision_census");
}

size_t hash4d_decompose_workspace_bytes(int64_t n) {
    if (n < 0 || n > kMaxQ) return 0;
    return decompose_workspace_bytes(n);
}

h4d_status hash4d_decompose(const float* dp, int64_t n, float k_percent, float lambda_s, int32_t* dynamic_idx,
                            int32_t* n_dynamic, uint8_t* is_dynamic, float* loss, float* d_dp, void* workspace,
                            size_t ws_bytes, void* stream) {
    g_last_error.clear();
    if (n < 0 || n > kMaxQ) return fail(H4D_EINVAL, "n=%lld outside 0..2^31-2^16", (long long)n);
    if (!(k_percent >= 0.f && k_percent <= 100.f)) return fail(H4D_EINVAL, "k_percent must be in [0, 100]");
    if (n == 0) return H4D_OK;
    if (!dp) return fail(H4D_EINVAL, "dp is NULL");
    if ((((uintptr_t)dp) | ((uintptr_t)d_dp)) & 3u) return fail(H4D_EINVAL, "dp and d_dp must be 4-byte aligned");
    const size_t need = decompose_workspace_bytes(n);
    if (!workspace || ws_bytes < need)
        return fail(H4D_EINVAL, "workspace of %zu bytes, %zu needed", workspace ? ws_bytes : (size_t)0, need);
    if (((uintptr_t)workspace) & 15u) return fail(H4D_EINVAL, "workspace is not 16-byte aligned");
    return hip_status(launch_decompose(dp, n, (double)k_percent, lambda_s, dynamic_idx, n_dynamic, is_dynamic, loss,
                                       d_dp, workspace, (hipStream_t)stream),
                      "hash4d_decompose");
}

h4d_status h4d_adam_step(float* params, float* grad, float* m, float* v, int64_t count, int32_t row,
                         const h4d_adam* hp, uint16_t* bf16_out, int32_t flags, void* stream) {
    g_last_error.clear();
    if (count < 0) return fail(H4D_EINVAL, "count=%lld is negative", (long long)count);
    if (!hp) return fail(H4D_EINVAL, "hyper-parameters are NULL");
    if (!(hp->lr >= 0.f) || !(hp->beta1 >= 0.f && hp->beta1 < 1.f) || !(hp->beta2 >= 0.f && hp->beta2 < 1.f) ||
        !(hp->eps > 0.f) || hp->step < 1)
        return fail(H4D_EINVAL, "need lr >= 0, 0 <= beta1, beta2 < 1, eps > 0, step >= 1");
    if (flags & ~(H4D_ADAM_LAZY | H4D_ADAM_ZERO_GRAD)) return fail(H4D_EINVAL, "unknown flags 0x%x", flags);
    const bool lazy = flags & H4D_ADAM_LAZY;
    if (lazy && row != 1 && row != 2 && row != 4 && row != 8) return fail(H4D_EINVAL, "row must be 1, 2, 4 or 8");
    if (lazy && count % row) return fail(H4D_EINVAL, "count is not a multiple of row");
    if (count == 0) return H4D_OK;
    if (!params || !grad || !m || !v) return fail(H4D_EINVAL, "params, grad, m or v is NULL");
    if ((((uintptr_t)params) | ((uintptr_t)grad) | ((uintptr_t)m) | ((uintptr_t)v)) & 15u)
        return fail(H4D_EINVAL, "params, grad, m and v must be 16-byte aligned");
    if (bf16_out && (((uintptr_t)bf16_out) & 7u)) return fail(H4D_EINVAL, "bf16_out is not 8-byte aligned");
    return hip_status(launch_adam(params, grad, m, v, count, lazy ? row : 1, hp->lr, hp->beta1, hp->beta2, hp->eps,
                                  hp->step, hp->grad_scale, bf16_out, lazy, flags & H4D_ADAM_ZERO_GRAD,
                                  (hipStream_t)stream),
                      "h4d_adam_step");
}

h4d_status h4d_cast_bf16(const float* src, uint16_t* dst, int64_t count, void* stream) {
    g_last_error.clear();
    if (count < 0) return fail(H4D_EINVAL, "count=%lld < 0", (long long)count);
    if (count == 0) return H4D_OK;
    if (!src || !dst) return fail(H4D_EINVAL, "src or dst is NULL");
    return hip_status(launch_cast_bf16(src, dst, count, (hipStream_t)stream), "h4d_cast_bf16");
}

h4d_status h4d_count_nonfinite(const float* p, int64_t count, int32_t* counter, void* stream) {
    g_last_error.clear();
    if (count < 0) return fail(H4D_EINVAL, "count=%lld < 0", (long long)count);
    if (count == 0) return H4D_OK;
    if (!p || !counter) return fail(H4D_EINVAL, "p or counter is NULL");
    return hip_status(launch_count_nonfinite(p, count, counter, (hipStream_t)stream), "h4d_count_nonfinite");
}

h4d_status h4d_probe_gather(const void* table, int64_t rows, int32_t row_bytes, int64_t n_loads, uint32_t seed,
                            float* sink, void* stream) {
    g_last_error.clear();
    if (rows < 1 || rows > 0xffffffffLL) return fail(H4D_EINVAL, "rows=%lld outside 1..2^32-1", (long long)rows);
    if (row_bytes != 4 && row_bytes != 8) return fail(H4D_EINVAL, "row_bytes must be 4 or 8");
    if (n_loads < 0 || n_loads > ((int64_t)1 << 40)) return fail(H4D_EINVAL, "n_loads out of range");
    if (n_loads == 0) return H4D_OK;
    if (!table || !sink) return fail(H4D_EINVAL, "table or sink is NULL");
    if (((uintptr_t)table) & 7u) return fail(H4D_EINVAL, "table is not 8-byte aligned");
    return hip_status(launch_probe_gather(table, (uint32_t)rows, row_bytes, n_loads, seed, sink, (hipStream_t)stream),
                      "h4d_probe_gather");
}

h4d_status h4d_probe_scatter(float* table, int64_t rows, int64_t n_updates, uint32_t seed, int32_t mode,
                             void* stream) {
    g_last_error.clear();
    if (rows < 1 || rows > 0xffffffffLL) return fail(H4D_EINVAL, "rows=%lld outside 1..2^32-1", (long long)rows);
    if (n_updates < 0 || n_updates > ((int64_t)1 << 40)) return fail(H4D_EINVAL, "n_updates out of range");
    if (n_updates == 0) return H4D_OK;
    if (!table) return fail(H4D_EINVAL, "table is NULL");
    if (mode != 0 && mode != 1) return fail(H4D_EINVAL, "mode must be 0 or 1");
    return hip_status(launch_probe_scatter(table, (uint32_t)rows, n_updates, seed, mode, (hipStream_t)stream),
                      "h4d_probe_scatter");
}

h4d_status h4d_probe_copy(const void* src, void* dst, int64_t bytes, void* stream) {
    g_last_error.clear();
    if (bytes < 0 || (bytes & 15)) return fail(H4D_EINVAL, "bytes must be a non-negative multiple of 16");
    if (bytes == 0) return H4D_OK;
    if (!src || !dst || ((((uintptr_t)src) | ((uintptr_t)dst)) & 15u))
        return fail(H4D_EINVAL, "src/dst NULL or not 16-byte aligned");
    return hip_status(launch_probe_copy(src, dst, bytes, (hipStream_t)stream), "h4d_probe_copy");
}

h4d_status h4d_probe_lds_atomic(int32_t blocks, int32_t per_thread, int32_t active, uint32_t seed, int32_t mode,
                                float* sink, void* stream) {
    g_last_error.clear();
    if (blocks < 1 || blocks > 1 << 20 || per_thread < 0 || per_thread > 1 << 16 || active < 1 || active > 64)
        return fail(H4D_EINVAL, "blocks 1..2^20, per_thread 0..65536, active 1..64");
    if (mode < 0 || mode > 2) return fail(H4D_EINVAL, "mode must be 0, 1 or 2");
    if (!sink) return fail(H4D_EINVAL, "sink is NULL");
    return hip_status(launch_probe_lds_atomic(blocks, per_thread, active, seed, mode, sink, (hipStream_t)stream),
                      "h4d_probe_lds_atomic");
}

size_t deform_mlp_workspace_bytes(const h4d_mlp* m, h4d_dtype dt, int64_t n) {
    if (check_mlp(m, dt) != H4D_OK || n < 0 || n > kMaxQ) return 0;
    return mlp_workspace_bytes(dt, m->in, m->out, (int)n);
}

// Feature strides of the decoder input for (layout, F); F = 1 for query-major.
static h4d_status mlp_strides(const h4d_mlp* m, int64_t n, h4d_layout layout, int32_t F, int* Fk, int64_t* ls,
                              int64_t* qs) {
    if (n < 0 || n > kMaxQ) return fail(H4D_EINVAL, "n=%lld outside 0..2^31-2^16", (long long)n);
    if ((int64_t)n * m->in > kMaxN) return fail(H4D_EINVAL, "n in exceeds 2^31-1 features");
    if (layout == H4D_QUERY_MAJOR) {
        *Fk = 1;
        *ls = 1;
        *qs = m->in;
        return H4D_OK;
    }
    if (layout != H4D_LEVEL_MAJOR) return fail(H4D_EINVAL, "unknown layout %d", (int)layout);
    if (!valid_F(F) || m->in % F) return fail(H4D_EINVAL, "level-major F=%d must be 1, 2, 4 or 8 and divide in", F);
    *Fk = F;
    *ls = n * F;
    *qs = F;
    return H4D_OK;
}

h4d_status deform_mlp_forward(const h4d_mlp* m, h4d_dtype dt, const void* params, const void* feat, int64_t n,
                              h4d_layout layout, int32_t F, void* out, void* stream) {
    g_last_error.clear();
    h4d_status st;
    int Fk;
    int64_t ls, qs;
    if ((st = check_mlp(m, dt)) || (st = mlp_strides(m, n, layout, F, &Fk, &ls, &qs))) return st;
    if (n == 0) return H4D_OK;
    if (!params || !feat || !out) return fail(H4D_EINVAL, "params, feat or out is NULL");
    return hip_status(launch_mlp_forward(dt, m->in, m->out, params, feat, Fk, ls, qs, (int)n, out,
                                         (hipStream_t)stream),
                      "deform_mlp_forward");
}

static h4d_status mlp_backward_call(const h4d_mlp* m, h4d_dtype dt, const void* params, const void* feat,
                                    int64_t n, h4d_layout layout, int32_t F, const void* d_out, float loss_scale,
                                    float grad_scale, void* d_feat, void* d_params, void* workspace, size_t ws_bytes,
                                    int32_t* nonfinite, void* stream) {
    h4d_status st;
    int Fk;
    int64_t ls, qs;
    const bool overwrite = (layout & H4D_GRAD_OVERWRITE) != 0;
    layout = (h4d_layout)(layout & ~H4D_GRAD_OVERWRITE);
    if ((st = check_mlp(m, dt)) || (st = mlp_strides(m, n, layout, F, &Fk, &ls, &qs))) return st;
    if (n == 0 && !overwrite) return H4D_OK;
    if (n == 0) {  // no query: the written parameter gradient is zero
        if (!d_params) return fail(H4D_EINVAL, "d_params is NULL");
        const int64_t H = H4D_HIDDEN, P = H * m->in + H + H * H + H + (int64_t)m->out * H + m->out;
        return hip_status(launch_zero_words(d_params, P * (dt == H4D_F64 ? 2 : 1), (hipStream_t)stream),
                          "deform_mlp_backward");
    }
    if (!params || !feat || !d_out || !d_feat || !d_params) return fail(H4D_EINVAL, "NULL data pointer");
    const size_t need = mlp_workspace_bytes(dt, m->in, m->out, (int)n);
    if (!workspace || ws_bytes < need)
        return fail(H4D_EINVAL, "workspace of %zu bytes, %zu needed", workspace ? ws_bytes : (size_t)0, need);
    if (((uintptr_t)workspace) & 15u) return fail(H4D_EINVAL, "workspace is not 16-byte aligned");
    return hip_status(launch_mlp_backward(dt, m->in, m->out, params, feat, Fk, ls, qs, (int)n, d_out, loss_scale,
                                          grad_scale, grad_scale, d_feat, ls, qs, d_params, workspace,
                                          (hipStream_t)stream, overwrite, nonfinite),
                      "deform_mlp_backward");
}

h4d_status deform_mlp_backward(const h4d_mlp* m, h4d_dtype dt, const void* params, const void* feat, int64_t n,
                               h4d_layout layout, int32_t F, const void* d_out, float loss_scale, float grad_scale,
                               void* d_feat, void* d_params, void* workspace, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return mlp_backward_call(m, dt, params, feat, n, layout, F, d_out, loss_scale, grad_scale, d_feat, d_params,
                             workspace, ws_bytes, nullptr, stream);
}

h4d_status deform_mlp_backward_checked(const h4d_mlp* m, h4d_dtype dt, const void* params, const void* feat,
                                       int64_t n, h4d_layout layout, int32_t F, const void* d_out, float loss_scale,
                                       float grad_scale, void* d_feat, void* d_params, void* workspace,
                                       size_t ws_bytes, int32_t* nonfinite, void* stream) {
    g_last_error.clear();
    if (!nonfinite || (((uintptr_t)nonfinite) & 3u)) return fail(H4D_EINVAL, "nonfinite is NULL or not 4-byte aligned");
    return mlp_backward_call(m, dt, params, feat, n, layout, F, d_out, loss_scale, grad_scale, d_feat, d_params,
                             workspace, ws_bytes, nonfinite, stream);
}

h4d_status hash4d_deform_apply(const float* delta, int64_t n, int32_t out, const float* xyz, const float* rot,
                               const float* scale, float* xyz_out, float* rot_out, float* scale_out, void* stream) {
    g_last_error.clear();
    if (n < 0 || n > kMaxQ) return fail(H4D_EINVAL, "n=%lld outside 0..2^31-2^16", (long long)n);
    if (out < 10 || out > H4D_MAX_OUT) return fail(H4D_EINVAL, "out=%d: the heads need 10 columns", out);
    if (n == 0) return H4D_OK;
    if (!delta || !xyz || !rot || !scale || !xyz_out || !rot_out || !scale_out)
        return fail(H4D_EINVAL, "NULL data pointer");
    return hip_status(launch_deform_apply(delta, (int)n, out, xyz, rot, scale, xyz_out, rot_out, scale_out,
                                          (hipStream_t)stream),
                      "hash4d_deform_apply");
}

size_t hash4d_deform_workspace_bytes(const h4d_grid* g, const h4d_mlp* m, h4d_dtype dt, int64_t n) {
    if (check_grid(g) != H4D_OK || check_mlp(m, dt) != H4D_OK || n < 0 || n > kMaxQ) return 0;
    return deform_ws(g, m, dt, n);
}

static h4d_status check_deform(const h4d_grid* g, const h4d_mlp* m, h4d_dtype dt, const float* xyzt, int64_t n) {
    h4d_status st;
    if ((st = check_grid(g)) || (st = check_mlp(m, dt)) || (st = check_xyzt(xyzt, n))) return st;
    if (m->in != g->L * g->F)
        return fail(H4D_EINVAL, "decoder input width %d != L F = %d", m->in, g->L * g->F);
    if ((int64_t)n * g->L * g->F > kMaxN) return fail(H4D_EINVAL, "n L F exceeds 2^31-1 features");
    return H4D_OK;
}

h4d_status hash4d_deform_forward(const h4d_grid* g, const h4d_mlp* m, h4d_dtype dt, const void* table,
                                 const void* params, const float* xyzt, int64_t n, void* feat, void* delta,
                                 void* stream) {
    g_last_error.clear();
    h4d_status st;
    if ((st = check_deform(g, m, dt, xyzt, n))) return st;
    if (n == 0) return H4D_OK;
    if (!table || !params || !feat || !delta) return fail(H4D_EINVAL, "NULL data pointer");
    if ((st = check_table_alignment(table, dt, g->F))) return st;
    const DevGrid d = to_device(*g);
    const hipStream_t s = (hipStream_t)stream;
    const int64_t ls = n * g->F, qs = g->F;
    if ((st = hip_status(launch_encode(d, dt, table, xyzt, (int)n, feat, ls, qs, s), "hash4d_deform_forward/encode")))
        return st;
    return hip_status(launch_mlp_forward(dt, m->in, m->out, params, feat, g->F, ls, qs, (int)n, delta, s),
                      "hash4d_deform_forward/decode");
}

h4d_status hash4d_deform_backward(const h4d_grid* g, const h4d_mlp* m, h4d_dtype dt, const void* params,
                                  const float* xyzt, int64_t n, const void* feat, const void* d_delta,
                                  float loss_scale, float grad_scale, void* d_table, void* d_params,
                                  void* workspace, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    h4d_status st;
    if ((st = check_deform(g, m, dt, xyzt, n))) return st;
    if (n == 0) return H4D_OK;
    if (!params || !feat || !d_delta || !d_table || !d_params) return fail(H4D_EINVAL, "NULL data pointer");
    const size_t need = deform_ws(g, m, dt, n);
    if (!workspace || ws_bytes < need)
        return fail(H4D_EINVAL, "workspace of %zu bytes, %zu needed", workspace ? ws_bytes : (size_t)0, need);
    if (((uintptr_t)workspace) & 15u) return fail(H4D_EINVAL, "workspace is not 16-byte aligned");
    const DevGrid d = to_device(*g);
    const hipStream_t s = (hipStream_t)stream;
    const int64_t ls = n * g->F, qs = g->F;
    char* ws = static_cast<char*>(workspace);
    const size_t el = dt == H4D_F64 ? sizeof(double) : sizeof(float);
    const size_t part = (mlp_workspace_bytes(dt, m->in, m->out, (int)n) + 255) / 256 * 256;
    void* d_feat = ws + part;
    void* masks = ws + part + ((size_t)n * g->L * g->F * el + 255) / 256 * 256;
    // decoder backward: d_feat keeps the loss scale, d_params gets grad_scale
    if ((st = hip_status(launch_mlp_backward(dt, m->in, m->out, params, feat, g->F, ls, qs, (int)n, d_delta,
                                             loss_scale, 1.0, grad_scale, d_feat, ls, qs, d_params, ws, s),
                         "hash4d_deform_backward/decode")))
        return st;
    int64_t rows[H4D_MAX_LEVELS];
    rows_of(*g, rows);
    return hip_status(launch_scatter_tiled(d, rows, dt == H4D_F64 ? H4D_F64 : H4D_F32, xyzt, nullptr, (int)n, d_feat,
                                           ls, qs, grad_scale, d_table, masks, s),
                      "hash4d_deform_backward/encode");
}

}  // extern "C"
