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
static const int64_t kMaxN = 2147483647;

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
    return d;
}

static h4d_status check_xyzt(const float* xyzt, int64_t n) {
    if (n < 0 || n > kMaxN) return fail(H4D_EINVAL, "n=%lld outside 0..2^31-1", (long long)n);
    if (n > 0 && !xyzt) return fail(H4D_EINVAL, "xyzt is NULL");
    if (((uintptr_t)xyzt) & 15u) return fail(H4D_EINVAL, "xyzt is not 16-byte aligned");
    return H4D_OK;
}

static h4d_status check_dtype(h4d_dtype dt) {
    if (dt != H4D_F32 && dt != H4D_BF16 && dt != H4D_F64) return fail(H4D_EINVAL, "unknown dtype %d", (int)dt);
    return H4D_OK;
}

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

int64_t h4d_grid_rows(const h4d_grid* g) {
    if (check_grid(g) != H4D_OK) return -1;
    return g->offset[g->L];
}

h4d_status hash4d_encode(const h4d_grid* g, h4d_dtype table_dt, const void* table, const float* xyzt, int64_t n,
                         void* feat, void* stream) {
    g_last_error.clear();
    h4d_status st;
    if ((st = check_grid(g)) || (st = check_dtype(table_dt)) || (st = check_xyzt(xyzt, n))) return st;
    if (n == 0) return H4D_OK;
    if (!table || !feat) return fail(H4D_EINVAL, "table or feat is NULL");
    const DevGrid d = to_device(*g);
    return hip_status(launch_encode(d, table_dt, table, xyzt, (int)n, feat, g->F, (int64_t)g->L * g->F,
                                    (hipStream_t)stream),
                      "hash4d_encode");
}

h4d_status hash4d_encode_backward(const h4d_grid* g, h4d_dtype grad_dt, const float* xyzt, int64_t n,
                                  const void* d_feat, float grad_scale, void* d_table, void* stream) {
    g_last_error.clear();
    h4d_status st;
    if ((st = check_grid(g)) || (st = check_xyzt(xyzt, n))) return st;
    if (grad_dt != H4D_F32 && grad_dt != H4D_F64) return fail(H4D_EINVAL, "grad dtype must be F32 or F64");
    if (n == 0) return H4D_OK;
    if (!d_feat || !d_table) return fail(H4D_EINVAL, "d_feat or d_table is NULL");
    const DevGrid d = to_device(*g);
    return hip_status(launch_encode_backward(d, grad_dt, xyzt, (int)n, d_feat, g->F, (int64_t)g->L * g->F,
                                             (double)grad_scale, d_table, (hipStream_t)stream),
                      "hash4d_encode_backward");
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

}  // extern "C"
