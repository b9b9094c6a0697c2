// Batched form: many scenes, each queried at several timestamps, in persistent
// launches (DASH Section 4.2 applied per scene; one deformation field per scene).
//
// Work is a list of items (segment = (scene, timestamp), level group, tile of
// queries), ordered scene by scene and, inside a scene, level group by level group,
// so that all timestamps of a scene reuse one level's slice of that scene's table
// while it is hot in L2.  A persistent grid walks the list with a fixed stride; the
// tile width (queries per thread) and the number of levels per item are the
// schedule the autotuner picks.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "h4d_device.h"

namespace h4d {

constexpr int kBatchBlock = 256;

struct BSeg {
    const float4* xyz;   // scene positions [n, 4]; the 4th value is replaced by t
    float t;
    int n;
    int scene;
    const void* table;   // [E, F] FP32 or BF16
    float* feat;         // [L, n, F]
    const float* d_feat; // [L, n, F]
    float* d_table;      // [E, F] FP32, +=
    uint32_t* mask;      // [L, n] tile masks of the scatter
};

struct BRange {          // items [first, first + ntiles) belong to (seg, level group lg)
    int first;
    int seg;
    int lg;
    int ntiles;
};

struct BSchedule {
    int qpt;             // queries per thread (tile = 256 qpt queries)
    int lpb;             // levels per item
    int grid;            // persistent workgroups
};

__device__ __forceinline__ int find_range(const BRange* __restrict__ r, int nr, int item) {
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (r[mid].first <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Workgroups go to the eight XCDs round-robin by id, so with a grid of whole rounds
// XCD x walks its own contiguous eighth of the item list: at any time each XCD's L2
// holds the level slices of its own part of the list instead of every XCD streaming
// the same slice.  PAIRS: row-pair corner loads (gather_corners).
template <typename TT, int F, bool PAIRS>
__global__ __launch_bounds__(kBatchBlock) void k_bencode(const BSeg* __restrict__ segs, const DevGrid* __restrict__ grids,
                                                         const BRange* __restrict__ ranges, int nranges, int total,
                                                         BSchedule sch) {
    const int nx = (gridDim.x % kXcds) == 0 ? kXcds : 1;
    const int x = (int)blockIdx.x % nx, slots = (int)gridDim.x / nx;
    const int per = (total + nx - 1) / nx;
    const int end = min(total, (x + 1) * per);
    for (int item = x * per + (int)blockIdx.x / nx; item < end; item += slots) {
        const BRange rg = ranges[find_range(ranges, nranges, item)];
        const BSeg sg = segs[rg.seg];
        const DevGrid& g = grids[sg.scene];
        const int tile = item - rg.first;
        const int l0 = rg.lg * sch.lpb, l1 = min(l0 + sch.lpb, g.L);
        const TT* __restrict__ table = static_cast<const TT*>(sg.table);
        for (int u = 0; u < sch.qpt; ++u) {
            const int q = (tile * sch.qpt + u) * kBatchBlock + (int)threadIdx.x;
            if (q >= sg.n) break;
            float4 x = sg.xyz[q];
            x.w = sg.t;
            for (int l = l0; l < l1; ++l) {
                const Cell c = level_cell(g, l, x);
                uint32_t row[16];
                level_rows(g, l, c, row);
                float v[16][F];
                gather_corners<TT, F, PAIRS>(g, table, row, v);
                float w[16];
                level_weights<float>(c, w);
                float acc[F];
#pragma unroll
                for (int f = 0; f < F; ++f) acc[f] = 0.f;
#pragma unroll
                for (int k = 0; k < 16; ++k)
#pragma unroll
                    for (int f = 0; f < F; ++f) acc[f] += w[k] * v[k][f];
                float* o = sg.feat + ((int64_t)l * sg.n + q) * F;
#pragma unroll
                for (int f = 0; f < F; ++f) o[f] = acc[f];
            }
        }
    }
}

// One workgroup per (scene, level, tile of rows): the owner-computes scatter of the
// plain path over every timestamp segment of its scene, each segment's queries
// filtered by the tile masks of k_bmask.
struct BTile {
    int scene, level, seg0, nseg;
    uint32_t base, cnt;  // table rows [base, base + cnt)
    uint32_t bit;        // the tile's bit in the query masks
};

__global__ __launch_bounds__(kBatchBlock) void k_bmask(const BSeg* __restrict__ segs, const DevGrid* __restrict__ grids,
                                                       const TileMap* __restrict__ tms) {
    const BSeg sg = segs[blockIdx.z];
    const int l = blockIdx.y;
    const int q = blockIdx.x * kBatchBlock + (int)threadIdx.x;
    const DevGrid& g = grids[sg.scene];
    if (q >= sg.n || l >= g.L) return;
    float4 x = sg.xyz[q];
    x.w = sg.t;
    sg.mask[(int64_t)l * mask_stride(sg.n) + q] = corner_tile_mask(g, tms[sg.scene], l, x);
}

template <int F>
struct BQuery {
    float4 x;
    float gv[F];
};

constexpr int kBatchScatterBlock = 1024;  // one workgroup per CU (128 KiB tile), 16 wavefronts

// XCD placement of the scatter tiles: the scene-ordered tile list is cut into eight
// runs of about equal work (queries scanned), run x going to XCD x (workgroup b runs
// on XCD b % 8), so each XCD's L2 holds the masks, gradients and positions of one or
// two scenes.
struct BXcdRuns {
    int start[kXcds + 1];
};

template <int F>
__global__ __launch_bounds__(kBatchScatterBlock) void k_bscatter(const BSeg* __restrict__ segs, const DevGrid* __restrict__ grids,
                                                                 const TileMap* __restrict__ tms,
                                                                 const BTile* __restrict__ tiles, BXcdRuns runs,
                                                                 float scale) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int queue[2 * kBatchScatterBlock];
    float* tile = reinterpret_cast<float*>(smem);
    const int x = (int)blockIdx.x % kXcds;
    const int ti = runs.start[x] + (int)blockIdx.x / kXcds;
    if (ti >= runs.start[x + 1]) return;
    const BTile tl = tiles[ti];
    const DevGrid& g = grids[tl.scene];
    const TileMap& tm = tms[tl.scene];
    const int l = tl.level;
    for (uint32_t i = threadIdx.x; i < tl.cnt * F; i += kBatchScatterBlock) tile[i] = 0.f;
    __syncthreads();
    for (int sgi = tl.seg0; sgi < tl.seg0 + tl.nseg; ++sgi) {
        const BSeg sg = segs[sgi];
        masked_queue_loop<kBatchScatterBlock>(
            sg.n, sg.mask + (int64_t)l * mask_stride(sg.n), tl.bit, queue,
            [&](int q) {
                BQuery<F> b;
                const float* gp = sg.d_feat + ((int64_t)l * sg.n + q) * F;
#pragma unroll
                for (int f = 0; f < F; ++f) b.gv[f] = gp[f];
                b.x = sg.xyz[q];
                return b;
            },
            [&](const BQuery<F>& b) {
                float gv[F];
#pragma unroll
                for (int f = 0; f < F; ++f) gv[f] = b.gv[f] * scale;
                float4 x = b.x;
                x.w = sg.t;
                tile_contrib<float, F>(g, tm, l, x, gv, tl.base, tl.cnt, tile);
            });
    }
    __syncthreads();
    float* out = segs[tl.seg0].d_table + (size_t)tl.base * F;
    for (uint32_t i = threadIdx.x; i < tl.cnt * F; i += kBatchScatterBlock) {
        const float v = tile[i];
        if (v != 0.f) out[i] += v;
    }
}

// Graph-safe zeroing (a kernel, not a memset node).
__global__ __launch_bounds__(256) void k_zero(float* __restrict__ p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) p[i] = 0.f;
}

}  // namespace h4d

// ------------------------------------------------------------------ plan ----
using namespace h4d;

struct h4d_batched_plan {
    int n_scenes = 0;
    h4d_mlp mlp{};
    h4d_dtype dt = H4D_F32;
    int flags = 0;
    float loss_scale = 1.f;
    std::vector<h4d_scene_desc> scenes;
    std::vector<DevGrid> grids_h;
    int nseg = 0;
    // device
    DevGrid* grids = nullptr;
    BSeg* segs = nullptr;
    BRange* ranges_enc = nullptr;
    BTile* tiles = nullptr;
    int ntiles = 0;
    BXcdRuns xcd_runs{};
    TileMap* tms = nullptr;
    uint32_t* masks = nullptr;
    int max_n = 0, max_L = 0;
    int nranges_enc = 0, total_enc = 0;
    float* d_feat = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    BSchedule enc{1, 1, 2048};
    MlpBatch fwd{}, bwd{};
    int fwd_blocks = 0, bwd_blocks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t queries = 0;
    std::vector<h4d_tune_result> tuned;
};

namespace h4d {

// Items for a schedule: scene by scene, level group by level group, every segment
// (timestamp) of the scene, every tile.
static std::vector<BRange> build_ranges(const h4d_batched_plan& p, const std::vector<BSeg>& segs, const BSchedule& s,
                                        int* total) {
    std::vector<BRange> r;
    int first = 0, seg0 = 0;
    for (int sc = 0; sc < p.n_scenes; ++sc) {
        const h4d_scene_desc& d = p.scenes[sc];
        const int L = d.grid.L;
        const int groups = (L + s.lpb - 1) / s.lpb;
        const int ntiles = (int)((d.n + (int64_t)kBatchBlock * s.qpt - 1) / ((int64_t)kBatchBlock * s.qpt));
        for (int lg = 0; lg < groups; ++lg)
            for (int k = 0; k < d.n_times; ++k) {
                if (ntiles == 0) continue;
                r.push_back(BRange{first, seg0 + k, lg, ntiles});
                first += ntiles;
            }
        seg0 += d.n_times;
    }
    (void)segs;
    *total = first;
    return r;
}

static hipError_t upload_ranges(BRange** dst, const std::vector<BRange>& r) {
    if (*dst) {
        hipError_t e = hipFree(*dst);
        *dst = nullptr;
        if (e != hipSuccess) return e;
    }
    const size_t bytes = std::max<size_t>(1, r.size()) * sizeof(BRange);
    hipError_t e = hipMalloc((void**)dst, bytes);
    if (e != hipSuccess) return e;
    if (!r.empty()) e = hipMemcpy(*dst, r.data(), r.size() * sizeof(BRange), hipMemcpyHostToDevice);
    return e;
}

static hipError_t launch_bencode(const h4d_batched_plan& p, const BSchedule& s, hipStream_t st) {
    if (p.total_enc == 0) return hipSuccess;
    const int F = p.scenes[0].grid.F;
    const dim3 grid(std::min(s.grid, p.total_enc)), block(kBatchBlock);
    // row-pair loads need every scene's table aligned to two rows
    const size_t pair_bytes = 2 * 2 * (p.dt == H4D_BF16 ? sizeof(uint16_t) : sizeof(float));
    bool pairs = F == 2;
    for (const h4d_scene_desc& d : p.scenes) pairs = pairs && ((uintptr_t)d.table % pair_bytes) == 0;
#define H4D_BENC(TT, FF, PP) hipLaunchKernelGGL((k_bencode<TT, FF, PP>), grid, block, 0, st, p.segs, p.grids, \
                                                p.ranges_enc, p.nranges_enc, p.total_enc, s)
    if (p.dt == H4D_BF16) {
        switch (F) {
            case 1: H4D_BENC(bf16_t, 1, false); break;
            case 2:
                if (pairs) H4D_BENC(bf16_t, 2, true);
                else H4D_BENC(bf16_t, 2, false);
                break;
            case 4: H4D_BENC(bf16_t, 4, false); break;
            default: H4D_BENC(bf16_t, 8, false); break;
        }
    } else {
        switch (F) {
            case 1: H4D_BENC(float, 1, false); break;
            case 2:
                if (pairs) H4D_BENC(float, 2, true);
                else H4D_BENC(float, 2, false);
                break;
            case 4: H4D_BENC(float, 4, false); break;
            default: H4D_BENC(float, 8, false); break;
        }
    }
#undef H4D_BENC
    return hipGetLastError();
}

static hipError_t launch_bscatter(const h4d_batched_plan& p, float scale, hipStream_t st) {
    if (p.ntiles == 0) return hipSuccess;
    if (p.max_n > 0) {
        hipLaunchKernelGGL(k_bmask, dim3((unsigned)((p.max_n + kBatchBlock - 1) / kBatchBlock), (unsigned)p.max_L,
                                         (unsigned)p.nseg),
                           dim3(kBatchBlock), 0, st, p.segs, p.grids, p.tms);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int F = p.scenes[0].grid.F;
    const size_t lds = (size_t)kTileBytes;
    int longest = 0;
    for (int x = 0; x < kXcds; ++x) longest = std::max(longest, p.xcd_runs.start[x + 1] - p.xcd_runs.start[x]);
    const dim3 grid((unsigned)(kXcds * longest)), block(kBatchScatterBlock);
#define H4D_BSCA(FF)                                                                                             \
    do {                                                                                                         \
        hipError_t e = hipFuncSetAttribute((const void*)k_bscatter<FF>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                           (int)lds);                                                            \
        if (e != hipSuccess) return e;                                                                           \
        hipLaunchKernelGGL((k_bscatter<FF>), grid, block, lds, st, p.segs, p.grids, p.tms, p.tiles, p.xcd_runs,      \
                           scale);                                                                               \
    } while (0)
    switch (F) {
        case 1: H4D_BSCA(1); break;
        case 2: H4D_BSCA(2); break;
        case 4: H4D_BSCA(4); break;
        default: H4D_BSCA(8); break;
    }
#undef H4D_BSCA
    return hipGetLastError();
}

static int64_t param_count(const h4d_mlp& m) {
    return (int64_t)m.hidden * m.in + m.hidden + (int64_t)m.hidden * m.hidden + m.hidden + (int64_t)m.out * m.hidden +
           m.out;
}

// Blocks of a persistent decoder grid split over scenes in proportion to their
// tiles (at least one each; blocks >= scenes).
static void split_blocks(h4d_batched_plan& p, MlpBatch& b, int blocks) {
    memset(&b, 0, sizeof b);
    b.count = p.n_scenes;
    std::vector<int64_t> tiles(p.n_scenes);
    int64_t total = 0;
    for (int s = 0; s < p.n_scenes; ++s) {
        tiles[s] = std::max<int64_t>(1, ((p.scenes[s].n + 15) / 16) * p.scenes[s].n_times);
        total += tiles[s];
    }
    std::vector<int> share(p.n_scenes);
    int used = 0;
    for (int s = 0; s < p.n_scenes; ++s) {
        share[s] = std::max(1, (int)((double)blocks * (double)tiles[s] / (double)total));
        used += share[s];
    }
    while (used > blocks) {
        int big = 0;
        for (int s = 1; s < p.n_scenes; ++s) if (share[s] > share[big]) big = s;
        --share[big];
        --used;
    }
    while (used < blocks) {
        int need = 0;
        for (int s = 1; s < p.n_scenes; ++s)
            if ((double)tiles[s] / share[s] > (double)tiles[need] / share[need]) need = s;
        ++share[need];
        ++used;
    }
    int b0 = 0;
    for (int s = 0; s < p.n_scenes; ++s) {
        const h4d_scene_desc& d = p.scenes[s];
        MlpSpan& sp = b.s[s];
        const int F = d.grid.F, L = d.grid.L;
        sp.params = d.params;
        sp.feat = d.feat;
        sp.delta = d.delta;
        sp.d_out = d.d_delta;
        sp.d_feat = nullptr;
        sp.d_params = d.d_params;
        sp.fv = FeatView{(int64_t)d.n * F, F, F == 1 ? 0 : F == 2 ? 1 : F == 4 ? 2 : 3};
        sp.feat_seg = (int64_t)L * d.n * F;
        sp.out_seg = (int64_t)d.n * p.mlp.out;
        sp.n = (int)d.n;
        sp.segs = d.n_times;
        sp.block0 = b0;
        sp.block1 = b0 + share[s];
        b0 += share[s];
    }
}

}  // namespace h4d

static h4d_status plan_fail(h4d_status st, const std::string& msg) { return set_error(st, msg.c_str()); }

namespace h4d {

static h4d_status plan_hip(hipError_t e, const char* where) {
    if (e == hipSuccess) return H4D_OK;
    return plan_fail(H4D_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

static hipError_t plan_forward(h4d_batched_plan& p, hipStream_t s) {
    hipError_t e;
    if (p.dt == H4D_BF16) {
        for (auto& d : p.scenes) {
            if (d.table_master && (e = launch_cast_bf16(d.table_master, static_cast<uint16_t*>(d.table),
                                                        d.grid.offset[d.grid.L] * d.grid.F, s)) != hipSuccess)
                return e;
            if (d.params_master && (e = launch_cast_bf16(d.params_master, static_cast<uint16_t*>(d.params),
                                                         param_count(p.mlp), s)) != hipSuccess)
                return e;
        }
    }
    if ((e = launch_bencode(p, p.enc, s)) != hipSuccess) return e;
    return launch_mlp_forward_batch(p.dt, p.mlp.in, p.mlp.out, p.fwd, p.fwd_blocks, s);
}

static hipError_t plan_backward(h4d_batched_plan& p, hipStream_t s) {
    hipError_t e;
    if (p.flags & H4D_PLAN_ZERO_GRADS) {
        for (auto& d : p.scenes) {
            const int64_t te = d.grid.offset[d.grid.L] * d.grid.F;
            hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<int64_t>((te + 255) / 256, 8192)), dim3(256), 0, s,
                               d.d_table, te);
            hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, s, d.d_params, param_count(p.mlp));
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const double S = p.loss_scale;
    if ((e = launch_mlp_backward_batch(p.dt, p.mlp.in, p.mlp.out, p.bwd, p.bwd_blocks, S, 1.0, 1.0 / S, p.ws, s)) !=
        hipSuccess)
        return e;
    return launch_bscatter(p, (float)(1.0 / S), s);
}

}  // namespace h4d

namespace h4d {

// Time every candidate schedule (queries per thread x levels per item x grid) of
// the batched encode kernel on the plan's own data and keep the fastest.  The
// stream is synchronised before a work list is replaced, so no launch ever reads
// a freed list.
static hipError_t autotune(h4d_batched_plan& p, const std::vector<BSeg>& segs, hipStream_t st) {
    const int qpts[] = {1, 2};
    const int lpbs[] = {1, 2, 4};
    const int grids[] = {1024, 2048, 4096, 8192};
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    float best = 1e30f;
    BSchedule best_s = p.enc;
    auto install = [&](const BSchedule& c) -> hipError_t {
        hipError_t e2 = hipStreamSynchronize(st);
        if (e2 != hipSuccess) return e2;
        std::vector<BRange> rr = build_ranges(p, segs, c, &p.total_enc);
        p.nranges_enc = (int)rr.size();
        return upload_ranges(&p.ranges_enc, rr);
    };
    for (int qpt : qpts)
        for (int lpb : lpbs)
            for (int gsz : grids) {
                if (e != hipSuccess) continue;
                const BSchedule cand{qpt, lpb, gsz};
                if ((e = install(cand)) != hipSuccess || (e = launch_bencode(p, cand, st)) != hipSuccess) continue;
                hipEventRecord(a, st);
                for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) e = launch_bencode(p, cand, st);
                hipEventRecord(b, st);
                if (e == hipSuccess) e = hipEventSynchronize(b);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                if (e != hipSuccess) continue;
                ms /= 3.f;
                p.tuned.push_back(h4d_tune_result{0, qpt, lpb, gsz, ms});
                if (ms < best) {
                    best = ms;
                    best_s = cand;
                }
            }
    if (e == hipSuccess) {
        e = install(best_s);
        p.enc = best_s;
    }
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    return e;
}

}  // namespace h4d

extern "C" {

h4d_status hash4d_batched_plan_create(h4d_batched_plan** out, const h4d_scene_desc* scenes, int32_t n_scenes,
                                      const h4d_mlp* m, h4d_dtype dt, float loss_scale, int32_t flags, void* stream) {
    clear_error();
    if (!out) return plan_fail(H4D_EINVAL, "plan output pointer is NULL");
    *out = nullptr;
    if (!scenes || n_scenes < 1 || n_scenes > H4D_MAX_SCENES)
        return plan_fail(H4D_EINVAL, "need 1..16 scenes");
    if (!m || m->hidden != H4D_HIDDEN || m->out < 1 || m->out > H4D_MAX_OUT ||
        (m->in != 8 && m->in != 16 && m->in != 32 && m->in != 64))
        return plan_fail(H4D_EINVAL, "bad decoder shape");
    if (dt != H4D_F32 && dt != H4D_BF16) return plan_fail(H4D_EUNSUPPORTED, "batched plans run F32 or BF16");
    if (!(loss_scale > 0.f)) return plan_fail(H4D_EINVAL, "loss_scale must be > 0");
    const int F0 = scenes[0].grid.F;
    int64_t queries = 0;
    for (int s = 0; s < n_scenes; ++s) {
        const h4d_scene_desc& d = scenes[s];
        h4d_status st = validate_grid(&d.grid);
        if (st != H4D_OK) return plan_fail(st, "scene " + std::to_string(s) + ": " + std::string(h4d_last_error()));
        if (d.grid.F != F0) return plan_fail(H4D_EINVAL, "all scenes need the same F");
        if (d.grid.L * d.grid.F != m->in) return plan_fail(H4D_EINVAL, "scene " + std::to_string(s) + ": L F != in");
        if (d.n < 0 || d.n * (int64_t)d.grid.L * d.grid.F > 2147483647LL)
            return plan_fail(H4D_EINVAL, "scene " + std::to_string(s) + ": n out of range");
        if (d.n_times < 1 || d.n_times > H4D_MAX_TIMES) return plan_fail(H4D_EINVAL, "n_times outside 1..8");
        if (d.n > 0 && (!d.xyz || !d.table || !d.params || !d.feat || !d.delta || !d.d_delta || !d.d_table ||
                        !d.d_params))
            return plan_fail(H4D_EINVAL, "scene " + std::to_string(s) + ": NULL buffer");
        if (((uintptr_t)d.xyz) & 15u) return plan_fail(H4D_EINVAL, "xyz not 16-byte aligned");
        queries += d.n * d.n_times;
    }
    h4d_batched_plan* p = new h4d_batched_plan();
    p->n_scenes = n_scenes;
    p->mlp = *m;
    p->dt = dt;
    p->flags = flags;
    p->loss_scale = loss_scale;
    p->scenes.assign(scenes, scenes + n_scenes);
    p->queries = queries;
    const hipStream_t st = (hipStream_t)stream;
    auto bail = [&](h4d_status s2) {
        hash4d_batched_plan_destroy(p);
        return s2;
    };
    // grids and segments
    std::vector<BSeg> segs;
    int64_t dfeat_elems = 0;
    for (int s = 0; s < n_scenes; ++s) {
        const h4d_scene_desc& d = scenes[s];
        p->grids_h.push_back(to_device(d.grid));
        dfeat_elems += (int64_t)d.n_times * d.grid.L * d.n * d.grid.F;
    }
    hipError_t e = hipMalloc((void**)&p->d_feat, std::max<int64_t>(dfeat_elems, 1) * sizeof(float));
    if (e != hipSuccess) return bail(plan_hip(e, "plan d_feat"));
    int64_t mask_elems = 0;
    for (int s = 0; s < n_scenes; ++s) mask_elems += (int64_t)scenes[s].n_times * scenes[s].grid.L * mask_stride(scenes[s].n);
    if ((e = hipMalloc((void**)&p->masks, std::max<int64_t>(mask_elems, 1) * sizeof(uint32_t))) != hipSuccess)
        return bail(plan_hip(e, "plan masks"));
    int64_t mo = 0;
    int64_t dfo = 0;
    for (int s = 0; s < n_scenes; ++s) {
        const h4d_scene_desc& d = scenes[s];
        const int64_t seg_elems = (int64_t)d.grid.L * d.n * d.grid.F;
        for (int k = 0; k < d.n_times; ++k) {
            BSeg b;
            b.xyz = reinterpret_cast<const float4*>(d.xyz);
            b.t = d.times[k];
            b.n = (int)d.n;
            b.scene = s;
            b.table = d.table;
            b.feat = d.feat + k * seg_elems;
            b.d_feat = p->d_feat + dfo + k * seg_elems;
            b.d_table = d.d_table;
            b.mask = p->masks + mo;
            mo += (int64_t)d.grid.L * mask_stride(d.n);
            segs.push_back(b);
        }
        dfo += d.n_times * seg_elems;
    }
    p->nseg = (int)segs.size();
    if ((e = hipMalloc((void**)&p->grids, p->grids_h.size() * sizeof(DevGrid))) != hipSuccess ||
        (e = hipMemcpy(p->grids, p->grids_h.data(), p->grids_h.size() * sizeof(DevGrid), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMalloc((void**)&p->segs, segs.size() * sizeof(BSeg))) != hipSuccess ||
        (e = hipMemcpy(p->segs, segs.data(), segs.size() * sizeof(BSeg), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(plan_hip(e, "plan tables"));
    // scatter tiles: (scene, level, rows) with at most kTileBytes of FP32 rows each
    {
        std::vector<BTile> tiles;
        std::vector<TileMap> tms;
        int seg0 = 0;
        for (int sc = 0; sc < n_scenes; ++sc) {
            const h4d_scene_desc& d = scenes[sc];
            int64_t lrows[H4D_MAX_LEVELS];
            for (int l = 0; l < d.grid.L; ++l) lrows[l] = d.grid.offset[l + 1] - d.grid.offset[l];
            const TileMap tm = make_tile_map(p->grids_h[sc], lrows, d.grid.F, (int)sizeof(float));
            tms.push_back(tm);
            for (int l = 0; l < d.grid.L; ++l) {
                const int P = tm.tile_start[l + 1] - tm.tile_start[l];
                for (int t = 0; t < P; ++t) {
                    const int64_t r = d.grid.offset[l] + ((int64_t)t << tm.tile_shift[l]);
                    const uint32_t cnt = (uint32_t)std::min<int64_t>((int64_t)1 << tm.tile_shift[l], d.grid.offset[l + 1] - r);
                    tiles.push_back(BTile{sc, l, seg0, d.n_times, (uint32_t)r, cnt, 1u << (t >> tm.bit_shift[l])});
                }
            }
            seg0 += d.n_times;
            p->max_n = std::max(p->max_n, (int)d.n);
            p->max_L = std::max(p->max_L, (int)d.grid.L);
        }
        p->ntiles = (int)tiles.size();
        // eight runs of about equal work: a tile scans its scene's queries at every timestamp
        {
            double total = 0.0;
            for (const BTile& t : tiles) total += (double)scenes[t.scene].n * t.nseg;
            double acc = 0.0;
            int x = 0;
            p->xcd_runs.start[0] = 0;
            for (int i = 0; i < (int)tiles.size(); ++i) {
                acc += (double)scenes[tiles[i].scene].n * tiles[i].nseg;
                while (x + 1 < kXcds && acc >= total * (x + 1) / kXcds) p->xcd_runs.start[++x] = i + 1;
            }
            while (x < kXcds) p->xcd_runs.start[++x] = (int)tiles.size();
        }
        if ((e = hipMalloc((void**)&p->tiles, std::max<size_t>(1, tiles.size()) * sizeof(BTile))) != hipSuccess ||
            (e = hipMemcpy(p->tiles, tiles.data(), tiles.size() * sizeof(BTile), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMalloc((void**)&p->tms, tms.size() * sizeof(TileMap))) != hipSuccess ||
            (e = hipMemcpy(p->tms, tms.data(), tms.size() * sizeof(TileMap), hipMemcpyHostToDevice)) != hipSuccess)
            return bail(plan_hip(e, "plan tiles"));
    }
    // decoder spans
    p->fwd_blocks = mlp_blocks_for(dt, false, queries);
    p->bwd_blocks = std::max(mlp_blocks_for(dt, true, queries), n_scenes);
    p->fwd_blocks = std::max(p->fwd_blocks, n_scenes);
    split_blocks(*p, p->fwd, p->fwd_blocks);
    split_blocks(*p, p->bwd, p->bwd_blocks);
    dfo = 0;
    for (int s = 0; s < n_scenes; ++s) {
        p->bwd.s[s].d_feat = p->d_feat + dfo;
        p->fwd.s[s].d_feat = nullptr;
        dfo += (int64_t)scenes[s].n_times * scenes[s].grid.L * scenes[s].n * scenes[s].grid.F;
    }
    p->ws_bytes = mlp_partial_bytes(dt, m->in, m->out, p->bwd_blocks, n_scenes);
    if ((e = hipMalloc(&p->ws, std::max<size_t>(p->ws_bytes, 16))) != hipSuccess) return bail(plan_hip(e, "plan ws"));
    // schedule: default, or the fastest measured candidate
    std::vector<BRange> r = build_ranges(*p, segs, p->enc, &p->total_enc);
    p->nranges_enc = (int)r.size();
    if ((e = upload_ranges(&p->ranges_enc, r)) != hipSuccess) return bail(plan_hip(e, "plan ranges"));
    if (flags & H4D_PLAN_AUTOTUNE) {
        if ((e = autotune(*p, segs, st)) != hipSuccess) return bail(plan_hip(e, "autotune"));
    }
    if (flags & H4D_PLAN_GRAPH) {
        hipStream_t cs;
        if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess)
            return bail(plan_hip(e, "capture stream"));
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e1 = plan_forward(*p, cs);
            hipError_t e2 = e1 == hipSuccess ? plan_backward(*p, cs) : e1;
            e = hipStreamEndCapture(cs, &p->graph);
            if (e == hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        hipStreamDestroy(cs);
        if (e != hipSuccess) return bail(plan_hip(e, "graph capture"));
    }
    *out = p;
    return H4D_OK;
}

h4d_status hash4d_batched_forward(h4d_batched_plan* p, void* stream) {
    clear_error();
    if (!p) return plan_fail(H4D_ENOPLAN, "plan is NULL");
    return plan_hip(plan_forward(*p, (hipStream_t)stream), "hash4d_batched_forward");
}

h4d_status hash4d_batched_backward(h4d_batched_plan* p, void* stream) {
    clear_error();
    if (!p) return plan_fail(H4D_ENOPLAN, "plan is NULL");
    return plan_hip(plan_backward(*p, (hipStream_t)stream), "hash4d_batched_backward");
}

h4d_status hash4d_batched_run(h4d_batched_plan* p, void* stream) {
    clear_error();
    if (!p) return plan_fail(H4D_ENOPLAN, "plan is NULL");
    if (!p->exec) {
        hipError_t e = plan_forward(*p, (hipStream_t)stream);
        if (e == hipSuccess) e = plan_backward(*p, (hipStream_t)stream);
        return plan_hip(e, "hash4d_batched_run");
    }
    return plan_hip(hipGraphLaunch(p->exec, (hipStream_t)stream), "hash4d_batched_run");
}

h4d_status hash4d_batched_plan_info(const h4d_batched_plan* p, h4d_batched_info* info) {
    clear_error();
    if (!p) return plan_fail(H4D_ENOPLAN, "plan is NULL");
    if (!info) return plan_fail(H4D_EINVAL, "info is NULL");
    memset(info, 0, sizeof *info);
    info->queries = p->queries;
    info->segments = p->nseg;
    info->encode_qpt = p->enc.qpt;
    info->encode_lpb = p->enc.lpb;
    info->encode_grid = p->enc.grid;
    info->scatter_tiles = p->ntiles;
    info->scatter_rows_per_tile = kTileBytes / (p->scenes[0].grid.F * (int)sizeof(float));
    info->graph = p->exec != nullptr;
    info->n_tuned = (int32_t)std::min<size_t>(p->tuned.size(), H4D_MAX_TUNED);
    for (int i = 0; i < info->n_tuned; ++i) info->tuned[i] = p->tuned[i];
    return H4D_OK;
}

void hash4d_batched_plan_destroy(h4d_batched_plan* p) {
    if (!p) return;
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    hipFree(p->grids);
    hipFree(p->segs);
    hipFree(p->ranges_enc);
    hipFree(p->tiles);
    hipFree(p->tms);
    hipFree(p->masks);
    hipFree(p->d_feat);
    hipFree(p->ws);
    delete p;
}

}  // extern "C"
