#!/usr/bin/env python3
"""Throughput of the DASH 4D hash deformation path (forward + backward) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-probes]

Workload: the paper-shaped scene -- 200k dynamic Gaussians in a 64-cluster cloud,
timestamps on a 300-frame grid, L = 16 levels, F = 2, T = 2^19 rows per hashed
level, spatial resolutions 16 -> 2048 and temporal 16 -> 150 (Eq. 7), decoder
32 -> 64 -> 64 -> 10.  Synthetic inputs (seed 0) stand in for the paper's scenes.

One step = zero the table / decoder gradients, encode (Eqs. 8-9), decode, decoder
backward, table scatter: every kernel of the path, inputs resident in HBM.  The
timed region is bracketed by device synchronisation; HIP events on the stream the
kernels run on split it per kernel.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "4D-hash deform queries/s fwd+bwd (N=200k, L=16, T=2^19), BF16 vs FP32"
HBM_PEAK_GBPS = 8000.0
KERNEL_SOURCES = ("encode.hip", "h4d_device.h", "h4d_internal.h", "mlp.hip")
# the library kernels behind each timed part of the step
STEP_KERNELS = {"cast": ["k_cast_bf16"], "encode": ["k_encode"], "decode": ["k_mlp_forward"],
                "decode_bwd": ["k_mlp_backward", "k_mlp_reduce"],
                "scatter": ["k_tile_mask", "k_tile_plan", "k_scatter_tiled", "k_tile_combine"]}
TRAFFIC_FILE = os.path.join("profiles", "traffic_deform_paper_scene_fp32.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-probes", action="store_true", help="skip the roofline probes")
    ap.add_argument("--no-batched", action="store_true", help="skip the multi-scene form")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the steps beyond the path (input gradient, optimiser, front end, whole scene)")
    ap.add_argument("--counters", action="store_true",
                    help="a few FP32 steps plus one 256 MiB copy kernel (the calibration reference of the "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE passes); prints the step kernels' names")
    ap.add_argument("--counters-form", default="fp32", choices=("fp32", "bf16"),
                    help="the form the --counters run steps")
    ap.add_argument("--fetch-calibration", action="store_true",
                    help="only 2^22 random 8-byte loads over a 2 GiB table (twice) and one 256 MiB copy: the "
                         "kernels that check the FETCH_SIZE scaling on random and streaming reads")
    ap.add_argument("--probe-sweep", action="store_true",
                    help="only run the gather / atomic probes over several footprints and print them")
    ap.add_argument("--cpu-sample", type=int, default=200000, help="queries the CPU oracle is timed on")
    return ap.parse_args()


def source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2507_19141_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


class Path:
    """Device buffers and the step of one form (fp32 or bf16) of the workload."""

    def __init__(self, torch, _lib, synth, form: str, n: int | None = None, shared_frame: int | None = None):
        self.torch, self.L_, self.form = torch, _lib, form
        w = synth.PAPER_SCENE
        self.w = w
        rng, x = synth.scene_inputs(w.n if n is None else n, 0, shared_frame=shared_frame)
        rs = _lib.h4d_grid_schedule(w.L, *w.space)
        rt = _lib.h4d_grid_schedule(w.L, *w.time)
        self.g = _lib.h4d_grid_init(w.L, w.F, rs, rt, w.T)
        self.m = _lib.mlp_shape(w.n_in)
        E, F, n = self.g.E, w.F, x.shape[0]
        table = synth.table_init(E, F, rng)
        params = synth.decoder_params(w.n_in, rng)
        gd = synth.upstream(n, 10, rng)
        dev = lambda a: torch.from_numpy(a).cuda()
        self.n, self.E = n, E
        self.xyzt = dev(x)
        self.table32 = dev(table)
        self.params32 = dev(params)
        self.d_delta = dev(gd)
        self.feat = torch.empty((w.L, n, F), device="cuda")
        self.delta = torch.empty((n, 10), device="cuda")
        self.d_feat = torch.empty((w.L, n, F), device="cuda")
        self.d_table = torch.zeros((E, F), device="cuda")
        self.d_params = torch.zeros(params.size, device="cuda")
        self.dt = _lib.BF16 if form == "bf16" else _lib.F32
        self.ws_bytes = _lib.deform_mlp_workspace_bytes(self.m, self.dt, n)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.sws_bytes = _lib.hash4d_encode_backward_workspace_bytes(self.g, n)
        self.sws = torch.empty(self.sws_bytes, dtype=torch.uint8, device="cuda")
        if form == "bf16":
            self.table_lo = torch.empty(E * F, dtype=torch.int16, device="cuda")
            self.params_lo = torch.empty(params.size, dtype=torch.int16, device="cuda")
            self.counter = torch.zeros(1, dtype=torch.int32, device="cuda")
            self.loss_scale = 4096.0
        self.names = (["cast"] if form == "bf16" else []) + ["encode", "decode", "decode_bwd", "scatter"]

    def step(self, ev=None):
        L_, t = self.L_, self.torch
        LM, F = L_.LEVEL_MAJOR, self.w.F
        k = 0

        def mark():
            nonlocal k
            if ev is not None:
                ev[k].record()
            k += 1
        # both backward calls write their gradient outputs (no separate zeroing pass)
        mark()
        if self.form == "bf16":
            # precision glue: BF16 copies of the FP32 masters, loss-scaled backward, overflow count
            L_.h4d_cast_bf16(self.table32, self.table_lo, self.E * F)
            L_.h4d_cast_bf16(self.params32, self.params_lo, self.params32.numel())
            self.counter.zero_()
            mark()
            table, params, S = self.table_lo, self.params_lo, self.loss_scale
        else:
            table, params, S = self.table32, self.params32, 1.0
        L_.hash4d_encode(self.g, self.dt, table, self.xyzt, self.n, self.feat, LM)
        mark()
        L_.deform_mlp_forward(self.m, self.dt, params, self.feat, self.n, self.delta, LM, F)
        mark()
        # the decoder backward scales d_delta by S on load and writes d_feat and
        # d_params times 1 / S, so the scatter takes d_feat unscaled (grad_scale 1)
        if self.form == "bf16":
            # the overflow test: both backward calls count the non-finite values they
            # write (all of d_params and d_table)
            L_.deform_mlp_backward_checked(self.m, self.dt, params, self.feat, self.n, self.d_delta, S, 1.0 / S,
                                           self.d_feat, self.d_params, self.ws, self.ws_bytes, self.counter,
                                           LM | L_.GRAD_OVERWRITE, F)
        else:
            L_.deform_mlp_backward(self.m, self.dt, params, self.feat, self.n, self.d_delta, S, 1.0 / S, self.d_feat,
                                   self.d_params, self.ws, self.ws_bytes, LM | L_.GRAD_OVERWRITE, F)
        mark()
        if self.form == "bf16":
            L_.hash4d_encode_backward_checked(self.g, L_.F32, self.xyzt, self.n, self.d_feat, 1.0, self.d_table,
                                              self.sws, self.sws_bytes, self.counter, LM | L_.GRAD_OVERWRITE)
        else:
            L_.hash4d_encode_backward(self.g, L_.F32, self.xyzt, self.n, self.d_feat, 1.0, self.d_table, self.sws,
                                      self.sws_bytes, LM | L_.GRAD_OVERWRITE)
        mark()

    def step_smooth(self, eps, loss, sws, swb, lam: float, merged: bool):
        """FP32 training step with the smoothness term: the step above plus Eq. 11,
        either as the two separate calls or with the table gradient of both in one
        scatter (hash4d_encode_backward_smooth)."""
        L_, LM, F, OW = self.L_, self.L_.LEVEL_MAJOR, self.w.F, self.L_.GRAD_OVERWRITE
        table, params = self.table32, self.params32
        L_.hash4d_encode(self.g, L_.F32, table, self.xyzt, self.n, self.feat, LM)
        L_.deform_mlp_forward(self.m, L_.F32, params, self.feat, self.n, self.delta, LM, F)
        L_.deform_mlp_backward(self.m, L_.F32, params, self.feat, self.n, self.d_delta, 1.0, 1.0, self.d_feat,
                               self.d_params, self.ws, self.ws_bytes, LM | OW, F)
        if merged:
            L_.hash4d_encode_backward_smooth(self.g, L_.F32, table, self.xyzt, eps, self.n, self.d_feat, 1.0, lam,
                                             loss, self.d_table, sws, swb, LM | OW)
        else:
            L_.hash4d_encode_backward(self.g, L_.F32, self.xyzt, self.n, self.d_feat, 1.0, self.d_table, self.sws,
                                      self.sws_bytes, LM | OW)
            L_.smoothness_reg(self.g, L_.F32, table, self.xyzt, eps, self.n, lam, loss, self.d_table, sws, swb)

    def run(self, steps: int, warmup: int):
        t = self.torch
        for _ in range(warmup):
            self.step()
        nev = len(self.names) + 1
        evs = [[t.cuda.Event(enable_timing=True) for _ in range(nev)] for _ in range(steps)]
        t.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            self.step(evs[s])
        t.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = {name: 0.0 for name in self.names}
        for s in range(steps):
            for i, name in enumerate(self.names):
                per[name] += evs[s][i].elapsed_time(evs[s][i + 1])
        per = {k: v / steps for k, v in per.items()}
        gpu_ms = evs[0][0].elapsed_time(evs[-1][-1]) / steps
        return wall, gpu_ms, per


def algorithmic_bytes(L, F, table_bytes, out=10):
    """Bytes per query each kernel must move: every corner row read or updated once
    (16 L per query), features read/written once, inputs and outputs once."""
    feat = L * F * 4
    return {
        "encode": 16 + 16 * L * F * table_bytes + feat,
        "decode": feat + out * 4,
        "decode_bwd": feat + out * 4 + feat,
        "scatter": 16 + feat + 16 * L * F * 4,
    }


def probes(torch, _lib, E, F, n_loads, reps=5):
    """Random-gather, random-atomic and copy ceilings at the workload's footprint."""
    out = {}
    buf = torch.rand((E, F), device="cuda")
    sink = torch.zeros(1, device="cuda")
    st = torch.cuda.current_stream()

    def timed(fn):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(reps):
            fn()
        b.record(st)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps / 1e3
    t = timed(lambda: _lib.h4d_probe_gather(buf, E, 8, n_loads, 7, sink))
    out["gather8_GBps"] = n_loads * 8 / t / 1e9
    t = timed(lambda: _lib.h4d_probe_gather(buf, 2 * E, 4, n_loads, 7, sink))
    out["gather4_GBps"] = n_loads * 4 / t / 1e9
    t = timed(lambda: _lib.h4d_probe_scatter(buf, E, n_loads, 9, 0))
    out["scatter8_GBps"] = n_loads * 8 / t / 1e9
    t = timed(lambda: _lib.h4d_probe_scatter(buf, E, n_loads, 9, 1))
    out["scatter8_xcd_owned_GBps"] = n_loads * 8 / t / 1e9
    t = timed(lambda: _lib.h4d_probe_scatter(buf, 1 << 17, n_loads, 9, 0))
    out["scatter8_1MiB_GBps"] = n_loads * 8 / t / 1e9
    # random 8-byte gathers over 4 MiB: the footprint one XCD's L2 holds, which is
    # what the level-placed encoder presents to each XCD
    t = timed(lambda: _lib.h4d_probe_gather(buf, 1 << 19, 8, n_loads, 7, sink))
    out["gather8_4MiB_Gloads_per_s"] = n_loads / t / 1e9
    # LDS compare-and-swap adds: 512 workgroups x 1024 threads x 256 adds each
    per, blocks = 256, 512
    t = timed(lambda: _lib.h4d_probe_lds_atomic(blocks, per, 64, 3, 2, sink))
    out["lds_cas_G_per_s"] = blocks * 1024 * per / t / 1e9
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, device="cuda")
    dst = torch.empty_like(src)
    t = timed(lambda: _lib.h4d_probe_copy(src, dst, nbytes))
    out["copy_GBps"] = 2 * nbytes / t / 1e9
    out["footprint_MiB"] = E * F * 4 / 2 ** 20
    out["n_loads"] = n_loads
    del buf, src, dst
    return out


def probe_sweep(torch, _lib, E, n_loads, reps=5):
    """Random FP32 atomics and random gathers over a range of footprints, both atomic
    modes (any row / rows of lines owned by the workgroup's XCC)."""
    buf = torch.zeros((E, 2), device="cuda")
    st = torch.cuda.current_stream()

    def timed(fn):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(reps):
            fn()
        b.record(st)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps / 1e3
    rows_list = [1 << 17, 1 << 19, 1 << 21, E]
    out = {"n": n_loads, "scatter": [], "gather": []}
    for rows in rows_list:
        for mode in (0, 1):
            t = timed(lambda: _lib.h4d_probe_scatter(buf, rows, n_loads, 9, mode))
            out["scatter"].append({"rows": rows, "MiB": rows * 8 / 2 ** 20, "mode": mode, "ms": t * 1e3,
                                   "G_atomics_per_s": 2 * n_loads / t / 1e9})
        t = timed(lambda: _lib.h4d_probe_gather(buf, rows, 8, n_loads, 7, buf))
        out["gather"].append({"rows": rows, "MiB": rows * 8 / 2 ** 20, "ms": t * 1e3, "GBps": n_loads * 8 / t / 1e9,
                              "G_loads_per_s": n_loads / t / 1e9})
    for mode in (0, 1):
        buf.zero_()
        _lib.h4d_probe_scatter(buf, E, n_loads, 9, mode)
        torch.cuda.synchronize()
        out[f"scatter_sum_mode{mode}"] = float(buf.double().sum())
    out["scatter_sum_expected"] = 2.0 * n_loads
    # LDS atomics, 128 KiB tile per 1024-thread workgroup, 512 workgroups
    sink = torch.zeros(1, device="cuda")
    out["lds_atomic"] = []
    for mode, kind in ((0, "ds_add_f32"), (1, "ds_add_u32"), (2, "f32 compare-and-swap")):
        for active in (64, 8):
            per = 256
            t = timed(lambda: _lib.h4d_probe_lds_atomic(512, per, active, 3, mode, sink))
            ops = 512 * 1024 * per * active / 64
            out["lds_atomic"].append({"kind": kind, "active_lanes": active, "ms": t * 1e3,
                                      "G_ops_per_s": ops / t / 1e9, "G_instr_per_s": 512 * 16 * per / t / 1e9})
    return out


def scatter_tile_count(rows_per_level, F=2, gbytes=4):
    """Tiles of the table scatter: per level about 32 tiles of a power of two of rows,
    at least 256 rows and at most 128 KiB of gradient."""
    max_rows = (128 * 1024) // (F * gbytes)
    tiles = 0
    for r in rows_per_level:
        want = -(-r // 32)
        sh = 8
        while (1 << sh) < max_rows and (1 << sh) < want:
            sh += 1
        tiles += -(-r // (1 << sh))
    return tiles


def achievable(torch, _lib, synth, per, pr, n):
    """Each kernel's time against the probe ceiling that matches its access pattern
    (each fraction at most 1 when the kernel runs at that ceiling):
    encode: its corner-row requests (one per x-pair whose rows are an aligned pair,
    two otherwise, counted from the corner rows) at the random-gather request rate of
    a 4 MiB, L2-resident footprint (the level slice each XCD holds);
    scatter: the owner-computes floor, the larger of the time to stream every tile's
    level of query masks at the copy rate and the time for the corner updates at the
    LDS compare-and-swap rate (the queries' own loads taken as free)."""
    w = synth.PAPER_SCENE
    g = _lib.h4d_grid_init(w.L, w.F, _lib.h4d_grid_schedule(w.L, *w.space), _lib.h4d_grid_schedule(w.L, *w.time),
                           w.T)
    _, x = synth.scene_inputs(w.n, 0)
    rows = torch.empty((n, w.L, 16), dtype=torch.int32, device="cuda")
    _lib.hash4d_corner_indices(g, torch.from_numpy(x).cuda(), n, rows, None)
    r0, r1 = rows[..., 0::2], rows[..., 1::2]
    paired = (r1 == (r0 ^ 1)) & ((r0 | 1) < g.E)
    requests = int(n * w.L * 8 + (~paired).sum().item())
    del rows, r0, r1, paired
    t_enc = requests / (pr["gather8_4MiB_Gloads_per_s"] * 1e9)
    level_rows = [g.offsets()[l + 1] - g.offsets()[l] for l in range(w.L)]
    tiles = scatter_tile_count(level_rows)
    mask_stream = tiles * n * 4                        # every tile scans its level's masks
    t_scan = mask_stream / (pr["copy_GBps"] * 1e9)
    t_lds = n * w.L * 16 / (pr["lds_cas_G_per_s"] * 1e9)
    t_sca = max(t_scan, t_lds)
    enc_ms, sca_ms = per["encode"], per["scatter"]
    return {"encode": {"requests": requests, "probe": "gather8_4MiB_Gloads_per_s", "floor_ms": t_enc * 1e3,
                       "ms": enc_ms, "frac": t_enc * 1e3 / enc_ms},
            "scatter": {"tiles": tiles, "mask_stream_bytes": mask_stream, "scan_floor_ms": t_scan * 1e3,
                        "lds_floor_ms": t_lds * 1e3, "floor_ms": t_sca * 1e3, "ms": sca_ms,
                        "frac": t_sca * 1e3 / sca_ms}}


def _oracle_levels(job):
    """One level of the oracle's encode (forward) or table gradient (backward), for the
    all-core CPU baseline: the oracle's own functions on a one-level grid."""
    import numpy as np
    from oracle import hash4d_oracle as O
    kind, l = job
    st = _CPU_STATE
    g = st["g"]
    gl = O.make_grid(1, g.F, [g.res_s[l]], [g.res_t[l]], g.T)
    sl = slice(g.offsets[l], g.offsets[l + 1])
    if kind == "fwd":
        return O.encode(st["x"], st["table"][sl], gl)
    d_feat = st["d_feat"][:, l * g.F:(l + 1) * g.F]
    return O.encode_backward(st["x"], np.ascontiguousarray(d_feat), gl)


_CPU_STATE = {}


def cpu_baseline(sample: int):
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import hash4d_oracle as O
    from paper_2507_19141_amd import synth
    w = synth.PAPER_SCENE
    rng, x = synth.scene_inputs(w.n, 0)
    g = O.make_grid(w.L, w.F, O.level_resolutions(*w.space, w.L), O.level_resolutions(*w.time, w.L), w.T)
    table = synth.table_init(g.E, w.F, rng)
    params = synth.decoder_params(w.n_in, rng)
    gd = synth.upstream(w.n, 10, rng)
    xs, gs = x[:sample], gd[:sample]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        O.deform_forward(xs, table, g, params)
        O.deform_backward(xs, table, g, params, gs)
        dt1 = time.perf_counter() - t0
    # all cores: the levels of the encoder and its table gradient in a process pool
    # (their rows are disjoint), the decoder with BLAS on every core; at most 16
    # workers, the host share one GPU has
    import multiprocessing as mp
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    _CPU_STATE.update({"g": g, "x": xs, "table": table})
    t0 = time.perf_counter()
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        f_h = np.concatenate(pool.map(_oracle_levels, [("fwd", l) for l in range(g.L)]), axis=1)
        with threadpool_limits(limits=cores):
            delta, _ = O.mlp_forward(params, f_h)
            d_feat, d_params = O.mlp_backward(params, f_h, gs)
        _CPU_STATE["d_feat"] = d_feat
    with ctx.Pool(cores) as pool:
        parts = pool.map(_oracle_levels, [("bwd", l) for l in range(g.L)])
        d_table = np.concatenate(parts, axis=0)
    dtn = time.perf_counter() - t0
    _CPU_STATE.clear()
    assert d_table.shape == (g.E, g.F) and delta.shape == (sample, 10) and d_params.size > 0
    return {"value": sample / dtn, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "one_thread_value": sample / dt1,
            "sample": f"first {sample} of the {w.n} clustered queries (all of them by default), full tables; FP64 "
                      f"oracle forward (f_h, delta) + backward (d_table, d_params): {dtn:.1f} s on {cores} cores (the "
                      f"encoder's levels in a process pool, the decoder with {cores} BLAS threads), {dt1:.1f} s on "
                      f"1 thread"}


def batched_form(torch, _lib, synth, steps: int, warmup: int):
    """The multi-scene workload: 8 clustered scenes of 50k..1.2M Gaussians, each at 4
    timestamps, BF16 tables and decoders rounded from FP32 masters every step, one
    autotuned plan replayed as a HIP graph.  Also times the same work as per-scene,
    per-timestamp calls of the plain path, for comparison."""
    import numpy as np
    w = synth.PAPER_SCENE
    m = _lib.mlp_shape(w.n_in)
    rs = _lib.h4d_grid_schedule(w.L, *w.space)
    rt = _lib.h4d_grid_schedule(w.L, *w.time)
    keep, descs = [], []
    for i, n in enumerate(synth.BATCHED_SCENE_N):
        rng = np.random.default_rng(i)
        xyz = synth.clustered_xyz(n, rng)
        x4 = np.concatenate([xyz, np.zeros((n, 1), np.float32)], axis=1)
        g = _lib.h4d_grid_init(w.L, w.F, rs, rt, 1 << synth.batched_table_rows_log2(n))
        table = synth.table_init(g.E, w.F, rng)
        params = synth.decoder_params(w.n_in, rng)
        nt = len(synth.BATCHED_TIMES)
        gd = synth.upstream(n * nt, 10, rng).reshape(nt, n, 10)
        s = {"g": g, "n": n, "xyz": torch.from_numpy(x4).cuda(), "tm": torch.from_numpy(table).cuda(),
             "pm": torch.from_numpy(params).cuda(),
             "t": torch.empty(table.size, dtype=torch.int16, device="cuda"),
             "p": torch.empty(params.size, dtype=torch.int16, device="cuda"),
             "feat": torch.empty((nt, w.L, n, w.F), device="cuda"), "delta": torch.empty((nt, n, 10), device="cuda"),
             "gd": torch.from_numpy(gd).cuda(), "dt": torch.zeros((g.E, w.F), device="cuda"),
             "dp": torch.zeros(params.size, device="cuda")}
        keep.append(s)
        descs.append(_lib.scene_desc(g, n, s["xyz"], synth.BATCHED_TIMES, s["t"], s["p"], s["feat"], s["delta"],
                                     s["gd"], s["dt"], s["dp"], table_master=s["tm"], params_master=s["pm"]))
    flags = _lib.PLAN_AUTOTUNE | _lib.PLAN_GRAPH | _lib.PLAN_ZERO_GRADS

    def timed(plan):
        for _ in range(warmup):
            plan.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.run()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # the same plan in FP32: the FP32 masters are the tables and decoders themselves
    descs32 = [_lib.scene_desc(s["g"], s["n"], s["xyz"], synth.BATCHED_TIMES, s["tm"], s["pm"], s["feat"],
                               s["delta"], s["gd"], s["dt"], s["dp"]) for s in keep]
    plan32 = _lib.BatchedPlan(descs32, m, _lib.F32, 1.0, flags)
    wall32 = timed(plan32)
    plan32.destroy()
    plan = _lib.BatchedPlan(descs, m, _lib.BF16, 4096.0, flags)
    info = plan.info()
    wall = timed(plan)
    q = info.queries
    # the same work as plain per-(scene, timestamp) calls
    ws = {}
    for s in keep:
        for k, tv in enumerate(synth.BATCHED_TIMES):
            s[("x", k)] = s["xyz"].clone().index_fill_(1, torch.tensor([3], device="cuda"), tv)
    def unbatched():
        for s in keep:
            s["dt"].zero_()
            s["dp"].zero_()
            _lib.h4d_cast_bf16(s["tm"], s["t"], s["tm"].numel())
            _lib.h4d_cast_bf16(s["pm"], s["p"], s["pm"].numel())
            for k, tv in enumerate(synth.BATCHED_TIMES):
                xt = s[("x", k)]
                n = s["n"]
                _lib.hash4d_deform_forward(s["g"], m, _lib.BF16, s["t"], s["p"], xt, n, s["feat"][k], s["delta"][k])
                wb = _lib.hash4d_deform_workspace_bytes(s["g"], m, _lib.BF16, n)
                if wb not in ws:
                    ws[wb] = torch.empty(wb, dtype=torch.uint8, device="cuda")
                _lib.hash4d_deform_backward(s["g"], m, _lib.BF16, s["p"], xt, n, s["feat"][k], s["gd"][k], 4096.0,
                                            1 / 4096.0, s["dt"], s["dp"], ws[wb], wb)
    unbatched()
    torch.cuda.synchronize()
    u_steps = max(1, steps // 2)
    t0 = time.perf_counter()
    for _ in range(u_steps):
        unbatched()
    torch.cuda.synchronize()
    u_wall = time.perf_counter() - t0
    plan.destroy()
    return {"value": q * steps / wall, "ms_per_step": wall * 1e3 / steps, "queries_per_step": q,
            "scenes": list(synth.BATCHED_SCENE_N), "timestamps": len(synth.BATCHED_TIMES), "dtype": "bf16",
            "schedule": {"encode_qpt_lpb_grid": [info.encode_qpt, info.encode_lpb, info.encode_grid],
                         "scatter_tiles": info.scatter_tiles},
            "graph": bool(info.graph), "unbatched_value": q * u_steps / u_wall,
            "unbatched_ms_per_step": u_wall * 1e3 / u_steps,
            "fp32": {"value": q * steps / wall32, "ms_per_step": wall32 * 1e3 / steps}}


def form_differences(ref32: dict, path) -> dict:
    """Per output of the step (features, decoder output, table and decoder
    gradients): max and mean |BF16 form - FP32 form| on the same inputs, and the
    max relative to the FP32 output's largest magnitude."""
    out = {}
    for k, a in ref32.items():
        b = getattr(path, k)
        d = (b.double() - a.double()).abs()
        top = float(a.double().abs().max())
        out[k] = {"max_abs": float(d.max()), "mean_abs": float(d.mean()), "fp32_max_abs": top,
                  "max_rel_to_fp32_max": float(d.max()) / top if top > 0 else None}
    return out


def smoothness_form(torch, _lib, synth, path, steps: int):
    """Eq. 11 on the paper scene: loss and table gradient for the 200k queries and
    their perturbed copies (sigma = 1e-3), FP32 table, timed on its own."""
    import numpy as np
    n = path.n
    eps = torch.from_numpy(synth.perturbation(n, np.random.default_rng(5))).cuda()
    loss = torch.zeros(1, device="cuda")
    wb = _lib.smoothness_workspace_bytes(path.g, _lib.F32, n)
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
    call = lambda: _lib.smoothness_reg(path.g, _lib.F32, path.table32, path.xyzt, eps, n, 1.0, loss, path.d_table,
                                       ws, wb)
    for _ in range(3):
        call()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        call()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    # the whole FP32 training step with the term: separate calls vs one scatter
    step_ms = {}
    for merged in (False, True):
        for _ in range(3):
            path.step_smooth(eps, loss, ws, wb, 1.0, merged)
        a.record()
        for _ in range(steps):
            path.step_smooth(eps, loss, ws, wb, 1.0, merged)
        b.record()
        torch.cuda.synchronize()
        step_ms["one_scatter" if merged else "separate"] = a.elapsed_time(b) / steps
    return {"ms": ms, "value": n / (ms / 1e3), "unit": "queries/s", "lambda": 1.0, "sigma": 1e-3,
            "kernels": ["k_smooth", "k_tile_mask", "k_tile_plan", "k_scatter_tiled", "k_tile_combine"],
            "training_step_ms": step_ms, "training_step_value": n / (step_ms["one_scatter"] / 1e3)}


def input_grad_form(torch, _lib, path, steps: int):
    """The next step beyond the path: the encoder's gradient with respect to the
    positions (table FP32, level-major upstream gradients of the last step), timed
    on its own with HIP events."""
    n, w = path.n, path.w
    d_xyzt = torch.zeros((n, 4), device="cuda")
    wb = _lib.hash4d_encode_backward_input_workspace_bytes(path.g, _lib.F32, n)
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")

    def timed(two_pass: bool) -> float:
        call = lambda: _lib.hash4d_encode_backward_input(path.g, _lib.F32, path.table32, path.xyzt, n, path.d_feat,
                                                         1.0, d_xyzt, _lib.LEVEL_MAJOR, ws if two_pass else None,
                                                         wb if two_pass else 0)
        for _ in range(3):
            call()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            call()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps
    ms, ms_one = timed(True), timed(False)
    bytes_q = 16 + 16 * w.L * w.F * 4 + w.L * w.F * 4 + 16
    return {"ms": ms, "value": n / (ms / 1e3), "unit": "queries/s", "algorithmic_bytes_per_query": bytes_q,
            "achieved_GBps": bytes_q * n / (ms / 1e3) / 1e9,
            "kernels": ["k_input_grad_levels", "k_input_grad_reduce"], "one_pass_ms": ms_one}


def adam_form(torch, _lib, E: int, F: int, steps: int):
    """The optimiser step over the paper scene's FP32 table master (E x F values):
    Adam on the touched rows, the BF16 copy and the gradient zeroing in one pass."""
    count = E * F
    p = torch.randn(count, device="cuda")
    gr = torch.randn(count, device="cuda")
    m = torch.zeros(count, device="cuda")
    v = torch.zeros(count, device="cuda")
    lo = torch.empty(count, dtype=torch.int16, device="cuda")
    flags = _lib.ADAM_LAZY | _lib.ADAM_ZERO_GRAD
    call = lambda t: _lib.h4d_adam_step(p, gr, m, v, count, 1e-3, 0.9, 0.999, 1e-15, t, 1 / 4096, lo, F, flags)
    for t in range(1, 4):
        call(t)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for t in range(steps):
        call(4 + t)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    bytes_el = 4 * 4 + 3 * 4 + 2 + 4   # read p g m v; write p m v, the BF16 copy, the zeroed gradient
    gbps = bytes_el * count / (ms / 1e3) / 1e9
    return {"ms": ms, "elements": count, "algorithmic_bytes_per_element": bytes_el, "achieved_GBps": gbps,
            "frac_of_hbm_peak": gbps / HBM_PEAK_GBPS, "kernel": "k_adam"}


def front_end_form(torch, _lib, synth, steps: int):
    """The step before the path (Section 4.1) on the paper-shaped cloud of 200k
    Gaussians: the 3D hash encoding G_3D of the positions (Eq. 3, L = 16, F = 2,
    T = 2^19, Eq. 7 from 16 to 2048), the 32-64-64-3 decoder for the linear motion dp,
    and the top-10% dynamic split with the static constraint and its gradient."""
    import numpy as np
    w = synth.PAPER_SCENE
    n = w.n
    rng, x = synth.scene_inputs(n, 0)
    g = _lib.h4d_grid3_init(w.L, w.F, _lib.h4d_grid_schedule(w.L, *w.space), w.T)
    table = torch.from_numpy(synth.table_init(g.E, w.F, rng, 1e-1)).cuda()
    params = torch.from_numpy(synth.decoder_params(w.n_in, rng, out=3)).cuda()
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    m = _lib.mlp_shape(w.n_in, out=3)
    feat = torch.empty((w.L, n, w.F), device="cuda")
    dp = torch.empty((n, 3), device="cuda")
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    loss = torch.zeros(1, device="cuda")
    d_dp = torch.zeros((n, 3), device="cuda")
    wb = _lib.hash4d_decompose_workspace_bytes(n)
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step(timed):
        if timed:
            ev[0].record()
        _lib.hash3d_encode(g, _lib.F32, table, xd, 4, n, feat, _lib.LEVEL_MAJOR)
        if timed:
            ev[1].record()
        _lib.deform_mlp_forward(m, _lib.F32, params, feat, n, dp, _lib.LEVEL_MAJOR, w.F)
        if timed:
            ev[2].record()
        _lib.hash4d_decompose(dp, n, 10.0, 1.0, idx, cnt, None, loss, d_dp, ws, wb)
        if timed:
            ev[3].record()
    for _ in range(3):
        step(False)
    torch.cuda.synchronize()
    enc = dec = split = 0.0
    for _ in range(steps):
        step(True)
        torch.cuda.synchronize()
        enc += ev[0].elapsed_time(ev[1])
        dec += ev[1].elapsed_time(ev[2])
        split += ev[2].elapsed_time(ev[3])
    # G_3D moves 12 B of position, 8 corner rows of 8 B and 8 B of features per (query, level)
    enc_bytes = n * (16 + w.L * (8 * 8 + 8))
    return {"gaussians": n, "k_percent": 10.0, "dynamic": int(cnt.item()), "encode3_ms": enc / steps,
            "encode3_GBps": enc_bytes / (enc / steps / 1e3) / 1e9, "decode_ms": dec / steps,
            "encode_decode_ms": (enc + dec) / steps, "split_ms": split / steps,
            "value": n / ((enc + dec + split) / steps / 1e3), "unit": "Gaussians/s"}


def whole_scene_form(torch, _lib, synth, steps: int):
    """The "w/o dec" setting: the same table (T = 2^19) hashing the whole scene, here
    1M clustered Gaussians instead of the 200k dynamic ones.  Reports the collision
    census (V distinct corner vertices, R distinct rows, 1 - R / V) at a middle and
    the finest level for both sets, and the FP32 step on the whole scene."""
    w = synth.PAPER_SCENE
    g = _lib.h4d_grid_init(w.L, w.F, _lib.h4d_grid_schedule(w.L, *w.space), _lib.h4d_grid_schedule(w.L, *w.time),
                           w.T)
    out = {"census": {}}
    for label, n in (("dynamic_200k", w.n), ("whole_1M", 1_000_000)):
        _, x = synth.scene_inputs(n, 0)
        xd = torch.from_numpy(x).cuda()
        counts = torch.zeros(2, dtype=torch.int64, device="cuda")
        out["census"][label] = {}
        for level in (9, w.L - 1):
            wb = _lib.hash4d_collision_workspace_bytes(g, level, n)
            ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
            _lib.hash4d_collision_census(g, level, xd, n, counts, ws, wb)
            V, R = (int(v) for v in counts.cpu())
            out["census"][label][f"level{level}"] = {"V": V, "R": R, "collision_rate": 1.0 - R / V}
            del ws
    path = Path(torch, _lib, synth, "fp32", n=1_000_000)
    wall, gpu_ms, per = path.run(steps, 2)
    out["whole_scene_step"] = {"n": path.n, "value": path.n * steps / wall, "ms_per_step": wall * 1e3 / steps,
                               "kernels_ms": per}
    return out


def traffic_record(dominant: str):
    """HBM bytes per launch of the dominant part of the step, from the committed
    rocprofv3 --pmc summary (its fenced json block), if that was taken for the current
    kernel sources; None otherwise."""
    p = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        text = fh.read()
    if "```json" not in text:
        return None
    rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    if rec.get("source_hash") != source_hash():
        return None
    total = 0.0
    for k in STEP_KERNELS[dominant]:
        if k not in rec.get("kernels", {}):
            return None
        total += rec["kernels"][k]["bytes_per_launch"]
    return total


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported "
                                   "(the multi-GPU sharding is described, not built)"}))
        sys.exit(2)
    import torch

    from paper_2507_19141_amd import _lib, synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    _lib.load()
    if args.counters:
        fp = Path(torch, _lib, synth, args.counters_form)
        fp.run(max(1, args.steps), 1)
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, device="cuda")
        dst = torch.empty_like(src)
        _lib.h4d_probe_copy(src, dst, nbytes)
        torch.cuda.synchronize()
        print(json.dumps({"counters_run": {"form": args.counters_form, "steps": args.steps + 1, "copy_bytes": nbytes,
                                           "copy_kernel": "k_probe_copy"}}), flush=True)
        return
    if args.fetch_calibration:
        big = torch.zeros(2 << 30, dtype=torch.uint8, device="cuda")
        sink = torch.zeros(1 << 20, device="cuda")
        for seed in (1, 2):
            _lib.h4d_probe_gather(big, (2 << 30) // 8, 8, 1 << 22, seed, sink)
        src = torch.ones(1 << 26, device="cuda")
        dst = torch.empty_like(src)
        _lib.h4d_probe_copy(src, dst, 1 << 28)
        torch.cuda.synchronize()
        print(json.dumps({"fetch_calibration": {"gather_loads": 1 << 22, "gather_table_bytes": 2 << 30,
                                                "copy_bytes": 1 << 28}}), flush=True)
        return
    if args.probe_sweep:
        w = synth.PAPER_SCENE
        E = _lib.h4d_grid_init(w.L, w.F, _lib.h4d_grid_schedule(w.L, *w.space),
                               _lib.h4d_grid_schedule(w.L, *w.time), w.T).E
        print(json.dumps({"probe_sweep": probe_sweep(torch, _lib, E, w.n * 16 * w.L)}), flush=True)
        return

    fp32 = Path(torch, _lib, synth, "fp32")
    wall, gpu_ms, per = fp32.run(args.steps, args.warmup)
    n = fp32.n
    # the FP32 step's outputs, kept to report the BF16 form against them
    ref32 = {k: getattr(fp32, k).clone() for k in ("feat", "delta", "d_table", "d_params")}
    ms_per_step = wall * 1e3 / args.steps
    value = n * args.steps / wall
    ab = algorithmic_bytes(fp32.w.L, fp32.w.F, 4)
    dominant = max(per, key=per.get)
    achieved = ab[dominant] * n / (per[dominant] / 1e3) / 1e9
    traffic = traffic_record(dominant)
    result = {
        "metric": METRIC, "value": value, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "deform-200k-clustered-L16F2T2^19 fwd+bwd", "n": n, "L": 16, "F": 2, "T": 1 << 19,
                   "res_s": "16->2048", "res_t": "16->150", "decoder": "32-64-64-10", "form": "fp32"},
        "roofline": {"bound": "hbm", "kernel": dominant, "kernels": STEP_KERNELS[dominant], "achieved": achieved,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "algorithmic_bytes_per_query": ab[dominant], "queries_per_launch": n,
                     "launch_ms": per[dominant]},
        "kernels_ms": per,
        "gpu_ms_per_step": gpu_ms,
    }
    if not args.no_next:
        result["next"] = {"input_grad": input_grad_form(torch, _lib, fp32, args.steps),
                          "adam_table": adam_form(torch, _lib, fp32.E, fp32.w.F, args.steps),
                          "front_end": front_end_form(torch, _lib, synth, min(args.steps, 20))}
        torch.cuda.empty_cache()
        result["next"]["whole_scene"] = whole_scene_form(torch, _lib, synth, min(args.steps, 10))
    smooth = smoothness_form(torch, _lib, synth, fp32, args.steps)
    del fp32
    torch.cuda.empty_cache()
    bf = Path(torch, _lib, synth, "bf16")
    wall_b, gpu_b, per_b = bf.run(args.steps, args.warmup)
    result["forms"] = {"bf16": {"value": n * args.steps / wall_b, "ms_per_step": wall_b * 1e3 / args.steps,
                                "kernels_ms": per_b, "loss_scale": bf.loss_scale,
                                "vs_fp32": form_differences(ref32, bf)},
                       "smoothness": smooth}
    del bf, ref32
    torch.cuda.empty_cache()
    # every query at frame 150 of 300: one view per training iteration
    sh = Path(torch, _lib, synth, "fp32", shared_frame=150)
    wall_s, _, per_s = sh.run(args.steps, args.warmup)
    result["forms"]["shared_t"] = {"value": n * args.steps / wall_s, "ms_per_step": wall_s * 1e3 / args.steps,
                                   "kernels_ms": per_s, "frame": 150, "form": "fp32"}
    del sh
    torch.cuda.empty_cache()
    if not args.no_batched:
        result["forms"]["batched"] = batched_form(torch, _lib, synth, max(3, args.steps // 5), 2)
        torch.cuda.empty_cache()
    if not args.no_probes:
        w = synth.PAPER_SCENE
        E = _lib.h4d_grid_init(w.L, w.F, _lib.h4d_grid_schedule(w.L, *w.space),
                               _lib.h4d_grid_schedule(w.L, *w.time), w.T).E
        pr = probes(torch, _lib, E, w.F, n * 16 * w.L)
        result["probes"] = pr
        result["achievable"] = achievable(torch, _lib, synth, per, pr, n)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
