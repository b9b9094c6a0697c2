"""GPU tests of the batched form: several scenes of uneven size, each queried at
several timestamps, in persistent launches with an autotuned schedule and a
captured HIP graph.  The batched outputs equal per-scene calls of the plain path
(bit-exact where no atomics are involved) and match the oracle on samples."""
import numpy as np
import pytest

from oracle import hash4d_oracle as O
from paper_2507_19141_amd import _lib, synth
from tests.util import (RTOL_BF16, RTOL_F32, RTOL_GRAD, mlp_backward_scale, mlp_forward_scale, needs_gpu,
                        scaled_close)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    needs_gpu()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


SCENES = [(1000, 1 << 10), (2500, 1 << 11), (4096 + 77, 1 << 12)]   # (n, T)
TIMES = [(0.0, 0.5), (0.25,), (0.0, 1 / 3, 2 / 3, 1.0)]


def make_scenes(dt, seed=300, masters=False):
    import torch
    L, F = 4, 2
    rs = O.doubling_resolutions(4, 32, L)
    rt = O.doubling_resolutions(4, 16, L)
    out = []
    for i, ((n, T), times) in enumerate(zip(SCENES, TIMES)):
        rng, x = synth.small_inputs(seed + i, n)
        og = O.make_grid(L, F, rs, rt, T)
        lg = _lib.h4d_grid_init(L, F, rs, rt, T)
        table = synth.table_init(og.E, F, rng)
        params = synth.decoder_params(L * F, rng)
        gd = synth.upstream(n * len(times), 10, rng).reshape(len(times), n, 10)
        s = {"n": n, "T": T, "og": og, "lg": lg, "x": x, "times": times, "table": table, "params": params, "gd": gd}
        s["xyz_d"] = dev(x)
        if dt == _lib.BF16:
            s["table_d"] = torch.empty(table.size, dtype=torch.int16, device="cuda")
            s["params_d"] = torch.empty(params.size, dtype=torch.int16, device="cuda")
            s["table_m"] = dev(table)
            s["params_m"] = dev(params)
            if not masters:
                _lib.h4d_cast_bf16(s["table_m"], s["table_d"], table.size)
                _lib.h4d_cast_bf16(s["params_m"], s["params_d"], params.size)
        else:
            s["table_d"], s["params_d"] = dev(table), dev(params)
            s["table_m"] = s["params_m"] = None
        nt = len(times)
        s["feat"] = torch.full((nt, L, n, F), float("nan"), device="cuda")
        s["delta"] = torch.full((nt, n, 10), float("nan"), device="cuda")
        s["gd_d"] = dev(gd)
        s["d_table"] = torch.zeros((og.E, F), device="cuda")
        s["d_params"] = torch.zeros(params.size, device="cuda")
        out.append(s)
    return out


def descs(scenes, masters=False):
    return [_lib.scene_desc(s["lg"], s["n"], s["xyz_d"], s["times"], s["table_d"], s["params_d"], s["feat"],
                            s["delta"], s["gd_d"], s["d_table"], s["d_params"],
                            table_master=s["table_m"] if masters else None,
                            params_master=s["params_m"] if masters else None) for s in scenes]


def oracle_grads(s):
    """Oracle table / decoder gradients of a scene summed over its timestamps, and
    their magnitude scales."""
    og, params = s["og"], s["params"]
    rt = np.zeros((og.E, og.F))
    rp = np.zeros(O.param_count(og.L * og.F))
    st = np.zeros_like(rt)
    sp = np.zeros_like(rp)
    for k, t in enumerate(s["times"]):
        xt = s["x"].copy()
        xt[:, 3] = t
        a, b, _ = O.deform_backward(xt, s["table"], og, params, s["gd"][k])
        f_ref = O.encode(xt, s["table"], og)
        sf, spk = mlp_backward_scale(params, f_ref, s["gd"][k])
        rt += a
        rp += b
        st += O.encode_backward(xt, sf, og)
        sp += spk
    return rt, rp, st, sp


def single_call_reference(s, dt):
    """The same scene through the plain per-call path, one timestamp at a time."""
    import torch
    L, F, n = s["og"].L, s["og"].F, s["n"]
    m = _lib.mlp_shape(L * F)
    feats, deltas = [], []
    d_table = torch.zeros_like(s["d_table"])
    d_params = torch.zeros_like(s["d_params"])
    for k, t in enumerate(s["times"]):
        xt = s["x"].copy()
        xt[:, 3] = t
        xd = dev(xt)
        feat = torch.empty((L, n, F), device="cuda")
        delta = torch.empty((n, 10), device="cuda")
        _lib.hash4d_deform_forward(s["lg"], m, dt, s["table_d"], s["params_d"], xd, n, feat, delta)
        ws_b = _lib.hash4d_deform_workspace_bytes(s["lg"], m, dt, n)
        ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
        _lib.hash4d_deform_backward(s["lg"], m, dt, s["params_d"], xd, n, feat, dev(s["gd"][k]), 1.0, 1.0, d_table,
                                    d_params, ws, ws_b)
        feats.append(host(feat))
        deltas.append(host(delta))
    return np.stack(feats), np.stack(deltas), host(d_table), host(d_params)


@pytest.mark.parametrize("flags", [0, _lib.PLAN_AUTOTUNE | _lib.PLAN_GRAPH])
def test_batched_equals_per_scene_calls_f32(flags):
    scenes = make_scenes(_lib.F32)
    plan = _lib.BatchedPlan(descs(scenes), _lib.mlp_shape(8), _lib.F32, 1.0, flags)
    info = plan.info()
    assert info.queries == sum(n * len(t) for (n, _), t in zip(SCENES, TIMES))
    assert info.segments == sum(len(t) for t in TIMES)
    if flags & _lib.PLAN_AUTOTUNE:
        assert info.n_tuned == 2 * 3 * 4 and info.graph == 1
    assert info.scatter_tiles >= sum(4 for _ in SCENES)
    plan.run()
    for s in scenes:
        feat, delta, _, _ = single_call_reference(s, _lib.F32)
        assert np.array_equal(host(s["feat"]), feat)          # same arithmetic, no atomics
        assert np.array_equal(host(s["delta"]), delta)
        rt, rp, st, sp = oracle_grads(s)
        scaled_close(host(s["d_table"]), rt, st, RTOL_GRAD, "batched d_table")
        scaled_close(host(s["d_params"]), rp, sp, RTOL_GRAD, "batched d_params")
    plan.destroy()


def test_batched_matches_oracle_and_graph_replays():
    import torch
    scenes = make_scenes(_lib.F32, seed=310)
    plan = _lib.BatchedPlan(descs(scenes), _lib.mlp_shape(8), _lib.F32, 1.0, _lib.PLAN_GRAPH | _lib.PLAN_ZERO_GRADS)
    plan.run()
    first = [(host(s["delta"]), host(s["d_table"]), host(s["d_params"])) for s in scenes]
    refs = [oracle_grads(s) for s in scenes]
    for s in scenes:   # oracle on the last timestamp of each scene
        k = len(s["times"]) - 1
        xt = s["x"].copy()
        xt[:, 3] = s["times"][k]
        f_ref, d_ref = O.deform_forward(xt, s["table"], s["og"], s["params"])
        fs = O.encode(xt, np.abs(s["table"]), s["og"])
        scaled_close(host(s["delta"])[k], d_ref, mlp_forward_scale(s["params"], fs), RTOL_F32, "batched delta")
    # replays with eager work in between: gradients are zeroed inside the graph, so every replay
    # must reproduce the first (up to atomic summation order)
    for rep in range(3):
        junk = torch.randn(1000, device="cuda") * 3
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        del junk
        for s, (dl, _, _), (rt, rp, st, sp) in zip(scenes, first, refs):
            assert np.array_equal(host(s["delta"]), dl)
            scaled_close(host(s["d_table"]), rt, st, RTOL_GRAD, f"replay {rep} d_table")
            scaled_close(host(s["d_params"]), rp, sp, RTOL_GRAD, f"replay {rep} d_params")
    plan.destroy()


def test_batched_bf16_with_masters_and_loss_scale():
    scenes = make_scenes(_lib.BF16, seed=320, masters=True)
    plan = _lib.BatchedPlan(descs(scenes, masters=True), _lib.mlp_shape(8), _lib.BF16, 1024.0,
                            _lib.PLAN_GRAPH | _lib.PLAN_ZERO_GRADS | _lib.PLAN_AUTOTUNE)
    plan.run()
    for s in scenes:
        assert np.array_equal(host(s["table_d"]).view(np.uint16), O.bf16_bits(s["table"]).ravel())
        k = 0
        xt = s["x"].copy()
        xt[:, 3] = s["times"][k]
        f_ref, d_ref = O.deform_forward(xt, s["table"], s["og"], s["params"])
        fs = O.encode(xt, np.abs(s["table"]), s["og"])
        scaled_close(host(s["delta"])[k], d_ref, mlp_forward_scale(s["params"], fs), RTOL_BF16, "bf16 delta")
        # loss-scaled BF16 gradients (d_delta times 1024 on load, 1/1024 on the way out)
        # against the oracle on the FP32 masters
        rt, rp, st, sp = oracle_grads(s)
        scaled_close(host(s["d_table"]), rt, st, RTOL_BF16, "bf16 batched d_table")
        scaled_close(host(s["d_params"]), rp, sp, RTOL_BF16, "bf16 batched d_params")
    plan.destroy()


def test_batched_bf16_multi_scene_workload_sampled():
    """The multi-scene workload at its own shape: 8 clustered scenes of 50k .. 1.2M
    Gaussians (seed = scene index), T = 2^17 / 2^18 / 2^19 by scene size, L = 16, F = 2,
    the paper scene's schedule and 32-64-64-10 decoder, 4 timestamps (frames 0, 99,
    199, 299), BF16 tables and decoders rounded from FP32 masters inside the captured
    step, loss scale 4096.  The upstream gradient is zero except on 4096 sampled
    queries per (scene, timestamp), so the whole d_table and d_params equal the
    oracle's sums over the samples (zero rows contribute exact zeros); feat and delta
    are compared on the samples."""
    import torch
    w = synth.PAPER_SCENE
    rs = O.level_resolutions(*w.space, w.L)
    rt_ = O.level_resolutions(*w.time, w.L)
    times = synth.BATCHED_TIMES
    nt = len(times)
    scenes, descriptors = [], []
    for i, n in enumerate(synth.BATCHED_SCENE_N):
        rng = np.random.default_rng(i)
        xyz = synth.clustered_xyz(n, rng)
        x4 = np.concatenate([xyz, np.zeros((n, 1), np.float32)], axis=1)
        T = 1 << synth.batched_table_rows_log2(n)
        og = O.make_grid(w.L, w.F, rs, rt_, T)
        lg = _lib.h4d_grid_init(w.L, w.F, rs, rt_, T)
        assert lg.offsets() == og.offsets
        table = synth.table_init(og.E, w.F, rng)
        params = synth.decoder_params(w.n_in, rng)
        samples = [np.sort(rng.choice(n, 4096, replace=False)) for _ in range(nt)]
        gd = np.zeros((nt, n, 10), np.float32)
        for k in range(nt):
            gd[k, samples[k]] = synth.upstream(4096, 10, rng)
        s = {"n": n, "og": og, "x": x4, "table": table, "params": params, "gd": gd, "samples": samples,
             "xyz_d": dev(x4), "table_m": dev(table), "params_m": dev(params),
             "table_d": torch.empty(table.size, dtype=torch.int16, device="cuda"),
             "params_d": torch.empty(params.size, dtype=torch.int16, device="cuda"),
             "feat": torch.full((nt, w.L, n, w.F), float("nan"), device="cuda"),
             "delta": torch.full((nt, n, 10), float("nan"), device="cuda"), "gd_d": dev(gd),
             "d_table": torch.full((og.E, w.F), float("nan"), device="cuda"),
             "d_params": torch.full((params.size,), float("nan"), device="cuda")}
        scenes.append(s)
        descriptors.append(_lib.scene_desc(lg, n, s["xyz_d"], times, s["table_d"], s["params_d"], s["feat"],
                                           s["delta"], s["gd_d"], s["d_table"], s["d_params"],
                                           table_master=s["table_m"], params_master=s["params_m"]))
    plan = _lib.BatchedPlan(descriptors, _lib.mlp_shape(w.n_in), _lib.BF16, 4096.0,
                            _lib.PLAN_AUTOTUNE | _lib.PLAN_GRAPH | _lib.PLAN_ZERO_GRADS)
    info = plan.info()
    assert info.queries == 4 * sum(synth.BATCHED_SCENE_N) and info.graph == 1
    plan.run()
    for i, s in enumerate(scenes):
        og, table, params = s["og"], s["table"], s["params"]
        feat, delta = host(s["feat"]), host(s["delta"])
        rt = np.zeros((og.E, og.F))
        rp = np.zeros(params.size)
        st, sp = np.zeros_like(rt), np.zeros_like(rp)
        for k, t in enumerate(times):
            idx = s["samples"][k]
            xt = s["x"][idx].copy()
            xt[:, 3] = np.float32(t)
            f_ref, d_ref = O.deform_forward(xt, table, og, params)
            f_scale = O.encode(xt, np.abs(table), og)
            got_f = np.transpose(feat[k][:, idx], (1, 0, 2)).reshape(len(idx), -1)
            scaled_close(got_f, f_ref, f_scale, RTOL_BF16, f"scene {i} t {k} feat")
            scaled_close(delta[k][idx], d_ref, mlp_forward_scale(params, f_scale), RTOL_BF16,
                         f"scene {i} t {k} delta")
            a, b, _ = O.deform_backward(xt, table, og, params, s["gd"][k][idx])
            sf, spk = mlp_backward_scale(params, f_ref, s["gd"][k][idx])
            rt += a
            rp += b
            st += O.encode_backward(xt, sf, og)
            sp += spk
        scaled_close(host(s["d_table"]), rt, st, RTOL_BF16, f"scene {i} d_table")
        scaled_close(host(s["d_params"]), rp, sp, RTOL_BF16, f"scene {i} d_params")
    plan.destroy()


def test_plan_rejects_bad_input():
    scenes = make_scenes(_lib.F32, seed=330)
    d = descs(scenes)
    d[1].n_times = 9
    with pytest.raises(_lib.H4DError):
        _lib.BatchedPlan(d, _lib.mlp_shape(8), _lib.F32)
    d = descs(scenes)
    with pytest.raises(_lib.H4DError):
        _lib.BatchedPlan(d, _lib.mlp_shape(16), _lib.F32)      # L F != in
    with pytest.raises(_lib.H4DError):
        _lib.BatchedPlan(descs(scenes), _lib.mlp_shape(8), _lib.F64)
    assert RTOL_GRAD > 0
