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
