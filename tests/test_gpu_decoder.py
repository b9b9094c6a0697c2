"""GPU parity of the decoder (Section 4.2: trunk of Eq. 9 and the three heads) and of
the whole deformation path through the C ABI, against the FP64 oracle."""
import numpy as np
import pytest

from oracle import hash4d_oracle as O
from paper_2507_19141_amd import _lib, synth
from tests.util import (RTOL_BF16, RTOL_F32, RTOL_GRAD, lib_grid, mlp_backward_scale, mlp_forward_scale, needs_gpu,
                        oracle_grid, scaled_close)

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


def nan_tensor(shape, dtype):
    import torch
    return torch.full(shape, float("nan"), dtype=dtype, device="cuda")


def decoder_case(n_in, n, seed, fscale=1.0):
    rng = np.random.default_rng(seed)
    params = synth.decoder_params(n_in, rng)
    f = (rng.standard_normal((n, n_in)) * fscale).astype(np.float32)
    g = synth.upstream(n, 10, rng)
    return params, f, g


def run_mlp_forward(dt, params_dev, f, n_in):
    import torch
    n = f.shape[0]
    tdt = torch.float64 if dt == _lib.F64 else torch.float32
    out = nan_tensor((n, 10), tdt)
    _lib.deform_mlp_forward(_lib.mlp_shape(n_in), dt, params_dev, dev(f), n, out)
    return host(out)


def run_mlp_backward(dt, params_dev, f, g, n_in, loss_scale=1.0, grad_scale=1.0, d_params_init=None):
    import torch
    n = f.shape[0]
    m = _lib.mlp_shape(n_in)
    tdt = torch.float64 if dt == _lib.F64 else torch.float32
    ws_bytes = _lib.deform_mlp_workspace_bytes(m, dt, n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    d_feat = nan_tensor((n, n_in), tdt)
    P = O.param_count(n_in)
    d_params = torch.zeros(P, dtype=tdt, device="cuda") if d_params_init is None else dev(d_params_init)
    _lib.deform_mlp_backward(m, dt, params_dev, dev(f), n, dev(g), loss_scale, grad_scale, d_feat, d_params, ws,
                             ws_bytes)
    return host(d_feat), host(d_params)


def bf16_dev(x32):
    return dev(O.bf16_bits(x32).view(np.int16))


# ------------------------------------------------------------ decoder ----
@pytest.mark.parametrize("n_in", [8, 16, 32, 64])
@pytest.mark.parametrize("n", [4096 + 13, 1, 15, 17])
def test_mlp_forward_f32(n_in, n):
    params, f, _ = decoder_case(n_in, n, 50 + n_in)
    got = run_mlp_forward(_lib.F32, dev(params), f, n_in)
    ref, _ = O.mlp_forward(params, f)
    scaled_close(got, ref, mlp_forward_scale(params, f), RTOL_F32, "delta")


@pytest.mark.parametrize("n_in", [8, 32])
def test_mlp_forward_bf16_and_f64(n_in):
    params, f, _ = decoder_case(n_in, 2048 + 5, 60 + n_in)
    ref, _ = O.mlp_forward(params, f)
    s = mlp_forward_scale(params, f)
    got = run_mlp_forward(_lib.BF16, bf16_dev(params), f, n_in)
    scaled_close(got, ref, s, RTOL_BF16, "delta bf16")
    p64 = params.astype(np.float64) * (1 + 1e-9)
    got64 = run_mlp_forward(_lib.F64, dev(p64), f.astype(np.float64), n_in)
    scaled_close(got64, O.mlp_forward(p64, f)[0], s, 1e-12, "delta f64")


@pytest.mark.parametrize("n_in", [8, 16, 32, 64])
@pytest.mark.parametrize("n", [4096 + 13, 3])
def test_mlp_backward_f32(n_in, n):
    params, f, g = decoder_case(n_in, n, 70 + n_in)
    d_feat, d_params = run_mlp_backward(_lib.F32, dev(params), f, g, n_in)
    rf, rp = O.mlp_backward(params, f, g)
    sf, sp = mlp_backward_scale(params, f, g)
    scaled_close(d_feat, rf, sf, RTOL_GRAD, "d_feat")
    scaled_close(d_params, rp, sp, RTOL_GRAD, "d_params")


def test_mlp_backward_scales_and_accumulates():
    n_in = 32
    params, f, g = decoder_case(n_in, 3000, 80)
    init = np.random.default_rng(81).standard_normal(O.param_count(n_in)).astype(np.float32)
    d_feat, d_params = run_mlp_backward(_lib.F32, dev(params), f, g, n_in, loss_scale=1024.0, grad_scale=1 / 2048,
                                        d_params_init=init)
    rf, rp = O.mlp_backward(params, f, g, 0.5)
    sf, sp = mlp_backward_scale(params, f, g)
    scaled_close(d_feat, rf, 0.5 * sf, RTOL_GRAD, "d_feat scaled")
    scaled_close(d_params, init + rp, np.abs(init) + 0.5 * sp, RTOL_GRAD, "d_params +=")


@pytest.mark.parametrize("dt", [_lib.F32, _lib.BF16, _lib.F64], ids=["f32", "bf16", "f64"])
def test_mlp_backward_overwrite(dt):
    # H4D_GRAD_OVERWRITE writes d_params (NaN beforehand) with exactly what accumulating
    # into zeros gives (the per-block sums are reduced in a fixed order); n = 0 writes
    # zeros.
    import torch
    n_in, n = 32, 2000
    params, f, g = decoder_case(n_in, n, 95)
    tdt, npdt = (torch.float64, np.float64) if dt == _lib.F64 else (torch.float32, np.float32)
    p_dev = bf16_dev(params) if dt == _lib.BF16 else dev(params.astype(npdt))
    f_dev, g_dev = dev(f.astype(npdt)), dev(g.astype(npdt))
    m = _lib.mlp_shape(n_in)
    ws_bytes = _lib.deform_mlp_workspace_bytes(m, dt, n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    d_feat = nan_tensor((n, n_in), tdt)
    P = O.param_count(n_in)
    acc = torch.zeros(P, dtype=tdt, device="cuda")
    _lib.deform_mlp_backward(m, dt, p_dev, f_dev, n, g_dev, 1.0, 0.25, d_feat, acc, ws, ws_bytes)
    wr = nan_tensor((P,), tdt)
    _lib.deform_mlp_backward(m, dt, p_dev, f_dev, n, g_dev, 1.0, 0.25, d_feat, wr, ws, ws_bytes,
                             _lib.QUERY_MAJOR | _lib.GRAD_OVERWRITE)
    assert np.array_equal(host(wr), host(acc))
    wr.fill_(float("nan"))
    _lib.deform_mlp_backward(m, dt, p_dev, f_dev, 0, g_dev, 1.0, 0.25, d_feat, wr, ws, ws_bytes,
                             _lib.QUERY_MAJOR | _lib.GRAD_OVERWRITE)
    assert (host(wr) == 0).all()


@pytest.mark.parametrize("dt", [_lib.F32, _lib.BF16], ids=["f32", "bf16"])
def test_mlp_backward_checked_counts_nonfinite(dt):
    # deform_mlp_backward_checked adds the NaN / infinite values among the d_params
    # values it writes to its counter; the gradients equal the unchecked call's.
    import torch
    n_in, n = 32, 3000
    params, f, g = decoder_case(n_in, n, 96)
    p_dev = bf16_dev(params) if dt == _lib.BF16 else dev(params)
    m = _lib.mlp_shape(n_in)
    wb = _lib.deform_mlp_workspace_bytes(m, dt, n)
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
    P = O.param_count(n_in)
    counter = torch.zeros(1, dtype=torch.int32, device="cuda")
    outs = []
    for checked in (False, True):
        d_feat = torch.empty((n, n_in), device="cuda")
        d_params = torch.full((P,), float("nan"), device="cuda")
        args = (m, dt, p_dev, dev(f), n, dev(g), 1.0, 1.0, d_feat, d_params, ws, wb)
        if checked:
            _lib.deform_mlp_backward_checked(*args, counter, _lib.QUERY_MAJOR | _lib.GRAD_OVERWRITE)
        else:
            _lib.deform_mlp_backward(*args, _lib.QUERY_MAJOR | _lib.GRAD_OVERWRITE)
        outs.append((host(d_feat), host(d_params)))
    assert int(host(counter)[0]) == 0
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    bad = g.copy()
    bad[5, 0] = np.inf
    bad[17, 3] = np.nan
    d_feat = torch.empty((n, n_in), device="cuda")
    for mode in (_lib.GRAD_OVERWRITE, 0):
        counter.zero_()
        d_params = torch.zeros(P, device="cuda")
        _lib.deform_mlp_backward_checked(m, dt, p_dev, dev(f), n, dev(bad), 1.0, 1.0, d_feat, d_params, ws, wb,
                                         counter, _lib.QUERY_MAJOR | mode)
        want = int((~torch.isfinite(d_params)).sum())
        assert want > 0
        assert int(host(counter)[0]) == want, (mode, int(host(counter)[0]), want)


@pytest.mark.parametrize("n_in", [8, 32])
def test_mlp_backward_bf16_and_f64(n_in):
    params, f, g = decoder_case(n_in, 2048 + 7, 90 + n_in)
    rf, rp = O.mlp_backward(params, f, g)
    sf, sp = mlp_backward_scale(params, f, g)
    d_feat, d_params = run_mlp_backward(_lib.BF16, bf16_dev(params), f, g, n_in)
    scaled_close(d_feat, rf, sf, RTOL_BF16, "d_feat bf16")
    scaled_close(d_params, rp, sp, RTOL_BF16, "d_params bf16")
    p64 = params.astype(np.float64)
    d_feat, d_params = run_mlp_backward(_lib.F64, dev(p64), f.astype(np.float64), g.astype(np.float64), n_in)
    scaled_close(d_feat, rf, sf, 1e-10, "d_feat f64")
    scaled_close(d_params, rp, sp, 1e-10, "d_params f64")


def test_mlp_backward_rejects_small_workspace():
    import torch
    m = _lib.mlp_shape(32)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    x = torch.zeros((64, 32), device="cuda")
    with pytest.raises(_lib.H4DError) as e:
        _lib.deform_mlp_backward(m, _lib.F32, x, x, 64, x, 1.0, 1.0, x, x, ws, 16)
    assert "workspace" in str(e.value)
    with pytest.raises(_lib.H4DError):
        _lib.deform_mlp_forward(_lib.mlp_shape(24), _lib.F32, x, x, 64, x)


# ---------------------------------------------------- precision helpers ----
def test_cast_bf16_bit_exact_and_nonfinite_count():
    import torch
    rng = np.random.default_rng(95)
    x = np.concatenate([rng.standard_normal(100003).astype(np.float32) * 1e-3,
                        np.float32([0, -0.0, np.inf, -np.inf, np.nan, 1.00390625, 3.4e38, 1e-40])])
    out = torch.empty(x.size, dtype=torch.int16, device="cuda")
    _lib.h4d_cast_bf16(dev(x), out, x.size)
    assert np.array_equal(host(out).view(np.uint16), O.bf16_bits(x))
    # odd offset (unaligned tail path)
    out2 = torch.empty(x.size - 1, dtype=torch.int16, device="cuda")
    _lib.h4d_cast_bf16(dev(x)[1:], out2, x.size - 1)
    assert np.array_equal(host(out2).view(np.uint16), O.bf16_bits(x[1:]))
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    _lib.h4d_count_nonfinite(dev(x), x.size, cnt)
    assert int(host(cnt)[0]) == 3


# ----------------------------------------------------- deformation path ----
def deform_case(w, n, seed, scene=False):
    og, lg = oracle_grid(w), lib_grid(w)
    assert lg.offsets() == og.offsets
    rng, x = synth.scene_inputs(n, seed) if scene else synth.small_inputs(seed, n)
    table = synth.table_init(og.E, w.F, rng)
    params = synth.decoder_params(w.n_in, rng)
    gd = synth.upstream(n, 10, rng)
    return og, lg, x, table, params, gd


def run_deform(lg, dt, table_dev, params_dev, x, gd, n_in, E, F, loss_scale=1.0, grad_scale=1.0):
    import torch
    n = x.shape[0]
    m = _lib.mlp_shape(n_in)
    tdt = torch.float64 if dt == _lib.F64 else torch.float32
    feat = nan_tensor((lg.L, n, F), tdt)
    delta = nan_tensor((n, 10), tdt)
    xd = dev(x)
    _lib.hash4d_deform_forward(lg, m, dt, table_dev, params_dev, xd, n, feat, delta)
    ws_bytes = _lib.hash4d_deform_workspace_bytes(lg, m, dt, n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    d_table = torch.zeros((E, F), dtype=tdt, device="cuda")
    d_params = torch.zeros(O.param_count(n_in), dtype=tdt, device="cuda")
    _lib.hash4d_deform_backward(lg, m, dt, params_dev, xd, n, feat, dev(gd.astype(np.float64 if dt == _lib.F64
                                                                                     else np.float32)),
                                loss_scale, grad_scale, d_table, d_params, ws, ws_bytes)
    return host(feat), host(delta), host(d_table), host(d_params)


def check_deform(og, x, table, params, gd, got, rtol_out, rtol_grad, tag):
    feat, delta, d_table, d_params = got
    n = x.shape[0]
    f_ref, d_ref = O.deform_forward(x, table, og, params)
    f_scale = O.encode(x, np.abs(table), og)
    qmajor = np.transpose(feat, (1, 0, 2)).reshape(n, -1)
    scaled_close(qmajor, f_ref, f_scale, rtol_out, f"feat {tag}")
    scaled_close(delta, d_ref, mlp_forward_scale(params, f_scale), rtol_out, f"delta {tag}")
    rt, rp, rf = O.deform_backward(x, table, og, params, gd)
    sf, sp = mlp_backward_scale(params, f_ref, gd)
    scaled_close(d_params, rp, sp, rtol_grad, f"d_params {tag}")
    scaled_close(d_table, rt, O.encode_backward(x, sf, og), rtol_grad, f"d_table {tag}")
    return {"delta": float(np.abs(delta - d_ref).max()), "d_table": float(np.abs(d_table - rt).max())}


def test_deform_path_f32_small():
    w = synth.SMALL_DECODER
    og, lg, x, table, params, gd = deform_case(w, 4096 + 100, 100)
    got = run_deform(lg, _lib.F32, dev(table), dev(params), x, gd, w.n_in, og.E, w.F)
    check_deform(og, x, table, params, gd, got, RTOL_F32, RTOL_GRAD, "f32")


def test_deform_path_bf16_small_with_loss_scale():
    # BF16 tables and decoder from FP32 masters (cast on the GPU), loss-scaled gradients.
    import torch
    w = synth.SMALL_DECODER
    og, lg, x, table, params, gd = deform_case(w, 4096, 101)
    tb = torch.empty(table.size, dtype=torch.int16, device="cuda")
    pb = torch.empty(params.size, dtype=torch.int16, device="cuda")
    _lib.h4d_cast_bf16(dev(table), tb, table.size)
    _lib.h4d_cast_bf16(dev(params), pb, params.size)
    assert np.array_equal(host(tb).view(np.uint16), O.bf16_bits(table).ravel())
    got = run_deform(lg, _lib.BF16, tb, pb, x, gd, w.n_in, og.E, w.F, loss_scale=4096.0, grad_scale=1 / 4096)
    check_deform(og, x, table, params, gd, got, RTOL_BF16, RTOL_BF16, "bf16")


def test_deform_path_f64_small():
    w = synth.SMALL_DECODER
    og, lg, x, table, params, gd = deform_case(w, 700, 102)
    t64, p64 = table.astype(np.float64), params.astype(np.float64)
    got = run_deform(lg, _lib.F64, dev(t64), dev(p64), x, gd.astype(np.float64), w.n_in, og.E, w.F)
    check_deform(og, x, t64, p64, gd, got, 1e-12, 1e-10, "f64")


@pytest.mark.parametrize("shared", [None, 150], ids=["own-frames", "shared-frame-150"])
def test_deform_path_paper_scene_full_size(shared):
    # The benchmark's configuration (n = 200k clustered, L = 16, T = 2^19), each query
    # at its own frame or all at frame 150: delta on 4096 sampled queries, d_params and
    # the whole d_table element by element against the oracle's chain (decoder
    # backward, then the transpose of Eq. 9).
    w = synth.PAPER_SCENE
    og, lg = oracle_grid(w), lib_grid(w)
    assert lg.offsets() == og.offsets
    rng, x = synth.scene_inputs(w.n, 103, shared_frame=shared)
    table = synth.table_init(og.E, w.F, rng)
    params = synth.decoder_params(w.n_in, rng)
    gd = synth.upstream(w.n, 10, rng)
    feat, delta, d_table, d_params = run_deform(lg, _lib.F32, dev(table), dev(params), x, gd, w.n_in, og.E, w.F)
    idx = np.random.default_rng(104).choice(w.n, 4096, replace=False)
    _, d_ref = O.deform_forward(x[idx], table, og, params)
    f_scale_s = O.encode(x[idx], np.abs(table), og)
    scaled_close(delta[idx], d_ref, mlp_forward_scale(params, f_scale_s), RTOL_F32, "delta 200k")
    f_ref = O.encode(x, table, og)
    rf, rp = O.mlp_backward(params, f_ref, gd)
    sf, sp = mlp_backward_scale(params, f_ref, gd)
    scaled_close(d_params, rp, sp, RTOL_GRAD, "d_params 200k")
    scaled_close(d_table, O.encode_backward(x, rf, og), O.encode_backward(x, sf, og), RTOL_GRAD, "d_table 200k")


def test_deform_path_paper_scene_full_size_bf16():
    # The BF16 form at the benchmark's configuration (n = 200k clustered, L = 16,
    # T = 2^19): BF16 tables and decoder cast on the GPU from FP32 masters, upstream
    # gradient loss-scaled by 4096; delta on 4096 sampled queries, d_params and the whole
    # d_table element by element against the oracle's chain on the FP32 masters.
    import torch
    w = synth.PAPER_SCENE
    og, lg = oracle_grid(w), lib_grid(w)
    rng, x = synth.scene_inputs(w.n, 105)
    table = synth.table_init(og.E, w.F, rng)
    params = synth.decoder_params(w.n_in, rng)
    gd = synth.upstream(w.n, 10, rng)
    tb = torch.empty(table.size, dtype=torch.int16, device="cuda")
    pb = torch.empty(params.size, dtype=torch.int16, device="cuda")
    _lib.h4d_cast_bf16(dev(table), tb, table.size)
    _lib.h4d_cast_bf16(dev(params), pb, params.size)
    feat, delta, d_table, d_params = run_deform(lg, _lib.BF16, tb, pb, x, gd, w.n_in, og.E, w.F,
                                                loss_scale=4096.0, grad_scale=1 / 4096.0)
    idx = np.random.default_rng(106).choice(w.n, 4096, replace=False)
    _, d_ref = O.deform_forward(x[idx], table, og, params)
    f_scale_s = O.encode(x[idx], np.abs(table), og)
    scaled_close(delta[idx], d_ref, mlp_forward_scale(params, f_scale_s), RTOL_BF16, "bf16 delta 200k")
    f_ref = O.encode(x, table, og)
    rf, rp = O.mlp_backward(params, f_ref, gd)
    sf, sp = mlp_backward_scale(params, f_ref, gd)
    scaled_close(d_params, rp, sp, RTOL_BF16, "bf16 d_params 200k")
    scaled_close(d_table, O.encode_backward(x, rf, og), O.encode_backward(x, sf, og), RTOL_BF16, "bf16 d_table 200k")


def test_deform_apply_eq10_bit_exact():
    import torch
    rng = np.random.default_rng(110)
    n = 5000 + 3
    delta = rng.standard_normal((n, 10)).astype(np.float32)
    x, r, s = (rng.standard_normal((n, k)).astype(np.float32) for k in (3, 4, 3))
    xo, ro, so = (torch.empty((n, k), device="cuda") for k in (3, 4, 3))
    _lib.hash4d_deform_apply(dev(delta), n, 10, dev(x), dev(r), dev(s), xo, ro, so)
    ref = O.deform(x, r, s, delta)
    for got, want in zip((xo, ro, so), ref):
        # one FP32 add each: bit-exact against the FP64 sum rounded to FP32
        assert np.array_equal(host(got), want.astype(np.float32))
    # in place
    xd = dev(x)
    _lib.hash4d_deform_apply(dev(delta), n, 10, xd, dev(r), dev(s), xd, ro, so)
    assert np.array_equal(host(xd), ref[0].astype(np.float32))
