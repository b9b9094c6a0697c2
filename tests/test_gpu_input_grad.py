"""GPU parity of the encoder's input gradient (the derivative of Eq. 9 with respect
to the positions) through the C ABI, against the FP64 oracle.

FP32 / BF16 tables: within 1e-5 of the oracle relative to its magnitude scale
sum_l sum_c |d w_c / d x| sum_f |theta_c,f g_f|; FP64: 1e-12.
"""
import numpy as np
import pytest

from oracle import hash4d_oracle as O
from paper_2507_19141_amd import _lib, synth
from tests.test_gpu_encoder import dev, edge_points, encoder_case, host
from tests.util import RTOL_F32, assert_same_layout, needs_gpu, scaled_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    needs_gpu()


def magnitude(x, table, g, gf):
    rows, _ = O.corners(x, g)
    dw = np.abs(O.corner_weight_derivatives(x, g))
    th = np.abs(np.asarray(table, np.float64))
    ga = np.abs(np.asarray(gf, np.float64))
    out = np.zeros((x.shape[0], 4))
    for l in range(g.L):
        gl = ga[:, l * g.F:(l + 1) * g.F]
        for c in range(16):
            out += dw[:, l, c, :] * np.sum(th[rows[:, l, c]] * gl, axis=1)[:, None]
    return out


def run(lg, dt, table_dev, x, gf, scale=1.0, layout=_lib.QUERY_MAJOR, start=None, two_pass=False):
    import torch
    n = x.shape[0]
    fdt = torch.float64 if dt == _lib.F64 else torch.float32
    out = torch.zeros((n, 4), dtype=fdt, device="cuda") if start is None else start.clone()
    g = np.asarray(gf, np.float64 if dt == _lib.F64 else np.float32)
    if layout == _lib.LEVEL_MAJOR:
        g = np.ascontiguousarray(g.reshape(n, lg.L, lg.F).transpose(1, 0, 2))
    ws, wb = None, 0
    if two_pass:   # the level-placed form: per-level terms in a workspace, then a sum
        wb = _lib.hash4d_encode_backward_input_workspace_bytes(lg, dt, n)
        assert wb == n * lg.L * 16
        ws = torch.full((wb // 4,), float("nan"), device="cuda")
    _lib.hash4d_encode_backward_input(lg, dt, table_dev, dev(x), n, dev(g), scale, out, layout, ws, wb)
    return host(out)


@pytest.mark.parametrize("dt,two_pass", [(_lib.F32, False), (_lib.F32, True), (_lib.F64, False)],
                         ids=["f32", "f32-two-pass", "f64"])
@pytest.mark.parametrize("layout", [_lib.QUERY_MAJOR, _lib.LEVEL_MAJOR], ids=["query-major", "level-major"])
def test_input_grad_small(dt, two_pass, layout):
    og, lg, x, table, rng = encoder_case(synth.ENCODER_SMALL, 4096, 30, table_scale=1.0)
    gf = synth.upstream(x.shape[0], og.L * og.F, rng)
    t = table.astype(np.float64) if dt == _lib.F64 else table
    got = run(lg, dt, dev(t), x, gf, 0.5, layout, two_pass=two_pass)
    ref = O.encode_backward_input(x, t, og, gf, 0.5)
    scaled_close(got, ref, 0.5 * magnitude(x, t, og, gf), 1e-12 if dt == _lib.F64 else RTOL_F32, "d_xyzt")
    # out-of-range and NaN coordinates carry no gradient
    bad = ~((x >= 0) & (x <= 1))
    assert np.all(got[bad] == 0)


@pytest.mark.parametrize("two_pass", [False, True], ids=["one-pass", "two-pass"])
def test_input_grad_bf16_table_exact_inputs(two_pass):
    og, lg, x, table, rng = encoder_case(synth.ENCODER_SMALL, 4096, 31, table_scale=1.0)
    gf = synth.upstream(x.shape[0], og.L * og.F, rng)
    bits = O.bf16_bits(table)
    tb = O.bf16_value(bits)
    got = run(lg, _lib.BF16, dev(bits.view(np.int16)), x, gf, two_pass=two_pass)
    scaled_close(got, O.encode_backward_input(x, tb, og, gf), magnitude(x, tb, og, gf), RTOL_F32, "d_xyzt bf16")


@pytest.mark.parametrize("two_pass", [False, True], ids=["one-pass", "two-pass"])
@pytest.mark.parametrize("F,T,n,L", [(1, 3000, 1037, 3), (4, 1 << 12, 777, 4), (8, 1 << 10, 300, 2)])
def test_input_grad_widths_and_ragged(F, T, n, L, two_pass):
    rs = O.doubling_resolutions(3, 40, L)
    rt = O.doubling_resolutions(2, 9, L)
    og = O.make_grid(L, F, rs, rt, T)
    lg = _lib.h4d_grid_init(L, F, rs, rt, T)
    assert_same_layout(og, lg)
    rng, x = synth.small_inputs(32, n)
    x = np.concatenate([x, edge_points(og)])
    table = synth.table_init(og.E, F, rng, 1.0)
    gf = synth.upstream(x.shape[0], L * F, rng)
    got = run(lg, _lib.F32, dev(table), x, gf, two_pass=two_pass)
    scaled_close(got, O.encode_backward_input(x, table, og, gf), magnitude(x, table, og, gf), RTOL_F32, "d_xyzt")


@pytest.mark.parametrize("two_pass", [False, True], ids=["one-pass", "two-pass"])
def test_input_grad_paper_scene_full_size_sampled(two_pass):
    # the whole 200k-query scene runs; 4096 sampled queries are checked (each output
    # row depends on its own query only)
    w = synth.PAPER_SCENE
    og, lg, x, table, rng = encoder_case(w, w.n, 33, edges=False, table_scale=1.0)
    gf = synth.upstream(w.n, og.L * og.F, rng)
    got = run(lg, _lib.F32, dev(table), x, gf, layout=_lib.LEVEL_MAJOR, two_pass=two_pass)
    idx = np.random.default_rng(34).choice(w.n, 4096, replace=False)
    xs, gs = x[idx], gf[idx]
    scaled_close(got[idx], O.encode_backward_input(xs, table, og, gs), magnitude(xs, table, og, gs), RTOL_F32,
                 "d_xyzt 200k")


@pytest.mark.parametrize("two_pass", [False, True], ids=["one-pass", "two-pass"])
def test_input_grad_accumulates_and_n0_is_noop(two_pass):
    import torch
    og, lg, x, table, rng = encoder_case(synth.ENCODER_SMALL, 1000, 35, edges=False, table_scale=1.0)
    gf = synth.upstream(x.shape[0], og.L * og.F, rng)
    start = torch.full((x.shape[0], 4), 2.0, device="cuda")
    got = run(lg, _lib.F32, dev(table), x, gf, start=start, two_pass=two_pass)
    ref = 2.0 + O.encode_backward_input(x, table, og, gf)
    scaled_close(got, ref, 2.0 + magnitude(x, table, og, gf), RTOL_F32, "d_xyzt +=")
    out = torch.full((4, 4), 7.0, device="cuda")
    _lib.hash4d_encode_backward_input(lg, _lib.F32, dev(table), dev(x[:4]), 0, dev(gf[:4]), 1.0, out)
    assert (host(out) == 7.0).all()


@pytest.mark.parametrize("two_pass", [False, True], ids=["one-pass", "two-pass"])
def test_position_gradient_through_the_decoder(two_pass):
    # dDelta/dP composed from the entry points: d_delta -> deform_mlp_backward ->
    # d_feat -> hash4d_encode_backward_input -> d_xyzt, against the same chain of
    # oracle functions (decoder backward on the oracle's features, then the input
    # gradient of the encoder).
    import torch
    from tests.util import RTOL_GRAD, mlp_backward_scale
    from tests.util import lib_grid, oracle_grid
    w = synth.SMALL_DECODER
    og, lg = oracle_grid(w), lib_grid(w)
    assert_same_layout(og, lg)
    rng, x = synth.small_inputs(41, 3000)
    n = x.shape[0]
    table = synth.table_init(og.E, w.F, rng)
    params = synth.decoder_params(w.n_in, rng)
    gd = synth.upstream(n, 10, rng)
    LM = _lib.LEVEL_MAJOR
    m = _lib.mlp_shape(w.n_in)
    td, xd = dev(table), dev(x)
    feat = torch.empty((w.L, n, w.F), device="cuda")
    _lib.hash4d_encode(lg, _lib.F32, td, xd, n, feat, LM)
    wb = _lib.deform_mlp_workspace_bytes(m, _lib.F32, n)
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
    d_feat = torch.empty((w.L, n, w.F), device="cuda")
    d_params = torch.empty(O.param_count(w.n_in), device="cuda")
    _lib.deform_mlp_backward(m, _lib.F32, dev(params), feat, n, dev(gd), 1.0, 1.0, d_feat, d_params, ws, wb,
                             LM | _lib.GRAD_OVERWRITE, w.F)
    d_xyzt = torch.zeros((n, 4), device="cuda")
    wi = _lib.hash4d_encode_backward_input_workspace_bytes(lg, _lib.F32, n) if two_pass else 0
    wsi = torch.empty(max(wi, 1), dtype=torch.uint8, device="cuda") if two_pass else None
    _lib.hash4d_encode_backward_input(lg, _lib.F32, td, xd, n, d_feat, 1.0, d_xyzt, LM, wsi, wi)
    f_ref = O.encode(x, table, og)
    rf, _ = O.mlp_backward(params, f_ref, gd)
    ref = O.encode_backward_input(x, table, og, rf)
    sf, _ = mlp_backward_scale(params, f_ref, gd)
    scaled_close(host(d_xyzt), ref, magnitude(x, table, og, sf), RTOL_GRAD, "dDelta/dP")
