"""GPU parity of the dynamic-static split and static constraint (Section 4.1,
Eqs. 4-5) through the C ABI.  The split and the dynamic indices are compared bit
for bit with the oracle on the same FP32 motion vectors; the loss and its gradient
within 1e-5 of the FP64 oracle."""
import numpy as np
import pytest

from oracle import hash4d_oracle as O
from paper_2507_19141_amd import _lib, synth
from tests.util import RTOL_F32, needs_gpu, scaled_close

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


def run(dp, k, lam=1.0):
    import torch
    n = dp.shape[0]
    idx = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    flag = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    loss = torch.zeros(1, device="cuda")
    grad = torch.zeros((n, 3), device="cuda")
    wb = _lib.hash4d_decompose_workspace_bytes(n)
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
    _lib.hash4d_decompose(dev(dp), n, k, lam, idx, cnt, flag, loss, grad, ws, wb)
    c = int(host(cnt)[0])
    return host(idx)[:c], host(flag), float(host(loss)[0]), host(grad)


def motion(n, seed):
    rng = np.random.default_rng(seed)
    # a few fast movers over a slow majority, like a mostly static scene
    dp = (rng.standard_normal((n, 3)) * np.where(rng.random((n, 1)) < 0.1, 1.0, 0.01)).astype(np.float32)
    return dp


@pytest.mark.parametrize("k", [0.0, 10.0, 33.3, 99.99, 100.0])
def test_split_matches_oracle(k):
    dp = motion(200_003, 80)
    dp[100:200] = dp[50]          # ties
    dp[300] = [np.nan, 0, 0]
    dp[400:410] = 0.0
    idx, flag, loss, grad = run(dp, k, 0.7)
    ridx, rloss, rgrad = O.decompose(dp, k, 0.7)
    assert np.array_equal(idx.astype(np.int64), ridx)
    want = np.zeros(dp.shape[0], np.uint8)
    want[ridx] = 1
    assert np.array_equal(flag, want)
    if np.isnan(rloss):   # the NaN Gaussian is static when k = 0: both sides carry the NaN
        assert np.isnan(loss)
    else:
        assert abs(loss - rloss) <= RTOL_F32 * abs(rloss) + 1e-30
    mags = np.linalg.norm(dp.astype(np.float64), axis=1)
    n_s = dp.shape[0] - len(ridx)
    scale = 0.7 / max(n_s, 1) * np.ones_like(rgrad)
    scaled_close(grad, rgrad, scale, RTOL_F32, "d_dp")


def test_split_small_and_ragged_sizes():
    for n, seed in ((1, 81), (63, 82), (257, 83), (5000, 84)):
        dp = motion(n, seed)
        for k in (0.0, 50.0, 100.0):
            idx, _, _, _ = run(dp, k)
            assert np.array_equal(idx.astype(np.int64), O.decompose(dp, k)[0]), (n, k)


def test_front_end_chain():
    # the whole front end on the paper-shaped cloud: the 3D multiresolution hash
    # encoding G_3D of the positions (Eq. 3), a 32-64-64-3 decoder for dp (phi_p then
    # phi_l), and the split on the decoder's FP32 output
    import torch
    w = synth.PAPER_SCENE
    n = 50_000
    rng, x = synth.scene_inputs(n, 85)
    rs = _lib.h4d_grid_schedule(w.L, *w.space)
    g = _lib.h4d_grid3_init(w.L, w.F, rs, w.T)
    og = O.make_grid3(w.L, w.F, list(rs), w.T)
    assert g.offsets() == og.offsets
    table = synth.table_init(og.E, w.F, rng, 1e-1)
    params = synth.decoder_params(w.n_in, rng, out=3)
    feat = torch.empty((n, w.L * w.F), device="cuda")
    _lib.hash3d_encode(g, _lib.F32, dev(table), dev(x), 4, n, feat)
    m = _lib.mlp_shape(w.n_in, out=3)
    dp = torch.empty((n, 3), device="cuda")
    _lib.deform_mlp_forward(m, _lib.F32, dev(params), feat, n, dp)
    f_ref = O.encode3(x, table, og)
    P = O.unpack_params(params, w.n_in, out=3)
    h1 = np.maximum(f_ref @ P["W1"].T + P["b1"], 0)
    h2 = np.maximum(h1 @ P["W2"].T + P["b2"], 0)
    d_ref = h2 @ P["W3"].T + P["b3"]
    A = {k: np.abs(v) for k, v in P.items()}
    mag = ((np.abs(f_ref) @ A["W1"].T + A["b1"]) @ A["W2"].T + A["b2"]) @ A["W3"].T + A["b3"]
    dph = host(dp)
    scaled_close(dph, d_ref, mag, RTOL_F32, "dp")
    idx, _, _, _ = run(dph, 10.0)
    assert np.array_equal(idx.astype(np.int64), O.decompose(dph, 10.0)[0])
    assert len(idx) == 5000
