"""GPU parity of the 3D hash encoder G_3D (Section 4.1, Eq. 3) through the C ABI:
features within 1e-5 (FP32), 2e-2 (BF16 tables) and 1e-12 (FP64) of the FP64 oracle,
relative to the oracle's magnitude scale; [n, 3] and [n, 4] position rows; ragged n;
dense, hashed and non-power-of-two-T levels; the dense threshold (N+1)^3 <= T; edge
points (vertices, just below vertex boundaries, out of range, NaN)."""
import numpy as np
import pytest

from oracle import hash4d_oracle as O
from paper_2507_19141_amd import _lib, synth
from tests.util import RTOL_BF16, RTOL_F32, needs_gpu, scaled_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    needs_gpu()


def grids(L, F, res, T):
    og = O.make_grid3(L, F, res, T)
    lg = _lib.h4d_grid3_init(L, F, res, T)
    assert lg.dense_list() == og.dense and lg.offsets() == og.offsets
    return og, lg


def edge_points3(og):
    pts = [[0, 0, 0], [1, 1, 1], [1, 0, 1], [-0.25, 1.75, 0.5], [np.nan, 0.5, np.nan], [np.inf, -np.inf, 0.5]]
    rng = np.random.default_rng(41)
    for N in og.res:
        for v in rng.integers(1, N + 1, size=4):
            d = int(rng.integers(0, 3))
            p = rng.random(3)
            p[d] = np.nextafter(np.float32(v / N), np.float32(0))
            pts.append(p)
            q = rng.random(3)
            q[d] = np.float32(v / N)
            pts.append(q)
    return np.asarray(pts, dtype=np.float32)


def run3(lg, dt, table, x, stride, layout=_lib.QUERY_MAJOR):
    import torch
    n = x.shape[0]
    rows = np.zeros((n, stride), dtype=np.float32)
    rows[:, :3] = x[:, :3]
    if stride == 4:
        rows[:, 3] = 0.625   # ignored
    if dt == _lib.BF16:
        td = torch.from_numpy(O.bf16_bits(table).view(np.int16)).cuda()
    else:
        td = torch.from_numpy(np.ascontiguousarray(table.astype(np.float64 if dt == _lib.F64 else np.float32))).cuda()
    odt = torch.float64 if dt == _lib.F64 else torch.float32
    shape = (n, lg.L * lg.F) if layout == _lib.QUERY_MAJOR else (lg.L, n, lg.F)
    out = torch.full(shape, float("nan"), dtype=odt, device="cuda")
    _lib.hash3d_encode(lg, dt, td, torch.from_numpy(rows).cuda(), stride, n, out, layout)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    if layout == _lib.LEVEL_MAJOR:
        o = o.transpose(1, 0, 2).reshape(n, lg.L * lg.F)
    return o


@pytest.mark.parametrize("F,T,res", [
    (2, 1 << 12, (4, 8, 16, 32)),        # dense then hashed
    (1, 5003, (3, 17, 40)),               # modulo hashing, F = 1
    (4, 1 << 16, (16, 31, 64)),           # F = 4
    (8, 1 << 14, (2, 9, 27)),             # F = 8
    (2, 600, (7,)),                       # 512 vertices, T = 600: dense in 3D
], ids=["mixed-F2", "modT-F1", "F4", "F8", "dense-threshold"])
@pytest.mark.parametrize("stride", [3, 4])
def test_encode3_f32_matches_oracle(F, T, res, stride):
    L = len(res)
    og, lg = grids(L, F, list(res), T)
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.random((2999, 3)).astype(np.float32), edge_points3(og)])
    table = synth.table_init(og.E, F, rng, scale=1.0)
    got = run3(lg, _lib.F32, table, x, stride)
    scaled_close(got, O.encode3(x, table, og), O.encode3(x, np.abs(table), og), RTOL_F32, "G_3D f32")


def test_encode3_bf16_and_f64():
    og, lg = grids(4, 2, [4, 8, 16, 32], 1 << 12)
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.random((1537, 3)).astype(np.float32), edge_points3(og)])
    table = synth.table_init(og.E, 2, rng, scale=1.0)
    tb = O.bf16_value(O.bf16_bits(table))      # the BF16 values the kernel reads
    got = run3(lg, _lib.BF16, table, x, 3, _lib.LEVEL_MAJOR)
    scaled_close(got, O.encode3(x, tb, og), O.encode3(x, np.abs(tb), og), RTOL_BF16, "G_3D bf16")
    got = run3(lg, _lib.F64, table.astype(np.float64), x, 4)
    scaled_close(got, O.encode3(x, table, og), O.encode3(x, np.abs(table), og), 1e-12, "G_3D f64")


def test_encode3_paper_cloud_sampled():
    # the front end's shape: 200k clustered positions, L = 16, F = 2, T = 2^19, Eq. 7 16 -> 2048
    w = synth.PAPER_SCENE
    res = O.level_resolutions(*w.space, w.L)
    og, lg = grids(w.L, w.F, res, w.T)
    rng, x = synth.scene_inputs(w.n, 12)
    table = synth.table_init(og.E, w.F, rng, scale=1e-1)
    got = run3(lg, _lib.F32, table, x, 4, _lib.LEVEL_MAJOR)
    idx = np.random.default_rng(43).choice(w.n, 4096, replace=False)
    xs = x[idx]
    scaled_close(got[idx], O.encode3(xs, table, og), O.encode3(xs, np.abs(table), og), RTOL_F32, "G_3D 200k")


def test_encode3_is_deterministic():
    og, lg = grids(3, 2, [4, 16, 64], 1 << 12)
    rng = np.random.default_rng(9)
    x = rng.random((777, 3)).astype(np.float32)
    table = synth.table_init(og.E, 2, rng)
    a = run3(lg, _lib.F32, table, x, 3)
    b = run3(lg, _lib.F32, table, x, 3)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
