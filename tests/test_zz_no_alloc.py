"""hash4d_encode_backward_noalloc (the table scatter with its masks in the library's
static workspace, no allocation) against hash4d_encode_backward with a caller
workspace: two calls in a row on one GPU, the second with a smaller input, each
compared element by element within the FP32 gradient tolerance (the LDS adds make
the summation order vary), and both pinned to the FP64 oracle."""
import numpy as np
import pytest

from oracle import hash4d_oracle as O
from paper_2507_19141_amd import _lib, synth
from tests.util import RTOL_GRAD, assert_same_layout, lib_grid, needs_gpu, oracle_grid, scaled_close

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20


def _scatter(lg, x, gf, base, noalloc, overwrite):
    """d_table after one call; it starts as `base` (accumulate) or as NaN (overwrite:
    every row must be written)."""
    import torch
    n = x.shape[0]
    xd = torch.from_numpy(x).cuda()
    gd = torch.from_numpy(gf).cuda()
    d_table = torch.from_numpy(np.full_like(base, np.nan) if overwrite else base).cuda()
    layout = _lib.QUERY_MAJOR | (_lib.GRAD_OVERWRITE if overwrite else 0)
    if noalloc:
        _lib.hash4d_encode_backward_noalloc(lg, _lib.F32, xd, n, gd, 0.5, d_table, layout=layout)
    else:
        wb = _lib.hash4d_encode_backward_workspace_bytes(lg, n)
        ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
        _lib.hash4d_encode_backward(lg, _lib.F32, xd, n, gd, 0.5, d_table, ws, wb, layout=layout)
    torch.cuda.synchronize()
    return d_table.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("overwrite", [False, True], ids=["accumulate", "overwrite"])
def test_noalloc_matches_workspace_form_twice(overwrite):
    needs_gpu()
    w = synth.PAPER_SCENE
    og, lg = oracle_grid(w), lib_grid(w)
    assert_same_layout(og, lg)
    # first call: 60k clustered queries (every level, many tiles), then 7k (ragged)
    for n, seed in ((60_000, 3), (7_001, 4)):
        print(f"noalloc scatter: n={n} seed={seed} overwrite={overwrite}", flush=True)
        assert _lib.hash4d_encode_backward_workspace_bytes(lg, n) <= STATIC_BYTES
        rng, x = synth.scene_inputs(n, seed)
        gf = synth.upstream(n, w.L * w.F, rng)
        base = synth.table_init(og.E, w.F, rng, scale=1e-3)
        got = _scatter(lg, x, gf, base, True, overwrite)
        ref_ws = _scatter(lg, x, gf, base, False, overwrite)
        ref = O.encode_backward(x, gf, og, 0.5)
        scale = O.encode_backward(x, np.abs(gf), og, 0.5)
        if not overwrite:  # the starting values join the sum (one FP32 rounding each)
            ref = ref + base
            scale = scale + np.abs(base)
        scaled_close(got, ref_ws, scale, RTOL_GRAD, f"noalloc vs workspace form, n={n}")
        scaled_close(got, ref, scale, RTOL_GRAD, f"noalloc vs oracle, n={n}")


def test_noalloc_rejects_more_than_the_static_workspace():
    needs_gpu()
    import torch
    w = synth.PAPER_SCENE
    lg = lib_grid(w)
    n = 1
    while _lib.hash4d_encode_backward_workspace_bytes(lg, n) <= STATIC_BYTES:
        n *= 2
    # the check comes before any launch or device access: the buffers are never read
    xd = torch.zeros((4, 4), device="cuda")
    with pytest.raises(RuntimeError, match="static workspace"):
        _lib.hash4d_encode_backward_noalloc(lg, _lib.F32, xd, n, xd, 1.0, xd)
