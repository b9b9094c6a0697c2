"""Shared helpers of the test-suite: workload grids on both sides and tolerance checks."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import hash4d_oracle as O
from paper_2507_19141_amd import synth

# Tolerances (relative to the oracle's magnitude scale, see scaled_close).
RTOL_F32 = 1e-5     # FP32 outputs
RTOL_BF16 = 2e-2    # BF16 outputs
RTOL_GRAD = 1e-4    # FP32 gradients


def oracle_grid(w: synth.Workload) -> O.Grid:
    if w.rule == "doubling":
        rs = O.doubling_resolutions(*w.space, w.L)
        rt = O.doubling_resolutions(*w.time, w.L)
    else:
        rs = O.level_resolutions(*w.space, w.L)
        rt = O.level_resolutions(*w.time, w.L)
    return O.make_grid(w.L, w.F, rs, rt, w.T)


def lib_grid(w: synth.Workload):
    from paper_2507_19141_amd import _lib
    rule = _lib.SCHEDULE_DOUBLING if w.rule == "doubling" else _lib.SCHEDULE_GEOMETRIC
    rs = _lib.h4d_grid_schedule(w.L, *w.space, rule)
    rt = _lib.h4d_grid_schedule(w.L, *w.time, rule)
    return _lib.h4d_grid_init(w.L, w.F, rs, rt, w.T)


def assert_same_layout(og: O.Grid, lg) -> None:
    assert list(lg.res_s[:og.L]) == og.res_s
    assert list(lg.res_t[:og.L]) == og.res_t
    assert lg.dense_list() == og.dense
    assert lg.offsets() == og.offsets


def scaled_close(got, ref, scale, rtol, what=""):
    """|got - ref| <= rtol * (|ref| + scale) elementwise, where scale is the oracle's
    own magnitude of the terms that were summed (so cancellation does not demand
    more than the arithmetic can give).  Returns (max scaled error, mean abs error)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.broadcast_to(np.asarray(scale, dtype=np.float64), ref.shape)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    den = np.abs(ref) + scale
    den = np.where(den > 0, den, 1.0)
    err = np.abs(got - ref) / den
    worst = float(err.max()) if err.size else 0.0
    if worst > rtol:
        i = np.unravel_index(int(np.argmax(err)), err.shape)
        raise AssertionError(f"{what}: scaled error {worst:.3e} > {rtol:.1e} at {i}: got {got[i]!r} ref {ref[i]!r} "
                             f"scale {scale[i]!r}")
    return worst, float(np.abs(got - ref).mean()) if err.size else 0.0


def needs_gpu():
    try:
        import torch
        ok = torch.cuda.is_available()
    except Exception:
        ok = False
    if not ok:
        pytest.skip("no GPU")


# ------------------------------------------------------- decoder scales ----
def mlp_forward_scale(flat, f):
    """Magnitude bound of the decoder forward: every layer on absolute values."""
    P = O.unpack_params(flat, np.asarray(f).shape[1])
    s1 = np.abs(f) @ np.abs(P["W1"]).T + np.abs(P["b1"])
    s2 = s1 @ np.abs(P["W2"]).T + np.abs(P["b2"])
    s3 = s2 @ np.abs(P["W3"]).T + np.abs(P["b3"])
    return s3


def mlp_backward_scale(flat, f, d_out):
    """Magnitude bounds of the decoder gradients (d_feat, d_params) on absolute values."""
    f = np.asarray(f, dtype=np.float64)
    P = O.unpack_params(flat, f.shape[1])
    A = {k: np.abs(v) for k, v in P.items()}
    s1 = np.abs(f) @ A["W1"].T + A["b1"]
    s2 = s1 @ A["W2"].T + A["b2"]
    g3 = np.abs(d_out)
    g2 = g3 @ A["W3"]
    g1 = g2 @ A["W2"]
    d_feat = g1 @ A["W1"]
    d_params = O.pack_params({"W1": g1.T @ np.abs(f), "b1": g1.sum(0), "W2": g2.T @ s1, "b2": g2.sum(0),
                              "W3": g3.T @ s2, "b3": g3.sum(0)})
    return d_feat, d_params
