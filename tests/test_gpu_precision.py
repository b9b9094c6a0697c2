"""Precision form of the small configuration (N = 4096, L = 4, F = 2, T = 2^12, seed
0): BF16 tables and BF16 MFMA decoder cast from FP32 masters, FP32 accumulation,
loss-scaled gradients.  Every output's max and mean error against the FP64 oracle
evaluated on the FP32 masters is printed as one JSON line (run pytest with -s to
see it), beside the plain FP32 path's errors on the same inputs, and bounded by the
tolerances: FP32 outputs 1e-5 and gradients 1e-4, BF16 2e-2, all relative to the
oracle's own magnitude of the summed terms."""
import json

import numpy as np
import pytest

from oracle import hash4d_oracle as O
from paper_2507_19141_amd import _lib, synth
from tests.test_gpu_decoder import deform_case, dev, host, run_deform
from tests.util import RTOL_BF16, RTOL_F32, RTOL_GRAD, mlp_backward_scale, mlp_forward_scale, needs_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    needs_gpu()


def errors(got, ref, scale):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(got - ref)
    den = np.abs(ref) + np.broadcast_to(scale, ref.shape)
    rel = err / np.where(den > 0, den, 1.0)  # rows no query reaches: ref = scale = 0
    return {"max_abs": float(err.max()), "mean_abs": float(err.mean()), "max_rel": float(rel.max()),
            "mean_rel": float(rel.mean()), "ref_max_abs": float(np.abs(ref).max())}


def test_precision_report_bf16_vs_fp32():
    import torch
    w = synth.SMALL_DECODER
    og, lg, x, table, params, gd = deform_case(w, w.n, 0)
    n = x.shape[0]
    f_ref, d_ref = O.deform_forward(x, table, og, params)
    rt, rp, _ = O.deform_backward(x, table, og, params, gd)
    f_scale = O.encode(x, np.abs(table), og)
    sf, sp = mlp_backward_scale(params, f_ref, gd)
    scales = {"feat": f_scale, "delta": mlp_forward_scale(params, f_scale), "d_table": O.encode_backward(x, sf, og),
              "d_params": sp}
    refs = {"feat": f_ref, "delta": d_ref, "d_table": rt, "d_params": rp}
    tb = torch.empty(table.size, dtype=torch.int16, device="cuda")
    pb = torch.empty(params.size, dtype=torch.int16, device="cuda")
    _lib.h4d_cast_bf16(dev(table), tb, table.size)
    _lib.h4d_cast_bf16(dev(params), pb, params.size)
    runs = {"fp32": run_deform(lg, _lib.F32, dev(table), dev(params), x, gd, w.n_in, og.E, w.F),
            "bf16": run_deform(lg, _lib.BF16, tb, pb, x, gd, w.n_in, og.E, w.F, loss_scale=4096.0,
                               grad_scale=1 / 4096)}
    report = {"workload": w.name, "n": n, "oracle": "FP64 on the FP32 masters", "loss_scale_bf16": 4096.0}
    for form, (feat, delta, d_table, d_params) in runs.items():
        got = {"feat": np.transpose(feat, (1, 0, 2)).reshape(n, -1), "delta": delta, "d_table": d_table,
               "d_params": d_params}
        report[form] = {k: errors(got[k], refs[k], scales[k]) for k in refs}
    print(json.dumps({"precision_report": report}), flush=True)
    for k in refs:
        bound32 = RTOL_F32 if k in ("feat", "delta") else RTOL_GRAD
        assert report["fp32"][k]["max_rel"] <= bound32, (k, report["fp32"][k])
        assert report["bf16"][k]["max_rel"] <= RTOL_BF16, (k, report["bf16"][k])
