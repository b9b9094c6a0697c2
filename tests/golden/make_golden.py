"""Writes oracle_snapshot_small.json: a frozen record of the CPU oracle on a small seeded case.

Calls only the oracle (and the seeded input generators).  The paper prints no
worked example of the encoder or the decoder, so this file is not a paper value:
it guards the oracle against unnoticed changes.  Regenerating it is a change of
the oracle's arithmetic and needs the justification such a change needs.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import hash4d_oracle as O                 # noqa: E402
from paper_2507_19141_amd import synth                # noqa: E402


def snapshot():
    g = O.make_grid(4, 2, O.doubling_resolutions(4, 32, 4), O.doubling_resolutions(4, 16, 4), 1 << 12)
    rng, x = synth.small_inputs(0, 8)
    table = synth.table_init(g.E, 2, rng)
    params = synth.decoder_params(8, rng)
    gd = synth.upstream(8, 10, rng)
    eps = synth.perturbation(8, rng)
    rows, w = O.corners(x, g)
    f, delta = O.deform_forward(x, table, g, params)
    d_table, d_params, d_feat = O.deform_backward(x, table, g, params, gd)
    loss, d_smooth = O.smoothness(x, eps, table, g, 1.0)
    return {
        "about": "CPU oracle on 8 uniform points, seed 0, L=4 F=2 T=4096, doubling schedule 4->32 / 4->16, "
                 "decoder 8->64->64->10 (Section 4.2 Eqs. 7-10, Section 4.3 Eq. 11)",
        "grid": {"res_s": g.res_s, "res_t": g.res_t, "dense": g.dense, "offsets": g.offsets},
        "rows_q0": rows[0].tolist(),
        "weights_q0": w[0].tolist(),
        "f_h": f.tolist(),
        "delta": delta.tolist(),
        "d_feat": d_feat.tolist(),
        "d_params_sum": float(d_params.sum()),
        "d_params_abs_sum": float(np.abs(d_params).sum()),
        "d_table_nonzero_rows": int(np.count_nonzero(np.abs(d_table).sum(1))),
        "d_table_abs_sum": float(np.abs(d_table).sum()),
        "smooth_loss": loss,
        "d_smooth_abs_sum": float(np.abs(d_smooth).sum()),
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "oracle_snapshot_small.json"), "w") as fh:
        json.dump(snapshot(), fh, indent=1)
