"""The oracle still reproduces its frozen snapshot (tests/golden/oracle_snapshot_small.json)."""
import json
import os

import numpy as np

from tests.golden.make_golden import snapshot

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_oracle_matches_frozen_snapshot():
    with open(os.path.join(HERE, "oracle_snapshot_small.json")) as fh:
        want = json.load(fh)
    got = snapshot()
    for k, v in want.items():
        if isinstance(v, (str, dict)) or k in ("rows_q0", "d_table_nonzero_rows"):
            assert got[k] == v, k
        else:
            assert np.allclose(np.asarray(got[k]), np.asarray(v), rtol=1e-12, atol=1e-300), k
