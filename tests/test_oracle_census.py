"""Pins of the oracle's collision census: a dense level is collision-free (its rows
are a bijection of the vertices), the counts match brute force on a tiny grid, and a
hashed level of few rows collides."""
import numpy as np

from oracle import hash4d_oracle as O
from paper_2507_19141_amd import synth


def test_dense_level_has_no_collisions():
    g = O.make_grid(2, 2, [4, 32], [4, 16], 1 << 12)
    assert g.dense == [True, False]
    _, x = synth.small_inputs(90, 2000)
    V, R = O.collision_census(x, g, 0)
    assert V == R and V <= 5 ** 3 * 5


def test_census_matches_brute_force():
    g = O.make_grid(1, 1, [6], [3], 37)
    assert g.dense == [False]
    rng = np.random.default_rng(91)
    x = rng.random((40, 4)).astype(np.float32)
    verts, rows = set(), set()
    for q in range(40):
        for c in range(16):
            v = []
            for d, N in enumerate((6, 6, 6, 3)):
                pos = np.float32(x[q, d]) * np.float32(N)
                v.append(min(int(np.floor(pos)), N - 1) + ((c >> d) & 1))
            verts.add(tuple(v))
            h = 0
            for vd, p in zip(v, O.PRIMES):
                h ^= (vd * p) & 0xFFFFFFFF
            rows.add(h % 37)
    assert O.collision_census(x, g, 0) == (len(verts), len(rows))
    assert len(rows) < len(verts)
