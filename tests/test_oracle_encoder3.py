"""Pins of the CPU oracle's 3D hash encoding G_3D (Section 4.1, Eq. 3; reading R12)
against what the mathematics fixes, each independent of the oracle's own code:
scipy's regular-grid linear interpolation (in 3D, trilinear interpolation) on dense
levels, Python-integer evaluation of the hash, brute force with exact rationals and
a hand-built vertex table on tiny hashed grids, the dense/hashed threshold, partition
of unity, vertex recovery, and the transpose identity of the backward."""
from fractions import Fraction

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from oracle import hash4d_oracle as O

P1, P2, P3 = 1, 2654435761, 805459861   # the spatial primes of the hash encoding (R4)


def bigint_hash3(vx, vy, vz, T):
    return (((vx * P1) & 0xFFFFFFFF) ^ ((vy * P2) & 0xFFFFFFFF) ^ ((vz * P3) & 0xFFFFFFFF)) % T


def test_dense_level_matches_scipy_trilinear():
    rng = np.random.default_rng(1)
    for N, F in ((5, 2), (12, 1), (7, 4)):
        S = N + 1
        g = O.make_grid3(1, F, [N], S ** 3)
        assert g.dense == [True]
        table = rng.uniform(-1, 1, size=(g.E, F)).astype(np.float32)
        x = rng.random((400, 3)).astype(np.float32)
        x[:5] = [[0, 0, 0], [1, 1, 1], [1, 0, 0.5], [0.5, 1, 0], [np.float32(3) / N, 0.25, 1]]
        got = O.encode3(x, table, g)
        # table row vx + S (vy + S vz)  ->  values[vx, vy, vz]
        vals = table.astype(np.float64).reshape(S, S, S, F).transpose(2, 1, 0, 3)
        axes = [np.arange(S, dtype=np.float64)] * 3
        for f in range(F):
            interp = RegularGridInterpolator(axes, vals[..., f], method="linear")
            pos = (x.astype(np.float32) * np.float32(N)).astype(np.float64)
            np.testing.assert_allclose(got[:, f], interp(pos), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("T", [1 << 12, 1 << 19, 5003])
def test_hash_matches_python_integers(T):
    rng = np.random.default_rng(2)
    v = rng.integers(0, 1 << 20, size=(500, 3))
    got = O.hash_index3(v[:, 0], v[:, 1], v[:, 2], T)
    want = [bigint_hash3(int(a), int(b), int(c), T) for a, b, c in v]
    assert got.tolist() == want


def test_brute_force_exact_on_tiny_hashed_grid():
    # N = 2 and T = 7: 27 vertices share 7 rows; every corner looked up through a dict
    # built by enumerating the vertices, every weight an exact rational
    N, T, F = 2, 7, 2
    g = O.make_grid3(1, F, [N], T)
    assert g.dense == [False]
    rng = np.random.default_rng(3)
    table = rng.uniform(-1, 1, size=(T, F)).astype(np.float32)
    row_of = {(a, b, c): bigint_hash3(a, b, c, T) for a in range(N + 1) for b in range(N + 1) for c in range(N + 1)}
    pts = [(Fraction(k, 8), Fraction(m, 16), Fraction(j, 4)) for k in range(9) for m in (0, 5, 16) for j in (1, 3)]
    x = np.array([[float(a), float(b), float(c)] for a, b, c in pts], dtype=np.float32)
    got = O.encode3(x, table, g)
    for q, p in enumerate(pts):
        pos = [c * N for c in p]                       # exact: N is a power of two
        lo = [min(int(c), N - 1) for c in pos]
        fr = [pos[d] - lo[d] for d in range(3)]
        for f in range(F):
            acc = Fraction(0)
            for c in range(8):
                up = [(c >> d) & 1 for d in range(3)]
                w = Fraction(1)
                for d in range(3):
                    w *= fr[d] if up[d] else 1 - fr[d]
                acc += w * Fraction(float(table[row_of[tuple(lo[d] + up[d] for d in range(3))], f]))
            assert got[q, f] == pytest.approx(float(acc), abs=1e-15)


def test_dense_threshold_is_the_3d_vertex_count():
    # dense iff (N+1)^3 <= T: the level of 8^3 = 512 vertices is dense at T = 512 and
    # at T = 600 (a 4D slab with one temporal cell would need 1024 rows), hashed at 511
    for T, dense in ((512, True), (600, True), (1023, True), (511, False)):
        g = O.make_grid3(1, 2, [7], T)
        assert g.dense == [dense]
        assert g.E == (512 if dense else T)
    g = O.make_grid3(3, 2, [4, 8, 16], 1 << 10)
    assert g.dense == [True, True, False]
    assert g.offsets == [0, 125, 125 + 729, 125 + 729 + 1024]


def test_partition_of_unity_and_vertex_recovery():
    rng = np.random.default_rng(4)
    g = O.make_grid3(3, 1, [4, 16, 64], 1 << 12)
    const = np.full((g.E, 1), 0.75, dtype=np.float32)
    x = rng.random((300, 3)).astype(np.float32)
    np.testing.assert_allclose(O.encode3(x, const, g), 0.75, rtol=0, atol=1e-15)
    _, w = O.corners3(x, g)
    np.testing.assert_allclose(w.sum(axis=2), 1.0, rtol=0, atol=1e-15)
    # at a vertex v / N (N a power of two: exact) the feature is that vertex's row
    table = rng.uniform(-1, 1, size=(g.E, 1)).astype(np.float32)
    for l, N in enumerate(g.res):
        v = rng.integers(0, N + 1, size=(50, 3))
        xv = (v / N).astype(np.float32)
        got = O.encode3(xv, table, g)[:, l]
        if g.dense[l]:
            rows = v[:, 0] + (N + 1) * (v[:, 1] + (N + 1) * v[:, 2])
        else:
            rows = np.array([bigint_hash3(int(a), int(b), int(c), g.T) for a, b, c in v])
        np.testing.assert_array_equal(got, table[g.offsets[l] + rows, 0].astype(np.float64))


def test_backward_is_the_transpose():
    rng = np.random.default_rng(5)
    g = O.make_grid3(3, 2, [4, 16, 64], 1 << 12)
    x = rng.random((500, 3)).astype(np.float32)
    u = rng.standard_normal((g.E, 2))
    gf = rng.standard_normal((500, 6))
    lhs = float(np.sum(O.encode3(x, u, g) * gf))
    rhs = float(np.sum(u * O.encode3_backward(x, gf, g)))
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # central differences on a few entries (exact: the encoding is linear in the table)
    grad = O.encode3_backward(x, gf, g)
    for r in rng.integers(0, g.E, size=8):
        for f in range(2):
            e = np.zeros_like(u)
            e[r, f] = 1e-3
            fd = (np.sum(O.encode3(x, u + e, g) * gf) - np.sum(O.encode3(x, u - e, g) * gf)) / 2e-3
            assert fd == pytest.approx(grad[r, f], rel=1e-9, abs=1e-9)


def test_out_of_range_and_nan_clamp():
    g = O.make_grid3(1, 1, [4], 1 << 10)
    table = np.arange(g.E, dtype=np.float32)[:, None]
    x = np.array([[-0.5, 2.0, np.nan], [0.0, 1.0, 0.0]], dtype=np.float32)
    got = O.encode3(x, table, g)
    assert got[0, 0] == got[1, 0]
