"""GPU parity of the collision census (distinct corner vertices and table rows of one
level) through the C ABI: exact integer counts against the oracle's Python sets."""
import numpy as np
import pytest

from oracle import hash4d_oracle as O
from paper_2507_19141_amd import _lib, synth
from tests.test_gpu_encoder import dev, edge_points, encoder_case, host
from tests.util import needs_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    needs_gpu()


def census(lg, level, x):
    import torch
    n = x.shape[0]
    counts = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    wb = _lib.hash4d_collision_workspace_bytes(lg, level, n)
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
    _lib.hash4d_collision_census(lg, level, dev(x), n, counts, ws, wb)
    return tuple(int(v) for v in host(counts))


def test_census_small_all_levels():
    og, lg, x, _, _ = encoder_case(synth.ENCODER_SMALL, 4096, 95)
    for level in range(og.L):
        got = census(lg, level, x)
        assert got == O.collision_census(x, og, level), level
        if og.dense[level]:
            assert got[0] == got[1]


@pytest.mark.parametrize("level", [0, 9, 15])
def test_census_paper_scene(level):
    w = synth.PAPER_SCENE
    og, lg, x, _, _ = encoder_case(w, w.n, 96, edges=False)
    got = census(lg, level, x)
    assert got == O.collision_census(x, og, level)
    if level == 15:
        assert got[1] < got[0]   # the finest hashed level collides


def test_census_twice_in_a_row_starts_clean():
    og, lg, x, _, _ = encoder_case(synth.ENCODER_SMALL, 1000, 97)
    a = census(lg, 3, x)
    b = census(lg, 3, x[:500])
    assert a == O.collision_census(x, og, 3) and b == O.collision_census(x[:500], og, 3)
