"""The C ABI library loads, exports every symbol include/hash4d.h declares, and its
host-only logic (level schedule, table layout, argument validation) agrees with
the oracle.  No call here launches GPU work."""
import os
import re

import numpy as np
import pytest

from oracle import hash4d_oracle as O
from paper_2507_19141_amd import _lib, synth
from tests.util import assert_same_layout, lib_grid, oracle_grid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hash4d.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+\*?([a-z0-9_]+)\s*\(",
                                 text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), f"{n} declared in hash4d.h but not exported"
    # every declared function has a binding of the same name, and vice versa
    assert sorted(_lib.SIGNATURES) == names


def test_version_and_empty_error():
    assert b"gfx950" in _lib.load().h4d_version()
    _lib.h4d_grid_schedule(4, 4, 16)
    assert _lib.last_error() == ""


@pytest.mark.parametrize("rule", [_lib.SCHEDULE_GEOMETRIC, _lib.SCHEDULE_DOUBLING])
def test_schedule_matches_oracle(rule):
    rng = np.random.default_rng(30)
    for _ in range(300):
        n_min = int(rng.integers(1, 100))
        n_max = int(rng.integers(n_min, 1 << 14))
        L = int(rng.integers(1, 33))
        want = (O.level_resolutions if rule == _lib.SCHEDULE_GEOMETRIC else O.doubling_resolutions)(n_min, n_max, L)
        assert _lib.h4d_grid_schedule(L, n_min, n_max, rule) == want


@pytest.mark.parametrize("w", [synth.ENCODER_SMALL, synth.PAPER_SCENE], ids=lambda w: w.name)
def test_layout_matches_oracle(w):
    og, lg = oracle_grid(w), lib_grid(w)
    assert_same_layout(og, lg)
    assert _lib.h4d_grid_rows(lg) == og.E
    assert list(lg.prime) == list(O.PRIMES)


def test_layout_random_grids():
    rng = np.random.default_rng(31)
    for _ in range(200):
        L = int(rng.integers(1, 33))
        F = int(rng.choice([1, 2, 4, 8]))
        T = int(rng.integers(1, 1 << 20))
        rs = rng.integers(1, 300, size=L).tolist()
        rt = rng.integers(1, 300, size=L).tolist()
        og = O.make_grid(L, F, rs, rt, T)
        if og.E * F >= 1 << 31:
            continue
        assert_same_layout(og, _lib.h4d_grid_init(L, F, rs, rt, T))


@pytest.mark.parametrize("args,frag", [
    ((0, 2, [4], [4], 64), "L=0"),
    ((33, 2, [4] * 33, [4] * 33, 64), "L=33"),
    ((2, 3, [4, 4], [4, 4], 64), "F=3"),
    ((2, 2, [0, 4], [4, 4], 64), "resolution"),
    ((2, 2, [4, 4], [4, 1 << 25], 64), "resolution"),
    ((2, 2, [4, 4], [4, 4], 0), "T=0"),
    ((2, 2, [4, 4], [4, 4], (1 << 30) + 1), "T="),
    ((3, 8, [1 << 20] * 3, [1 << 20] * 3, 1 << 30), "exceeds 2^31"),
])
def test_grid_init_rejects(args, frag):
    L = args[0]
    g = _lib.Grid()
    rs = (_lib.ctypes.c_int32 * max(L, 1))(*args[2][:max(L, 1)])
    rt = (_lib.ctypes.c_int32 * max(L, 1))(*args[3][:max(L, 1)])
    st = _lib.load().h4d_grid_init(_lib.ctypes.byref(g), L, args[1], rs, rt, args[4])
    assert st == -1
    assert frag in _lib.last_error()


def test_schedule_rejects():
    for args in [(0, 4, 16, 0), (4, 0, 16, 0), (4, 16, 4, 0), (4, 4, 1 << 25, 0), (4, 4, 16, 7)]:
        with pytest.raises(_lib.H4DError) as e:
            _lib.h4d_grid_schedule(*args)
        assert e.value.status == -1


def test_corrupted_grid_is_rejected_before_launch():
    g = lib_grid(synth.ENCODER_SMALL)
    g.offset[2] += 1
    assert _lib.h4d_grid_rows(g) == -1
    fake = 1 << 20   # never dereferenced: validation fails first
    st = _lib.load().hash4d_encode(_lib.ctypes.byref(g), 0, fake, fake, 10, 0, fake, None)
    assert st == -1 and "inconsistent" in _lib.last_error()


def test_entry_points_validate_without_launching():
    lib = _lib.load()
    g = lib_grid(synth.ENCODER_SMALL)
    gp = _lib.ctypes.byref(g)
    fake = 1 << 20
    assert lib.hash4d_encode(gp, 0, fake, fake, 0, 0, fake, None) == 0                 # n = 0: no-op
    assert lib.hash4d_encode(gp, 0, None, fake, 5, 0, fake, None) == -1                # NULL table
    assert lib.hash4d_encode(gp, 0, fake, fake + 4, 5, 0, fake, None) == -1            # misaligned xyzt
    assert "aligned" in _lib.last_error()
    assert lib.hash4d_encode(gp, 0, fake + 4, fake, 5, 0, fake, None) == -1            # table not row-aligned
    assert "row size" in _lib.last_error()
    assert lib.hash4d_encode(gp, 7, fake, fake, 5, 0, fake, None) == -1                # unknown dtype
    assert lib.hash4d_encode(gp, 0, fake, fake, 5, 2, fake, None) == -1                # unknown layout
    assert lib.hash4d_encode(gp, 0, fake, fake, -1, 0, fake, None) == -1               # negative n
    assert lib.hash4d_encode(gp, 0, fake, fake, 1 << 31, 0, fake, None) == -1          # n too large
    assert lib.hash4d_encode_backward(gp, 1, fake, 5, 0, fake, 1.0, fake, fake, 1 << 20, None) == -1  # F32/F64 grads
    assert lib.hash4d_encode_backward(gp, 0, fake, 5, 0, fake, 1.0, fake, fake, 4, None) == -1        # small workspace
    assert "workspace" in _lib.last_error()
    assert lib.hash4d_encode_backward(gp, 0, fake, 5, 0, fake, 1.0, fake, fake + 8, 1 << 20, None) == -1  # misaligned
    assert "aligned" in _lib.last_error()
    OW = _lib.GRAD_OVERWRITE
    assert lib.hash4d_encode_backward(gp, 0, fake, 5, 0x200, fake, 1.0, fake, fake, 1 << 20, None) == -1  # bad flag
    assert "layout" in _lib.last_error()
    assert lib.hash4d_encode_backward(gp, 0, fake, 0, OW, fake, 1.0, None, fake, 0, None) == -1  # n = 0 writes: NULL
    assert lib.hash4d_encode(gp, 0, fake, fake, 5, OW, fake, None) == -1              # the forward has no gradient
    assert lib.hash4d_encode_backward_input(gp, 0, fake, fake, 5, OW, fake, 1.0, fake, None, 0, None) == -1
    # masks (4 bytes) and pair tile bytes (8 bytes) per (query, level), level-major with
    # the query count padded to a multiple of four, then a load-balance plan whose size
    # does not depend on n within one chunk of queries
    w1000 = _lib.hash4d_encode_backward_workspace_bytes(g, 1000)
    w1001 = _lib.hash4d_encode_backward_workspace_bytes(g, 1001)
    assert w1000 >= 1000 * 4 * 12 and w1001 >= 1004 * 4 * 12
    assert abs((w1001 - 1004 * 4 * 12) - (w1000 - 1000 * 4 * 12)) <= 512
    assert lib.hash4d_corner_indices(gp, fake, 5, None, None, None) == -1
    assert lib.hash4d_encode_backward_input(gp, 0, fake, fake, 5, 0, fake, 1.0, None, None, 0, None) == -1  # NULL d_xyzt
    assert lib.hash4d_encode_backward_input(gp, 0, fake, fake, 5, 0, fake, 1.0, fake + 8, None, 0, None) == -1
    assert "d_xyzt" in _lib.last_error()
    assert lib.hash4d_encode_backward_input(gp, 0, fake, fake, 0, 0, None, 1.0, None, None, 0, None) == 0  # n = 0
    wbi = _lib.hash4d_encode_backward_input_workspace_bytes(g, 0, 5)
    assert wbi == 5 * g.L * 16 and _lib.hash4d_encode_backward_input_workspace_bytes(g, 2, 5) == 0
    assert lib.hash4d_encode_backward_input(gp, 0, fake, fake, 5, 0, fake, 1.0, fake, fake, wbi - 1, None) == -1
    assert "workspace" in _lib.last_error()
    assert lib.hash4d_encode_backward_input(gp, 0, fake, fake, 5, 0, fake, 1.0, fake, fake + 8, wbi, None) == -1
    assert "aligned" in _lib.last_error()
    assert lib.hash4d_encode(None, 0, fake, fake, 5, 0, fake, None) == -1
    sm = lib.hash4d_encode_backward_smooth
    wbs = _lib.smoothness_workspace_bytes(g, 0, 5)
    assert sm(gp, 0, fake, fake, fake, 5, 1, None, 1.0, 1.0, fake, fake, fake, wbs, None) == -1   # NULL d_feat
    assert sm(gp, 0, fake, fake, fake + 4, 5, 1, fake, 1.0, 1.0, fake, fake, fake, wbs, None) == -1  # eps aligned
    assert "eps" in _lib.last_error()
    assert sm(gp, 0, fake, fake, fake, 5, 1, fake, 1.0, 1.0, fake, fake, fake, wbs - 4, None) == -1  # workspace
    assert "workspace" in _lib.last_error()
    assert sm(gp, 0, fake, fake, fake, 5, 1, fake, 1.0, 1.0, fake, None, fake, wbs, None) == -1     # NULL d_table
    assert sm(gp, 0, fake, fake, fake, 5, 2, fake, 1.0, 1.0, fake, fake, fake, wbs, None) == -1     # unknown layout
    assert sm(gp, 0, fake, fake, fake, 0, 1, None, 1.0, 1.0, None, fake, None, 0, None) == 0        # n = 0: no-op
    assert sm(gp, 0, fake, fake, fake, 0, 0x101, None, 1.0, 1.0, None, None, None, 0, None) == -1   # writes: NULL
    hp = _lib.Adam(1e-3, 0.9, 0.999, 1e-8, 1, 1.0)
    hpp = _lib.ctypes.byref(hp)
    assert lib.h4d_adam_step(fake, fake, fake, fake + 4, 8, 1, hpp, None, 0, None) == -1   # misaligned v
    assert lib.h4d_adam_step(fake, fake, fake, fake, 9, 2, hpp, None, 1, None) == -1       # count % row
    assert lib.h4d_adam_step(fake, fake, fake, fake, 8, 3, hpp, None, 1, None) == -1       # row 3
    assert lib.h4d_adam_step(fake, fake, fake, fake, 8, 1, hpp, None, 4, None) == -1       # unknown flag
    assert lib.h4d_adam_step(fake, fake, fake, fake, 8, 1, None, None, 0, None) == -1      # no hyper-parameters
    bad = _lib.Adam(1e-3, 1.0, 0.999, 1e-8, 1, 1.0)
    assert lib.h4d_adam_step(fake, fake, fake, fake, 8, 1, _lib.ctypes.byref(bad), None, 0, None) == -1  # beta1 = 1
    bad = _lib.Adam(1e-3, 0.9, 0.999, 1e-8, 0, 1.0)
    assert lib.h4d_adam_step(fake, fake, fake, fake, 8, 1, _lib.ctypes.byref(bad), None, 0, None) == -1  # step 0
    assert lib.h4d_adam_step(None, None, None, None, 0, 1, hpp, None, 0, None) == 0        # count 0
    assert lib.hash4d_decompose(fake, 10, 101.0, 1.0, None, None, None, None, None, fake, 1 << 20, None) == -1  # k
    assert lib.hash4d_decompose(None, 10, 10.0, 1.0, None, None, None, None, None, fake, 1 << 20, None) == -1  # dp
    assert lib.hash4d_decompose(fake, 10, 10.0, 1.0, None, None, None, None, None, fake, 8, None) == -1       # ws
    assert lib.hash4d_decompose(fake, 0, 10.0, 1.0, None, None, None, None, None, None, 0, None) == 0          # n 0
    assert _lib.hash4d_decompose_workspace_bytes(1000) == 256 + 1024 + 12 * 4
    assert lib.hash4d_collision_census(gp, 9, fake, 5, fake, fake, 1 << 30, None) == -1       # level out of range
    assert lib.hash4d_collision_census(gp, 0, fake, 5, None, fake, 1 << 30, None) == -1       # counts NULL
    assert lib.hash4d_collision_census(gp, 0, fake, 5, fake, fake, 8, None) == -1             # workspace
    assert _lib.hash4d_collision_workspace_bytes(g, 0, 1000) == 32768 * 8 + ((625 + 31) // 32) * 4
    m = _lib.mlp_shape(32)
    mp = _lib.ctypes.byref(m)
    assert lib.deform_mlp_forward(mp, 0, fake, fake, 5, 1, 3, fake, None) == -1            # F must divide in
    assert lib.deform_mlp_forward(mp, 0, fake, fake, 0, 1, 2, fake, None) == 0             # n = 0
    bad = _lib.mlp_shape(24)
    assert lib.deform_mlp_forward(_lib.ctypes.byref(bad), 0, fake, fake, 5, 0, 0, fake, None) == -2
    assert _lib.deform_mlp_workspace_bytes(m, 0, 200_000) > 0
    assert _lib.deform_mlp_workspace_bytes(bad, 0, 200_000) == 0
    assert lib.deform_mlp_backward(mp, 0, fake, fake, 5, 0, 0, fake, 1.0, 1.0, fake, fake, fake, 8, None) == -1
    OW = _lib.GRAD_OVERWRITE
    assert lib.deform_mlp_backward(mp, 0, fake, fake, 0, OW, 0, fake, 1.0, 1.0, fake, None, fake, 8, None) == -1
    assert lib.deform_mlp_backward(mp, 0, fake, fake, 0, 0, 0, fake, 1.0, 1.0, fake, None, fake, 8, None) == 0
    assert lib.deform_mlp_forward(mp, 0, fake, fake, 5, OW, 0, fake, None) == -1            # no gradient there
    # the overflow-counting forms check their counter before anything else
    ck = lib.deform_mlp_backward_checked
    assert ck(mp, 0, fake, fake, 5, 0, 0, fake, 1.0, 1.0, fake, fake, fake, 1 << 20, None, None) == -1  # NULL
    assert "nonfinite" in _lib.last_error()
    assert ck(mp, 0, fake, fake, 5, 0, 0, fake, 1.0, 1.0, fake, fake, fake, 1 << 20, fake + 2, None) == -1
    assert "aligned" in _lib.last_error()
    eck = lib.hash4d_encode_backward_checked
    assert eck(gp, 0, fake, 5, 0, fake, 1.0, fake, fake, 1 << 20, None, None) == -1              # NULL counter
    assert "nonfinite" in _lib.last_error()
    assert eck(gp, 0, fake, 5, 0, fake, 1.0, fake, fake, 1 << 20, fake + 1, None) == -1          # misaligned
    assert eck(gp, 0, fake, 5, 0, fake, 1.0, fake, fake, 4, fake, None) == -1                   # then the rest
    assert "workspace" in _lib.last_error()
    assert lib.h4d_count_nonfinite(fake, -1, fake, None) == -1
    assert lib.h4d_count_nonfinite(None, 0, None, None) == 0                                  # count 0: no-op
    assert lib.h4d_count_nonfinite(None, 5, fake, None) == -1


def test_query_count_limit_boundary():
    """n up to 2^31 - 2^16 passes the size checks (validation then stops at a NULL
    pointer, before any launch); one more query is rejected as out of range, so no
    kernel sees a count whose padding to whole workgroups overflows 32 bits."""
    lib = _lib.load()
    limit = (1 << 31) - (1 << 16)
    g = _lib.h4d_grid_init(1, 1, [4], [4], 1 << 12)
    gp = _lib.ctypes.byref(g)
    fake = 1 << 20
    assert lib.hash4d_encode(gp, 0, None, fake, limit, 0, fake, None) == -1
    assert "NULL" in _lib.last_error()
    assert lib.hash4d_encode(gp, 0, None, fake, limit + 1, 0, fake, None) == -1
    assert "outside" in _lib.last_error()
    assert _lib.hash4d_encode_backward_workspace_bytes(g, limit) > 0
    assert _lib.hash4d_encode_backward_workspace_bytes(g, limit + 1) == 0
    m = _lib.mlp_shape(8)
    mp = _lib.ctypes.byref(m)
    lim8 = ((1 << 31) - 1) // 8   # n in <= 2^31 - 1 features binds first for in = 8
    assert lib.deform_mlp_forward(mp, 0, None, fake, lim8, 0, 0, fake, None) == -1
    assert "NULL" in _lib.last_error()
    assert lib.deform_mlp_forward(mp, 0, None, fake, limit + 1, 0, 0, fake, None) == -1
    assert "outside" in _lib.last_error()
    assert lib.hash4d_decompose(None, limit, 10.0, 1.0, None, None, None, None, None, fake, 1 << 20, None) == -1
    assert "dp" in _lib.last_error()
    assert lib.hash4d_decompose(fake, limit + 1, 10.0, 1.0, None, None, None, None, None, fake, 1 << 20,
                                None) == -1
    assert "outside" in _lib.last_error()
    assert lib.hash4d_deform_apply(None, limit + 1, 10, fake, fake, fake, fake, fake, fake, None) == -1
    assert "outside" in _lib.last_error()


def test_grid3_layout_matches_oracle():
    rng = np.random.default_rng(33)
    for _ in range(200):
        L = int(rng.integers(1, 17))
        F = int(rng.choice([1, 2, 4, 8]))
        T = int(rng.choice([1 << int(rng.integers(4, 21)), int(rng.integers(1, 1 << 20))]))
        res = sorted(int(v) for v in rng.integers(1, 300, size=L))
        og = O.make_grid3(L, F, res, T)
        if og.E * F >= 1 << 31:
            continue
        lg = _lib.h4d_grid3_init(L, F, res, T)
        assert lg.dense_list() == og.dense and lg.offsets() == og.offsets
        assert list(lg.prime) == list(O.PRIMES[:3])


def test_hash3d_encode_validates_without_launching():
    lib = _lib.load()
    g = _lib.h4d_grid3_init(3, 2, [4, 8, 16], 1 << 10)
    gp = _lib.ctypes.byref(g)
    fake = 1 << 20   # never dereferenced: validation fails first
    assert lib.hash3d_encode(gp, 0, fake, fake, 3, 0, 0, fake, None) == 0        # n = 0: no-op
    assert lib.hash3d_encode(gp, 0, fake, fake, 5, 4, 0, fake, None) == -1       # stride
    assert "stride" in _lib.last_error()
    assert lib.hash3d_encode(gp, 0, None, fake, 3, 4, 0, fake, None) == -1       # NULL table
    assert lib.hash3d_encode(gp, 0, fake, fake + 4, 4, 4, 0, fake, None) == -1   # [n, 4] rows not 16-byte aligned
    assert lib.hash3d_encode(gp, 0, fake, fake + 2, 3, 4, 0, fake, None) == -1   # not 4-byte aligned
    assert lib.hash3d_encode(gp, 0, fake, fake, 3, -1, 0, fake, None) == -1      # negative n
    g.offset[2] += 1
    assert lib.hash3d_encode(gp, 0, fake, fake, 3, 4, 0, fake, None) == -1       # corrupted grid
    assert "inconsistent" in _lib.last_error()
