"""GPU parity of the fused optimiser step (Adam + BF16 copy + gradient zeroing)
through the C ABI, against the FP64 oracle (itself pinned to torch.optim.Adam and
SparseAdam).  FP32 arithmetic: parameters within 1e-5 of (|p| + lr), moments within
1e-5 of their magnitude; the BF16 copy is the RNE of the kernel's own FP32 result,
bit for bit; untouched rows of the lazy step are bit-identical to their inputs."""
import numpy as np
import pytest

from oracle import hash4d_oracle as O
from paper_2507_19141_amd import _lib
from tests.util import needs_gpu, scaled_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    needs_gpu()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


HP = dict(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8)


def state(count, seed, zero_rows=None, row=1):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(count).astype(np.float32)
    g = (rng.standard_normal(count) * 50).astype(np.float32)
    m = (rng.standard_normal(count) * 0.1).astype(np.float32)
    v = (rng.random(count) * 0.01).astype(np.float32)
    if zero_rows is not None:
        gr = g.reshape(-1, row)
        gr[zero_rows] = 0.0
    return p, g, m, v


def check(got, ref, g, lr, grad_scale):
    p, m, v = got
    rp, rm, rv = ref
    gs = np.abs(g.astype(np.float64) * grad_scale)
    scaled_close(p, rp, lr, 1e-5, "params")
    scaled_close(m, rm, gs, 1e-5, "m")
    scaled_close(v, rv, gs * gs, 1e-5, "v")


@pytest.mark.parametrize("count", [10001, 4096 + 3])
def test_adam_dense_two_steps_with_bf16_copy_and_zeroing(count):
    import torch
    p, g, m, v = state(count, 60)
    P, G, M, V = dev(p), dev(g), dev(m), dev(v)
    lo = torch.empty(count, dtype=torch.int16, device="cuda")
    rp, rm, rv = p, m, v
    for t in (1, 2):
        G.copy_(dev(g))
        _lib.h4d_adam_step(P, G, M, V, count, step=t, grad_scale=0.5, bf16_out=lo,
                           flags=_lib.ADAM_ZERO_GRAD, **HP)
        rp, rm, rv = O.adam_step(rp, g, rm, rv, t=t, grad_scale=0.5, **HP)
        got = (host(P), host(M), host(V))
        check(got, (rp, rm, rv), g, HP["lr"], 0.5)
        assert np.array_equal(host(lo).view(np.uint16), O.bf16_bits(got[0]))
        assert not host(G).any()


@pytest.mark.parametrize("row", [1, 2, 4, 8])
def test_adam_lazy_rows(row):
    count = row * 3001
    zero_rows = np.arange(0, 3001, 3)
    p, g, m, v = state(count, 61, zero_rows, row)
    P, G, M, V = dev(p), dev(g), dev(m), dev(v)
    _lib.h4d_adam_step(P, G, M, V, count, step=7, row=row, flags=_lib.ADAM_LAZY, **HP)
    rp, rm, rv = O.adam_step(p, g, m, v, t=7, lazy_row=row, **HP)
    got = (host(P), host(M), host(V))
    check(got, (rp, rm, rv), g, HP["lr"], 1.0)
    idle = np.zeros(count, bool)
    idle.reshape(-1, row)[zero_rows] = True
    for a, b in zip(got, (p, m, v)):
        assert np.array_equal(a[idle].view(np.uint32), b[idle].view(np.uint32))
    assert np.array_equal(host(G), g)   # no ZERO_GRAD flag: the gradient is left alone


def test_adam_paper_table_sampled():
    # the whole table of the paper-shaped scene (7 654 726 rows x 2) in one call;
    # the step is elementwise, so sampled elements are checked exactly as computed
    count = 7654726 * 2
    p, g, m, v = state(count, 62)
    P, G, M, V = dev(p), dev(g), dev(m), dev(v)
    _lib.h4d_adam_step(P, G, M, V, count, step=3, grad_scale=1 / 4096, row=2,
                       flags=_lib.ADAM_LAZY | _lib.ADAM_ZERO_GRAD, **HP)
    idx = np.random.default_rng(63).choice(count, 20000, replace=False)
    idx = np.unique(np.concatenate([idx, idx ^ 1]))   # whole rows
    rp, rm, rv = O.adam_step(p[idx], g[idx], m[idx], v[idx], t=3, grad_scale=1 / 4096, lazy_row=2, **HP)
    got = (host(P)[idx], host(M)[idx], host(V)[idx])
    check(got, (rp, rm, rv), g[idx], HP["lr"], 1 / 4096)


def test_adam_count_zero_is_noop():
    import torch
    t = torch.ones(4, device="cuda")
    _lib.h4d_adam_step(t, t, t, t, 0, step=1, **HP)
    assert (host(t) == 1).all()
