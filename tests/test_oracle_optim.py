"""Pins of the oracle's optimiser step against torch's own CPU optimisers (library
routines, FP64): torch.optim.Adam for the dense step and torch.optim.SparseAdam for
the lazy step that touches only rows with a gradient."""
import numpy as np
import torch

from oracle import hash4d_oracle as O


def test_adam_matches_torch_adam_over_three_steps():
    rng = np.random.default_rng(50)
    p0 = rng.standard_normal(600)
    grads = [rng.standard_normal(600) for _ in range(3)]
    hp = dict(lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-15)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=hp["lr"], betas=(hp["beta1"], hp["beta2"]), eps=hp["eps"])
    p, m, v = p0, np.zeros(600), np.zeros(600)
    for t, g in enumerate(grads, 1):
        tp.grad = torch.tensor(g * 0.25)
        opt.step()
        p, m, v = O.adam_step(p, g, m, v, t=t, grad_scale=0.25, **hp)
        assert np.allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)
        st = opt.state[tp]
        assert np.allclose(m, st["exp_avg"].numpy(), rtol=1e-12, atol=1e-17)
        assert np.allclose(v, st["exp_avg_sq"].numpy(), rtol=1e-12, atol=1e-19)


def test_lazy_adam_matches_torch_sparse_adam():
    # SparseAdam adds eps to sqrt(v) before the bias correction of v is applied,
    # Adam after it; with a vanishing eps the two definitions coincide.
    rng = np.random.default_rng(51)
    rows, R = 50, 2
    p0 = rng.standard_normal((rows, R))
    hp = dict(lr=5e-3, beta1=0.8, beta2=0.99, eps=1e-300)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.SparseAdam([tp], lr=hp["lr"], betas=(hp["beta1"], hp["beta2"]), eps=hp["eps"])
    p, m, v = p0.reshape(-1), np.zeros(rows * R), np.zeros(rows * R)
    for t in range(1, 4):
        touched = np.sort(rng.choice(rows, 17, replace=False))
        g = np.zeros((rows, R))
        g[touched] = rng.standard_normal((17, R))
        tp.grad = torch.sparse_coo_tensor(torch.tensor(touched)[None], torch.tensor(g[touched]), (rows, R))
        opt.step()
        p, m, v = O.adam_step(p, g.reshape(-1), m, v, t=t, lazy_row=R, **hp)
        assert np.allclose(p.reshape(rows, R), tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_untouched_rows_keep_everything_in_the_lazy_step():
    rng = np.random.default_rng(52)
    p, m, v = rng.standard_normal(40), rng.standard_normal(40), rng.random(40)
    g = rng.standard_normal(40)
    g[10:20] = 0.0
    p1, m1, v1 = O.adam_step(p, g, m, v, 1e-3, 0.9, 0.999, 1e-8, 5, lazy_row=2)
    assert np.array_equal(p1[10:20], p[10:20]) and np.array_equal(m1[10:20], m[10:20])
    assert np.array_equal(v1[10:20], v[10:20])
    # the dense step moves them (momentum and the second moment decay)
    p2, m2, _ = O.adam_step(p, g, m, v, 1e-3, 0.9, 0.999, 1e-8, 5)
    assert not np.array_equal(p2[10:20], p[10:20]) and np.allclose(m2[10:20], 0.9 * m[10:20])
