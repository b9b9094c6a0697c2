"""Planted mistakes: each test breaks the CPU oracle in one plausible way and checks
that at least one pin notices.  The mistakes are planted in the oracle, on the CPU,
through monkeypatching; the oracle's own file is never changed."""
import math

import numpy as np
import pytest

from oracle import hash4d_oracle as O
from tests import test_oracle_decoder as D
from tests import test_oracle_encoder as E


def expect_pin_failure(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_schedule_without_level_exponent_is_caught(monkeypatch):
    def garbled(n_min, n_max, L):   # Eq. 7 as printed, b not raised to l
        b = math.exp((math.log(n_max) - math.log(n_min)) / (L - 1))
        return [n_min] + [int(n_min * b)] * (L - 2) + [n_max]
    monkeypatch.setattr(O, "level_resolutions", garbled)
    expect_pin_failure(E.test_schedule_matches_exact_integer_floor, 16, 2048, 16)


def test_schedule_without_fp_guard_is_caught(monkeypatch):
    def unguarded(n_min, n_max, L):
        b = math.exp((math.log(n_max) - math.log(n_min)) / (L - 1))
        return [int(math.floor(n_min * b ** l)) for l in range(L)]
    monkeypatch.setattr(O, "level_resolutions", unguarded)
    expect_pin_failure(E.test_schedule_fp_guard_case)


def test_swapped_weights_are_caught(monkeypatch):
    real = O.cell_position

    def swapped(x32, N):
        i, fr = real(x32, N)
        return i, 1.0 - fr
    monkeypatch.setattr(O, "cell_position", swapped)
    expect_pin_failure(E.test_affine_reproduction_on_dense_level)
    expect_pin_failure(E.test_dense_level_matches_scipy_regular_grid_interpolation)


def test_fp64_scaling_is_caught(monkeypatch):
    def fp64_scale(x32, N):
        pos = x32.astype(np.float64) * N
        i = np.minimum(np.floor(pos).astype(np.int64), N - 1)
        return i, pos - i
    monkeypatch.setattr(O, "cell_position", fp64_scale)
    expect_pin_failure(E.test_affine_reproduction_on_dense_level)


def test_transposed_dense_order_is_caught(monkeypatch):
    def z_fastest(vx, vy, vz, vt, Ns):
        S = Ns + 1
        return vz + S * (vy + S * (vx + S * vt))
    monkeypatch.setattr(O, "dense_index", z_fastest)
    expect_pin_failure(E.test_dense_index_is_bijection, 2, 3)


def test_corner_bits_out_of_step_with_weights_is_caught(monkeypatch):
    def mixed(xyzt, grid):
        x32 = O.clamp_unit_f32(xyzt)
        n = x32.shape[0]
        rows = np.zeros((n, grid.L, 16), dtype=np.int64)
        wts = np.zeros((n, grid.L, 16))
        for l in range(grid.L):
            res = (grid.res_s[l],) * 3 + (grid.res_t[l],)
            lo, fr = zip(*(O.cell_position(x32[:, d], res[d]) for d in range(4)))
            for c in range(16):
                up = [(c >> d) & 1 for d in range(4)]
                v = [lo[d] + up[d] for d in range(4)]
                w = np.ones(n)
                for d in range(4):
                    w = w * (fr[d] if up[3 - d] else 1.0 - fr[d])
                idx = O.dense_index(*v, grid.res_s[l]) if grid.dense[l] else O.hash_index(*v, grid.T)
                rows[:, l, c] = grid.offsets[l] + idx
                wts[:, l, c] = w
        return rows, wts
    monkeypatch.setattr(O, "corners", mixed)
    expect_pin_failure(E.test_dense_level_matches_scipy_regular_grid_interpolation)
    expect_pin_failure(E.test_brute_force_unit_grid_dense_T16)


def test_hash_without_32bit_wrap_is_caught(monkeypatch):
    def no_wrap(vx, vy, vz, vt, T):
        h = np.zeros(np.shape(vx), dtype=np.uint64)
        for v, p in zip((vx, vy, vz, vt), O.PRIMES):
            h ^= np.asarray(v, dtype=np.uint64) * np.uint64(p)
        return (h % np.uint64(T)).astype(np.int64)
    monkeypatch.setattr(O, "hash_index", no_wrap)
    expect_pin_failure(E.test_hash_against_python_bigints, 3 ** 9)


def test_hash_with_sum_instead_of_xor_is_caught(monkeypatch):
    def summed(vx, vy, vz, vt, T):
        h = np.zeros(np.shape(vx), dtype=np.uint64)
        for v, p in zip((vx, vy, vz, vt), O.PRIMES):
            h = (h + np.asarray(v, dtype=np.uint64) * np.uint64(p)) & np.uint64(0xFFFFFFFF)
        return (h % np.uint64(T)).astype(np.int64)
    monkeypatch.setattr(O, "hash_index", summed)
    expect_pin_failure(E.test_hash_against_python_bigints, 1 << 12)


def test_backward_without_weights_is_caught(monkeypatch):
    def unweighted(xyzt, d_feat, grid, scale=1.0):
        rows, _ = O.corners(xyzt, grid)
        out = np.zeros((grid.E, grid.F))
        for l in range(grid.L):
            for c in range(16):
                np.add.at(out, rows[:, l, c], scale * d_feat[:, l * grid.F:(l + 1) * grid.F] / 16)
        return out
    monkeypatch.setattr(O, "encode_backward", unweighted)
    expect_pin_failure(E.test_backward_is_exact_transpose)


def test_dropped_bias_is_caught(monkeypatch):
    real = O.unpack_params

    def no_b2(flat, n_in, hidden=64, out=10):
        d = real(flat, n_in, hidden, out)
        d["b2"] = np.zeros_like(d["b2"])
        return d
    monkeypatch.setattr(O, "unpack_params", no_b2)
    expect_pin_failure(D.test_decoder_forward_and_backward_match_torch, 8)


def test_one_sided_smoothness_gradient_is_caught(monkeypatch):
    def one_sided(xyzt, eps, table, grid, lam=1.0):
        n = xyzt.shape[0]
        xp = O.perturbed(xyzt, eps)
        d = O.encode(xyzt, table, grid) - O.encode(xp, table, grid)
        return lam / n * float(np.sum(d * d)), O.encode_backward(xyzt, 2 * lam / n * d, grid)
    monkeypatch.setattr(O, "smoothness", one_sided)
    # the value check passes, the central differences do not
    expect_pin_failure(D.test_smoothness_value_and_central_differences)


def test_input_grad_without_resolution_factor_is_caught(monkeypatch):
    # d frac / d x = N was dropped: the derivative is taken in cell units
    real = O.corner_weight_derivatives

    def per_cell(xyzt, grid):
        out = real(xyzt, grid)
        for l in range(grid.L):
            res = np.array((grid.res_s[l],) * 3 + (grid.res_t[l],), dtype=np.float64)
            out[:, l] /= res
        return out
    monkeypatch.setattr(O, "corner_weight_derivatives", per_cell)
    expect_pin_failure(E.test_input_grad_affine_closed_form)
    expect_pin_failure(E.test_input_grad_matches_central_differences)


def test_input_grad_ignoring_the_clamp_is_caught(monkeypatch):
    # the derivative of the clamp taken as 1 everywhere (out-of-range inputs moved inside)
    real = O.encode_backward_input

    def unclamped(xyzt, table, grid, d_feat, scale=1.0):
        x = np.asarray(xyzt, np.float32)
        inside = np.where(np.isnan(x), np.float32(0.5), np.clip(x, np.float32(0.01), np.float32(0.99)))
        return real(inside, table, grid, d_feat, scale)
    monkeypatch.setattr(O, "encode_backward_input", unclamped)
    expect_pin_failure(E.test_input_grad_is_zero_where_the_clamp_is_active)


def test_adam_without_bias_correction_is_caught(monkeypatch):
    from tests import test_oracle_optim as Opt
    real = O.adam_step

    def uncorrected(p, g, m, v, lr, beta1, beta2, eps, t, grad_scale=1.0, lazy_row=0):
        # t = 1e9 makes both bias corrections 1, i.e. drops them
        return real(p, g, m, v, lr, beta1, beta2, eps, 10 ** 9, grad_scale, lazy_row)
    monkeypatch.setattr(O, "adam_step", uncorrected)
    expect_pin_failure(Opt.test_adam_matches_torch_adam_over_three_steps)


def test_split_taking_ties_as_dynamic_is_caught(monkeypatch):
    from tests import test_oracle_decompose as Dec
    real_keys = O.motion_keys

    def ties_up(dp, k_percent, lam_s=1.0):   # ">= tau" instead of "> tau"
        key = real_keys(dp)
        n = len(key)
        n_d = int(math.floor(k_percent / 100.0 * n))
        dyn = np.ones(n, bool) if n_d >= n else key >= np.sort(key)[::-1][n_d]
        return np.nonzero(dyn)[0], 0.0, np.zeros((n, 3))
    monkeypatch.setattr(O, "decompose", ties_up)
    expect_pin_failure(Dec.test_split_matches_brute_force_with_ties_and_nan)


# ---- G_3D (reading R12) ----
from tests import test_oracle_encoder3 as E3  # noqa: E402


def test_g3d_slab_dense_criterion_is_caught(monkeypatch):
    # the 4D encoder on a t = 0 slab with one temporal cell: dense iff 2 (N+1)^3 <= T
    real = O.make_grid3

    def slab(L, F, res, T):
        g = real(L, F, res, T)
        off = [0]
        g.dense, g.sizes = [], []
        for N in g.res:
            nv = 2 * (N + 1) ** 3
            g.dense.append(nv <= g.T)
            g.sizes.append(nv if nv <= g.T else g.T)
            off.append(off[-1] + g.sizes[-1])
        g.offsets = off
        return g
    monkeypatch.setattr(O, "make_grid3", slab)
    expect_pin_failure(E3.test_dense_threshold_is_the_3d_vertex_count)


def test_g3d_swapped_primes_are_caught(monkeypatch):
    def swapped(vx, vy, vz, T):   # pi_2 and pi_3 exchanged
        h = np.zeros(np.shape(vx), dtype=np.uint64)
        for v, p in zip((vx, vy, vz), (O.PRIMES[0], O.PRIMES[2], O.PRIMES[1])):
            h ^= (np.asarray(v, dtype=np.uint64) * np.uint64(p)) & np.uint64(O.MASK32)
        return (h % np.uint64(T)).astype(np.int64)
    monkeypatch.setattr(O, "hash_index3", swapped)
    expect_pin_failure(E3.test_hash_matches_python_integers, 1 << 19)
    expect_pin_failure(E3.test_brute_force_exact_on_tiny_hashed_grid)


def test_g3d_corner_bits_out_of_step_are_caught(monkeypatch):
    real = O.cell_position

    def swapped(x32, N):   # the upper corner given the lower corner's weight
        i, fr = real(x32, N)
        return i, 1.0 - fr
    monkeypatch.setattr(O, "cell_position", swapped)
    expect_pin_failure(E3.test_dense_level_matches_scipy_trilinear)
