"""Seeded synthetic inputs for the 4D hash deformation path.

This module draws random numbers and nothing else: it holds no part of the
method's arithmetic (no schedule, no hashing, no interpolation, no decoder).
Tests, the benchmark and the smoke check use it to feed the same host arrays to
the HIP library and to the CPU checker.

The shapes stand in for the paper's real-world scenes (multi-view videos of
300 frames, scene Gaussian counts around 1e5, point clouds from structure from
motion, Section 5): the datasets themselves are not used.  All draws come from
``numpy.random.default_rng(seed)`` in a fixed order: positions, times, table,
decoder parameters, upstream gradients, perturbations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

FRAMES = 300            # frames per video in the paper's N3DV setting (Section 5.1)


def uniform_xyzt(n: int, rng: np.random.Generator) -> np.ndarray:
    """n points uniform in [0, 1)^4 as FP32 [n, 4] (x, y, z, t)."""
    xyz = rng.random((n, 3), dtype=np.float64)
    t = rng.random(n, dtype=np.float64)
    return np.concatenate([xyz, t[:, None]], axis=1).astype(np.float32)


def clustered_xyz(n: int, rng: np.random.Generator, clusters: int = 64) -> np.ndarray:
    """Gaussian-mixture cloud: centres U[0.1, 0.9]^3, isotropic sigma log-uniform in
    [0.01, 0.06], equal weights, clipped to [0, 1].  FP32 [n, 3]."""
    centres = rng.uniform(0.1, 0.9, size=(clusters, 3))
    sigma = np.exp(rng.uniform(math.log(0.01), math.log(0.06), size=clusters))
    k = rng.integers(0, clusters, size=n)
    pts = centres[k] + rng.standard_normal((n, 3)) * sigma[k, None]
    return np.clip(pts, 0.0, 1.0).astype(np.float32)


def frame_times(n: int, rng: np.random.Generator, frames: int = FRAMES) -> np.ndarray:
    """Per-point timestamps k / (frames - 1), k uniform on {0, ..., frames - 1}.  FP32 [n]."""
    k = rng.integers(0, frames, size=n)
    return (k / (frames - 1)).astype(np.float32)


def table_init(rows: int, F: int, rng: np.random.Generator, scale: float = 1e-4) -> np.ndarray:
    """Hash-table features uniform in (-scale, scale).  FP32 [rows, F]."""
    return rng.uniform(-scale, scale, size=(rows, F)).astype(np.float32)


def decoder_params(n_in: int, rng: np.random.Generator, hidden: int = 64, out: int = 10) -> np.ndarray:
    """Flat FP32 decoder parameters, each layer U(+-1/sqrt(fan_in)), in the order
    W1[hidden, n_in], b1, W2[hidden, hidden], b2, W3[out, hidden], b3."""
    parts = []
    for fan_in, fan_out in ((n_in, hidden), (hidden, hidden), (hidden, out)):
        k = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-k, k, size=fan_out * fan_in))
        parts.append(rng.uniform(-k, k, size=fan_out))
    return np.concatenate(parts).astype(np.float32)


def upstream(n: int, width: int, rng: np.random.Generator) -> np.ndarray:
    """Upstream gradients N(0, 1).  FP32 [n, width]."""
    return rng.standard_normal((n, width)).astype(np.float32)


def perturbation(n: int, rng: np.random.Generator, sigma: float = 1e-3) -> np.ndarray:
    """Smoothness perturbations eps ~ N(0, sigma^2) on all four coordinates.  FP32 [n, 4]."""
    return (rng.standard_normal((n, 4)) * sigma).astype(np.float32)


# ----------------------------------------------------------------------------
# Workload recipes.  Level resolutions are described by (n_min, n_max, rule);
# turning that into per-level numbers is method arithmetic and is done by each
# side on its own.
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    n: int
    L: int
    F: int
    T: int
    space: tuple          # (n_min, n_max)
    time: tuple           # (n_min, n_max)
    rule: str             # "geometric" (Eq. 7) or "doubling" (growth x2, clamped)
    n_in: int = 0         # decoder input width (L*F), 0 = encoder only


ENCODER_SMALL = Workload("encoder-4k-uniform-L4F2T4096", 4096, 4, 2, 1 << 12,
                         (4, 32), (4, 16), "doubling", 0)
SMALL_DECODER = Workload("deform-4k-uniform-L4F2T4096", 4096, 4, 2, 1 << 12,
                         (4, 32), (4, 16), "doubling", 8)
PAPER_SCENE = Workload("deform-200k-clustered-L16F2T2^19", 200_000, 16, 2, 1 << 19,
                       (16, 2048), (16, 150), "geometric", 32)

BATCHED_SCENE_N = (50_000, 100_000, 200_000, 400_000, 600_000, 800_000, 1_000_000, 1_200_000)
BATCHED_TIMES = tuple(k / (FRAMES - 1) for k in (0, 99, 199, 299))


def batched_table_rows_log2(n: int) -> int:
    """Per-scene hash table size used by the multi-scene workload."""
    if n < 200_000:
        return 17
    if n < 800_000:
        return 18
    return 19


def small_inputs(seed: int = 0, n: int = 4096):
    """Uniform points for the small parity workloads: positions then times."""
    rng = np.random.default_rng(seed)
    return rng, uniform_xyzt(n, rng)


def scene_inputs(n: int, seed: int = 0, shared_frame: int | None = None):
    """Clustered cloud with timestamps on the 300-frame grid.

    With ``shared_frame`` every point gets the same timestamp (one view per
    training iteration); otherwise each point draws its own frame.
    """
    rng = np.random.default_rng(seed)
    xyz = clustered_xyz(n, rng)
    if shared_frame is None:
        t = frame_times(n, rng)
    else:
        t = np.full(n, shared_frame / (FRAMES - 1), dtype=np.float32)
    return rng, np.concatenate([xyz, t[:, None]], axis=1).astype(np.float32)
