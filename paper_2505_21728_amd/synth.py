"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module draws random inputs only; it holds none of the transform's
arithmetic. The workloads it imitates are the paper's: intra-prediction
residual blocks of 4x4 and 8x8 pixels (Sec. VI), one class per block out of
35 intra modes per size (Sec. VI), and one angle per butterfly (Sec. IV). The
paper's training and test video data are not available; separable 2-D AR(1)
fields stand in for residual blocks.

All generators use numpy's PCG64 through ``default_rng(seed)``.
"""

from __future__ import annotations

import math

import numpy as np

SEED_ANGLES = 1
SEED_DATA = 2
SEED_CLASSES = 3
SEED_SERVING = 4


def angles(nclasses: int, rounds: int, d: int, seed: int = SEED_ANGLES) -> np.ndarray:
    """float32 [C, R, d, N/2] angles, uniform in [-pi, pi)."""
    rng = np.random.default_rng(seed)
    half = 1 << (d - 1)
    return rng.uniform(-math.pi, math.pi, (nclasses, rounds, d, half)).astype(np.float32)


def gaussian_blocks(nblocks: int, n_elems: int, sigma: float = 32.0,
                    seed: int = SEED_DATA) -> np.ndarray:
    """float32 [B, N] i.i.d. N(0, sigma^2) residuals."""
    rng = np.random.default_rng(seed)
    return (sigma * rng.standard_normal((nblocks, n_elems))).astype(np.float32)


def ar1_filter(width: int, rho: float) -> np.ndarray:
    """Lower-triangular W x W filter whose output is a unit-variance AR(1) row.

    Row i combines white noise as z_0*rho^i + sqrt(1-rho^2)*sum_{j=1..i} rho^(i-j) z_j,
    so the output covariance is rho^|i-j|.
    """
    a = np.zeros((width, width), dtype=np.float64)
    g = math.sqrt(1.0 - rho * rho)
    for i in range(width):
        a[i, 0] = rho ** i
        for j in range(1, i + 1):
            a[i, j] = rho ** (i - j) * g
    return a


def ar1_blocks(nblocks: int, width: int, rho: float = 0.9, sigma: float = 40.0,
               seed: int = SEED_DATA, clip: float = 255.0, integer: bool = True,
               chunk: int = 1 << 16) -> np.ndarray:
    """float32 [B, W*W] separable 2-D AR(1) blocks in row-major raster order.

    X = sigma * A Z A^T with Z ~ N(0, 1) of shape W x W, so that
    cov(X[r1,c1], X[r2,c2]) = sigma^2 rho^|r1-r2| rho^|c1-c2|. With
    ``integer`` the values are rounded half-to-even and clipped to
    [-clip, clip] (the int16 range used by the 8x8 workload), then stored as
    float32. ``rho`` may be a scalar or a per-block array.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((nblocks, width * width), dtype=np.float32)
    rho_arr = np.broadcast_to(np.asarray(rho, dtype=np.float64), (nblocks,))
    per_block = np.ndim(rho) > 0
    a_fixed = None if per_block else ar1_filter(width, float(rho))
    for start in range(0, nblocks, chunk):
        stop = min(nblocks, start + chunk)
        z = rng.standard_normal((stop - start, width, width))
        if per_block:
            a = np.stack([ar1_filter(width, float(r)) for r in rho_arr[start:stop]])
            x = sigma * (a @ z @ np.transpose(a, (0, 2, 1)))
        else:
            x = sigma * (a_fixed @ z @ a_fixed.T)
        if integer:
            x = np.clip(np.rint(x), -clip, clip)
        out[start:stop] = x.reshape(stop - start, width * width).astype(np.float32)
    return out


def classes(nblocks: int, nclasses: int, seed: int = SEED_CLASSES) -> np.ndarray:
    """int32 [B] class indices, uniform in [0, C)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, nclasses, nblocks, dtype=np.int32)
