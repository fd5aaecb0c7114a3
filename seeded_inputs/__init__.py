"""Seeded synthetic inputs for the tile Cholesky path.

This module is shared by the CPU oracle's tests and by the GPU path. It
holds no arithmetic of the factorization, of the covariance function or of
the likelihood: only random draws, a spatial ordering of the points, small
integer/test matrices built from random draws, and the workload sizes.

Workloads (Matern covariance over points in the unit square, Section III-D,
Eq. 2; the paper's own experiments use synthetic Matern fields with
theta = (1, beta, 0.5)):

  small    n=2048,   nb=256,  nu=0.5, range=0.1,  nugget=1e-4  (FP64)
  fp64     n=65536,  nb=1024, nu=1.5, range=0.1,  nugget=1e-6  (FP64, in HBM)
  mxp      n=131072, nb=1024, nu=0.5, range=0.03, nugget=1e-4  (4 precisions,
           target accuracy 1e-9, 16 right-hand sides, refined solve)
  grad     n=32768,  nb=512,  nu=0.5, range=0.1,  nugget=1e-4  (likelihood
           gradient; 4000 base points translated to reach n)
  ooc      n=294912, nb=2048, nu=1.0, range=0.05, nugget=1e-4  (out of core)
"""
from __future__ import annotations

import numpy as np

WORKLOADS = {
    "small": dict(n=2048, nb=256, nu=0.5, sigma2=1.0, range=0.1, nugget=1e-4, seed=1),
    "fp64": dict(n=65536, nb=1024, nu=1.5, sigma2=1.0, range=0.1, nugget=1e-6, seed=2),
    "mxp": dict(n=131072, nb=1024, nu=0.5, sigma2=1.0, range=0.03, nugget=1e-4,
                eps=1e-9, nrhs=16, seed=3),
    "grad": dict(n=32768, nb=512, nu=0.5, sigma2=1.0, range=0.1, nugget=1e-4,
                 base_points=4000, seed=4, theta_eval=(1.2, 0.08, 2e-4)),
    "ooc": dict(n=294912, nb=2048, nu=1.0, sigma2=1.0, range=0.05, nugget=1e-4,
                eps=1e-9, seed=5),
}


def rhs_seed(points_seed: int) -> int:
    """Seed of the right-hand sides / latent draws that go with a point seed."""
    return 10 * points_seed + 1


def morton_order(pts: np.ndarray, bits: int = 16) -> np.ndarray:
    """Stable permutation sorting 2-D points in [0,1)^2 along the Z-order curve.

    Each coordinate is quantised to `bits` bits and the two codes are
    interleaved (x in the even bits, y in the odd bits). Nearby points then
    get nearby indices, which is what gives a covariance matrix its decaying
    off-diagonal tiles.
    """
    pts = np.asarray(pts, dtype=np.float64)
    scale = float(1 << bits)
    q = np.clip(np.floor(pts * scale), 0, scale - 1).astype(np.uint64)
    code = np.zeros(len(pts), dtype=np.uint64)
    for b in range(bits):
        one = np.uint64(1)
        code |= ((q[:, 0] >> np.uint64(b)) & one) << np.uint64(2 * b)
        code |= ((q[:, 1] >> np.uint64(b)) & one) << np.uint64(2 * b + 1)
    return np.argsort(code, kind="stable")


def points(n: int, seed: int, sort: bool = True) -> np.ndarray:
    """n seeded uniform points in the unit square, (n, 2) float64, C order.

    With sort=True they are reordered along the Z-order curve."""
    pts = np.random.default_rng(seed).random((n, 2))
    if sort:
        pts = pts[morton_order(pts)]
    return np.ascontiguousarray(pts)


def translated_points(n: int, base: int, seed: int) -> np.ndarray:
    """n points made from `base` seeded points: point i is base point i % base
    shifted by (i // base, 0), so that all n locations are distinct. The base
    set is Z-order sorted; the copies follow one another."""
    b = points(base, seed, sort=True)
    reps = -(-n // base)
    out = np.concatenate([b + np.array([r, 0.0]) for r in range(reps)], axis=0)
    return np.ascontiguousarray(out[:n])


def standard_normal(shape, seed: int) -> np.ndarray:
    """Seeded N(0,1) draws, float64, Fortran (column-major) order."""
    x = np.random.default_rng(seed).standard_normal(shape)
    return np.asfortranarray(x)


def integer_factor(n: int, seed: int, band: int = 3) -> np.ndarray:
    """Lower-triangular n x n float64 matrix with small integer entries.

    Diagonal entries are drawn from {1, 2, 4}; entries within `band` below the
    diagonal from {-1, 0, 1}. A = L0 L0^T then has small integer entries, and
    every product, sum, division by a diagonal entry and square root of a
    diagonal pivot met while factoring A is exact in binary64.
    """
    rng = np.random.default_rng(seed)
    L = np.zeros((n, n))
    L[np.arange(n), np.arange(n)] = rng.choice([1.0, 2.0, 4.0], size=n)
    for d in range(1, band + 1):
        idx = np.arange(d, n)
        L[idx, idx - d] = rng.choice([-1.0, 0.0, 1.0], size=n - d)
    return L


def random_factor(n: int, seed: int) -> np.ndarray:
    """Well-conditioned random lower-triangular matrix: unit-scale normal
    entries below the diagonal scaled by 1/sqrt(n), diagonal in [1, 2]."""
    rng = np.random.default_rng(seed)
    L = np.tril(rng.standard_normal((n, n)) / np.sqrt(n), -1)
    L[np.arange(n), np.arange(n)] = 1.0 + rng.random(n)
    return L


def tridiagonal(n: int) -> np.ndarray:
    """The n x n second-difference matrix tridiag(-1, 2, -1), float64."""
    A = 2.0 * np.eye(n)
    i = np.arange(n - 1)
    A[i + 1, i] = -1.0
    A[i, i + 1] = -1.0
    return A
