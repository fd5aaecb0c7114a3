"""CPU oracle for the tile Cholesky path.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product library. It
shares no code with the GPU path. Everything is binary64.

Paper: arXiv 2410.09819 ("Accelerating Mixed-Precision Out-of-Core Cholesky
Factorization with Static Task Scheduling").

  tile_cholesky        left-looking tile Cholesky, Section III-A, Algorithm 1
                       (plain C loops in oracle.c)
  cholesky_unblocked   row-by-row Cholesky on the whole matrix (cross-check)
  solve, logdet        Sigma^{-1} y and log|Sigma| from the factor, used by the
                       likelihood of Eq. 1 (Section III-D)
  matern, matern_*     Eq. 2, C(h) = sigma^2 / (2^(nu-1) Gamma(nu)) (h/a)^nu
                       K_nu(h/a), written out with scipy's K_nu; the nugget
                       tau^2 is added on the diagonal
  tile_norms, fro_norm, precision_map
                       the per-tile precision criterion of Section IV-C:
                       tile (i,j) may be stored in a lower precision p when
                       Nt ||A_ij||_F / ||A||_F < eps_target / eps_p

Pins (what ties each function to something other than itself) live in
tests/test_oracle_*.py: exact integer factors, the closed-form factor of the
second-difference matrix, brute force on small matrices, LAPACK's Cholesky,
closed forms of the Matern function at half-integer smoothness, the
norm bound that the precision criterion guarantees, and hand-worked
scalar-tile factors for the low classes' update arithmetic (class_update).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build as _build

_LIB = None
_c_dbl_p = ctypes.POINTER(ctypes.c_double)


def _bind(lib):
    i64 = ctypes.c_int64
    lib.oracle_tile_cholesky.restype = i64
    lib.oracle_tile_cholesky.argtypes = [i64, i64, _c_dbl_p, i64, ctypes.c_int]
    lib.oracle_cholesky_unblocked.restype = i64
    lib.oracle_cholesky_unblocked.argtypes = [i64, _c_dbl_p, i64]
    for f in (lib.oracle_forward_solve, lib.oracle_back_solve):
        f.restype = None
        f.argtypes = [i64, _c_dbl_p, i64, _c_dbl_p, i64, i64]
    lib.oracle_mutant_id.restype = ctypes.c_int
    return lib


def load(path: str | None = None):
    """The oracle's C library (built with gcc on first use if missing)."""
    global _LIB
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _LIB = _bind(ctypes.CDLL(_build.LIB))
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_c_dbl_p)


# ---------------------------------------------------------------------------
# Factorization, solves, log-determinant
# ---------------------------------------------------------------------------

def tile_cholesky(A: np.ndarray, nb: int, threads: int = 1, lib=None):
    """Left-looking tile Cholesky of the symmetric n x n matrix A with tile
    size nb (Algorithm 1). Returns (L, info): L lower triangular with zero
    strict upper part; info = 0, or the 1-based global column of the first
    non-positive pivot (L is then partial)."""
    lib = lib or load()
    n = A.shape[0]
    a = np.array(A, dtype=np.float64, order="F", copy=True)
    info = lib.oracle_tile_cholesky(n, nb, _ptr(a), n, threads)
    if info < 0:
        raise ValueError("bad arguments: n=%d nb=%d" % (n, nb))
    return np.tril(a), int(info)


def cholesky_unblocked(A: np.ndarray, lib=None):
    """Unblocked row-by-row Cholesky (a different code path). (L, info)."""
    lib = lib or load()
    n = A.shape[0]
    a = np.array(A, dtype=np.float64, order="F", copy=True)
    info = lib.oracle_cholesky_unblocked(n, _ptr(a), n)
    return np.tril(a), int(info)


def solve(L: np.ndarray, B: np.ndarray, lib=None) -> np.ndarray:
    """X = (L L^T)^{-1} B by forward then back substitution."""
    lib = lib or load()
    Lf = np.asfortranarray(L, dtype=np.float64)
    X = np.array(B, dtype=np.float64, order="F", copy=True)
    if X.ndim == 1:
        X = X.reshape(-1, 1, order="F")
    n, nrhs = X.shape
    lib.oracle_forward_solve(n, _ptr(Lf), n, _ptr(X), n, nrhs)
    lib.oracle_back_solve(n, _ptr(Lf), n, _ptr(X), n, nrhs)
    return X.reshape(B.shape) if np.ndim(B) == 1 else X


def forward_solve(L: np.ndarray, B: np.ndarray, lib=None) -> np.ndarray:
    """Y = L^{-1} B."""
    lib = lib or load()
    Lf = np.asfortranarray(L, dtype=np.float64)
    X = np.array(B, dtype=np.float64, order="F", copy=True)
    if X.ndim == 1:
        X = X.reshape(-1, 1, order="F")
    n, nrhs = X.shape
    lib.oracle_forward_solve(n, _ptr(Lf), n, _ptr(X), n, nrhs)
    return X.reshape(B.shape) if np.ndim(B) == 1 else X


def logdet(L: np.ndarray) -> float:
    """log|A| = 2 sum_i log L_ii, summed with math.fsum (correctly rounded
    sum of the rounded logarithms)."""
    return 2.0 * math.fsum(np.log(np.diag(L)).tolist())


def backward_error(A: np.ndarray, L: np.ndarray) -> float:
    """||A - L L^T||_F / ||A||_F on the full symmetric matrix (A symmetric;
    only its lower triangle is used)."""
    As = np.tril(A) + np.tril(A, -1).T
    R = As - L @ L.T
    return float(np.linalg.norm(R) / np.linalg.norm(As))


# ---------------------------------------------------------------------------
# Matern covariance (Eq. 2) with a nugget on the diagonal
# ---------------------------------------------------------------------------

def matern(h, sigma2: float, rng: float, nu: float) -> np.ndarray:
    """C(h) = sigma2 / (2^(nu-1) Gamma(nu)) * x^nu * K_nu(x), x = h / rng,
    with its limit C(0) = sigma2."""
    from scipy.special import gamma, kv
    h = np.asarray(h, dtype=np.float64)
    x = h / rng
    out = np.full(x.shape, float(sigma2))
    pos = x > 0
    xp = x[pos]
    out[pos] = sigma2 / (2.0 ** (nu - 1.0) * gamma(nu)) * xp ** nu * kv(nu, xp)
    return out


def distances(pts: np.ndarray, I, J) -> np.ndarray:
    """Euclidean distance between points I and J (index arrays)."""
    d = pts[np.asarray(I)] - pts[np.asarray(J)]
    return np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1])


def matern_entries(pts, I, J, sigma2, rng, nu, nugget) -> np.ndarray:
    """Entries Sigma[I, J] = C(||s_I - s_J||) + nugget * [I == J]."""
    I = np.asarray(I)
    J = np.asarray(J)
    v = matern(distances(pts, I, J), sigma2, rng, nu)
    return v + nugget * (I == J)


def matern_matrix(pts, sigma2, rng, nu, nugget) -> np.ndarray:
    """Dense symmetric Sigma (n x n, Fortran order)."""
    n = len(pts)
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.asfortranarray(matern_entries(pts, I, J, sigma2, rng, nu, nugget))


# ---------------------------------------------------------------------------
# Per-tile precision criterion (Section IV-C)
# ---------------------------------------------------------------------------

# Storage classes, in the library's numbering.
FP64, FP32, FP16, BF16, FP8 = 0, 1, 2, 3, 4
# Significand bits p (including the implicit bit) of each class; the machine
# epsilon of the class is 2^(1-p), its unit roundoff 2^-p.
SIGNIFICAND_BITS = {FP64: 53, FP32: 24, FP16: 11, BF16: 8, FP8: 4}


def tile_index(Nt: int, i: int, j: int) -> int:
    """Position of lower tile (i, j), i >= j, when the lower tiles are listed
    column of tiles by column of tiles, top to bottom."""
    return j * Nt - j * (j - 1) // 2 + (i - j)


def tile_norms(A: np.ndarray, nb: int) -> np.ndarray:
    """||A_ij||_F of every lower tile (i >= j), in tile_index order."""
    n = A.shape[0]
    Nt = n // nb
    out = np.empty(Nt * (Nt + 1) // 2)
    for j in range(Nt):
        for i in range(j, Nt):
            out[tile_index(Nt, i, j)] = np.linalg.norm(A[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb])
    return out


def fro_norm(norms: np.ndarray, Nt: int) -> float:
    """||A||_F of the full symmetric matrix from the lower tiles' norms:
    diagonal tiles once, off-diagonal tiles twice."""
    s = 0.0
    for j in range(Nt):
        for i in range(j, Nt):
            v = norms[tile_index(Nt, i, j)] ** 2
            s += v if i == j else 2.0 * v
    return math.sqrt(s)


def class_eps(c: int, unit_roundoff: bool = False) -> float:
    p = SIGNIFICAND_BITS[c]
    return 2.0 ** (-p if unit_roundoff else 1 - p)


def precision_map(norms: np.ndarray, fro: float, Nt: int, eps: float,
                  allowed=(FP64, FP32, FP16, FP8), unit_roundoff: bool = False) -> np.ndarray:
    """Class of every lower tile (uint8, tile_index order). A tile takes the
    lowest allowed class p (largest eps_p) for which
        Nt * ||A_ij||_F / ||A||_F < eps / eps_p
    holds; if none does, or the tile is on the diagonal, FP64."""
    low_first = sorted((c for c in allowed if c != FP64),
                       key=lambda c: -class_eps(c, unit_roundoff))
    out = np.zeros(len(norms), dtype=np.uint8)
    for j in range(Nt):
        for i in range(j + 1, Nt):
            t = tile_index(Nt, i, j)
            lhs = Nt * norms[t] / fro
            for c in low_first:
                if lhs < eps / class_eps(c, unit_roundoff):
                    out[t] = c
                    break
    return out


# ---------------------------------------------------------------------------
# Rounding to the storage classes (Section IV-C: tiles kept in FP32, FP16 or
# FP8 instead of FP64). Round-to-nearest-even from binary64 in one step,
# saturating at the class's largest finite value. FP8 is the OCP E4M3 format
# (4 exponent bits, bias 7, 3 fraction bits, largest finite 448).
# ---------------------------------------------------------------------------

# (significand bits p, smallest normal exponent emin, largest finite value)
CLASS_FORMAT = {
    FP32: (24, -126, float(np.finfo(np.float32).max)),
    FP16: (11, -14, 65504.0),
    BF16: (8, -126, float.fromhex("0x1.fep127")),
    FP8: (4, -6, 448.0),
}


def round_to_class(x: np.ndarray, c: int) -> np.ndarray:
    """Round binary64 values to class c (RNE, saturating), returned as
    binary64. The quantum at |x| in [2^e, 2^(e+1)) is 2^(max(e, emin)-p+1),
    which also covers the subnormal range."""
    x = np.asarray(x, dtype=np.float64)
    if c == FP64:
        return x.copy()
    p, emin, vmax = CLASS_FORMAT[c]
    _, e2 = np.frexp(x)                      # x = m 2^e2, 0.5 <= |m| < 1
    e = np.maximum(e2.astype(np.int64) - 1, emin)
    q = np.ldexp(1.0, e - (p - 1))
    r = np.round(x / q) * q                  # np.round: half to even
    return np.clip(r, -vmax, vmax)


def scale_exponent(amax: float, c: int) -> int:
    """Per-tile power-of-two scale for the narrow-range classes: the tile is
    stored as x * 2^-e with e = ceil(log2(amax / largest finite)), so its
    largest entry lands in the top binade. FP32/BF16/FP64 are not scaled."""
    if c not in (FP16, FP8) or not (amax > 0.0):
        return 0
    return int(math.ceil(math.log2(amax / CLASS_FORMAT[c][2])))


def round_tile(t: np.ndarray, c: int) -> tuple[np.ndarray, int]:
    """Round one tile to class c with its per-tile scale. Returns the value
    it stands for (binary64, already multiplied back by 2^e) and e."""
    e = scale_exponent(float(np.max(np.abs(t))) if t.size else 0.0, c)
    return np.ldexp(round_to_class(np.ldexp(t, -e), c), e), e


# ---------------------------------------------------------------------------
# Mixed-precision tile Cholesky (Section IV-C), emulated on the CPU.
#
# Reading of the paper used here (the paper does not spell the arithmetic
# out): a tile's class governs how it is stored and how the updates *into*
# it are computed.
#   * diagonal tiles are FP64: SYRK in FP64 on the stored operands, POTRF in
#     FP64;
#   * an off-diagonal tile (m, k) of class p gets
#       C = A_mk - sum_{n<k} Q_p(Lh_mn) Q_p(Lh_kn)^T
#     where Q_p rounds a stored tile to class p (with its per-tile scale for
#     FP16 / FP8) and the products are accumulated in FP32 (FP64 for p =
#     FP64); then L_mk = C L_kk^{-T} in FP64 and the stored tile is
#     Lh_mk = Q_p(L_mk).
# Products of operands of class <= FP32 are exact in binary64; the FP32
# accumulation is emulated with float32 matrix products per operand tile,
# summed in float32. The GPU accumulates in a different order, so results
# agree to within the error bounds, not bitwise.
#
# Variant (fp64_update = FP32): the updates into FP64-class tiles, the
# diagonal tiles' SYRK included, are computed like those of FP32-class tiles
# (operands rounded to binary32, FP32 accumulation), so binary64 arithmetic
# remains only in POTRF, TRSM and the refinement residuals; FP64 tiles are
# still stored in binary64.
# ---------------------------------------------------------------------------

def class_update(C: np.ndarray, ops, q: int) -> np.ndarray:
    """C - sum_{(a, b) in ops} a b^T in the arithmetic of class q (the
    reading of Section IV-C above). ops: the stored operand tiles
    (Lh_mn, Lh_kn) for n = 0 .. k-1, in that order. q = FP64: binary64
    products and sums. Otherwise each stored operand is first rounded to
    the output tile's class q with its own per-tile scale (Q_q: an operand
    stored in a wider class loses its extra bits here), each tile product
    is a float32 matrix product of the rounded operands, and the products
    are summed into a float32 accumulator; the accumulated update is
    subtracted from C in binary64."""
    if q == FP64:
        for a, b in ops:
            C -= a @ b.T
        return C
    acc = np.zeros(C.shape, dtype=np.float32)
    for a, b in ops:
        ra, _ = round_tile(a, q)
        rb, _ = round_tile(b, q)
        acc += (ra.astype(np.float32) @ rb.astype(np.float32).T).astype(np.float32)
    return C - acc.astype(np.float64)


def mxp_tile_cholesky(A: np.ndarray, nb: int, cmap: np.ndarray, fp64_update: int = FP64,
                      reverse_sums: bool = False):
    """Mixed-precision left-looking tile Cholesky. Returns (Lh, info): Lh the
    stored factor as binary64 values (each tile exactly representable in
    its class with its scale), info as in tile_cholesky. fp64_update: the
    class whose arithmetic computes the updates into FP64-class tiles and
    the diagonal SYRK (FP64, or FP32 for the variant above). Every update
    goes through class_update. reverse_sums: sum each update's terms from
    n = k-1 down to 0 instead of upwards -- the reading fixes no order, so
    the two results differ only by rounding and their difference measures
    how much of a quantity is rounding-order noise."""
    from scipy.linalg import solve_triangular
    n = A.shape[0]
    Nt = n // nb
    As = np.tril(A) + np.tril(A, -1).T
    Lh = np.zeros((n, n))

    def T(M, i, j):
        return M[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]

    def ops(m, k):
        order = range(k - 1, -1, -1) if reverse_sums else range(k)
        return [(T(Lh, m, n2), T(Lh, k, n2)) for n2 in order]

    for k in range(Nt):
        C = class_update(T(As, k, k).copy(), ops(k, k), fp64_update)
        Lkk, info = tile_cholesky(C, nb)
        if info:
            return Lh, k * nb + info
        T(Lh, k, k)[:] = Lkk
        for m in range(k + 1, Nt):
            p = int(cmap[tile_index(Nt, m, k)])
            C = class_update(T(As, m, k).copy(), ops(m, k), fp64_update if p == FP64 else p)
            X = solve_triangular(Lkk, C.T, lower=True).T  # C L_kk^{-T}
            T(Lh, m, k)[:] = round_tile(X, p)[0]
    return Lh, 0


def refine(A: np.ndarray, Lh: np.ndarray, B: np.ndarray, tol: float = 1e-9, max_iter: int = 30):
    """Iterative refinement with a (possibly low-precision) factor Lh, all
    arithmetic binary64: x = (Lh Lh^T)^{-1} b, then repeat r = b - A x,
    x += (Lh Lh^T)^{-1} r until max_j ||r_j|| / ||b_j|| <= tol.
    Returns (X, iterations, relative residuals)."""
    As = np.tril(A) + np.tril(A, -1).T
    B = np.asarray(B, dtype=np.float64)
    X = solve(Lh, B)
    bn = np.linalg.norm(B, axis=0)
    it = 0
    while True:
        R = B - As @ X
        rel = np.linalg.norm(R, axis=0) / bn
        if rel.max() <= tol or it >= max_iter:
            return X, it, rel
        X = X + solve(Lh, R)
        it += 1


# ---------------------------------------------------------------------------
# Gaussian log-likelihood (Eq. 1) and its gradient with respect to
# theta = (sigma2, range, nugget) at fixed smoothness nu.
# ---------------------------------------------------------------------------

def loglik(pts, y, sigma2, rng, nu, nugget, nb=None):
    """l = -n/2 log(2 pi) - 1/2 log|Sigma| - 1/2 y^T Sigma^{-1} y, through the
    oracle's tile Cholesky."""
    n = len(pts)
    A = matern_matrix(pts, sigma2, rng, nu, nugget)
    L, info = tile_cholesky(A, nb or n, threads=8)
    if info:
        raise ValueError("not positive definite")
    z = forward_solve(L, np.asarray(y, dtype=np.float64))
    return -0.5 * n * math.log(2.0 * math.pi) - 0.5 * logdet(L) - 0.5 * float(np.sum(z * z))


def matern_dcov(pts, sigma2, rng, nu):
    """(dSigma/dsigma2, dSigma/drange) as dense matrices (dSigma/dnugget = I).
    dC/dsigma2 = C / sigma2; with x = h / a and d/dx[x^nu K_nu(x)] =
    -x^nu K_{nu-1}(x), dC/da = sigma2 / (2^(nu-1) Gamma(nu)) x^(nu+1)
    K_{nu-1}(x) / a, which is 0 at h = 0."""
    from scipy.special import gamma, kv
    n = len(pts)
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    h = distances(pts, I, J)
    C = matern(h, sigma2, rng, nu)
    x = h / rng
    dA = np.zeros_like(x)
    pos = x > 0
    xp = x[pos]
    dA[pos] = sigma2 / (2.0 ** (nu - 1.0) * gamma(nu)) * xp ** (nu + 1.0) * kv(nu - 1.0, xp) / rng
    return C / sigma2, dA


def loglik_grad(pts, y, sigma2, rng, nu, nugget, nb=None):
    """Gradient of l by the trace formula
        dl/dtheta_p = 1/2 alpha^T (dSigma/dtheta_p) alpha
                      - 1/2 tr(Sigma^{-1} dSigma/dtheta_p),
    alpha = Sigma^{-1} y, Sigma^{-1} from the oracle's factor. Returns
    (l, [dl/dsigma2, dl/drange, dl/dnugget])."""
    n = len(pts)
    A = matern_matrix(pts, sigma2, rng, nu, nugget)
    L, info = tile_cholesky(A, nb or n, threads=8)
    if info:
        raise ValueError("not positive definite")
    y = np.asarray(y, dtype=np.float64)
    z = forward_solve(L, y)
    alpha = solve(L, y)
    Sinv = solve(L, np.eye(n))
    l = -0.5 * n * math.log(2.0 * math.pi) - 0.5 * logdet(L) - 0.5 * float(np.sum(z * z))
    d_s2, d_a = matern_dcov(pts, sigma2, rng, nu)
    g = []
    for D in (d_s2, d_a, np.eye(n)):
        g.append(0.5 * float(alpha @ D @ alpha) - 0.5 * float(np.sum(Sinv * D)))
    return l, np.array(g)
