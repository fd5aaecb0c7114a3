"""Pins for the oracle's mixed-precision tile Cholesky emulation (Section
IV-C) and its refinement solve.

* With every tile in FP64 the emulation is the FP64 tile Cholesky.
* Every stored tile is exactly representable in its class (with its
  per-tile scale).
* The criterion targets accuracy eps: the factor's backward error stays
  below eps, and falls as eps tightens.
* Refinement with an FP64 factor converges at once; with the mixed factor
  it reaches 1e-9 relative residual and the solution of A x = b.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import FP8, FP16, FP32, FP64


@pytest.fixture(scope="module")
def mat():
    n, nb = 1024, 128
    pts = si.points(n, seed=3)
    A = oracle.matern_matrix(pts, 1.0, 0.03, 0.5, 1e-4)
    Nt = n // nb
    norms = oracle.tile_norms(A, nb)
    return A, nb, Nt, norms, oracle.fro_norm(norms, Nt)


def test_all_fp64_map_is_fp64_cholesky(mat):
    A, nb, Nt, _, _ = mat
    cm = np.zeros(Nt * (Nt + 1) // 2, dtype=np.uint8)
    Lh, info = oracle.mxp_tile_cholesky(A, nb, cm)
    L, _ = oracle.tile_cholesky(A, nb)
    assert info == 0
    assert np.linalg.norm(Lh - L) <= 1e-13 * np.linalg.norm(L)


@pytest.mark.parametrize("eps", [1e-5, 1e-9])
def test_mixed_factor_tiles_representable_and_accurate(mat, eps):
    A, nb, Nt, norms, fro = mat
    cm = oracle.precision_map(norms, fro, Nt, eps)
    assert len(set(cm.tolist())) >= 3
    Lh, info = oracle.mxp_tile_cholesky(A, nb, cm)
    assert info == 0
    for j in range(Nt):
        for i in range(j + 1, Nt):
            t = Lh[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
            c = int(cm[oracle.tile_index(Nt, i, j)])
            assert np.array_equal(oracle.round_tile(t, c)[0], t)
    be = oracle.backward_error(A, Lh)
    assert be <= eps, be


def test_error_falls_with_target(mat):
    A, nb, Nt, norms, fro = mat
    bes = []
    for eps in (1e-4, 1e-6, 1e-8):
        Lh, _ = oracle.mxp_tile_cholesky(A, nb, oracle.precision_map(norms, fro, Nt, eps))
        bes.append(oracle.backward_error(A, Lh))
    assert bes[0] > bes[1] > bes[2]


def test_all_fp32_offdiagonal_error_scale(mat):
    A, nb, Nt, _, _ = mat
    cm = np.full(Nt * (Nt + 1) // 2, FP32, dtype=np.uint8)
    for k in range(Nt):
        cm[oracle.tile_index(Nt, k, k)] = FP64
    Lh, _ = oracle.mxp_tile_cholesky(A, nb, cm)
    be = oracle.backward_error(A, Lh)
    assert 1e-10 < be < 64 * 2.0 ** -24, be


def test_refinement(mat):
    A, nb, Nt, norms, fro = mat
    n = A.shape[0]
    B = si.standard_normal((n, 4), seed=31)
    L, _ = oracle.tile_cholesky(A, nb)
    X, it, rel = oracle.refine(A, L, B)
    assert it == 0 and rel.max() <= 1e-12
    Lh, _ = oracle.mxp_tile_cholesky(A, nb, oracle.precision_map(norms, fro, Nt, 1e-5))
    X, it, rel = oracle.refine(A, Lh, B, tol=1e-9)
    assert rel.max() <= 1e-9 and 1 <= it <= 10
    Xnp = np.linalg.solve(A, B)
    assert np.linalg.norm(X - Xnp) <= 1e-6 * np.linalg.norm(Xnp)


def test_fp32_update_exact_on_integer_factor():
    """A = L0 L0^T with small integers: every partial sum stays below 2^24,
    so updates in binary32 arithmetic are exact and the FP32-update variant
    must return L0 bit for bit (a dropped or transposed term, a wrong sign
    or tile index would not), for FP64 and FP32 storage alike."""
    n, nb = 48, 16
    Nt = n // nb
    rng = np.random.default_rng(7)
    L0 = np.tril(rng.integers(-2, 3, size=(n, n)).astype(np.float64), -1)
    L0 += np.diag(rng.integers(1, 4, size=n).astype(np.float64))
    A = L0 @ L0.T
    assert np.abs(A).max() < 2 ** 24
    for cm in (np.zeros(Nt * (Nt + 1) // 2, dtype=np.uint8),
               np.array([FP32 if i != j else FP64 for j in range(Nt) for i in range(j, Nt)],
                        dtype=np.uint8)):
        Lh, info = oracle.mxp_tile_cholesky(A, nb, cm, fp64_update=FP32)
        assert info == 0
        assert np.array_equal(Lh, L0)


def test_fp32_update_rounds_like_fp32(mat):
    """With an all-FP64 map the variant still computes every update in
    binary32 arithmetic: its backward error is at the FP32 level, far above
    the FP64 factorization's, and the FP64 variant stays exact-FP64."""
    A, nb, Nt, _, _ = mat
    cm = np.zeros(Nt * (Nt + 1) // 2, dtype=np.uint8)
    L64, _ = oracle.mxp_tile_cholesky(A, nb, cm)
    L32, info = oracle.mxp_tile_cholesky(A, nb, cm, fp64_update=FP32)
    assert info == 0
    be64, be32 = oracle.backward_error(A, L64), oracle.backward_error(A, L32)
    assert be64 < 1e-14
    assert 1e-10 < be32 < 64 * 2.0 ** -24, be32


def test_fp32_update_refines_to_target(mat):
    A, nb, Nt, norms, fro = mat
    n = A.shape[0]
    B = si.standard_normal((n, 4), seed=31)
    cm = oracle.precision_map(norms, fro, Nt, 1e-9)
    Lh, info = oracle.mxp_tile_cholesky(A, nb, cm, fp64_update=FP32)
    assert info == 0
    X, it, rel = oracle.refine(A, Lh, B, tol=1e-9)
    assert rel.max() <= 1e-9 and 1 <= it <= 10
