"""Pins for the oracle's mixed-precision tile Cholesky emulation (Section
IV-C) and its refinement solve.

* With every tile in FP64 the emulation is the FP64 tile Cholesky.
* Every stored tile is exactly representable in its class (with its
  per-tile scale).
* The criterion targets accuracy eps: the factor's backward error stays
  below eps, and falls as eps tightens.
* Refinement with an FP64 factor converges at once; with the mixed factor
  it reaches 1e-9 relative residual and the solution of A x = b.
* The low classes' update arithmetic: two hand-worked scalar-tile factors
  pin that operands are rounded to the output tile's class and that the
  products are summed in FP32; two planted mistakes (binary64 sums,
  operands in their own stored class) each fail one of them.
"""
import math

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
        for rev in (False, True):  # either summation order is exact here
            Lh, info = oracle.mxp_tile_cholesky(A, nb, cm, fp64_update=FP32, reverse_sums=rev)
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


# --- the low classes' update arithmetic (Section IV-C) ----------------------
#
# Two scalar-tile (nb = 1) factors built so that the reading of Section IV-C
# (operands rounded to the *output* tile's class, products summed in FP32)
# gives a different stored factor than either plausible alternative
# (operands kept in their own stored class; sums in binary64). Expected
# values are worked out by hand below with numpy's own float32 / float16
# casts, not with the oracle's rounding helpers.

def _accumulation_case():
    """Nt = 4, nb = 1. L has L20 = L30 = 2^12, L21 = L31 = 1, L32 = 1/2 and a
    diagonal (1, 1, 1, 2) (L10 = 0; L33 = 2 leaves room for the FP32 error
    in L32). The update into tile (3, 2) sums the products
    L30 L20 = 2^24 and L31 L21 = 1: binary64 keeps 2^24 + 1, binary32 rounds
    the sum to 2^24 (a tie, to even)."""
    L = np.eye(4)
    L[2, 0] = L[3, 0] = 2.0 ** 12
    L[2, 1] = L[3, 1] = 1.0
    L[3, 2] = 0.5
    L[3, 3] = 2.0
    A = L @ L.T  # every entry below 2^53: exact
    cm = np.full(10, FP32, dtype=np.uint8)
    for k in range(4):
        cm[oracle.tile_index(4, k, k)] = FP64
    return A, cm


def _operand_class_case():
    """Nt = 3, nb = 1. Tiles (1, 0) and (2, 0) are FP32-class and hold
    1 + 2^-12 (exact in binary32, not in binary16); tile (2, 1) is FP16-class.
    Its update multiplies the two operands after rounding them to FP16 (to
    1.0 each), not in their stored binary32 form."""
    v = 1.0 + 2.0 ** -12
    L = np.eye(3)
    L[1, 0] = L[2, 0] = v
    L[2, 1] = 0.5
    A = L @ L.T  # entries need at most 26 significant bits: exact
    cm = np.array([FP64, FP32, FP32, FP64, FP16, FP64], dtype=np.uint8)
    assert [oracle.tile_index(3, i, j) for (i, j) in ((1, 0), (2, 0), (2, 1))] == [1, 2, 4]
    return A, cm


def pin_fp32_accumulation():
    A, cm = _accumulation_case()
    Lh, info = oracle.mxp_tile_cholesky(A, 1, cm)
    assert info == 0
    # C = A32 - fl32(fl32(2^24) + fl32(1)) in FP32 arithmetic
    acc = np.float32(np.float32(2.0 ** 12) * np.float32(2.0 ** 12)) + np.float32(1.0)
    assert float(acc) == 2.0 ** 24  # the binary32 sum drops the 1
    c = A[3, 2] - float(acc)
    expected = float(np.float32(c / 1.0))  # L22 = 1, stored in binary32
    assert expected == 1.5
    assert Lh[3, 2] == expected, Lh[3, 2]
    # the diagonal tiles' SYRK is binary64 (FP64 class), with the stored
    # L32: L22 = 1 and L33 = sqrt(A33 - 2^24 - 1 - 1.5^2) = sqrt(2)
    assert Lh[2, 2] == 1.0 and Lh[3, 3] == math.sqrt(2.0)


def pin_output_class_operands():
    A, cm = _operand_class_case()
    Lh, info = oracle.mxp_tile_cholesky(A, 1, cm)
    assert info == 0
    v = 1.0 + 2.0 ** -12
    assert Lh[1, 0] == v and Lh[2, 0] == v  # FP32 tiles keep the 2^-12 bit
    q = np.float16(v)  # the operand in the output tile's class
    assert float(q) == 1.0
    prod = float(np.float32(q) * np.float32(q))
    c = A[2, 1] - prod  # = 1/2 + 2^-11 + 2^-24
    expected = float(np.float16(c / Lh[1, 1]))
    assert expected == 0.5 + 2.0 ** -11
    assert Lh[2, 1] == expected, Lh[2, 1]


def test_low_class_update_accumulates_in_fp32():
    pin_fp32_accumulation()


def test_low_class_update_rounds_operands_to_output_class():
    pin_output_class_operands()


def _mutant_float64_accumulation(C, ops, q):
    """Planted mistake: the low classes' products summed in binary64."""
    if q == FP64:
        for a, b in ops:
            C -= a @ b.T
        return C
    acc = np.zeros(C.shape)
    for a, b in ops:
        acc += oracle.round_tile(a, q)[0] @ oracle.round_tile(b, q)[0].T
    return C - acc


def _mutant_own_class_operands(C, ops, q):
    """Planted mistake: each operand used in its own stored class (no
    rounding to the output tile's class), FP32 accumulation kept."""
    if q == FP64:
        for a, b in ops:
            C -= a @ b.T
        return C
    acc = np.zeros(C.shape, dtype=np.float32)
    for a, b in ops:
        acc += (a.astype(np.float32) @ b.astype(np.float32).T).astype(np.float32)
    return C - acc.astype(np.float64)


@pytest.mark.parametrize("mutant", [_mutant_float64_accumulation, _mutant_own_class_operands])
def test_pins_catch_planted_update_mistakes(monkeypatch, mutant):
    """Each planted mistake in the low classes' update arithmetic fails at
    least one of the two pins above (and the unmutated oracle passes both,
    see the tests above)."""
    monkeypatch.setattr(oracle, "class_update", mutant)
    failed = 0
    for pin in (pin_fp32_accumulation, pin_output_class_operands):
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed >= 1, mutant.__name__
