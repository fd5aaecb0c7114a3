"""Pins for the CPU oracle's Cholesky, solves and log-determinant.

Each pin ties the oracle to something other than itself: exact integer
arithmetic, a closed-form factor, an independent unblocked code path,
LAPACK's Cholesky (numpy.linalg), or the uniqueness of the factor. The
mutant test at the end builds the oracle with planted mistakes (a dropped
update term, a transposed operand, a wrong triangular index, swapped GEMM
operands) and checks that the pins catch every one.
"""
import math

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import build as obuild

U = 2.0 ** -53


def divisors(n):
    return [d for d in range(1, n + 1) if n % d == 0]


# --- exact integer factors (Section III-A: the factor is unique) -----------

@pytest.mark.parametrize("n", [16, 48, 64])
def test_exact_integer_factor_bitwise(n):
    L0 = si.integer_factor(n, seed=n)
    A = L0 @ L0.T  # small integers, exact
    for nb in divisors(n):
        L, info = oracle.tile_cholesky(A, nb)
        assert info == 0
        assert np.array_equal(L, L0), "nb=%d" % nb
    L, info = oracle.cholesky_unblocked(A)
    assert info == 0 and np.array_equal(L, L0)


def test_exact_integer_solve():
    n = 64
    L0 = si.integer_factor(n, seed=7)
    A = L0 @ L0.T
    x = np.round(si.standard_normal((n, 3), seed=8) * 4.0)
    b = A @ x  # exact small integers
    X = oracle.solve(L0, b)
    assert np.array_equal(X, x)


def test_exact_integer_forward_solve():
    """L^{-1} b, the first term of the likelihood's quadratic form (Eq. 1):
    with b = L0 x in small integers every step is exact."""
    n = 64
    L0 = si.integer_factor(n, seed=9)
    x = np.round(si.standard_normal((n, 2), seed=10) * 4.0)
    assert np.array_equal(oracle.forward_solve(L0, L0 @ x), x)
    assert np.array_equal(oracle.forward_solve(L0, L0 @ x[:, 0]), x[:, 0])


def test_forward_solve_matches_library_routine():
    """Against LAPACK's triangular solve (scipy) on a well-conditioned
    lower-triangular matrix with random entries."""
    from scipy.linalg import solve_triangular
    n = 200
    M = si.standard_normal((n, n), seed=11)
    L = np.tril(M) * 0.1 + np.diag(2.0 + np.abs(np.diag(M)))
    B = si.standard_normal((n, 5), seed=12)
    Y = oracle.forward_solve(L, B)
    ref = solve_triangular(L, B, lower=True)
    assert np.max(np.abs(Y - ref)) <= 1e-13 * np.max(np.abs(ref))


# --- closed form: second-difference matrix ---------------------------------

@pytest.mark.parametrize("nb", [1, 8, 16, 64])
def test_tridiagonal_closed_form(nb):
    n = 64
    A = si.tridiagonal(n)
    L, info = oracle.tile_cholesky(A, nb)
    assert info == 0
    j = np.arange(1, n + 1, dtype=np.float64)  # 1-based
    diag = np.sqrt((j + 1) / j)
    sub = -np.sqrt(j[:-1] / (j[:-1] + 1))
    assert np.allclose(np.diag(L), diag, rtol=8 * U * n, atol=0)
    assert np.allclose(np.diag(L, -1), sub, rtol=8 * U * n, atol=0)
    assert np.count_nonzero(np.tril(L, -2)) == 0
    assert abs(oracle.logdet(L) - math.log(n + 1)) <= 64 * U * math.log(n + 1)


# --- independent code path: unblocked Cholesky on small matrices -----------

@pytest.mark.parametrize("n", [8, 24, 64])
def test_tile_equals_unblocked(n):
    L0 = si.random_factor(n, seed=100 + n)
    A = L0 @ L0.T
    Lu, info = oracle.cholesky_unblocked(A)
    assert info == 0
    for nb in divisors(n):
        L, info = oracle.tile_cholesky(A, nb)
        assert info == 0
        err = np.linalg.norm(L - Lu) / np.linalg.norm(Lu)
        assert err <= 16 * n * U, (nb, err)
    # factor recovered: forward error within kappa * u (A = L0 L0^T)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(Lu - L0) / np.linalg.norm(L0) <= 8 * n * kappa * U


# --- LAPACK agreement on a Matern covariance matrix (small workload) ------

@pytest.mark.parametrize("n,nb", [(512, 64), (2048, 256)])
def test_matern_against_lapack(n, nb):
    w = si.WORKLOADS["small"]
    pts = si.points(n, seed=w["seed"])
    A = oracle.matern_matrix(pts, w["sigma2"], w["range"], w["nu"], w["nugget"])
    L, info = oracle.tile_cholesky(A, nb, threads=8)
    assert info == 0
    Lnp = np.linalg.cholesky(A)
    be = oracle.backward_error(A, L)
    be_np = oracle.backward_error(A, Lnp)
    assert be <= 1e-14 and be_np <= 1e-14, (be, be_np)
    # perturbation bound for the Cholesky factor: ||dL||/||L|| <~ kappa(A) u
    kappa = np.linalg.cond(A)
    diff = np.linalg.norm(L - Lnp) / np.linalg.norm(Lnp)
    assert diff <= 4 * kappa * n * U, (diff, kappa)
    assert abs(oracle.logdet(L) - np.linalg.slogdet(A)[1]) <= 1e-10 * n


def test_threads_do_not_change_result():
    n, nb = 512, 64
    L0 = si.random_factor(n, seed=5)
    A = L0 @ L0.T
    L1, _ = oracle.tile_cholesky(A, nb, threads=1)
    L4, _ = oracle.tile_cholesky(A, nb, threads=4)
    assert np.array_equal(L1, L4)


# --- failure reporting (LAPACK convention) ---------------------------------

@pytest.mark.parametrize("bad", [0, 5, 37, 63])
def test_not_spd_reports_column(bad):
    n, nb = 64, 16
    A = np.eye(n) * 4.0
    A[bad, bad] = -1.0
    for f in (lambda M: oracle.tile_cholesky(M, nb), oracle.cholesky_unblocked):
        _, info = f(A)
        assert info == bad + 1


def test_nan_reports_column():
    n, nb = 32, 8
    A = np.eye(n)
    A[20, 20] = np.nan
    _, info = oracle.tile_cholesky(A, nb)
    assert info == 21


def test_bad_arguments():
    with pytest.raises(ValueError):
        oracle.tile_cholesky(np.eye(10), 3)


# --- log-determinant pins ---------------------------------------------------

def test_logdet_of_known_factor():
    n = 64
    L0 = si.integer_factor(n, seed=3)
    L, _ = oracle.tile_cholesky(L0 @ L0.T, 16)
    assert oracle.logdet(L) == 2.0 * math.fsum(np.log(np.diag(L0)).tolist())


def test_logdet_uncorrelated_limit():
    # range -> 0: every off-diagonal covariance underflows, Sigma = (s2+t2) I
    n = 128
    pts = si.points(n, seed=1)
    A = oracle.matern_matrix(pts, 1.3, 1e-9, 0.5, 0.2)
    assert np.count_nonzero(A - np.diag(np.diag(A))) == 0
    L, _ = oracle.tile_cholesky(A, 32)
    assert abs(oracle.logdet(L) - n * math.log(1.5)) <= 1e-12 * n


# --- mutants: each planted mistake must fail at least one pin --------------

def _pins_pass(lib):
    try:
        n = 48
        L0 = si.integer_factor(n, seed=n)
        A = L0 @ L0.T
        for nb in (4, 8, 16):
            L, info = oracle.tile_cholesky(A, nb, lib=lib)
            if info or not np.array_equal(L, L0):
                return False
        A = si.tridiagonal(32)
        L, info = oracle.tile_cholesky(A, 8, lib=lib)
        j = np.arange(1, 33.0)
        if info or not np.allclose(np.diag(L), np.sqrt((j + 1) / j), rtol=1e-13):
            return False
        L0 = si.random_factor(24, seed=124)
        A = L0 @ L0.T
        Lu, _ = oracle.cholesky_unblocked(A)
        for nb in (4, 6, 8):
            L, info = oracle.tile_cholesky(A, nb, lib=lib)
            if info or np.linalg.norm(L - Lu) > 1e-12 * np.linalg.norm(Lu):
                return False
        return True
    except Exception:
        return False


def test_pins_pass_on_real_oracle():
    assert oracle.load().oracle_mutant_id() == 0
    assert _pins_pass(oracle.load())


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5])
def test_pins_catch_planted_mistake(mutant, tmp_path):
    path = obuild.build(out=str(tmp_path / ("liboracle_m%d.so" % mutant)), mutant=mutant)
    lib = oracle.load(path)
    assert lib.oracle_mutant_id() == mutant
    assert not _pins_pass(lib)
