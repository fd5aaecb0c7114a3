"""Pins for the oracle's Matern covariance (Eq. 2) and nugget.

The oracle evaluates Eq. 2 through scipy's K_nu for every smoothness. At
half-integer smoothness the Matern function has textbook closed forms
(exponential for nu = 1/2, (1+x)e^-x for 3/2, (1+x+x^2/3)e^-x for 5/2), and
its limit at h = 0 is sigma^2; those pin the normalising constant, the power
of x and the argument scaling h/a.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

CLOSED = {
    0.5: lambda x: np.exp(-x),
    1.5: lambda x: (1.0 + x) * np.exp(-x),
    2.5: lambda x: (1.0 + x + x * x / 3.0) * np.exp(-x),
}


@pytest.mark.parametrize("nu", sorted(CLOSED))
def test_half_integer_closed_forms(nu):
    a, s2 = 0.07, 1.7
    x = np.concatenate([np.geomspace(1e-8, 690.0, 4000), [1.0, 2.0, 10.0]])
    got = oracle.matern(x * a, s2, a, nu)
    want = s2 * CLOSED[nu](x)
    assert np.all(np.abs(got - want) <= 1e-13 * np.abs(want))


def test_nu_one_small_argument_limit():
    # x K_1(x) -> 1 as x -> 0, so C -> sigma^2 (nu = 1: 2^0 Gamma(1) = 1)
    got = oracle.matern(np.array([1e-12, 1e-9]), 2.0, 1.0, 1.0)
    assert np.allclose(got, 2.0, rtol=1e-12)


def test_zero_distance_is_variance():
    assert oracle.matern(np.array([0.0]), 1.3, 0.1, 1.0)[0] == 1.3


def test_matrix_symmetric_spd_and_nugget():
    pts = si.points(256, seed=9)
    A = oracle.matern_matrix(pts, 1.0, 0.1, 1.5, 1e-3)
    assert np.array_equal(A, A.T)
    assert np.all(np.diag(A) == 1.0 + 1e-3)
    assert np.linalg.eigvalsh(A).min() > 0
    A0 = oracle.matern_matrix(pts, 1.0, 0.1, 1.5, 0.0)
    assert np.array_equal(A, A0 + 1e-3 * np.eye(256))


def test_entries_match_matrix():
    pts = si.points(100, seed=2)
    A = oracle.matern_matrix(pts, 1.0, 0.05, 0.5, 1e-4)
    I = np.array([0, 5, 99, 42])
    J = np.array([0, 7, 3, 42])
    assert np.array_equal(oracle.matern_entries(pts, I, J, 1.0, 0.05, 0.5, 1e-4), A[I, J])


def test_morton_order_makes_neighbours_close():
    pts = si.points(4096, seed=1, sort=True)
    raw = si.points(4096, seed=1, sort=False)
    step = np.linalg.norm(np.diff(pts, axis=0), axis=1).mean()
    step_raw = np.linalg.norm(np.diff(raw, axis=0), axis=1).mean()
    assert step < step_raw / 10
    assert sorted(map(tuple, pts)) == sorted(map(tuple, raw))


def test_translated_points_distinct():
    p = si.translated_points(10000, 4000, seed=4)
    assert len(np.unique(p, axis=0)) == 10000
    assert np.allclose(p[4000:8000] - [1.0, 0.0], p[:4000], rtol=0, atol=1e-15)
