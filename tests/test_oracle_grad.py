"""Pins for the oracle's Gaussian log-likelihood (Eq. 1) and its gradient
with respect to (sigma2, range, nugget).

* Central finite differences of the log-likelihood, evaluated away from the
  data-generating parameters (where the score is not zero on average).
* The closed form in the uncorrelated limit (range -> 0): Sigma = s I with
  s = sigma2 + nugget, dl/dsigma2 = dl/dnugget = -n/(2s) + y^T y/(2 s^2).
* The nugget identity dl/dnugget = 1/2 alpha^T alpha - 1/2 tr(Sigma^{-1}).
* The log-likelihood against scipy's multivariate normal.
* The range derivative of the Matern function at nu = 1/2 against its
  closed form sigma2 x e^{-x} / a.
"""
import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal

import oracle
import seeded_inputs as si


def data(n=96, seed=4, theta0=(1.0, 0.1, 1e-4), nu=0.5):
    pts = si.translated_points(n, 40, seed=seed)
    A = oracle.matern_matrix(pts, theta0[0], theta0[1], nu, theta0[2])
    y = np.linalg.cholesky(A) @ si.standard_normal(n, seed=si.rhs_seed(seed))
    return pts, y


def test_loglik_matches_scipy():
    pts, y = data()
    l = oracle.loglik(pts, y, 1.2, 0.08, 0.5, 2e-4)
    A = oracle.matern_matrix(pts, 1.2, 0.08, 0.5, 2e-4)
    assert abs(l - multivariate_normal(mean=np.zeros(len(y)), cov=A).logpdf(y)) <= 1e-9 * abs(l)


@pytest.mark.parametrize("nu", [0.5, 1.5, 1.0])
def test_gradient_against_central_differences(nu):
    pts, y = data(nu=nu)
    th = np.array([1.2, 0.08, 2e-4])
    _, g = oracle.loglik_grad(pts, y, th[0], th[1], nu, th[2])
    for p in range(3):
        h = 1e-6 * max(th[p], 1e-3) if p < 2 else 1e-7
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (oracle.loglik(pts, y, tp[0], tp[1], nu, tp[2]) -
              oracle.loglik(pts, y, tm[0], tm[1], nu, tm[2])) / (2 * h)
        assert abs(fd - g[p]) <= 1e-4 * abs(g[p]) + 1e-6, (p, fd, g[p])


def test_uncorrelated_limit_closed_form():
    pts, y = data()
    s2, tau2 = 1.3, 0.2
    _, g = oracle.loglik_grad(pts, y, s2, 1e-9, 0.5, tau2)
    s = s2 + tau2
    want = -len(y) / (2 * s) + float(y @ y) / (2 * s * s)
    assert abs(g[0] - want) <= 1e-12 * abs(want) and abs(g[2] - want) <= 1e-12 * abs(want)
    assert g[1] == 0.0


def test_nugget_identity():
    pts, y = data()
    _, g = oracle.loglik_grad(pts, y, 1.2, 0.08, 0.5, 2e-4)
    A = oracle.matern_matrix(pts, 1.2, 0.08, 0.5, 2e-4)
    alpha = np.linalg.solve(A, y)
    want = 0.5 * alpha @ alpha - 0.5 * np.trace(np.linalg.inv(A))
    assert abs(g[2] - want) <= 1e-9 * abs(want)


def test_range_derivative_closed_form():
    pts = si.points(50, seed=2)
    s2, a = 1.7, 0.07
    _, dA = oracle.matern_dcov(pts, s2, a, 0.5)
    I, J = np.meshgrid(np.arange(50), np.arange(50), indexing="ij")
    x = oracle.distances(pts, I, J) / a
    assert np.allclose(dA, s2 * x * np.exp(-x) / a, rtol=1e-12, atol=0)
