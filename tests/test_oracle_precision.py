"""Pins for the oracle's per-tile precision criterion (Section IV-C) and its
rounding to the storage classes.

The criterion exists to bound the error of storing A tile by tile in lower
precision: if every tile stored in class p satisfies
Nt ||A_ij|| / ||A|| < eps / eps_p, then ||A - A_hat||_F <= eps ||A||_F (each
tile contributes at most eps_p ||A_ij|| < eps ||A|| / Nt, and there are at
most Nt^2 tiles). That bound is checked on real rounding. The rounding itself
is pinned against numpy's and torch's own binary16 / binary32 / bfloat16 /
float8_e4m3fn conversions.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si
from oracle import FP8, FP16, FP32, FP64, BF16


@pytest.mark.parametrize("c,dt", [(FP64, torch.float64), (FP32, torch.float32), (FP16, torch.float16),
                                  (BF16, torch.bfloat16), (FP8, torch.float8_e4m3fn)])
def test_class_eps_matches_format(c, dt):
    """eps_p of the criterion: the format's machine epsilon (spacing above
    1), or half of it as the unit roundoff, from torch's own description of
    each format."""
    assert oracle.class_eps(c) == torch.finfo(dt).eps
    assert oracle.class_eps(c, unit_roundoff=True) == torch.finfo(dt).eps / 2


def test_tile_index_is_packed_column_order():
    Nt = 7
    idx = [oracle.tile_index(Nt, i, j) for j in range(Nt) for i in range(j, Nt)]
    assert idx == list(range(Nt * (Nt + 1) // 2))


def test_fro_norm_counts_offdiagonal_twice():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((64, 64))
    A = M + M.T
    norms = oracle.tile_norms(A, 16)
    assert abs(oracle.fro_norm(norms, 4) - np.linalg.norm(A)) <= 1e-13 * np.linalg.norm(A)


@pytest.mark.parametrize("c,dt", [(FP32, np.float32), (FP16, np.float16)])
def test_rounding_matches_numpy(c, dt):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(200000) * np.exp(rng.uniform(-30, 10, 200000))
    vmax = float(np.finfo(dt).max)
    x = x[np.abs(x) < vmax]
    assert np.array_equal(oracle.round_to_class(x, c), x.astype(dt).astype(np.float64))


@pytest.mark.parametrize("c,dt", [(BF16, torch.bfloat16), (FP8, torch.float8_e4m3fn)])
def test_rounding_matches_torch(c, dt):
    # inputs exactly representable in binary32, so torch's float->narrow
    # conversion is a single rounding
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-14, 6, 200000))).astype(np.float32)
    x = x.astype(np.float64)
    if c == FP8:
        x = x[np.abs(x) <= 448.0]
    want = torch.from_numpy(x.astype(np.float32)).to(dt).to(torch.float64).numpy()
    assert np.array_equal(oracle.round_to_class(x, c), want)


def test_fp8_saturates_and_keeps_subnormals():
    r = oracle.round_to_class(np.array([1e6, -500.0, 2.0 ** -9, 2.0 ** -10 * 1.5, 2.0 ** -11]), FP8)
    assert list(r) == [448.0, -448.0, 2.0 ** -9, 2.0 ** -9, 0.0]


def test_scale_puts_amax_in_top_binade():
    for amax in (1e-12, 3e-7, 0.5, 447.0, 449.0, 1e5):
        e = oracle.scale_exponent(amax, FP8)
        assert 224.0 < amax * 2.0 ** -e <= 448.0
        e = oracle.scale_exponent(amax, FP16)
        assert 32752.0 < amax * 2.0 ** -e <= 65504.0
    assert oracle.scale_exponent(1e-30, FP32) == 0


def _matern(n, rng_, seed=3):
    pts = si.points(n, seed=seed)
    return oracle.matern_matrix(pts, 1.0, rng_, 0.5, 1e-4)


@pytest.mark.parametrize("eps", [1e-3, 1e-5, 1e-7, 1e-9])
def test_map_norm_bound(eps):
    n, nb = 2048, 64
    Nt = n // nb
    A = _matern(n, 0.03)
    norms = oracle.tile_norms(A, nb)
    fro = oracle.fro_norm(norms, Nt)
    cmap = oracle.precision_map(norms, fro, Nt, eps)
    err2 = 0.0
    for j in range(Nt):
        for i in range(j, Nt):
            c = int(cmap[oracle.tile_index(Nt, i, j)])
            if i == j:
                assert c == FP64
            t = A[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
            r, _ = oracle.round_tile(t, c)
            d = np.linalg.norm(t - r) ** 2
            err2 += d if i == j else 2 * d
    assert math.sqrt(err2) <= 1.05 * eps * fro
    if eps <= 1e-5:
        assert len(set(cmap.tolist())) >= 3  # the map really mixes classes


def test_map_extremes_and_monotone():
    n, nb = 1024, 64
    Nt = n // nb
    A = _matern(n, 0.03)
    norms = oracle.tile_norms(A, nb)
    fro = oracle.fro_norm(norms, Nt)
    diag = np.array([i == j for j in range(Nt) for i in range(j, Nt)])
    m_hi = oracle.precision_map(norms, fro, Nt, 10.0)
    assert np.all(m_hi[~diag] == FP8) and np.all(m_hi[diag] == FP64)
    m_lo = oracle.precision_map(norms, fro, Nt, 1e-30)
    assert np.all(m_lo == FP64)
    # precision needed (smaller eps_p) never decreases as eps tightens
    order = {FP8: 0, BF16: 1, FP16: 2, FP32: 3, FP64: 4}
    prev = None
    for eps in (1e-3, 1e-5, 1e-7, 1e-9, 1e-11):
        m = np.array([order[c] for c in oracle.precision_map(norms, fro, Nt, eps)])
        if prev is not None:
            assert np.all(m >= prev)
        prev = m


def test_map_threshold_is_strict_and_mask_respected():
    Nt = 4
    norms = np.ones(10)
    fro = 1.0
    eps = 4.0 * 2.0 ** -23  # Nt*1/1 == eps/eps_fp32 exactly -> not below
    m = oracle.precision_map(norms, fro, Nt, eps, allowed=(FP64, FP32))
    assert np.all(m == FP64)
    m = oracle.precision_map(norms, fro, Nt, eps * 1.0000001, allowed=(FP64, FP32))
    assert sorted(set(m.tolist())) == [FP64, FP32]
    m = oracle.precision_map(norms, fro, Nt, 1.0, allowed=(FP64, FP16))
    assert set(m.tolist()) == {FP64, FP16}


def test_unsorted_points_give_no_low_precision():
    # without a spatial ordering every off-diagonal tile has about the same
    # norm, so at a tight target the map stays FP64
    n, nb = 2048, 128
    Nt = n // nb
    pts = si.points(n, seed=3, sort=False)
    A = oracle.matern_matrix(pts, 1.0, 0.03, 0.5, 1e-4)
    norms = oracle.tile_norms(A, nb)
    m = oracle.precision_map(norms, oracle.fro_norm(norms, Nt), Nt, 1e-9)
    assert np.all(m == FP64)
