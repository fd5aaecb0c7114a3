"""Host checks of the benchmark's measurement helpers (no GPU): the tile
products behind the probe backward error, and the map-weighted roofline."""
import numpy as np
import pytest
import torch

import bench
import paper_2410_09819_amd as tc


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n))
    return X @ X.T / n + np.eye(n)


@pytest.mark.parametrize("n,nb", [(384, 128), (256, 256), (512, 128)])
def test_tile_products_match_dense(n, nb):
    A = _spd(n, 3)
    L = np.linalg.cholesky(A)
    G = np.random.default_rng(4).standard_normal((n, 5))
    Ap = torch.from_numpy(tc.pack_lower(A, nb))
    Lp = torch.from_numpy(tc.pack_lower(L, nb))
    Gt = torch.from_numpy(G)
    # A G from the lower tiles (diagonal tiles in full) and the mirrored upper part
    AG = bench._tiles_times(Ap, n, nb, Gt) + bench._tiles_t_times(Ap, n, nb, Gt, diag=False)
    np.testing.assert_allclose(AG.numpy(), A @ G, rtol=0, atol=1e-12 * np.abs(A @ G).max())
    np.testing.assert_allclose(bench._tiles_t_times(Lp, n, nb, Gt).numpy(), L.T @ G, rtol=0,
                               atol=1e-12 * np.abs(L.T @ G).max())
    np.testing.assert_allclose(bench._tiles_times(Lp, n, nb, Gt).numpy(), L @ G, rtol=0,
                               atol=1e-12 * np.abs(L @ G).max())


def test_probe_backward_error_matches_dense():
    """The probe estimate equals the dense formula with the same probes, and
    sees a planted perturbation of one factor tile at its size."""
    n, nb = 384, 128
    A = _spd(n, 5)
    L = np.linalg.cholesky(A)
    gen = torch.Generator(device="cpu").manual_seed(97)
    G = torch.randn(n, 32, generator=gen, dtype=torch.float64).numpy()
    Ap = torch.from_numpy(tc.pack_lower(A, nb))
    for delta in (0.0, 1e-9, 1e-5):
        Lq = L.copy()
        Lq[300:340, 130:170] += delta
        be = bench.probe_backward_error(Ap, torch.from_numpy(tc.pack_lower(Lq, nb)), n, nb)
        ref = np.linalg.norm((A - Lq @ Lq.T) @ G) / np.linalg.norm(A @ G)
        assert abs(be - ref) <= 1e-3 * ref + 1e-15, (delta, be, ref)
        if delta > 0:
            assert be > 0.1 * delta


def test_map_roofline_all_fp64_and_mixed():
    n = 4096
    tot = n ** 3 / 3.0
    upd = 0.9 * tot
    r = bench.map_roofline(n, [upd, 0, 0, 0, 0], 1000.0)
    assert abs(r["t_star_s"] - tot / 78.6e12) <= 1e-12 * r["t_star_s"]
    assert abs(r["frac"] - r["t_star_s"] / 1.0) <= 1e-15
    # moving update flops to FP8 shrinks t* by exactly their FP64 time less their FP8 time
    r2 = bench.map_roofline(n, [0.5 * upd, 0, 0, 0, 0.5 * upd], 1000.0)
    want = r["t_star_s"] - 0.5 * upd / 78.6e12 + 0.5 * upd / 5000e12
    assert abs(r2["t_star_s"] - want) <= 1e-12 * want
    # the FP32 class is priced at a third of the FP16 rate (three products)
    r3 = bench.map_roofline(n, [0, upd, 0, 0, 0], 1000.0)
    want3 = (tot - upd) / 78.6e12 + 3 * upd / 2500e12
    assert abs(r3["t_star_s"] - want3) <= 1e-12 * want3
