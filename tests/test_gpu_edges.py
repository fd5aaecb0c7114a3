"""Edge cases of every path on the GPU, through the C ABI, against the CPU
oracle: one and two tile columns (Nt = 1, 2), the smallest tile (nb = 128),
a tile size that is not a power of two (nb = 640, which also splits the
refinement residual into five column segments), and more right-hand sides
than one residual pass takes (17 = 16 + 1).

Tolerances are those of the main parity tests: the first-order perturbation
bound 4 kappa n u for factors and solves, the closed form of dl/dSigma for
the reverse sweep, max_j ||b_j - A x_j|| / ||b_j|| for refinement checked in
binary64 on the CPU.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def tc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_09819_amd as tc
    tc.lib()
    return tc


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.device("cuda", 0))


def matern(n, seed=7, rng=0.1, nugget=1e-4):
    pts = si.points(n, seed=seed)
    return pts, oracle.matern_matrix(pts, 1.0, rng, 0.5, nugget)


@pytest.mark.parametrize("n,nb", [(128, 128), (256, 128), (640, 640), (1280, 640)])
def test_fp64_factor_solve_small_tile_counts(tc, n, nb):
    _, A = matern(n)
    ctx = tc.Context(n, nb, nrhs=17)
    Ad = to_dev(tc.pack_lower(A, nb))
    F = tc.factorize(ctx, Ad, n, nb)
    L = tc.unpack_lower(tc.export(ctx, F).cpu().numpy(), n, nb)
    Lo, info = oracle.tile_cholesky(A, nb)
    assert info == 0
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(L - Lo) <= 4 * kappa * n * U * np.linalg.norm(Lo)
    assert abs(tc.logdet(ctx, F) - oracle.logdet(Lo)) <= 1e-12 * abs(oracle.logdet(Lo)) + 1e-10
    B = si.standard_normal((n, 17), seed=n)
    Bd = to_dev(np.ascontiguousarray(B.T))
    st = tc.solve_refine(ctx, F, Ad, Bd, max_iter=5, tol=1e-12)
    X = Bd.cpu().numpy().T
    rel = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert st["converged"] and rel.max() <= 1e-12, (st, rel.max())
    # the library's and the CPU's residuals differ by the rounding of forming
    # b - A x: at most gamma_n ||A|| ||x_j|| / ||b_j|| each
    floor = (n * U / (1 - n * U)) * np.max(np.linalg.norm(A) * np.linalg.norm(X, axis=0) /
                                          np.linalg.norm(B, axis=0))
    assert abs(st["rel_residual"] - rel.max()) <= 1e-2 * rel.max() + 2 * floor


@pytest.mark.parametrize("n,nb", [(256, 128), (640, 640)])
def test_mixed_two_tile_columns(tc, n, nb):
    """The smallest mixed-precision factor: one FP32 tile below the diagonal
    (Nt = 2), or a single diagonal tile (no low-precision tile: the FP64 path)."""
    _, A = matern(n, rng=0.02)
    Nt = n // nb
    cm = np.zeros(Nt * (Nt + 1) // 2, dtype=np.uint8)
    if Nt > 1:
        cm[1] = tc.FP32
    ctx = tc.Context(n, nb)
    Ad = to_dev(tc.pack_lower(A, nb))
    F = tc.factorize(ctx, Ad, n, nb, cmap=cm)
    L = tc.unpack_lower(tc.export(ctx, F).cpu().numpy(), n, nb)
    Lo, info = oracle.mxp_tile_cholesky(A, nb, cm)
    assert info == 0
    be_g, be_o = oracle.backward_error(A, L), oracle.backward_error(A, Lo)
    assert be_g <= 10 * be_o + 1e-15, (be_g, be_o)
    if Nt > 1:
        t = L[nb:, :nb]
        assert np.array_equal(t.astype(np.float32).astype(np.float64), t)


@pytest.mark.parametrize("n,nb,slots", [(128, 128, 2), (256, 128, 4), (384, 128, 6)])
def test_ooc_minimal_cache(tc, n, nb, slots):
    """Out of core with the smallest allowed cache (2 Nt tiles)."""
    import torch
    _, A = matern(n)
    Nt = n // nb
    assert slots == 2 * Nt
    Ah = torch.empty(tc.num_tiles(n, nb) * nb * nb, dtype=torch.float64, pin_memory=True)
    Ah.copy_(torch.from_numpy(tc.pack_lower(A, nb)))
    ctx = tc.Context(n, nb)
    cache = torch.empty(slots * nb * nb * 8, dtype=torch.uint8, device="cuda")
    st = tc.factorize_ooc(ctx, Ah, n, nb, cache)
    assert st["info"] == 0
    L = np.tril(tc.unpack_lower(Ah.numpy(), n, nb))
    Lo, _ = oracle.tile_cholesky(A, nb)
    assert np.linalg.norm(L - Lo) <= 4 * np.linalg.cond(A) * n * U * np.linalg.norm(Lo)


@pytest.mark.parametrize("n,nb", [(128, 128), (256, 128), (1280, 640)])
def test_reverse_sweep_small_tile_counts(tc, n, nb):
    import torch
    pts, A0 = matern(n, seed=9)
    y = np.linalg.cholesky(A0) @ si.standard_normal(n, seed=11)
    th = (1.2, 0.08, 2e-4)
    A = oracle.matern_matrix(pts, th[0], th[1], 0.5, th[2])
    ctx = tc.Context(n, nb)
    locs = to_dev(pts)
    Ad, _, _ = tc.matern_tiles(ctx, locs, (th[0], th[1], 0.5, th[2]), nb, norms=False)
    F = tc.factorize(ctx, Ad, n, nb, inplace=True)
    Lbar = torch.empty_like(Ad)
    tc.loglik_seed(ctx, F, to_dev(y), Lbar)
    tc.factor_adjoint(ctx, F, Lbar)
    Ab = tc.unpack_lower(Lbar.cpu().numpy(), n, nb)
    Lo, _ = oracle.tile_cholesky(A, nb)
    alpha = oracle.solve(Lo, y)
    Sinv = oracle.solve(Lo, np.eye(n))
    G = 0.5 * (np.outer(alpha, alpha) - Sinv)
    want = np.tril(2.0 * G, -1) + np.diag(np.diag(G))
    err = np.linalg.norm(Ab - want) / np.linalg.norm(want)
    assert err <= 4 * np.linalg.cond(A) * n * U, err


def test_zero_right_hand_sides(tc):
    import torch
    n, nb = 256, 128
    _, A = matern(n)
    ctx = tc.Context(n, nb)
    F = tc.factorize(ctx, to_dev(tc.pack_lower(A, nb)), n, nb)
    B = torch.empty((0, n), dtype=torch.float64, device="cuda")
    tc.solve(ctx, F, B)  # nothing to do, no error


@pytest.mark.parametrize("n,nb,upd", [(128, 128, 0), (256, 128, 0), (256, 128, 1)])
def test_ooc_mixed_all_fp64_map(tc, n, nb, upd):
    """The mixed out-of-core path with a map that has no low-precision tile
    (one and two tile columns, the minimal 2 Nt-slot cache): with binary64
    updates the factor is an all-FP64 factor, the host image holds binary64
    tiles on 256-byte boundaries followed by zero scale exponents, and the
    factor matches the oracle's like the in-core FP64 path; with FP32-class
    updates (upd = 1) it matches the oracle's emulation of that variant."""
    import torch
    _, A = matern(n)
    Nt = n // nb
    ntiles = Nt * (Nt + 1) // 2
    cm = np.zeros(ntiles, dtype=np.uint8)
    assert tc.ooc_mixed_host_bytes(n, nb, cm) == ntiles * nb * nb * 8 + (4 * ntiles + 255) // 256 * 256
    Ah = torch.empty(ntiles * nb * nb, dtype=torch.float64, pin_memory=True)
    Ah.copy_(torch.from_numpy(tc.pack_lower(A, nb)))
    ctx = tc.Context(n, nb)
    cache = torch.empty(tc.ooc_mixed_cache_bytes(n, nb, cm, 2 * Nt, fp64_update=upd),
                        dtype=torch.uint8, device="cuda")
    st, img = tc.factorize_ooc_mixed(ctx, Ah, n, nb, cm, cache, fp64_update=upd)
    assert st["info"] == 0
    raw = img.numpy()
    tiles = raw[:ntiles * nb * nb * 8].view(np.float64)
    assert np.all(raw[ntiles * nb * nb * 8:][:4 * ntiles].view(np.int32) == 0)
    L = np.tril(tc.unpack_lower(tiles, n, nb))
    assert st["bytes_d2h"] == ntiles * nb * nb * 8
    if upd == 0:
        Lo, info = oracle.tile_cholesky(A, nb)
        assert info == 0
        assert np.linalg.norm(L - Lo) <= 4 * np.linalg.cond(A) * n * U * np.linalg.norm(Lo)
    else:
        Lo, info = oracle.mxp_tile_cholesky(A, nb, cm, fp64_update=oracle.FP32)
        assert info == 0
        be_g, be_o = oracle.backward_error(A, L), oracle.backward_error(A, Lo)
        assert be_g <= 10 * be_o + 1e-15, (be_g, be_o)
