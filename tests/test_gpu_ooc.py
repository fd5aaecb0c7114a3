"""GPU parity of the out-of-core factorization (Sections III-C, IV-B): the
matrix and factor in pinned host memory, a device tile cache of a given
size. Checked against the CPU oracle (same perturbation bound as the
in-core FP64 path) and for its transfer volume:
  * with a cache that holds every column's working set, each tile crosses
    the link exactly once in each direction (A in, L out);
  * with a cache of 2*Nt tiles the update is chunked, tiles are evicted by
    the static next use and reloaded from the host copy of L, and the factor
    is unchanged up to rounding.
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


@pytest.fixture(scope="module")
def case():
    n, nb = 2048, 128
    w = si.WORKLOADS["small"]
    pts = si.points(n, seed=w["seed"])
    A = oracle.matern_matrix(pts, w["sigma2"], w["range"], w["nu"], w["nugget"])
    Lo, info = oracle.tile_cholesky(A, nb, threads=8)
    assert info == 0
    return dict(n=n, nb=nb, A=A, Lo=Lo, kappa=np.linalg.cond(A))


def pinned(x):
    import torch
    t = torch.empty(x.size, dtype=torch.float64, pin_memory=True)
    t.copy_(torch.from_numpy(x))
    return t


@pytest.mark.parametrize("slots,inplace", [(400, False), (32, False), (40, True)])
def test_ooc_matches_oracle(tc, case, slots, inplace):
    import torch
    n, nb, A, Lo = case["n"], case["nb"], case["A"], case["Lo"]
    Nt = n // nb
    ntiles = Nt * (Nt + 1) // 2
    tbytes = nb * nb * 8
    Ah = pinned(tc.pack_lower(A, nb))
    Lh = Ah if inplace else pinned(np.zeros(ntiles * nb * nb))
    ctx = tc.Context(n, nb)
    cache = torch.empty(slots * tbytes, dtype=torch.uint8, device="cuda")
    st = tc.factorize_ooc(ctx, Ah, n, nb, cache, L_host=Lh)
    assert st["info"] == 0 and st["cache_slots"] == slots
    L = np.tril(tc.unpack_lower(Lh.numpy(), n, nb))
    assert np.linalg.norm(L - Lo) <= 4 * case["kappa"] * n * U * np.linalg.norm(Lo)
    assert oracle.backward_error(A, L) <= 1e-14
    assert st["bytes_d2h"] == ntiles * tbytes
    if slots >= Nt * Nt // 4 + Nt:
        assert st["bytes_h2d"] == ntiles * tbytes and st["tiles_reloaded"] == 0
        assert st["chunks"] == Nt - 1
    else:
        assert st["evictions"] > 0 and st["tiles_reloaded"] > 0
        assert st["bytes_h2d"] == (ntiles + st["tiles_reloaded"]) * tbytes


def test_ooc_matches_in_core(tc, case):
    import torch
    n, nb, A = case["n"], case["nb"], case["A"]
    ctx = tc.Context(n, nb)
    Ad = torch.from_numpy(tc.pack_lower(A, nb)).cuda()
    Lin = tc.unpack_lower(tc.export(ctx, tc.factorize(ctx, Ad, n, nb)).cpu().numpy(), n, nb)
    Ah = pinned(tc.pack_lower(A, nb))
    cache = torch.empty(400 * nb * nb * 8, dtype=torch.uint8, device="cuda")
    tc.factorize_ooc(ctx, Ah, n, nb, cache)
    L = np.tril(tc.unpack_lower(Ah.numpy(), n, nb))
    assert np.linalg.norm(L - Lin) <= 4 * case["kappa"] * n * U * np.linalg.norm(Lin)


def test_ooc_errors(tc, case):
    import torch
    n, nb = case["n"], case["nb"]
    ctx = tc.Context(n, nb)
    Ah = pinned(np.eye(n)[:1].ravel()[:1].repeat(tc.num_tiles(n, nb) * nb * nb))
    small = torch.empty(10 * nb * nb * 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(tc.TileCholError) as e:
        tc.factorize_ooc(ctx, Ah, n, nb, small)
    assert e.value.status == tc.TC_ENOMEM
    bad = np.eye(n) * 3.0
    bad[700, 700] = -1.0
    Bh = pinned(tc.pack_lower(bad, nb))
    cache = torch.empty(64 * nb * nb * 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(tc.NotPositiveDefinite) as e:
        tc.factorize_ooc(ctx, Bh, n, nb, cache)
    assert e.value.info == 701


@pytest.mark.parametrize("sync,no_reuse,no_v3", [(True, False, False), (False, True, False),
                                                  (True, True, False), (False, False, True),
                                                  (True, False, True)])
def test_ooc_strategy_variants(tc, case, sync, no_reuse, no_v3):
    """The reduced strategies (copies on the compute stream; no operand
    reuse across columns; no diagonal tile kept through the TRSMs) compute
    every entry with the same kernels in the same order, so the factor is
    bitwise the default's; without reuse every column reloads its operand
    tiles, and without V3 every TRSM reloads the diagonal factor (written
    back once, right after POTRF)."""
    import torch
    n, nb, A = case["n"], case["nb"], case["A"]
    Nt = n // nb
    ntiles = Nt * (Nt + 1) // 2
    tbytes = nb * nb * 8
    cache = torch.empty(400 * tbytes, dtype=torch.uint8, device="cuda")
    Ah = pinned(tc.pack_lower(A, nb))
    st0 = tc.factorize_ooc(tc.Context(n, nb), Ah, n, nb, cache)
    L0 = Ah.numpy().copy()
    Ah = pinned(tc.pack_lower(A, nb))
    ctx = tc.Context(n, nb, ooc_sync=sync, ooc_no_reuse=no_reuse, ooc_no_v3=no_v3)
    st = tc.factorize_ooc(ctx, Ah, n, nb, cache)
    assert st["info"] == 0
    assert np.array_equal(Ah.numpy(), L0)
    assert st["bytes_d2h"] == st0["bytes_d2h"] == ntiles * tbytes
    if no_v3:
        diag_loads = Nt * (Nt - 1) // 2  # one per tile below the diagonal
        assert st["tiles_reloaded"] == st0["tiles_reloaded"] + diag_loads
        assert st["bytes_h2d"] == st0["bytes_h2d"] + diag_loads * tbytes
        assert st["cache_slots"] == st0["cache_slots"] - 2
    elif no_reuse:
        # operands (m, n), m >= k > n, loaded in every column k
        loads = sum((Nt - k) * k for k in range(1, Nt))
        assert st["tiles_reloaded"] == loads
        assert st["bytes_h2d"] == (ntiles + loads) * tbytes
    else:
        assert st["bytes_h2d"] == st0["bytes_h2d"] and st["tiles_reloaded"] == st0["tiles_reloaded"]


@pytest.mark.parametrize("slots", [32, 40])
def test_ooc_lru_eviction(tc, case, slots):
    """Least-recently-used eviction in place of next-use eviction, with a
    cache smaller than the working set: the same kernels on the same tile
    values (bitwise the same factor); every operand load is counted once in
    the transfer volume; on the left-looking schedule's cyclic reads LRU
    reloads at least as many tiles as next-use eviction."""
    import torch
    n, nb, A = case["n"], case["nb"], case["A"]
    Nt = n // nb
    ntiles = Nt * (Nt + 1) // 2
    tbytes = nb * nb * 8
    cache = torch.empty(slots * tbytes, dtype=torch.uint8, device="cuda")
    res = {}
    for lru in (False, True):
        Ah = pinned(tc.pack_lower(A, nb))
        st = tc.factorize_ooc(tc.Context(n, nb, ooc_lru=lru), Ah, n, nb, cache)
        assert st["info"] == 0 and st["evictions"] > 0
        assert st["bytes_h2d"] == (ntiles + st["tiles_reloaded"]) * tbytes
        assert st["bytes_d2h"] == ntiles * tbytes
        res[lru] = (Ah.numpy().copy(), st)
    print("slots %d: reloads next-use %d, LRU %d" % (slots, res[False][1]["tiles_reloaded"],
                                                     res[True][1]["tiles_reloaded"]))
    assert np.array_equal(res[True][0], res[False][0])
    assert res[True][1]["tiles_reloaded"] >= res[False][1]["tiles_reloaded"]


@pytest.fixture(scope="module")
def big_tiles():
    """The out-of-core workload's tile size (nb = 2048) at n = 20480 (Nt = 10).
    The cache holds finished factor tiles only (the working columns live in
    the context workspace): during column k the live tiles are (r, n) with
    r >= k > n, (Nt - k) k of them, 25 at k = 5. So the minimal 2 Nt =
    20-slot cache must evict and reload, and a 32-slot cache holds every
    column's set (after column k, (Nt - k - 1)(k + 1) <= 30 tiles)."""
    n, nb = 20480, 2048
    w = si.WORKLOADS["ooc"]
    return dict(n=n, nb=nb, w=w, pts=si.points(n, seed=w["seed"]))


@pytest.mark.parametrize("slots", [20, 32])
def test_ooc_nb2048_exact_integer_factor(tc, big_tiles, slots):
    """A = L0 L0^T with a dense small-integer L0 (entries in {-1, 0, 1}
    below a diagonal from {1, 2, 4}): every partial sum is an integer below
    2^53, so any summation order is exact and the factor must be L0 bit for
    bit -- the result the oracle's own exact-integer pin reproduces for any
    tiling. A is formed on the device in binary64 (exact for the same
    reason)."""
    import torch
    n, nb = big_tiles["n"], big_tiles["nb"]
    Nt = n // nb
    L0 = si.integer_factor(n, seed=29, band=n - 1)
    L0d = torch.from_numpy(L0).cuda()
    Ad = (L0d @ L0d.t()).cpu().numpy()
    del L0d
    Ah = pinned(tc.pack_lower(Ad, nb))
    ctx = tc.Context(n, nb)
    cache = torch.empty(slots * nb * nb * 8, dtype=torch.uint8, device="cuda")
    st = tc.factorize_ooc(ctx, Ah, n, nb, cache)
    assert st["info"] == 0 and st["cache_slots"] == slots
    ntiles = Nt * (Nt + 1) // 2
    tbytes = nb * nb * 8
    assert st["bytes_d2h"] == ntiles * tbytes
    if slots == 2 * Nt:
        assert st["evictions"] > 0 and st["tiles_reloaded"] > 0
    else:
        assert st["tiles_reloaded"] == 0 and st["bytes_h2d"] == ntiles * tbytes
    assert st["bytes_h2d"] == (ntiles + st["tiles_reloaded"]) * tbytes
    L = np.tril(tc.unpack_lower(Ah.numpy(), n, nb))
    assert np.array_equal(L, L0)


@pytest.mark.parametrize("slots", [20, 32])
def test_ooc_nb2048_matern_rows(tc, big_tiles, slots):
    """The out-of-core workload's covariance (nu = 1, range 0.05, nugget
    1e-4) at nb = 2048: 24 sampled rows of the factor satisfy the
    componentwise backward-error bound |A - L L^T|_ij <= gamma_{n+1}
    (|L| |L|^T)_ij against covariance entries computed by the oracle, and
    the factor agrees with the in-core factor within the perturbation bound
    (the out-of-core update is summed in chunks of tile columns): both are
    exact factors of matrices within gamma_{n+1} of A, and kappa(A) <=
    ||A||_F / nugget (the Matern part is positive semidefinite)."""
    import torch
    n, nb, w, pts = big_tiles["n"], big_tiles["nb"], big_tiles["w"], big_tiles["pts"]
    theta = (w["sigma2"], w["range"], w["nu"], w["nugget"])
    ctx = tc.Context(n, nb)
    Ad, _, fro = tc.matern_tiles(ctx, torch.from_numpy(pts).cuda(), theta, nb)
    Ah = torch.empty(Ad.numel(), dtype=torch.float64, pin_memory=True)
    Ah.copy_(Ad)
    Lin = tc.unpack_lower(tc.export(ctx, tc.factorize(ctx, Ad, n, nb)).cpu().numpy(), n, nb)
    del Ad
    cache = torch.empty(slots * nb * nb * 8, dtype=torch.uint8, device="cuda")
    st = tc.factorize_ooc(ctx, Ah, n, nb, cache)
    assert st["info"] == 0
    L = np.tril(tc.unpack_lower(Ah.numpy(), n, nb))
    rows = np.unique(np.concatenate([np.arange(0, n, n // 16),
                                     np.random.default_rng(41).integers(0, n, 8), [n - 1]]))
    g = (n + 1) * U / (1 - (n + 1) * U)
    absL = np.abs(L)
    for i in rows:
        J = np.arange(i + 1)
        a = oracle.matern_entries(pts, np.full(i + 1, i), J, *theta)
        r = a - L[i, :i + 1] @ L[:i + 1, :i + 1].T
        bound = g * (absL[i, :i + 1] @ absL[:i + 1, :i + 1].T)
        assert np.all(np.abs(r) <= bound), (i, float(np.max(np.abs(r) / bound)))
    be = np.linalg.norm(L - Lin) / np.linalg.norm(Lin)
    print("slots %d: |L_ooc - L_in| / |L_in| = %.2e, reloads %d" % (slots, be, st["tiles_reloaded"]))
    kappa_max = fro / theta[3]
    assert be <= 4 * kappa_max * n * U, (be, kappa_max)
