"""The factorization entry point that allocates nothing (tc_factorize_noalloc)
against tc_factorize, the FP64 factorization it is a variant of, through
the C ABI.

The bar is the FP64 one: bitwise for an exact-integer matrix (every
operation is exact in binary64, so any summation order gives L0), and for a
Matern covariance a probe backward error ||(A - L L^T) G||_F / ||A G||_F of
at most 1e-12, plus agreement with tc_factorize's factor within the
first-order perturbation bound 4 kappa(A) n u (the two sum the panel
updates in different orders). The calls come in a row on one context, the
second with a smaller input, so the second runs on the fixed scratch array
the first one left behind.
"""
import numpy as np
import pytest

import bench
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


def _zero_upper(tc, L, n, nb):
    """Zero the strict upper triangles of the diagonal tiles (in place)."""
    Nt = n // nb
    nb2 = nb * nb
    for k in range(Nt):
        t = tc.tile_offset(Nt, k, k)
        L[t * nb2:(t + 1) * nb2].view(nb, nb).triu_()  # view[c][r] = L[r][c]: keep r >= c
    return L


def test_noalloc_matches_factorize_two_calls(tc):
    import torch
    dev = torch.device("cuda", 0)
    # call 1: the n = 65536 workload's covariance at n = 16384, nb = 1024
    # (the late columns' split-K is held to the fixed array)
    n, nb = 16384, 1024
    w = si.WORKLOADS["fp64"]
    theta = (w["sigma2"], w["range"], w["nu"], w["nugget"])
    ctx = tc.Context(n, nb)
    A, _, fro = tc.matern_tiles(ctx, torch.from_numpy(si.points(n, seed=w["seed"])).to(dev), theta, nb)
    F = tc.factorize(ctx, A, n, nb)
    Lref = tc.export(ctx, F)
    F.close()
    Lna = torch.empty_like(A)
    print("noalloc call 1: n=%d nb=%d" % (n, nb), flush=True)
    assert tc.factorize_noalloc(ctx, A, n, nb, Lna) == 0
    _zero_upper(tc, Lna, n, nb)
    be = bench.probe_backward_error(A, Lna, n, nb)
    be_ref = bench.probe_backward_error(A, Lref, n, nb)
    rel = float(torch.linalg.norm(Lna - Lref) / torch.linalg.norm(Lref))
    kappa_max = fro / theta[3]
    print("noalloc: probe backward error %.2e (tc_factorize %.2e), |L - Lref| / |Lref| = %.2e"
          % (be, be_ref, rel))
    assert be <= 1e-12 and be_ref <= 1e-12
    assert rel <= 4 * kappa_max * n * U
    del A, Lref, Lna, F
    ctx.close()
    # call 2, smaller: exact integer matrix, bitwise equal to L0 and to tc_factorize
    n, nb = 1536, 256
    L0 = si.integer_factor(n, seed=31, band=n - 1)
    ctx = tc.Context(n, nb)
    A = torch.from_numpy(tc.pack_lower(L0 @ L0.T, nb)).to(dev)
    F = tc.factorize(ctx, A, n, nb)
    Lref = tc.unpack_lower(tc.export(ctx, F).cpu().numpy(), n, nb)
    F.close()
    out = torch.empty_like(A)
    print("noalloc call 2: n=%d nb=%d" % (n, nb), flush=True)
    assert tc.factorize_noalloc(ctx, A, n, nb, out) == 0
    L = np.tril(tc.unpack_lower(out.cpu().numpy(), n, nb))
    assert np.array_equal(L, L0)
    assert np.array_equal(L, Lref)


def test_noalloc_failure_then_success(tc):
    """A pivot failure reports tc_factorize's info; the next call starts
    from a cleared flag (the array keeps the failed call's contents)."""
    import torch
    dev = torch.device("cuda", 0)
    n, nb = 1024, 256
    L0 = si.integer_factor(n, seed=37, band=n - 1)
    Abad = L0 @ L0.T
    Abad[700, 700] = -1.0
    ctx = tc.Context(n, nb)
    Ad = torch.from_numpy(tc.pack_lower(Abad, nb)).to(dev)
    with pytest.raises(tc.NotPositiveDefinite) as ref:
        tc.factorize(ctx, Ad, n, nb)
    out = torch.empty_like(Ad)
    print("noalloc: failing call n=%d nb=%d" % (n, nb), flush=True)
    with pytest.raises(tc.NotPositiveDefinite) as got:
        tc.factorize_noalloc(ctx, Ad, n, nb, out)
    assert got.value.info == ref.value.info == 701
    # in place this time (out == A)
    n2 = 512
    L1 = si.integer_factor(n2, seed=38, band=n2 - 1)
    A2 = torch.from_numpy(tc.pack_lower(L1 @ L1.T, nb)).to(dev)
    print("noalloc: call after the failure n=%d nb=%d in place" % (n2, nb), flush=True)
    assert tc.factorize_noalloc(ctx, A2, n2, nb, A2) == 0
    assert np.array_equal(np.tril(tc.unpack_lower(A2.cpu().numpy(), n2, nb)), L1)


def test_noalloc_rejects_bad_arguments(tc):
    import torch
    ctx = tc.Context(1024, 256)
    A = torch.zeros(tc.num_tiles(1024, 256) * 256 * 256, dtype=torch.float64, device="cuda")
    with pytest.raises(tc.TileCholError):
        tc.factorize_noalloc(ctx, A, 1000, 256, A)  # n not a multiple of nb
    with pytest.raises(tc.TileCholError):
        tc.factorize_noalloc(ctx, A, 1024, 100, A)  # nb not a multiple of 128
