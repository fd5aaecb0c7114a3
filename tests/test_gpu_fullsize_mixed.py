"""Full-size checks of the mixed-precision paths in the launch
configuration bench.py times, on quantities the oracle computes at any
size:
  * mxp workload (n = 131072, nb = 1024, map at 1e-9, 16 right-hand sides
    refined to 1e-9), with the updates into FP64 tiles in binary64 or in
    the FP32 class's arithmetic: sampled rows of the residual b - A x
    recomputed from the oracle's own covariance entries (independent of the
    GPU's A) stay within the reported relative residual, and a
    Gaussian-probe backward error of the mixed factor is within its bound;
  * out of core, mixed precision (n = 90112, nb = 2048, the ooc workload's
    parameters, map at 1e-9, a cache holding the working set): sampled
    tiles of the host image equal the in-core mixed factor of the same map
    bit for bit (the two schedules launch the same tile-column pieces), each
    factor tile crosses the link once in its class's bytes and A once in
    binary64.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu

BYTES = {0: 8, 1: 4, 2: 2, 3: 2, 4: 1}


@pytest.fixture(scope="module")
def tc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_09819_amd as tc
    tc.lib()
    return tc


def probe_backward_error(tc, A, L, n, nb, k=4, seed=0):
    """||(A - L L^T) G||_F / ||A G||_F for Gaussian G, tile by tile (torch
    products on the device, not the library's kernels)."""
    import torch
    Nt = n // nb
    G = torch.from_numpy(si.standard_normal((n, k), seed=seed)).to(A.device)
    AG = torch.zeros_like(G)
    Z = torch.zeros_like(G)
    for j in range(Nt):
        for i in range(j, Nt):
            t = oracle.tile_index(Nt, i, j)
            Aij = A[t * nb * nb:(t + 1) * nb * nb].view(nb, nb).t()
            Lij = L[t * nb * nb:(t + 1) * nb * nb].view(nb, nb).t()
            AG[i * nb:(i + 1) * nb] += Aij @ G[j * nb:(j + 1) * nb]
            if i != j:
                AG[j * nb:(j + 1) * nb] += Aij.t() @ G[i * nb:(i + 1) * nb]
            Z[j * nb:(j + 1) * nb] += Lij.t() @ G[i * nb:(i + 1) * nb]
    W = torch.zeros_like(G)
    for j in range(Nt):
        for i in range(j, Nt):
            t = oracle.tile_index(Nt, i, j)
            Lij = L[t * nb * nb:(t + 1) * nb * nb].view(nb, nb).t()
            W[i * nb:(i + 1) * nb] += Lij @ Z[j * nb:(j + 1) * nb]
    return float(torch.linalg.norm(AG - W) / torch.linalg.norm(AG))


@pytest.mark.parametrize("fp64_update", [0, 1])
def test_mxp_workload_full_size(tc, fp64_update):
    """fp64_update 0: the updates into FP64 tiles in binary64; 1 (FP32):
    in the FP32 class's arithmetic. The backward-error bound is the map's
    target for the former, and sqrt(n) * 2^-22 (FP32-class products summed
    over growing columns) for the latter, whose accuracy refinement
    restores."""
    import torch
    w = si.WORKLOADS["mxp"]
    n, nb, nrhs, eps = w["n"], w["nb"], w["nrhs"], w["eps"]
    theta = (w["sigma2"], w["range"], w["nu"], w["nugget"])
    pts = si.points(n, seed=w["seed"])
    ctx = tc.Context(n, nb, nrhs=nrhs)
    A, tf, fro = tc.matern_tiles(ctx, torch.from_numpy(pts).cuda(), theta, nb)
    Nt = n // nb
    cm = tc.precision_map(Nt, tf.cpu().numpy(), fro, eps)
    assert len(set(cm.tolist())) == 4
    F = tc.factorize(ctx, A, n, nb, cmap=cm, fp64_update=fp64_update)
    assert F.stats.info == 0
    B0 = si.standard_normal((n, nrhs), seed=si.rhs_seed(w["seed"]))
    B = torch.from_numpy(np.ascontiguousarray(B0.T)).cuda()
    st = tc.solve_refine(ctx, F, A, B, max_iter=30, tol=1e-9)
    assert st["converged"] and st["rel_residual"] <= 1e-9
    X = B.cpu().numpy()  # (nrhs, n)
    rng = np.random.default_rng(5)
    rows = rng.choice(n, 6, replace=False)
    bnorm = np.linalg.norm(B0, axis=0)
    for i in rows:
        a = oracle.matern_entries(pts, np.full(n, i), np.arange(n), *theta)
        r = B0[i] - X @ a
        # one row of b - A x is at most the whole residual (plus the
        # rounding of forming it in binary64 here)
        floor = n * 2.0 ** -53 * (np.abs(X) @ np.abs(a) + np.abs(B0[i]))
        assert np.all(np.abs(r) <= st["rel_residual"] * bnorm * (1 + 1e-6) + 2 * floor), i
    L = tc.export(ctx, F)
    F.close()
    be = probe_backward_error(tc, A, L, n, nb)
    assert be <= (eps if fp64_update == 0 else np.sqrt(n) * 2.0 ** -22), be


def decode_tile(raw, cm, nb, t):
    nb2 = nb * nb
    sizes = [(nb2 * BYTES[int(c)] + 255) // 256 * 256 for c in cm]
    off, end = sum(sizes[:t]), sum(sizes)
    e = int(raw[end:end + 4 * len(cm)].view(np.int32)[t])
    c = int(cm[t])
    b = raw[off:off + nb2 * BYTES[c]]
    if c == 0:
        v = b.view(np.float64)
    elif c == 1:
        v = b.view(np.float32).astype(np.float64)
    elif c == 2:
        v = b.view(np.float16).astype(np.float64)
    elif c == 3:
        v = (b.view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    else:
        ex, m = (b >> 3) & 15, (b & 7).astype(np.float64)
        v = np.where(ex == 0, m * 2.0 ** -9, (1 + m / 8) * np.ldexp(1.0, ex.astype(np.int64) - 7))
        v = np.where(b & 0x80, -v, v)
    return np.ldexp(v, e).reshape(nb, nb).T


def test_ooc_mixed_bench_size(tc):
    import torch
    w = si.WORKLOADS["ooc"]
    n, nb, eps = 90112, 2048, 1e-9
    theta = (w["sigma2"], w["range"], w["nu"], w["nugget"])
    pts = torch.from_numpy(si.points(n, seed=w["seed"])).cuda()
    ctx = tc.Context(n, nb)
    A, tf, fro = tc.matern_tiles(ctx, pts, theta, nb)
    Nt = n // nb
    cm = tc.precision_map(Nt, tf.cpu().numpy(), fro, eps)
    F = tc.factorize(ctx, A, n, nb, cmap=cm)
    L64 = tc.export(ctx, F)
    F.close()
    nb2 = nb * nb
    samples = [(Nt - 1, 0), (Nt // 2, Nt // 3), (Nt - 1, Nt - 2), (7, 6), (Nt - 1, Nt - 1), (0, 0)]
    ref = {ij: L64[tc.tile_offset(Nt, *ij) * nb2:(tc.tile_offset(Nt, *ij) + 1) * nb2].view(nb, nb).t().cpu().numpy()
           for ij in samples}
    del L64
    torch._C._host_emptyCache()
    Abuf = tc.PinnedBuffer(A.numel() * 8)
    Abuf.view(torch.float64).copy_(A)
    del A
    torch.cuda.empty_cache()
    Ibuf = tc.PinnedBuffer(tc.ooc_mixed_host_bytes(n, nb, cm))
    cache = torch.empty(40 << 30, dtype=torch.uint8, device="cuda")
    st, img = tc.factorize_ooc_mixed(ctx, Abuf.view(torch.float64), n, nb, cm, cache, L_host=Ibuf.tensor)
    del cache
    torch.cuda.empty_cache()
    assert st["info"] == 0 and st["tiles_reloaded"] == 0
    assert st["bytes_h2d"] == len(cm) * nb2 * 8
    assert st["bytes_d2h"] == sum(nb2 * BYTES[int(c)] for c in cm)
    raw = img.numpy()
    for ij in samples:
        t = tc.tile_offset(Nt, *ij)
        a, b = ref[ij], decode_tile(raw, cm, nb, t)
        if ij[0] == ij[1]:
            a, b = np.tril(a), np.tril(b)
        c = int(cm[t])
        # exactly representable in the tile's class
        assert np.array_equal(oracle.round_tile(b, c)[0] if c else b, b), ij
        # with the working set in the cache the out-of-core group launches
        # are the in-core ones (same tile-column pieces, same kernels): the
        # same factor bit for bit
        assert np.array_equal(a, b), (ij, float(np.abs(a - b).max()))
    Abuf.close()
    Ibuf.close()
