"""GPU parity of the 256 x 256-block update kernels of the low classes
(tc_opts.wide_tiles = 1) against the CPU oracle (Section IV-C).

What pins what:
  * The factor under a map with FP32 (two-term FP16 split), FP16 or BF16,
    and FP8 tiles has every stored tile representable in its class, a
    backward error within 10x of the oracle's emulation of the same map and
    update arithmetic (and below the map's target), and agrees with the
    oracle's factor and with the 128 x 128-block kernels' factor
    (wide_tiles = -1) within the perturbation bound 4 kappa (be + be'); the
    two block shapes sum in a different binary32 order, so their factors
    are not bitwise equal (which shows the wide kernels ran).
  * The same with the updates into FP64 tiles in FP32-class arithmetic.
  * Out of core (n = 4096, nb = 256, the minimal cache, which evicts):
    the host image decodes to a factor with the same bounds.
  * Refined solves with the wide factor reach 1e-9.
  * nb = 256 (one block per tile) and nb = 512 (four), tile columns walked
    in ascending order of their product scale inside each block.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from test_gpu_ooc_mixed import decode_image, pinned

pytestmark = pytest.mark.gpu


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


_CASES = {}


def case(n, nb):
    if (n, nb) not in _CASES:
        pts = si.points(n, seed=3)
        A = oracle.matern_matrix(pts, 1.0, 0.03, 0.5, 1e-4)
        Nt = n // nb
        norms = oracle.tile_norms(A, nb)
        _CASES[(n, nb)] = dict(n=n, nb=nb, Nt=Nt, A=A, norms=norms,
                               fro=oracle.fro_norm(norms, Nt), kappa=np.linalg.cond(A))
    return _CASES[(n, nb)]


def class_map(tc, c, eps, bf16):
    allowed = ((tc.FP64, tc.FP32, tc.BF16, tc.FP8E4M3) if bf16 else
               (tc.FP64, tc.FP32, tc.FP16, tc.FP8E4M3))
    return tc.precision_map(c["Nt"], c["norms"], c["fro"], eps, allowed=allowed)


def representable(tc, L, cm, Nt, nb):
    for j in range(Nt):
        for i in range(j + 1, Nt):
            t = L[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
            cl = int(cm[oracle.tile_index(Nt, i, j)])
            assert np.array_equal(oracle.round_tile(t, cl)[0], t), (i, j, cl)


@pytest.mark.parametrize("n,nb,eps,bf16,upd", [
    (2048, 256, 1e-4, False, 0),
    (2048, 256, 1e-4, True, 0),
    (3072, 512, 1e-6, False, 0),
    (2048, 256, 1e-9, False, 1),
    (2048, 256, 1e-4, True, 1),
])
def test_wide_factor_matches_oracle(tc, n, nb, eps, bf16, upd):
    c = case(n, nb)
    Nt, A = c["Nt"], c["A"]
    cm = class_map(tc, c, eps, bf16)
    low = set(cm.tolist()) - {tc.FP64}
    assert len(low) >= 2 and (not bf16 or tc.BF16 in low), np.bincount(cm, minlength=5)
    ctx = tc.Context(n, nb, nrhs=3)
    Ad = to_dev(tc.pack_lower(A, nb))
    fu = tc.FP32 if upd else tc.FP64
    Fw = tc.factorize(ctx, Ad, n, nb, cmap=cm, fp64_update=fu, wide_tiles=1)
    Fn = tc.factorize(ctx, Ad, n, nb, cmap=cm, fp64_update=fu, wide_tiles=-1)
    assert Fw.stats.info == 0 and Fn.stats.info == 0
    assert list(Fw.stats.class_flops) == list(Fn.stats.class_flops)
    Lw = tc.unpack_lower(tc.export(ctx, Fw).cpu().numpy(), n, nb)
    Ln = tc.unpack_lower(tc.export(ctx, Fn).cpu().numpy(), n, nb)
    representable(tc, Lw, cm, Nt, nb)
    assert not np.array_equal(Lw, Ln)  # a different summation order ran
    Lo, info = oracle.mxp_tile_cholesky(A, nb, cm, fp64_update=oracle.FP32 if upd else oracle.FP64)
    assert info == 0
    be_w, be_n, be_o = (oracle.backward_error(A, X) for X in (Lw, Ln, Lo))
    assert be_w <= 10 * be_o and (upd or be_w <= eps), (be_w, be_o)
    k4 = 4 * c["kappa"]
    assert np.linalg.norm(Lw - Lo) / np.linalg.norm(Lo) <= k4 * (be_w + be_o) + 1e-13
    assert np.linalg.norm(Lw - Ln) / np.linalg.norm(Ln) <= k4 * (be_w + be_n) + 1e-13
    B = si.standard_normal((n, 3), seed=si.rhs_seed(3))
    Bd = to_dev(np.ascontiguousarray(B.T))
    st = tc.solve_refine(ctx, Fw, Ad, Bd, max_iter=30, tol=1e-9)
    X = Bd.cpu().numpy().T
    rel = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert st["converged"] and rel.max() <= 1e-9, (st, rel.max())
    Fw.close()
    Fn.close()


def test_wide_ooc_mixed(tc):
    """Out of core with the wide kernels and the minimal 2 Nt-slot cache
    (evictions and reloads), against the oracle and the in-core wide
    factor."""
    import torch
    n, nb = 4096, 256
    c = case(n, nb)
    Nt, A = c["Nt"], c["A"]
    cm = class_map(tc, c, 1e-4, False)
    ctx = tc.Context(n, nb)
    Ah = pinned(tc.pack_lower(A, nb))
    slots = 2 * Nt
    cache = torch.empty(tc.ooc_mixed_cache_bytes(n, nb, cm, slots), dtype=torch.uint8,
                        device="cuda")
    st, img = tc.factorize_ooc_mixed(ctx, Ah, n, nb, cm, cache, wide_tiles=1)
    assert st["info"] == 0 and st["evictions"] > 0
    L = np.tril(tc.unpack_lower(decode_image(img, n, nb, cm), n, nb))
    representable(tc, L, cm, Nt, nb)
    Ad = to_dev(tc.pack_lower(A, nb))
    Lin = tc.unpack_lower(tc.export(ctx, tc.factorize(ctx, Ad, n, nb, cmap=cm, wide_tiles=1))
                          .cpu().numpy(), n, nb)
    Lo, info = oracle.mxp_tile_cholesky(A, nb, cm)
    assert info == 0
    be, be_in, be_o = (oracle.backward_error(A, X) for X in (L, Lin, Lo))
    assert be <= 10 * be_o and be <= 1e-4, (be, be_o)
    assert np.linalg.norm(L - Lin) / np.linalg.norm(Lin) <= 4 * c["kappa"] * (be + be_in) + 1e-13


def test_wide_tiles_option_checked(tc):
    n, nb = 1024, 256
    c = case(n, nb)
    cm = class_map(tc, c, 1e-4, False)
    ctx = tc.Context(n, nb)
    Ad = to_dev(tc.pack_lower(c["A"], nb))
    with pytest.raises(tc.TileCholError) as e:
        tc.factorize(ctx, Ad, n, nb, cmap=cm, wide_tiles=2)
    assert e.value.status == tc.TC_EINVAL
    # nb = 128 cannot hold a 256 x 256 block: wide_tiles = 1 falls back
    n2, nb2 = 1024, 128
    c2 = case(n2, nb2)
    cm2 = class_map(tc, c2, 1e-4, False)
    ctx2 = tc.Context(n2, nb2)
    A2 = to_dev(tc.pack_lower(c2["A"], nb2))
    L1 = tc.export(ctx2, tc.factorize(ctx2, A2, n2, nb2, cmap=cm2, wide_tiles=1)).cpu().numpy()
    L0 = tc.export(ctx2, tc.factorize(ctx2, A2, n2, nb2, cmap=cm2, wide_tiles=-1)).cpu().numpy()
    assert np.array_equal(L1, L0)
