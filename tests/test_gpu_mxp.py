"""GPU parity of the mixed-precision factorization (Section IV-C) and the
FP64 refinement solve against the CPU oracle.

The GPU and the oracle run the same algorithm (operands rounded to the
output tile's class, FP32 accumulation, FP64 POTRF/TRSM, results rounded to
the tile's class) but accumulate in different orders, so they are compared
through properties and bounds:
  * every stored tile is exactly representable in its class;
  * the backward error ||A - Lh Lh^T||_F / ||A||_F is at most the target
    accuracy eps and within 10x of the oracle's (the per-map bound);
  * both factors are exact factors of A + E with ||E|| <= be ||A||, so they
    differ by at most ~4 kappa(A) (be_gpu + be_oracle) relative;
  * refinement reaches max_j ||b_j - A x_j|| / ||b_j|| <= 1e-9, checked on the
    CPU in binary64 from A;
  * the log-determinant, through D_KL of Eq. 3 at y = 0,
    D = (log|Lh Lh^T| - log|A|) / 2: the GPU's D against the oracle
    emulation's, with the same sign and within a stated factor where the
    stored tiles' rounding sets D, and within 10x of the emulation's
    magnitude where the FP32 accumulation's rounding noise sets it (the
    oracle's two summation orders then disagree in sign);
  * the FP32 class's update in isolation: recomputed in binary64 from the
    GPU's own stored binary32 operands, componentwise within the split's
    per-product bound plus the FP32 accumulation bound.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

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


@pytest.fixture(scope="module")
def case():
    n, nb = 2048, 128
    pts = si.points(n, seed=3)
    A = oracle.matern_matrix(pts, 1.0, 0.03, 0.5, 1e-4)
    Nt = n // nb
    norms = oracle.tile_norms(A, nb)
    L64, info = oracle.tile_cholesky(A, nb, threads=8)
    assert info == 0
    return dict(n=n, nb=nb, Nt=Nt, pts=pts, A=A, norms=norms, fro=oracle.fro_norm(norms, Nt),
                kappa=np.linalg.cond(A), ld64=oracle.logdet(L64))


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-9])
def test_mixed_factor_matches_oracle(tc, case, eps):
    n, nb, Nt, A = case["n"], case["nb"], case["Nt"], case["A"]
    cm = tc.precision_map(Nt, case["norms"], case["fro"], eps)
    assert len(set(cm.tolist())) >= 3
    ctx = tc.Context(n, nb)
    Ad = to_dev(tc.pack_lower(A, nb))
    F = tc.factorize(ctx, Ad, n, nb, cmap=cm)
    assert F.stats.info == 0
    assert list(F.stats.class_tiles) == np.bincount(cm, minlength=5).tolist()
    Lg = tc.unpack_lower(tc.export(ctx, F).cpu().numpy(), n, nb)
    for j in range(Nt):
        for i in range(j + 1, Nt):
            t = Lg[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
            c = int(cm[oracle.tile_index(Nt, i, j)])
            assert np.array_equal(oracle.round_tile(t, c)[0], t), (i, j, c)
    Lo, info = oracle.mxp_tile_cholesky(A, nb, cm)
    assert info == 0
    be_g, be_o = oracle.backward_error(A, Lg), oracle.backward_error(A, Lo)
    assert be_g <= eps and be_g <= 10 * be_o, (be_g, be_o)
    diff = np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo)
    assert diff <= 4 * case["kappa"] * (be_g + be_o) + 1e-13, diff
    # log-determinant: the GPU's and the oracle's mixed factors may differ
    # by at most 10x the oracle's own mixed-precision effect on it (D_KL of
    # Eq. 3 at y = 0, times 2) or its rounding-order noise, whichever is
    # larger, plus the binary64 floor of the two FP64 log-determinants
    ld = tc.logdet(ctx, F)
    ld64, ld_o = case["ld64"], oracle.logdet(Lo)
    Lr, _ = oracle.mxp_tile_cholesky(A, nb, cm, reverse_sums=True)
    scale = max(abs(ld_o - ld64), abs(oracle.logdet(Lr) - ld_o))
    assert abs(ld - ld_o) <= 10 * scale + 1e-12 * abs(ld64), (ld - ld_o, scale)


def test_all_fp64_map_equals_fp64_path(tc, case):
    n, nb, Nt, A = case["n"], case["nb"], case["Nt"], case["A"]
    ctx = tc.Context(n, nb)
    Ad = to_dev(tc.pack_lower(A, nb))
    L1 = tc.export(ctx, tc.factorize(ctx, Ad, n, nb)).cpu().numpy()
    cm = np.zeros(Nt * (Nt + 1) // 2, dtype=np.uint8)
    L2 = tc.export(ctx, tc.factorize(ctx, Ad, n, nb, cmap=cm)).cpu().numpy()
    assert np.array_equal(L1, L2)


@pytest.mark.parametrize("eps,nrhs", [(1e-5, 16), (1e-9, 3)])
def test_refined_solve(tc, case, eps, nrhs):
    n, nb, Nt, A = case["n"], case["nb"], case["Nt"], case["A"]
    cm = tc.precision_map(Nt, case["norms"], case["fro"], eps)
    ctx = tc.Context(n, nb, nrhs=nrhs)
    Ad = to_dev(tc.pack_lower(A, nb))
    F = tc.factorize(ctx, Ad, n, nb, cmap=cm)
    B = si.standard_normal((n, nrhs), seed=si.rhs_seed(3))
    Bd = to_dev(np.ascontiguousarray(B.T))
    st = tc.solve_refine(ctx, F, Ad, Bd, max_iter=30, tol=1e-9)
    X = Bd.cpu().numpy().T
    rel = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert st["converged"] and rel.max() <= 1e-9, (st, rel.max())
    assert abs(st["rel_residual"] - rel.max()) <= 1e-3 * rel.max() + 1e-15
    Xo = np.linalg.solve(A, B)
    assert np.linalg.norm(X - Xo) <= case["kappa"] * 1e-9 * np.linalg.norm(Xo) * 4
    # the oracle's refinement with the oracle's factor needs a similar count
    Lo, _ = oracle.mxp_tile_cholesky(A, nb, cm)
    _, it_o, _ = oracle.refine(A, Lo, B, tol=1e-9)
    assert abs(st["iterations"] - it_o) <= 2


def test_bf16_map_factor_and_refined_solve(tc, case):
    """A map with BF16 in place of FP16 (classes FP64 / FP32 / BF16 / FP8 at
    target 1e-5: 16 / 52 / 25 / 43 tiles): the factor against the oracle's
    emulation of the same map, and a refined solve of 20 right-hand sides
    (two groups of 16 through every solve kernel, K-split forward panels and
    ragged backward splits included)."""
    n, nb, Nt, A = case["n"], case["nb"], case["Nt"], case["A"]
    eps, nrhs = 1e-5, 20
    cm = tc.precision_map(Nt, case["norms"], case["fro"], eps,
                          allowed=(tc.FP64, tc.FP32, tc.BF16, tc.FP8E4M3))
    assert np.count_nonzero(cm == tc.BF16) >= 8
    ctx = tc.Context(n, nb, nrhs=nrhs)
    Ad = to_dev(tc.pack_lower(A, nb))
    F = tc.factorize(ctx, Ad, n, nb, cmap=cm)
    assert F.stats.info == 0
    Lg = tc.unpack_lower(tc.export(ctx, F).cpu().numpy(), n, nb)
    for j in range(Nt):
        for i in range(j + 1, Nt):
            t = Lg[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
            c = int(cm[oracle.tile_index(Nt, i, j)])
            assert np.array_equal(oracle.round_tile(t, c)[0], t), (i, j, c)
    Lo, info = oracle.mxp_tile_cholesky(A, nb, cm)
    assert info == 0
    be_g, be_o = oracle.backward_error(A, Lg), oracle.backward_error(A, Lo)
    assert be_g <= eps and be_g <= 10 * be_o, (be_g, be_o)
    diff = np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo)
    assert diff <= 4 * case["kappa"] * (be_g + be_o) + 1e-13, diff
    B = si.standard_normal((n, nrhs), seed=si.rhs_seed(5))
    Bd = to_dev(np.ascontiguousarray(B.T))
    st = tc.solve_refine(ctx, F, Ad, Bd, max_iter=30, tol=1e-9)
    X = Bd.cpu().numpy().T
    rel = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert st["converged"] and rel.max() <= 1e-9, (st, rel.max())
    _, it_o, _ = oracle.refine(A, Lo, B, tol=1e-9)
    assert abs(st["iterations"] - it_o) <= 2


def test_refinement_reports_nonconvergence(tc, case):
    n, nb, Nt, A = case["n"], case["nb"], case["Nt"], case["A"]
    cm = tc.precision_map(Nt, case["norms"], case["fro"], 1e-3)
    ctx = tc.Context(n, nb)
    Ad = to_dev(tc.pack_lower(A, nb))
    F = tc.factorize(ctx, Ad, n, nb, cmap=cm)
    Bd = to_dev(np.ascontiguousarray(si.standard_normal((n, 2), seed=5).T))
    with pytest.raises(tc.TileCholError) as e:
        tc.solve_refine(ctx, F, Ad, Bd, max_iter=0, tol=1e-14)
    assert e.value.status == tc.TC_ENOTCONV
    st = tc.solve_refine(ctx, F, Ad, Bd, max_iter=0, tol=1e-14, check=False)
    assert st["iterations"] == 0 and not st["converged"]


def test_fp64_refinement_converges_immediately(tc, case):
    n, nb, A = case["n"], case["nb"], case["A"]
    ctx = tc.Context(n, nb)
    Ad = to_dev(tc.pack_lower(A, nb))
    F = tc.factorize(ctx, Ad, n, nb)
    Bd = to_dev(np.ascontiguousarray(si.standard_normal((n, 4), seed=6).T))
    st = tc.solve_refine(ctx, F, Ad, Bd, tol=1e-12)
    assert st["iterations"] <= 1 and st["rel_residual"] <= 1e-12


@pytest.mark.parametrize("eps", [1e-6, 1e-9, None])
def test_fp32_update_matches_oracle(tc, case, eps):
    """Updates into FP64-class tiles (diagonal SYRK included) in the FP32
    class's arithmetic: no FP64 GEMM/SYRK flops remain; stored tiles are
    representable in their classes; the backward error is within 10x of the
    oracle's emulation of the same variant (the split's per-product error,
    at most 3 * 2^-22, is within 6x of binary32 product rounding plus one
    FP32 addition) and well above binary64's, so the option took effect;
    the factors agree within the perturbation bound; refinement reaches
    1e-9. eps=None: an all-FP64 map."""
    n, nb, Nt, A = case["n"], case["nb"], case["Nt"], case["A"]
    if eps is None:
        cm = np.zeros(Nt * (Nt + 1) // 2, dtype=np.uint8)
    else:
        cm = tc.precision_map(Nt, case["norms"], case["fro"], eps)
    ctx = tc.Context(n, nb, nrhs=3)
    Ad = to_dev(tc.pack_lower(A, nb))
    F = tc.factorize(ctx, Ad, n, nb, cmap=cm, fp64_update=tc.FP32)
    assert F.stats.info == 0 and F.mixed
    assert F.stats.class_flops[tc.FP64] == 0
    # every panel-update flop (SYRK nb^2 K, GEMM 2 nb^2 K per tile) is counted once
    upd = sum(nb ** 3 * k * (1 + 2 * (Nt - k - 1)) for k in range(Nt))
    assert sum(F.stats.class_flops) == upd
    assert list(F.stats.class_tiles) == np.bincount(cm, minlength=5).tolist()
    Lg = tc.unpack_lower(tc.export(ctx, F).cpu().numpy(), n, nb)
    for j in range(Nt):
        for i in range(j + 1, Nt):
            t = Lg[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
            c = int(cm[oracle.tile_index(Nt, i, j)])
            assert np.array_equal(oracle.round_tile(t, c)[0], t), (i, j, c)
    Lo, info = oracle.mxp_tile_cholesky(A, nb, cm, fp64_update=oracle.FP32)
    assert info == 0
    be_g, be_o = oracle.backward_error(A, Lg), oracle.backward_error(A, Lo)
    assert be_g <= 10 * be_o and be_g > 1e-12, (be_g, be_o)
    diff = np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo)
    assert diff <= 4 * case["kappa"] * (be_g + be_o) + 1e-13, diff
    B = si.standard_normal((n, 3), seed=si.rhs_seed(3))
    Bd = to_dev(np.ascontiguousarray(B.T))
    st = tc.solve_refine(ctx, F, Ad, Bd, max_iter=30, tol=1e-9)
    X = Bd.cpu().numpy().T
    rel = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert st["converged"] and rel.max() <= 1e-9, (st, rel.max())


# --- D_KL (Eq. 3 at y = 0) against the oracle's emulation -------------------

KL_N, KL_NB = 2048, 128


@pytest.fixture(scope="module")
def kl_mats():
    """Matern nu = 1/2 fields at the paper's weak and strong correlation
    (range 0.02627 and 0.210158), nugget 1e-4, 2048 Z-ordered points: the
    matrix, its tile norms and the oracle's FP64 log-determinant."""
    pts = si.points(KL_N, seed=3)
    out = {}
    for beta in (0.02627, 0.210158):
        A = oracle.matern_matrix(pts, 1.0, beta, 0.5, 1e-4)
        L, info = oracle.tile_cholesky(A, KL_NB, threads=8)
        assert info == 0
        norms = oracle.tile_norms(A, KL_NB)
        out[beta] = dict(A=A, norms=norms, fro=oracle.fro_norm(norms, KL_N // KL_NB),
                         ld0=oracle.logdet(L))
    return out


# (beta, eps, mode): "ratio2" -- D set by the stored tiles' rounding (the
# oracle's summation orders agree to 0.1%): same sign, within 2x;
# "ratio10" -- same sign, within 10x; "magnitude" -- D set by the FP32
# accumulation's rounding noise (the oracle's two orders disagree in sign):
# |D_gpu| <= 10 max(|D_oracle|, |D_oracle, reversed sums|).
KL_CELLS = [(0.02627, 1e-4, "ratio2"), (0.02627, 1e-5, "ratio10"),
            (0.210158, 1e-3, "ratio10"), (0.210158, 1e-5, "magnitude")]


@pytest.mark.parametrize("beta,eps,mode", KL_CELLS)
def test_kl_divergence_matches_oracle(tc, kl_mats, beta, eps, mode):
    n, nb = KL_N, KL_NB
    Nt = n // nb
    m = kl_mats[beta]
    A = m["A"]
    cm = tc.precision_map(Nt, m["norms"], m["fro"], eps)
    ctx = tc.Context(n, nb)
    Ad = to_dev(tc.pack_lower(A, nb))
    F64 = tc.factorize(ctx, Ad, n, nb)
    ld64_g = tc.logdet(ctx, F64)
    F64.close()
    F = tc.factorize(ctx, Ad, n, nb, cmap=cm)
    d_g = 0.5 * (tc.logdet(ctx, F) - ld64_g)
    Lo, info = oracle.mxp_tile_cholesky(A, nb, cm)
    assert info == 0
    d_o = 0.5 * (oracle.logdet(Lo) - m["ld0"])
    print("beta=%g eps=%g classes=%s D_gpu=%.4e D_oracle=%.4e" % (
        beta, eps, np.bincount(cm, minlength=5).tolist(), d_g, d_o))
    # the binary64 factors' own log-determinants agree to rounding
    assert abs(ld64_g - m["ld0"]) <= 1e-12 * abs(m["ld0"])
    if mode == "magnitude":
        Lr, _ = oracle.mxp_tile_cholesky(A, nb, cm, reverse_sums=True)
        d_r = 0.5 * (oracle.logdet(Lr) - m["ld0"])
        assert abs(d_g) <= 10 * max(abs(d_o), abs(d_r)), (d_g, d_o, d_r)
    else:
        f = 2.0 if mode == "ratio2" else 10.0
        assert d_g * d_o > 0 and abs(d_o) / f <= abs(d_g) <= f * abs(d_o), (d_g, d_o)


# --- the FP32 class's update in isolation ----------------------------------

def test_fp32_split_update_componentwise(tc):
    """One FP32-class tile's update, C_76 = A_76 - sum_{n<6} Lh_7n Lh_6n^T
    (K = 768), computed by the GPU on the FP16 matrix cores from the
    two-term split of each binary32 operand, against the same sum in binary64
    from the GPU's own stored binary32 operands. The operands span 2^30 in
    magnitude. The GPU's C is recovered from the stored L_76 = fl32(C
    L_66^{-T}) as Lh_76 L_66^T. Componentwise bound per entry (i, j), with
    P_ij = sum_l |a_il| |b_jl|:
      split: each operand x (scaled by its copy's 2^-ce into FP16's range)
        is held as hi + lo with |x - hi - lo| <= 2^-22 |x| + 2^-25 and
        |lo| <= 2^-11 |x|, so a product is off by at most
        3 * 2^-22 |a||b| plus the absolute terms 2^-25 (2^ce_b |a| +
        2^ce_a |b|) (dropped lo_a lo_b included);
      accumulation: FP32 over 3 nb products per tile column plus the fold
        of each tile column, gamma_{3 nb + Nt + 2} P_ij with u = 2^-24;
      storage: rounding X to binary32, 2^-24 (|X| |L_66|^T)_ij, and the
        binary64 TRSM, 1e-12 (|X| |L_66|^T)_ij.
    The binary32 GEMM of the same operands, emulated on the CPU, is within
    the same bound; the split's error is compared with it norm-wise too."""
    n, nb = 1024, 128
    Nt = n // nb
    rng = np.random.default_rng(19)
    L0 = np.tril(rng.standard_normal((n, n)) * np.exp2(-30.0 * rng.random((n, n))), -1) / np.sqrt(n)
    L0[np.arange(n), np.arange(n)] = 1.0 + rng.random(n)
    A = L0 @ L0.T
    cm = np.array([tc.FP64 if i == j else tc.FP32 for j in range(Nt) for i in range(j, Nt)],
                  dtype=np.uint8)
    ctx = tc.Context(n, nb)
    F = tc.factorize(ctx, to_dev(tc.pack_lower(A, nb)), n, nb, cmap=cm)
    assert F.stats.info == 0
    L = tc.unpack_lower(tc.export(ctx, F).cpu().numpy(), n, nb)

    def T(M, i, j):
        return M[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]

    m, k = Nt - 1, Nt - 2
    K = k * nb
    a = np.hstack([T(L, m, j) for j in range(k)])  # nb x K, binary32 values
    b = np.hstack([T(L, k, j) for j in range(k)])
    assert np.array_equal(a.astype(np.float32).astype(np.float64), a)
    span = np.log2(np.abs(a[a != 0]).max() / np.abs(a[a != 0]).min())
    assert span >= 30, span
    C = T(A, m, k) - a @ b.T
    Lkk = np.tril(T(L, k, k))
    X = T(L, m, k)
    Cg = X @ Lkk.T
    # copy scales: the largest entry of each operand tile in FP16's top
    # binade, e = ceil(log2(amax / 65504))
    def ce(t):
        r = float(np.abs(t).max()) / 65504.0
        e = int(np.frexp(r)[1]) - 1  # 2^e <= r < 2^(e+1)
        return e + 1 if np.ldexp(1.0, e) < r else e
    sa = np.hstack([np.full(nb, 2.0 ** (ce(T(L, m, j)) - 25)) for j in range(k)])
    sb = np.hstack([np.full(nb, 2.0 ** (ce(T(L, k, j)) - 25)) for j in range(k)])
    absa, absb = np.abs(a), np.abs(b)
    u32 = 2.0 ** -24
    mm = 3 * nb + Nt + 2
    gam = mm * u32 / (1 - mm * u32)
    P = absa @ absb.T
    # per product: 3 * 2^-22 |a||b| + 2^(ce_b - 25) |a| + 2^(ce_a - 25) |b| + s_a s_b
    bound = (3 * 2.0 ** -22 + gam) * P + (absa * sb[None, :]).sum(axis=1)[:, None] \
        + (absb * sa[None, :]).sum(axis=1)[None, :] + float(np.sum(sa * sb))
    XL = np.abs(X) @ np.abs(Lkk).T
    bound += (u32 + 1e-12) * XL
    err = np.abs(Cg - C)
    ratio = err / bound
    print("max err/bound %.3e, median %.3e" % (ratio.max(), np.median(ratio)))
    assert np.all(err <= bound), float(ratio.max())
    # norm-wise against a binary32 GEMM of the same operands (binary32
    # products and sums, emulated with numpy): the split keeps FP32's error
    # level; the GPU's recovered C also carries the rounding of X to binary32
    c32 = T(A, m, k) - (a.astype(np.float32) @ b.astype(np.float32).T).astype(np.float64)
    e32 = np.linalg.norm(c32 - C)
    eg = np.linalg.norm(Cg - C)
    print("||C_gpu - C|| = %.3e, ||C_fp32 - C|| = %.3e" % (eg, e32))
    assert eg <= 4 * e32 + 2 * u32 * np.linalg.norm(XL)
