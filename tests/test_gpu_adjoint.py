"""GPU parity of the log-likelihood gradient: the reverse sweep of the tile
Cholesky (C-ABI through the Python binding) against the CPU oracle.

What pins what:
  * Abar for the log-likelihood seed equals, for the lower-triangle
    convention, 2 dl/dSigma off the diagonal and dl/dSigma on it, where
    dl/dSigma = (alpha alpha^T - Sigma^{-1}) / 2 is the textbook closed form;
    the oracle computes alpha and Sigma^{-1} with its own substitutions.
  * For an arbitrary seed Lbar the sweep is the adjoint of the
    factorization's derivative: <Lbar, dL> = sum_{i>=j} Abar_ij E_ij for a
    symmetric direction E, with dL from central differences of the oracle's
    Cholesky (error O(h^2) + O(u/h), about 1e-9 relative here).
  * The gradient equals the oracle's trace formula (Eq. 1 differentiated,
    an independent route) within 1e-8 relative per component, and the
    log-likelihood equals the oracle's.
  * The FP32-mixed variant ({FP64, FP32} map at target 1e-7) against the
    FP64 oracle within the stated bound of 1e-4 relative.
  * At full size (n = 32768, nb = 512, 4000 base points translated), the
    gradient equals central differences of the GPU log-likelihood within
    1e-4 relative (step 1e-6 relative: truncation ~1e-12, rounding of l
    divided by the step ~1e-6 relative).
  * The memory-short form of the sweep (scratch of tc_adjoint_min_bytes:
    no transposed copy of Abar, mixed factors decoded one column at a time)
    gives the full form's Abar bit for bit, for binary64 and mixed factors
    over every class, at small sizes and at the full gradient size; the
    autograd function's "recompute" mode (factor and seed recomputed in
    backward) gives the "store" mode's log-likelihood and gradient.
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


def dev():
    import torch
    return torch.device("cuda", 0)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev())


def data(n, nu=0.5, theta0=(1.0, 0.1, 1e-4), base=4000, seed=4):
    pts = si.translated_points(n, base, seed=seed)
    A = oracle.matern_matrix(pts, theta0[0], theta0[1], nu, theta0[2])
    y = np.linalg.cholesky(A) @ si.standard_normal(n, seed=si.rhs_seed(seed))
    return pts, y


def gpu_loglik_grad(tc, pts, y, theta, nu, nb, ctx=None):
    """(l, grad, Abar as dense lower) through the C-ABI."""
    import torch
    n = len(pts)
    ctx = ctx or tc.Context(n, nb)
    locs = to_dev(pts)
    A, _, _ = tc.matern_tiles(ctx, locs, (theta[0], theta[1], nu, theta[2]), nb, norms=False)
    F = tc.factorize(ctx, A, n, nb, inplace=True)
    Lbar = torch.empty_like(A)
    ll = tc.loglik_seed(ctx, F, to_dev(y), Lbar)
    tc.factor_adjoint(ctx, F, Lbar)
    g = tc.matern_grad(ctx, locs, (theta[0], theta[1], nu, theta[2]), nb, Lbar)
    F.close()
    return ll, g, Lbar


@pytest.mark.parametrize("n,nb", [(1024, 256), (1536, 128), (768, 384)])
def test_abar_matches_closed_form(tc, n, nb):
    pts, y = data(n)
    th = (1.2, 0.08, 2e-4)
    ll, g, Lbar = gpu_loglik_grad(tc, pts, y, th, 0.5, nb)
    Ab = tc.unpack_lower(Lbar.cpu().numpy(), n, nb)
    A = oracle.matern_matrix(pts, th[0], th[1], 0.5, th[2])
    Lo, info = oracle.tile_cholesky(A, nb, threads=8)
    assert info == 0
    alpha = oracle.solve(Lo, y)
    Sinv = oracle.solve(Lo, np.eye(n))
    G = 0.5 * (np.outer(alpha, alpha) - Sinv)
    want = np.tril(2.0 * G, -1) + np.diag(np.diag(G))
    kappa = np.linalg.cond(A)
    err = np.linalg.norm(Ab - want) / np.linalg.norm(want)
    assert err <= 4 * kappa * n * U, (err, kappa)
    assert np.all(np.triu(Ab, 1) == 0.0)


@pytest.mark.parametrize("n,nb", [(256, 128), (384, 128), (768, 256)])
def test_adjoint_identity_random_seed(tc, n, nb):
    import torch
    L0 = si.random_factor(n, seed=n)
    A = L0 @ L0.T
    ctx = tc.Context(n, nb)
    F = tc.factorize(ctx, to_dev(tc.pack_lower(A, nb)), n, nb)
    Lb = np.tril(np.asarray(si.standard_normal((n, n), seed=n + 1)))
    P = tc.pack_lower(Lb, nb)
    # garbage in the strict upper triangle of the diagonal tiles is ignored
    Nt = n // nb
    for k in range(Nt):
        t = oracle.tile_index(Nt, k, k)
        tile = P[t * nb * nb:(t + 1) * nb * nb].reshape(nb, nb).T  # column-major view
        tile[np.triu_indices(nb, 1)] = 7.0
    Lbar = to_dev(P)
    tc.factor_adjoint(ctx, F, Lbar)
    Ab = tc.unpack_lower(Lbar.cpu().numpy(), n, nb)
    for d in range(3):
        E = np.asarray(si.standard_normal((n, n), seed=100 * n + d))
        E = E + E.T
        h = 1e-6 * np.linalg.norm(A) / np.linalg.norm(E)
        Lp, ip = oracle.tile_cholesky(A + h * E, nb, threads=8)
        Lm, im = oracle.tile_cholesky(A - h * E, nb, threads=8)
        assert ip == im == 0
        dL = (Lp - Lm) / (2 * h)
        lhs = float(np.sum(Lb * dL))
        rhs = float(np.sum(np.tril(Ab) * np.tril(E)))
        scale = float(np.sum(np.abs(Lb) * np.abs(dL)))
        assert abs(lhs - rhs) <= 1e-7 * scale, (lhs, rhs, scale)


@pytest.mark.parametrize("nu,n,nb", [(0.5, 1024, 256), (1.5, 1024, 128), (1.0, 1024, 256),
                                     (0.8, 768, 128), (2.5, 512, 128)])
def test_gradient_matches_trace_formula(tc, nu, n, nb):
    pts, y = data(n, nu=nu)
    th = (1.2, 0.08, 2e-4)
    ll, g, _ = gpu_loglik_grad(tc, pts, y, th, nu, nb)
    lo, go = oracle.loglik_grad(pts, y, th[0], th[1], nu, th[2], nb=nb)
    assert abs(ll - lo) <= 1e-10 * abs(lo), (ll, lo)
    for p in range(3):
        assert abs(g[p] - go[p]) <= 1e-8 * abs(go[p]), (p, g[p], go[p])


def test_autograd_function(tc):
    import torch
    n, nb = 1024, 256
    pts, y = data(n)
    ctx = tc.Context(n, nb)
    theta = torch.tensor([1.2, 0.08, 2e-4], dtype=torch.float64, requires_grad=True)
    ll = tc.matern_loglik(theta, to_dev(pts), to_dev(y), 0.5, nb, ctx)
    (2.0 * ll).backward()
    lo, go = oracle.loglik_grad(pts, y, 1.2, 0.08, 0.5, 2e-4, nb=nb)
    assert abs(float(ll.detach()) - lo) <= 1e-10 * abs(lo)
    gg = theta.grad.numpy()
    assert np.all(np.abs(gg - 2 * go) <= 1e-8 * np.abs(2 * go)), (gg, go)


def test_errors(tc):
    import torch
    n, nb = 512, 128
    L0 = si.random_factor(n, seed=5)
    ctx = tc.Context(n, nb)
    F = tc.factorize(ctx, to_dev(tc.pack_lower(L0 @ L0.T, nb)), n, nb)
    Lbar = torch.zeros(tc.num_tiles(n, nb) * nb * nb, dtype=torch.float64, device=dev())
    small = torch.empty(tc.adjoint_min_bytes(n, nb) - 8, dtype=torch.uint8, device=dev())
    with pytest.raises(tc.TileCholError) as e:
        tc.factor_adjoint(ctx, F, Lbar, scratch=small)
    assert e.value.status == tc.TC_ENOMEM
    # a mixed-precision factor needs room for its binary64 column decode
    cm = np.zeros(tc.num_tiles(n, nb), dtype=np.uint8)
    cm[1] = tc.FP32
    Fm = tc.factorize(ctx, to_dev(tc.pack_lower(L0 @ L0.T, nb)), n, nb, cmap=cm)
    assert Fm.mixed
    fp64_sized = torch.empty(tc.adjoint_min_bytes(n, nb), dtype=torch.uint8, device=dev())
    assert tc.adjoint_min_bytes(n, nb, True) > tc.adjoint_min_bytes(n, nb)
    with pytest.raises(tc.TileCholError) as e:
        tc.factor_adjoint(ctx, Fm, Lbar, scratch=fp64_sized)
    assert e.value.status == tc.TC_ENOMEM


def _random_seed_lbar(tc, n, nb, seed):
    """Random lower seed, packed, with garbage in the strict upper triangle
    of the diagonal tiles (which the sweep ignores)."""
    Lb = np.tril(np.asarray(si.standard_normal((n, n), seed=seed)))
    P = tc.pack_lower(Lb, nb)
    Nt = n // nb
    for k in range(Nt):
        t = oracle.tile_index(Nt, k, k)
        tile = P[t * nb * nb:(t + 1) * nb * nb].reshape(nb, nb).T
        tile[np.triu_indices(nb, 1)] = -3.0
    return P


@pytest.mark.parametrize("n,nb,eps,bf16", [(2048, 128, None, False), (1536, 256, None, False),
                                           (512, 512, None, False), (2048, 128, 1e-4, False),
                                           (1024, 256, 1e-6, False), (1536, 128, 1e-4, True)])
def test_short_form_equals_full_form(tc, n, nb, eps, bf16):
    """Memory-short sweep (scratch of exactly tc_adjoint_min_bytes, and one
    just below the full size) against the full form on the same factor and
    seed: Abar bit for bit. eps: a mixed factor under the map at that
    target over FP64/FP32/FP16/FP8 (bf16: BF16 in place of FP16), every
    stored class decoded column by column."""
    import torch
    pts = si.points(n, seed=11)
    A = oracle.matern_matrix(pts, 1.0, 0.03, 0.5, 1e-4)
    ctx = tc.Context(n, nb)
    Ad = to_dev(tc.pack_lower(A, nb))
    if eps is None:
        F = tc.factorize(ctx, Ad, n, nb)
    else:
        norms = oracle.tile_norms(A, nb)
        allowed = ((tc.FP64, tc.FP32, tc.BF16, tc.FP8E4M3) if bf16 else
                   (tc.FP64, tc.FP32, tc.FP16, tc.FP8E4M3))
        cm = tc.precision_map(n // nb, norms, oracle.fro_norm(norms, n // nb), eps,
                              allowed=allowed)
        assert len(set(cm.tolist())) >= 3 and (not bf16 or tc.BF16 in cm)
        F = tc.factorize(ctx, Ad, n, nb, cmap=cm)
        assert F.mixed
    assert F.stats.info == 0
    P = to_dev(_random_seed_lbar(tc, n, nb, seed=n + nb))
    full = P.clone()
    st_f = tc.factor_adjoint(ctx, F, full)
    lo = tc.adjoint_min_bytes(n, nb, F.mixed)
    hi = tc.adjoint_bytes(n, nb, F.mixed)
    assert lo < hi or n == nb
    for nbytes in sorted({lo, max(lo, hi - 8)}):
        short = P.clone()
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=dev())
        st_s = tc.factor_adjoint(ctx, F, short, scratch=scratch)
        assert torch.equal(full, short), (nbytes, float((full - short).abs().max()))
        assert st_s.flops_total == st_f.flops_total
    F.close()


@pytest.mark.parametrize("eps", [None, 1e-7])
def test_autograd_recompute_mode(tc, eps):
    """memory="recompute": nothing kept between the passes; backward
    factorizes again and sweeps in the memory-short form. Same
    log-likelihood and gradient as "store" (both binary64 and the
    FP32-mixed variant), and the FP64 oracle's gradient within 1e-8
    (binary64) or the stated 1e-4 (FP32-mixed)."""
    import torch
    n, nb = 1536, 128
    pts, y = data(n)
    th = (1.2, 0.08, 2e-4)
    ctx = tc.Context(n, nb)
    locs, yd = to_dev(pts), to_dev(y)
    out = {}
    for mode in ("store", "recompute", "auto"):
        theta = torch.tensor(th, dtype=torch.float64, requires_grad=True)
        ll = tc.matern_loglik(theta, locs, yd, 0.5, nb, ctx, eps=eps, memory=mode)
        resolved = ll.grad_fn.memory
        ll.backward()
        out[mode] = (float(ll.detach()), theta.grad.numpy().copy(), resolved)
    assert out["store"][2] == "store" and out["recompute"][2] == "recompute"
    assert out["auto"][2] == "store"  # ample free memory at this size
    ls, gs, _ = out["store"]
    lr, gr, _ = out["recompute"]
    assert lr == ls
    assert np.allclose(gr, gs, rtol=1e-13, atol=0), (gr, gs)
    print("recompute vs store gradient bitwise equal:", np.array_equal(gr, gs), flush=True)
    lo, go = oracle.loglik_grad(pts, y, th[0], th[1], 0.5, th[2], nb=nb)
    tol = 1e-8 if eps is None else 1e-4
    assert np.all(np.abs(gr - go) <= tol * np.abs(go)), (gr, go)
    with pytest.raises(ValueError):
        tc.matern_loglik(torch.tensor(th, dtype=torch.float64), locs, yd, 0.5, nb, ctx,
                         memory="never")


def test_fp32_mixed_gradient(tc):
    """The FP32-mixed variant: factorization under the {FP64, FP32} map at
    target accuracy 1e-7 (Section IV-C), gradient of the mixed factor
    against the FP64 oracle's trace formula. Stated bound: 1e-4 relative per
    component (the oracle's own emulation of the mixed factor is within
    3e-6 at this map); log-likelihood within 1e-6 relative."""
    import torch
    n, nb, eps = 2048, 128, 1e-7
    pts, y = data(n)
    th = (1.2, 0.08, 2e-4)
    ctx = tc.Context(n, nb)
    locs = to_dev(pts)
    full = (th[0], th[1], 0.5, th[2])
    A, tf, fro = tc.matern_tiles(ctx, locs, full, nb)
    cm = tc.precision_map(n // nb, tf.cpu().numpy(), fro, eps, allowed=(tc.FP64, tc.FP32))
    assert np.count_nonzero(cm == tc.FP32) > 40
    F = tc.factorize(ctx, A, n, nb, cmap=cm)
    assert F.mixed
    Lbar = torch.empty_like(A)
    ll = tc.loglik_seed(ctx, F, to_dev(y), Lbar)
    tc.factor_adjoint(ctx, F, Lbar)
    g = tc.matern_grad(ctx, locs, full, nb, Lbar)
    lo, go = oracle.loglik_grad(pts, y, th[0], th[1], 0.5, th[2], nb=nb)
    assert abs(ll - lo) <= 1e-6 * abs(lo), (ll, lo)
    assert np.all(np.abs(g - go) <= 1e-4 * np.abs(go)), (g, go)
    # the same through the autograd function
    theta = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    l2 = tc.matern_loglik(theta, locs, to_dev(y), 0.5, nb, ctx, eps=eps)
    l2.backward()
    assert abs(float(l2.detach()) - ll) <= 1e-12 * abs(ll)
    assert np.allclose(theta.grad.numpy(), g, rtol=1e-12, atol=0)


def _lower_matvec(tc, L, z, n, nb):
    """y = L z for packed lower tiles L (device), by tiles (input synthesis)."""
    import torch
    Nt = n // nb
    y = torch.zeros(n, dtype=torch.float64, device=L.device)
    for j in range(Nt):
        zj = z[j * nb:(j + 1) * nb]
        for i in range(j, Nt):
            t = oracle.tile_index(Nt, i, j)
            Lij = L[t * nb * nb:(t + 1) * nb * nb].view(nb, nb).t()
            if i == j:
                Lij = torch.tril(Lij)
            y[i * nb:(i + 1) * nb] += Lij @ zj
    return y


def test_full_size_gradient_central_differences(tc):
    """The gradient workload: n = 32768, nb = 512, 4000 base points
    translated, data y = L(theta0) z, gradient at theta_eval, in binary64
    and in the FP32-mixed variant."""
    import torch
    w = si.WORKLOADS["grad"]
    n, nb, nu = w["n"], w["nb"], w["nu"]
    pts = si.translated_points(n, w["base_points"], seed=w["seed"])
    locs = to_dev(pts)
    ctx = tc.Context(n, nb)
    A0, _, _ = tc.matern_tiles(ctx, locs, (w["sigma2"], w["range"], nu, w["nugget"]), nb,
                               norms=False)
    F0 = tc.factorize(ctx, A0, n, nb, inplace=True)
    z = to_dev(si.standard_normal(n, seed=si.rhs_seed(w["seed"])))
    y = _lower_matvec(tc, A0, z, n, nb)
    F0.close()
    del A0
    th = np.array(w["theta_eval"])

    def loglik(t):
        A, _, _ = tc.matern_tiles(ctx, locs, (t[0], t[1], nu, t[2]), nb, norms=False)
        F = tc.factorize(ctx, A, n, nb, inplace=True)
        Lb = torch.empty_like(A)
        v = tc.loglik_seed(ctx, F, y, Lb)
        F.close()
        return v

    A, _, _ = tc.matern_tiles(ctx, locs, (th[0], th[1], nu, th[2]), nb, norms=False)
    F = tc.factorize(ctx, A, n, nb, inplace=True)
    Lbar = torch.empty_like(A)
    l0 = tc.loglik_seed(ctx, F, y, Lbar)
    Lshort = Lbar.clone()
    st = tc.factor_adjoint(ctx, F, Lbar)
    g = tc.matern_grad(ctx, locs, (th[0], th[1], nu, th[2]), nb, Lbar)
    # the memory-short form at this size: the same Abar bit for bit
    st_s = tc.factor_adjoint(ctx, F, Lshort, short=True)
    assert torch.equal(Lshort, Lbar)
    F.close()
    del A, Lbar, Lshort
    torch.cuda.empty_cache()
    print("l =", l0, "grad =", g, "reverse sweep ms = %.1f (full), %.1f (memory-short)"
          % (st.ms_total, st_s.ms_total), flush=True)
    assert np.all(np.isfinite(g))
    fds = []
    for p in range(3):
        h = 1e-6 * th[p]
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (loglik(tp) - loglik(tm)) / (2 * h)
        fds.append(fd)
        print("p", p, "fd", fd, "adjoint", g[p], flush=True)
        assert abs(fd - g[p]) <= 1e-4 * abs(g[p]), (p, fd, g[p])
    # the FP32-mixed variant at the same size: {FP64, FP32} map at target
    # 1e-9 (Section IV-C), the forward factor in mixed precision and the
    # reverse sweep in binary64 on its upcast tiles; stated bound 1e-4
    # relative per component against the binary64 gradient and against the
    # central differences of the binary64 log-likelihood
    full = (th[0], th[1], nu, th[2])
    A, tf, fro = tc.matern_tiles(ctx, locs, full, nb)
    cm = tc.precision_map(n // nb, tf.cpu().numpy(), fro, 1e-9, allowed=(tc.FP64, tc.FP32))
    n32 = int(np.count_nonzero(cm == tc.FP32))
    assert n32 > 0
    Fm = tc.factorize(ctx, A, n, nb, cmap=cm)
    assert Fm.mixed and Fm.stats.info == 0
    del A
    Lbar = torch.empty(tc.num_tiles(n, nb) * nb * nb, dtype=torch.float64, device=dev())
    lm = tc.loglik_seed(ctx, Fm, y, Lbar)
    Lshort = Lbar.clone()
    tc.factor_adjoint(ctx, Fm, Lbar)
    gm = tc.matern_grad(ctx, locs, full, nb, Lbar)
    tc.factor_adjoint(ctx, Fm, Lshort, short=True)  # columns decoded one at a time
    assert torch.equal(Lshort, Lbar)
    Fm.close()
    del Lbar, Lshort
    torch.cuda.empty_cache()
    print("FP32-mixed (%d FP32 tiles): l = %r grad = %r" % (n32, lm, gm), flush=True)
    assert abs(lm - l0) <= 1e-6 * abs(l0), (lm, l0)
    for p in range(3):
        assert abs(gm[p] - g[p]) <= 1e-4 * abs(g[p]), (p, gm[p], g[p])
        assert abs(gm[p] - fds[p]) <= 1e-4 * abs(fds[p]), (p, gm[p], fds[p])
