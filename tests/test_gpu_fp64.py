"""GPU parity of the FP64 path (C-ABI through the Python binding) against
the CPU oracle.

Tolerances:
  * exact integer matrices: bitwise (every operation is exact in binary64);
  * factors of general SPD matrices: L is unique, but computed factors
    differ by rounding amplified by the conditioning, so the GPU factor is
    compared entrywise with the oracle's under the first-order perturbation
    bound ||dL||_F <= 4 kappa(A) n u ||L||_F, and its backward error
    ||A - L L^T||_F / ||A||_F must be <= 1e-12;
  * sampled checks at full size use the componentwise backward-error bound
    of Cholesky, |A - L L^T|_ij <= gamma_{n+1} (|L| |L|^T)_ij (valid for any
    summation order), plus the difference between the GPU's and the oracle's
    covariance entries.
"""
import math
import os

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
    tc.lib()  # raises if the HIP library is missing
    return tc


def dev():
    import torch
    return torch.device("cuda", 0)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev())


def gpu_factor(tc, A_dense, nb, ctx=None):
    n = A_dense.shape[0]
    ctx = ctx or tc.Context(n, nb)
    A = to_dev(tc.pack_lower(A_dense, nb))
    F = tc.factorize(ctx, A, n, nb)
    L = tc.unpack_lower(tc.export(ctx, F).cpu().numpy(), n, nb)
    return ctx, F, L


@pytest.mark.parametrize("n,nb", [(512, 128), (768, 256), (1024, 256), (1536, 384)])
def test_integer_factor_bitwise(tc, n, nb):
    L0 = si.integer_factor(n, seed=n + nb)
    _, F, L = gpu_factor(tc, L0 @ L0.T, nb)
    assert F.stats.info == 0
    assert np.array_equal(L, L0)


@pytest.mark.parametrize("n,nb,seed", [(256, 128, 11), (1280, 256, 12), (1152, 384, 13)])
def test_random_spd_matches_oracle(tc, n, nb, seed):
    L0 = si.random_factor(n, seed=seed)
    A = L0 @ L0.T
    _, F, L = gpu_factor(tc, A, nb)
    Lo, info = oracle.tile_cholesky(A, nb, threads=8)
    assert info == 0
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(L - Lo) <= 4 * kappa * n * U * np.linalg.norm(Lo)
    assert oracle.backward_error(A, L) <= 1e-14


def _small_workload_matrix(n=None):
    w = si.WORKLOADS["small"]
    n = n or w["n"]
    pts = si.points(n, seed=w["seed"])
    A = oracle.matern_matrix(pts, w["sigma2"], w["range"], w["nu"], w["nugget"])
    return w, pts, A


def test_small_workload_factor_logdet_solve(tc):
    import torch
    w, pts, A = _small_workload_matrix()
    n, nb = w["n"], w["nb"]
    ctx, F, L = gpu_factor(tc, A, nb)
    Lo, info = oracle.tile_cholesky(A, nb, threads=8)
    assert info == 0
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(L - Lo) <= 4 * kappa * n * U * np.linalg.norm(Lo)
    be = oracle.backward_error(A, L)
    assert be <= 1e-12, be
    ld = tc.logdet(ctx, F)
    assert abs(ld - oracle.logdet(Lo)) <= 1e-12 * abs(oracle.logdet(Lo)) + 1e-10
    for nrhs in (1, 16, 20):
        B = si.standard_normal((n, nrhs), seed=si.rhs_seed(w["seed"]) + nrhs)
        Bd = to_dev(np.ascontiguousarray(B.T))
        tc.solve(ctx, F, Bd)
        X = Bd.cpu().numpy().T
        Xo = oracle.solve(Lo, B)
        assert np.linalg.norm(X - Xo) <= 8 * kappa * n * U * np.linalg.norm(Xo)
        res = np.linalg.norm(B - A @ X, axis=0) / (np.linalg.norm(A, 2) * np.linalg.norm(X, axis=0))
        assert res.max() <= 1e-14


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5, 1.0, 0.8])
def test_matern_generator_matches_oracle(tc, nu):
    import torch
    n, nb = 1024, 256
    pts = si.points(n, seed=3)
    rng_, s2, tau2 = 0.05, 1.3, 1e-4
    ctx = tc.Context(n, nb)
    A, tf, fro = tc.matern_tiles(ctx, to_dev(pts), (s2, rng_, nu, tau2), nb)
    G = tc.unpack_lower(A.cpu().numpy(), n, nb)
    Ao = oracle.matern_matrix(pts, s2, rng_, nu, tau2)
    low = np.tril(np.ones((n, n), dtype=bool))
    err = np.abs(G - Ao)[low]
    assert np.all(err <= 2e-13 * np.abs(Ao[low]) + 1e-300)
    # diagonal tiles are filled in full (symmetric)
    for k in range(n // nb):
        blk = G[k * nb:(k + 1) * nb, k * nb:(k + 1) * nb]
        assert np.array_equal(blk, blk.T)
    norms = oracle.tile_norms(Ao, nb)
    assert np.allclose(tf.cpu().numpy(), norms, rtol=1e-13, atol=0)
    assert abs(fro - np.linalg.norm(Ao)) <= 1e-13 * np.linalg.norm(Ao)


def test_not_positive_definite_reports_column(tc):
    n, nb = 1024, 256
    for bad in (0, 300, 511, 1023):
        A = np.eye(n) * 4.0
        A[bad, bad] = -2.0
        _, info_o = oracle.tile_cholesky(A, nb)
        ctx = tc.Context(n, nb)
        with pytest.raises(tc.NotPositiveDefinite) as e:
            tc.factorize(ctx, to_dev(tc.pack_lower(A, nb)), n, nb)
        assert e.value.info == info_o == bad + 1


def test_errors_are_reported(tc):
    ctx = tc.Context(1024, 256)
    A = to_dev(np.zeros(tc.num_tiles(1024, 256) * 256 * 256))
    with pytest.raises(tc.TileCholError):
        tc.factorize(ctx, A, 1024, 200)
    cm = np.zeros(10, dtype=np.uint8)
    cm[0] = tc.FP32  # diagonal tiles must stay FP64
    with pytest.raises(tc.TileCholError) as e:
        tc.factorize(ctx, A, 1024, 256, cmap=cm)
    assert e.value.status == tc.TC_EINVAL
    small = tc.Context(256, 128)
    with pytest.raises(tc.TileCholError) as e:
        tc.factorize(small, A, 1024, 256)
    assert e.value.status == tc.TC_ENOMEM


def _rows_of_factor(L, n, nb, rows):
    """Rows of a packed lower factor (device tensor) as a dense (len(rows), n)
    host array."""
    import torch
    Nt = n // nb
    out = np.zeros((len(rows), n))
    Lh = None
    for q, i in enumerate(rows):
        it, r = divmod(int(i), nb)
        idx = []
        for jt in range(it + 1):
            t = oracle.tile_index(Nt, it, jt)
            idx.append(t * nb * nb + np.arange(nb) * nb + r)
        idx = torch.from_numpy(np.concatenate(idx)).to(L.device)
        vals = L[idx].cpu().numpy()
        out[q, :vals.size] = vals
    return out


def _probe_residual(A, L, n, nb, k=4, seed=0):
    """||(A - L L^T) G||_F / (||A G||_F) with Gaussian probes, by tiles."""
    import torch
    Nt = n // nb
    G = torch.from_numpy(si.standard_normal((n, k), seed=seed)).to(A.device)
    AG = torch.zeros_like(G)
    Z = torch.zeros_like(G)
    for j in range(Nt):
        for i in range(j, Nt):
            t = oracle.tile_index(Nt, i, j)
            Aij = A[t * nb * nb:(t + 1) * nb * nb].view(nb, nb).t()  # column-major tile
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


@pytest.mark.parametrize("name", ["small", "fp64"])
def test_workload_full_size_sampled(tc, name):
    """Full-size factorization in the benchmark's launch configuration:
    generated on the GPU, factored out of place, checked on sampled rows
    against the oracle's covariance entries and by a probe residual."""
    import torch
    w = si.WORKLOADS[name]
    n, nb = w["n"], w["nb"]
    theta = (w["sigma2"], w["range"], w["nu"], w["nugget"])
    pts = si.points(n, seed=w["seed"])
    ctx = tc.Context(n, nb)
    A, tf, fro = tc.matern_tiles(ctx, to_dev(pts), theta, nb)
    rng = np.random.default_rng(77)
    # sampled covariance entries
    Nt = n // nb
    I = rng.integers(0, n, 4000)
    J = rng.integers(0, n, 4000)
    I, J = np.maximum(I, J), np.minimum(I, J)
    t = np.array([oracle.tile_index(Nt, i // nb, j // nb) for i, j in zip(I, J)])
    pos = t * nb * nb + (J % nb) * nb + (I % nb)
    got = A[torch.from_numpy(pos).to(A.device)].cpu().numpy()
    want = oracle.matern_entries(pts, I, J, *theta)
    assert np.all(np.abs(got - want) <= 2e-13 * np.abs(want) + 1e-300)

    F = tc.factorize(ctx, A, n, nb)
    assert F.stats.info == 0
    L = tc.export(ctx, F, out=F.storage)
    rows = np.sort(rng.choice(n, 48, replace=False))
    R = _rows_of_factor(L, n, nb, rows)
    LLt = R @ R.T
    bound = (n + 1) * U / (1 - (n + 1) * U) * (np.abs(R) @ np.abs(R).T)
    Aij = oracle.matern_entries(pts, rows[:, None], rows[None, :], *theta)
    assert np.all(np.abs(LLt - Aij) <= 2 * bound + 2e-13 * np.abs(Aij))
    pr = _probe_residual(A, L, n, nb)
    assert pr <= 1e-12, pr
