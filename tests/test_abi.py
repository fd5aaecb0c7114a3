"""The C-ABI library loads and exports every entry point that
include/tilechol.h declares; host-only entry points and layout helpers
behave as documented (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tilechol.h")


def _lib():
    import paper_2410_09819_amd as tc
    if not os.path.exists(tc.LIB_PATH):
        from paper_2410_09819_amd import build
        build.build()
    return tc


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared_functions()
    for f in ("tc_factorize", "tc_solve", "tc_logdet", "tc_matern_tiles", "tc_ctx_create",
              "tc_factor_export", "tc_tile_offset", "tc_last_error"):
        assert f in names


def test_every_declared_symbol_is_exported():
    tc = _lib()
    raw = ctypes.CDLL(tc.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(raw, f)]
    assert not missing, missing


def test_tile_offset_matches_packed_order():
    tc = _lib()
    Nt = 9
    offs = [tc.tile_offset(Nt, i, j) for j in range(Nt) for i in range(j, Nt)]
    assert offs == list(range(Nt * (Nt + 1) // 2))
    assert tc.tile_offset(Nt, 2, 3) == -1 and tc.tile_offset(Nt, 9, 0) == -1


def test_sizes_and_validation():
    tc = _lib()
    assert tc.factor_bytes(2048, 256) == 36 * 256 * 256 * 8
    cm = np.array([tc.FP64] * 36, dtype=np.uint8)
    cm[1] = tc.FP32
    cm[2] = tc.FP8E4M3
    # tiles in their classes, plus operand copies and tables
    assert tc.factor_bytes(2048, 256, cm) >= (34 * 8 + 4 + 1) * 256 * 256
    assert tc.workspace_bytes(2048, 256) > 0
    for n, nb in [(2048, 100), (2000, 256), (0, 256), (4096, 4096)]:
        assert tc.workspace_bytes(n, nb) == 0
        assert tc.factor_bytes(n, nb) == 0
    L = tc.lib()
    st = L.tc_factorize(None, 2048, 256, None, None, None, None, 0, None, None)
    assert st == tc.TC_EINVAL
    assert b"NULL" in L.tc_last_error()
    assert L.tc_version().startswith(b"tilechol")


def test_adjoint_scratch_sizes():
    """Full form: transposed copies of every Abar tile (+ the binary64
    upcast of a mixed factor); memory-short form: H_m per tile row (+ one
    decoded column). Both share three tile columns' worth of panels and
    tiles and the same split-K partials, so their difference is exact."""
    tc = _lib()
    for n, nb in [(32768, 512), (4096, 256), (512, 512)]:
        Nt = n // nb
        tri = Nt * (Nt + 1) // 2 * nb * nb * 8
        col = Nt * nb * nb * 8
        full, short = tc.adjoint_bytes(n, nb), tc.adjoint_min_bytes(n, nb)
        fullm, shortm = tc.adjoint_bytes(n, nb, True), tc.adjoint_min_bytes(n, nb, True)
        assert full - short == tri - col
        assert fullm - full == tri and shortm - short == col
        assert short < full or Nt == 1
    # the gradient workload: about 0.9 GiB instead of 4.8 GiB of scratch
    assert tc.adjoint_min_bytes(32768, 512) < tc.adjoint_bytes(32768, 512) / 4
    assert tc.adjoint_min_bytes(2000, 256) == 0 == tc.adjoint_bytes(2000, 256)


def test_pack_unpack_roundtrip():
    tc = _lib()
    rng = np.random.default_rng(0)
    n, nb = 640, 128
    M = rng.standard_normal((n, n))
    A = M + M.T
    P = tc.pack_lower(A, nb)
    assert P.size == tc.num_tiles(n, nb) * nb * nb
    B = tc.unpack_lower(P, n, nb, symmetric=True)
    assert np.array_equal(B, A)
    # tile (3,1) sits where tile_offset says, column-major
    t = tc.tile_offset(n // nb, 3, 1)
    assert np.array_equal(P[t * nb * nb:(t + 1) * nb * nb].reshape(nb, nb, order="F"),
                          A[3 * nb:4 * nb, nb:2 * nb])


@pytest.mark.parametrize("eps", [1e-3, 1e-5, 1e-7, 1e-9])
@pytest.mark.parametrize("unit", [False, True])
def test_library_precision_map_equals_oracle(eps, unit):
    """tc_precision_map (host code in the library) takes the same decisions
    as the oracle's criterion on the same norms."""
    import oracle
    import seeded_inputs as si
    tc = _lib()
    n, nb = 2048, 128
    A = oracle.matern_matrix(si.points(n, seed=3), 1.0, 0.03, 0.5, 1e-4)
    Nt = n // nb
    norms = oracle.tile_norms(A, nb)
    fro = oracle.fro_norm(norms, Nt)
    for allowed in [(0, 1, 2, 4), (0, 1), (0, 3, 4), (0, 1, 2, 3, 4)]:
        got = tc.precision_map(Nt, norms, fro, eps, allowed=allowed, unit_roundoff=unit)
        want = oracle.precision_map(norms, fro, Nt, eps, allowed=allowed, unit_roundoff=unit)
        assert np.array_equal(got, want)


def test_mixed_factor_bytes_cover_tiles():
    tc = _lib()
    Nt, nb = 6, 128
    cm = np.zeros(Nt * (Nt + 1) // 2, dtype=np.uint8)
    cm[[1, 2, 3]] = [tc.FP32, tc.FP16, tc.FP8E4M3]
    # tiles in their classes, and L_kk^{-T} of the Nt diagonal tiles for the solves
    assert tc.factor_bytes(Nt * nb, nb, cm) > (18 * 8 + 4 + 2 + 1 + Nt * 8) * nb * nb
    bad = cm.copy()
    bad[0] = tc.FP32  # diagonal tile must stay FP64
    assert tc.factor_bytes(Nt * nb, nb, bad) == 0


def test_fp32_update_factor_bytes():
    """With the updates into FP64 tiles in FP32 arithmetic, every
    off-diagonal tile (an operand of a later column or of its row's
    diagonal SYRK) also gets an FP32 operand copy (two FP16 planes), even
    for an all-FP64 map; other arithmetic codes are rejected."""
    tc = _lib()
    Nt, nb = 6, 128
    ntiles = Nt * (Nt + 1) // 2
    cm = np.zeros(ntiles, dtype=np.uint8)
    plain = tc.factor_bytes(Nt * nb, nb, cm)
    assert plain == ntiles * nb * nb * 8
    low = tc.factor_bytes(Nt * nb, nb, cm, fp64_update=tc.FP32)
    assert low >= (ntiles * 8 + (ntiles - Nt) * 4) * nb * nb
    assert tc.factor_bytes(Nt * nb, nb, None, fp64_update=tc.FP32) == low
    assert tc.factor_bytes(Nt * nb, nb, cm, fp64_update=tc.FP16) == 0
