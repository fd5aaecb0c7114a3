"""Python binding of libtilechol: a tile-based left-looking Cholesky
factorization on one AMD Instinct MI355X (gfx950).

Argument marshalling only: every step of the factorization, solve,
log-determinant and covariance generation runs in the library's HIP
kernels. PyTorch supplies device memory and the stream. The binding fails
loudly if the library has not been built.

Method: arXiv 2410.09819, Section III-A (Algorithm 1: left-looking tile
Cholesky), Section III-B (static schedule), Section III-D (Matern
covariance, Eq. 2, and the Gaussian log-likelihood of Eq. 1).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libtilechol.so")

FP64, FP32, FP16, BF16, FP8E4M3 = 0, 1, 2, 3, 4
TC_OK, TC_EINVAL, TC_ENOMEM, TC_EHIP, TC_ENOTCONV, TC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5


class TileCholError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("tilechol error %d: %s" % (status, msg))
        self.status = status


class NotPositiveDefinite(TileCholError):
    def __init__(self, info: int, msg: str):
        super().__init__(info, msg)
        self.info = info


class Matern(ctypes.Structure):
    _fields_ = [("sigma2", ctypes.c_double), ("range", ctypes.c_double),
                ("nu", ctypes.c_double), ("nugget", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("inplace", ctypes.c_int32), ("fp64_update", ctypes.c_int32),
                ("wide_tiles", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class Stats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("ms_gemm", ctypes.c_double),
                ("gemm_flops", ctypes.c_double), ("gemm_launches", ctypes.c_int32),
                ("info", ctypes.c_int32), ("flops_total", ctypes.c_double),
                ("class_flops", ctypes.c_double * 5), ("class_tiles", ctypes.c_int32 * 5),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}
        d["class_flops"] = list(self.class_flops)
        d["class_tiles"] = list(self.class_tiles)
        return d


class IrStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("history", ctypes.c_double * 32),
                ("ms_total", ctypes.c_double)]

    def as_dict(self):
        return {"iterations": self.iterations, "converged": bool(self.converged),
                "rel_residual": self.rel_residual,
                "history": list(self.history[:min(self.iterations + 1, 32)]),
                "ms_total": self.ms_total}


class OocStats(ctypes.Structure):
    _fields_ = [("bytes_h2d", ctypes.c_uint64), ("bytes_d2h", ctypes.c_uint64),
                ("tiles_reloaded", ctypes.c_int32), ("evictions", ctypes.c_int32),
                ("chunks", ctypes.c_int32), ("cache_slots", ctypes.c_int32),
                ("ms_total", ctypes.c_double), ("flops_total", ctypes.c_double),
                ("info", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


_LIB = None
_vp = ctypes.c_void_p
_i32, _i64, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t


def lib():
    """The loaded libtilechol (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libtilechol.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "tc_tile_offset": (_i64, [_i32, _i32, _i32]),
        "tc_version": (ctypes.c_char_p, []),
        "tc_last_error": (ctypes.c_char_p, []),
        "tc_workspace_bytes": (_sz, [_i64, _i32, _i32]),
        "tc_ctx_create": (_i32, [ctypes.POINTER(_vp), ctypes.c_int, _vp, _sz, _vp, ctypes.c_uint32]),
        "tc_ctx_destroy": (_i32, [_vp]),
        "tc_matern_tiles": (_i32, [_vp, _i64, _i32, _vp, ctypes.POINTER(Matern), _vp, _vp,
                                   ctypes.POINTER(ctypes.c_double)]),
        "tc_factor_bytes": (_sz, [_i64, _i32, _vp, ctypes.POINTER(Opts)]),
        "tc_factorize": (_i32, [_vp, _i64, _i32, _vp, _vp, ctypes.POINTER(Opts), _vp, _sz,
                                ctypes.POINTER(_vp), ctypes.POINTER(Stats)]),
        "tc_solve": (_i32, [_vp, _vp, _vp, _i64, _i32]),
        "tc_solve_refine": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, _i32, ctypes.c_double,
                                   ctypes.POINTER(IrStats)]),
        "tc_precision_map": (_i32, [_i32, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_uint32,
                                    _i32, _vp]),
        "tc_logdet": (_i32, [_vp, _vp, ctypes.POINTER(ctypes.c_double)]),
        "tc_factorize_ooc": (_i32, [_vp, _i64, _i32, _vp, _vp, _vp, _sz, ctypes.POINTER(OocStats)]),
        "tc_ooc_mixed_host_bytes": (_sz, [_i64, _i32, _vp]),
        "tc_host_alloc": (_i32, [_sz, ctypes.POINTER(_vp)]),
        "tc_host_free": (_i32, [_vp]),
        "tc_ooc_mixed_cache_bytes": (_sz, [_i64, _i32, _vp, _i64, ctypes.POINTER(Opts)]),
        "tc_factorize_ooc_mixed": (_i32, [_vp, _i64, _i32, _vp, _vp, _vp, _sz, _vp, _sz,
                                          ctypes.POINTER(Opts), ctypes.POINTER(OocStats)]),
        "tc_factorize_noalloc": (_i32, [_vp, _i64, _i32, _vp, _vp, ctypes.POINTER(_i32)]),
        "tc_factor_export": (_i32, [_vp, _vp, _vp]),
        "tc_factor_destroy": (_i32, [_vp]),
        "tc_loglik_seed": (_i32, [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]),
        "tc_adjoint_bytes": (_sz, [_i64, _i32, _i32]),
        "tc_adjoint_min_bytes": (_sz, [_i64, _i32, _i32]),
        "tc_factor_adjoint": (_i32, [_vp, _vp, _vp, _vp, _sz, ctypes.POINTER(Stats)]),
        "tc_matern_grad": (_i32, [_vp, _i64, _i32, _vp, ctypes.POINTER(Matern), _vp,
                                  ctypes.POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def _check(status: int):
    if status == 0:
        return
    msg = (lib().tc_last_error() or b"").decode()
    if status > 0:
        raise NotPositiveDefinite(status, msg)
    raise TileCholError(status, msg)


# --- host-side helpers (no device work) -------------------------------------

def tile_offset(Nt: int, i: int, j: int) -> int:
    return lib().tc_tile_offset(Nt, i, j)


def workspace_bytes(n: int, nb: int, nrhs: int = 16) -> int:
    return lib().tc_workspace_bytes(n, nb, nrhs)


def factor_bytes(n: int, nb: int, cmap=None, fp64_update: int = 0) -> int:
    """Bytes of storage tc_factorize needs for this map (None: all FP64) and
    the arithmetic of the updates into FP64 tiles (FP64 or FP32)."""
    opts = Opts(0, fp64_update)
    if cmap is None:
        return lib().tc_factor_bytes(n, nb, None, ctypes.byref(opts))
    m = np.ascontiguousarray(cmap, dtype=np.uint8)
    return lib().tc_factor_bytes(n, nb, m.ctypes.data, ctypes.byref(opts))


def precision_map(Nt: int, tile_fro, fro: float, eps: float,
                  allowed=(FP64, FP32, FP16, FP8E4M3), unit_roundoff: bool = False) -> np.ndarray:
    """Per-tile class codes (uint8, packed order) from the tile norms
    (Section IV-C criterion, computed by the library on the host)."""
    tf = np.ascontiguousarray(np.asarray(tile_fro, dtype=np.float64))
    out = np.zeros(Nt * (Nt + 1) // 2, dtype=np.uint8)
    mask = 0
    for c in allowed:
        mask |= 1 << int(c)
    _check(lib().tc_precision_map(Nt, tf.ctypes.data, float(fro), float(eps), mask,
                                  1 if unit_roundoff else 0, out.ctypes.data))
    return out


def num_tiles(n: int, nb: int) -> int:
    Nt = n // nb
    return Nt * (Nt + 1) // 2


def pack_lower(A: np.ndarray, nb: int) -> np.ndarray:
    """Dense n x n -> packed lower tiles (layout conversion only)."""
    n = A.shape[0]
    Nt = n // nb
    out = np.empty(num_tiles(n, nb) * nb * nb, dtype=np.float64)
    t = 0
    for j in range(Nt):
        for i in range(j, Nt):
            out[t * nb * nb:(t + 1) * nb * nb] = np.ravel(A[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb],
                                                          order="F")
            t += 1
    return out


def unpack_lower(P: np.ndarray, n: int, nb: int, symmetric: bool = False) -> np.ndarray:
    """Packed lower tiles -> dense n x n (upper triangle outside the
    diagonal tiles zero, or mirrored when symmetric=True)."""
    Nt = n // nb
    A = np.zeros((n, n), dtype=np.float64, order="F")
    t = 0
    for j in range(Nt):
        for i in range(j, Nt):
            A[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb] = \
                P[t * nb * nb:(t + 1) * nb * nb].reshape(nb, nb, order="F")
            t += 1
    if symmetric:
        A = np.tril(A) + np.tril(A, -1).T
    return A


# --- device API -------------------------------------------------------------

class Context:
    """Device, stream and workspace for matrices up to order n with tile nb."""

    def __init__(self, n: int, nb: int, device: int = 0, stream=None, timed: bool = False,
                 nrhs: int = 16, ooc_sync: bool = False, ooc_no_reuse: bool = False,
                 ooc_lru: bool = False, ooc_no_v3: bool = False):
        import torch
        self.device = device
        self.dev = torch.device("cuda", device)
        nbytes = workspace_bytes(n, nb, nrhs)
        if nbytes == 0:
            raise TileCholError(TC_EINVAL, "invalid shape n=%d nb=%d" % (n, nb))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        h = _vp()
        _check(lib().tc_ctx_create(ctypes.byref(h), device, self.workspace.data_ptr(), nbytes,
                                   self.stream.cuda_stream,
                                   (1 if timed else 0) | (2 if ooc_sync else 0) | (4 if ooc_no_reuse else 0)
                                   | (8 if ooc_lru else 0) | (16 if ooc_no_v3 else 0)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().tc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def matern_tiles(ctx: Context, locs, theta, nb: int, out=None, norms: bool = True):
    """Packed lower Matern tiles (Eq. 2 + nugget) for device locations
    `locs` (n x 2 float64). theta = (sigma2, range, nu, nugget).
    Returns (A, tile_fro or None, fro_A or None)."""
    import torch
    n = locs.shape[0]
    assert locs.dtype == torch.float64 and locs.is_contiguous() and locs.shape[1] == 2
    th = Matern(*[float(v) for v in theta])
    A = out if out is not None else torch.empty(num_tiles(n, nb) * nb * nb, dtype=torch.float64,
                                                 device=locs.device)
    tf = torch.empty(num_tiles(n, nb), dtype=torch.float64, device=locs.device) if norms else None
    fro = ctypes.c_double(0.0)
    _check(lib().tc_matern_tiles(ctx.handle, n, nb, locs.data_ptr(), ctypes.byref(th),
                                 A.data_ptr(), tf.data_ptr() if norms else None,
                                 ctypes.byref(fro) if norms else None))
    return A, tf, (fro.value if norms else None)


class Factor:
    def __init__(self, handle, n, nb, storage, stats: Stats, mixed: bool = False):
        self.handle, self.n, self.nb, self.storage, self.stats = handle, n, nb, storage, stats
        self.mixed = mixed

    def close(self):
        if getattr(self, "handle", None):
            lib().tc_factor_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def factorize(ctx: Context, A, n: int, nb: int, cmap=None, inplace: bool = False,
              storage=None, fp64_update: int = 0, wide_tiles: int = 0) -> Factor:
    """Tile Cholesky of the packed lower tiles A (device float64). With
    inplace=True the factor overwrites A. fp64_update=FP32 computes the
    updates into FP64-class tiles (diagonal SYRK included) in the FP32
    class's arithmetic. wide_tiles: block shape of the low-class update
    kernels (tc_opts.wide_tiles: 0 auto, 1 256 x 256 when nb allows, -1
    128 x 128). Raises NotPositiveDefinite."""
    import torch
    if inplace:
        storage = A
    elif storage is None:
        storage = torch.empty(factor_bytes(n, nb, cmap, fp64_update) // 8, dtype=torch.float64,
                              device=A.device)
    m = None if cmap is None else np.ascontiguousarray(cmap, dtype=np.uint8)
    opts = Opts(1 if inplace else 0, fp64_update, wide_tiles)
    st = Stats()
    h = _vp()
    status = lib().tc_factorize(ctx.handle, n, nb, A.data_ptr(), None if m is None else m.ctypes.data,
                                ctypes.byref(opts), storage.data_ptr(),
                                storage.numel() * storage.element_size(), ctypes.byref(h),
                                ctypes.byref(st))
    F = Factor(h, n, nb, storage, st) if h.value else None
    if F is not None:
        F.mixed = (m is not None and bool(np.any(m != FP64))) or fp64_update != FP64
    if status != 0:
        if F is not None:
            F.close()
        _check(status)
    return F


def factorize_noalloc(ctx: Context, A, n: int, nb: int, out) -> int:
    """FP64 factorization of the packed lower tiles A (device float64) into
    `out` (device float64 of A's size; may be A) with the library's fixed
    per-GPU scratch instead of the context workspace (no device allocation).
    Returns 0; raises NotPositiveDefinite like factorize."""
    Nt = n // nb if nb > 0 else 0
    assert out.numel() >= Nt * (Nt + 1) // 2 * nb * nb and out.dtype == A.dtype
    info = _i32(0)
    _check(lib().tc_factorize_noalloc(ctx.handle, n, nb, A.data_ptr(), out.data_ptr(),
                                      ctypes.byref(info)))
    return info.value


def solve(ctx: Context, F: Factor, B):
    """In place: B <- Sigma^{-1} B. B is a device float64 tensor of shape
    (nrhs, n) (each row one right-hand side; column-major n x nrhs)."""
    assert B.is_contiguous() and B.shape[-1] == F.n
    nrhs = 1 if B.dim() == 1 else B.shape[0]
    _check(lib().tc_solve(ctx.handle, F.handle, B.data_ptr(), F.n, nrhs))
    return B


def solve_refine(ctx: Context, F: Factor, A, B, max_iter: int = 30, tol: float = 1e-9,
                 check: bool = True):
    """In place: B <- x refined to max_j ||b_j - A x_j|| / ||b_j|| <= tol, A the
    packed lower tiles that were factored. Returns the statistics dict;
    raises TileCholError(TC_ENOTCONV) when check is set and tol is not met."""
    assert B.is_contiguous() and B.shape[-1] == F.n
    nrhs = 1 if B.dim() == 1 else B.shape[0]
    st = IrStats()
    status = lib().tc_solve_refine(ctx.handle, F.handle, A.data_ptr(), B.data_ptr(), F.n, nrhs,
                                   max_iter, tol, ctypes.byref(st))
    if status != 0 and (check or status != TC_ENOTCONV):
        _check(status)
    return st.as_dict()


def factorize_ooc(ctx: Context, A_host, n: int, nb: int, cache, L_host=None) -> dict:
    """Out-of-core factorization: A_host (pinned CPU float64 tensor, packed
    lower tiles) streams through the device tile cache `cache` (a device
    tensor); the factor is written to L_host (default: in place over A_host).
    Returns the transfer statistics. Raises NotPositiveDefinite."""
    assert A_host.device.type == "cpu" and A_host.is_pinned()
    L_host = A_host if L_host is None else L_host
    assert L_host.device.type == "cpu" and L_host.is_pinned()
    st = OocStats()
    _check(lib().tc_factorize_ooc(ctx.handle, n, nb, A_host.data_ptr(), L_host.data_ptr(),
                                  cache.data_ptr(), cache.numel() * cache.element_size(),
                                  ctypes.byref(st)))
    return st.as_dict()


class PinnedBuffer:
    """Pinned host memory of an exact size (tc_host_alloc), exposed as a CPU
    uint8 tensor (`.tensor`, or typed views through `.view(dtype)`); freed
    by close() or when the object is collected. Views must not outlive it."""

    def __init__(self, nbytes: int):
        import torch
        p = _vp()
        _check(lib().tc_host_alloc(nbytes, ctypes.byref(p)))
        self._ptr = p
        self.nbytes = nbytes
        raw = (ctypes.c_uint8 * nbytes).from_address(p.value)
        self.tensor = torch.frombuffer(raw, dtype=torch.uint8)

    def view(self, dtype):
        return self.tensor.view(dtype)

    def close(self):
        if self._ptr is not None and self._ptr.value:
            self.tensor = None
            lib().tc_host_free(self._ptr)
        self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ooc_mixed_host_bytes(n: int, nb: int, cmap) -> int:
    """Bytes of the host image of an out-of-core mixed-precision factor
    (tiles in their classes, then one int32 scale exponent per tile)."""
    m = np.ascontiguousarray(cmap, dtype=np.uint8)
    b = lib().tc_ooc_mixed_host_bytes(n, nb, m.ctypes.data)
    if b == 0:
        raise TileCholError(TC_EINVAL, "invalid shape or precision map")
    return b


def ooc_mixed_cache_bytes(n: int, nb: int, cmap, slots: int, fp64_update: int = 0) -> int:
    """Device cache bytes of factorize_ooc_mixed with `slots` tile slots."""
    m = np.ascontiguousarray(cmap, dtype=np.uint8)
    opts = Opts(0, fp64_update)
    b = lib().tc_ooc_mixed_cache_bytes(n, nb, m.ctypes.data, slots, ctypes.byref(opts))
    if b == 0:
        raise TileCholError(TC_EINVAL, "invalid shape or precision map")
    return b


def factorize_ooc_mixed(ctx: Context, A_host, n: int, nb: int, cmap, cache, L_host=None,
                        fp64_update: int = 0, wide_tiles: int = 0):
    """Out-of-core mixed-precision factorization: A_host (pinned CPU float64
    tensor, packed lower tiles) streams through the device cache `cache`;
    the factor image (tiles in their classes, then the tile scale exponents)
    goes to L_host (pinned CPU uint8 tensor, allocated if None). fp64_update
    as in factorize (size the cache with the same value), wide_tiles as in
    factorize. Returns (transfer statistics, L_host). Raises
    NotPositiveDefinite."""
    import torch
    assert A_host.device.type == "cpu" and A_host.is_pinned()
    m = np.ascontiguousarray(cmap, dtype=np.uint8)
    nbytes = ooc_mixed_host_bytes(n, nb, m)
    if L_host is None:
        L_host = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    assert L_host.device.type == "cpu" and L_host.is_pinned()
    st = OocStats()
    _check(lib().tc_factorize_ooc_mixed(ctx.handle, n, nb, A_host.data_ptr(), m.ctypes.data,
                                        L_host.data_ptr(), L_host.numel() * L_host.element_size(),
                                        cache.data_ptr(), cache.numel() * cache.element_size(),
                                        ctypes.byref(Opts(0, fp64_update, wide_tiles)),
                                        ctypes.byref(st)))
    return st.as_dict(), L_host


def logdet(ctx: Context, F: Factor) -> float:
    out = ctypes.c_double(0.0)
    _check(lib().tc_logdet(ctx.handle, F.handle, ctypes.byref(out)))
    return out.value


def export(ctx: Context, F: Factor, out=None):
    """FP64 packed lower tiles of the factor with zero strict upper parts."""
    import torch
    if out is None:
        out = torch.empty(num_tiles(F.n, F.nb) * F.nb * F.nb, dtype=torch.float64,
                          device=F.storage.device)
    _check(lib().tc_factor_export(ctx.handle, F.handle, out.data_ptr()))
    return out


# --- log-likelihood gradient (reverse mode through the tile Cholesky) ------

def adjoint_bytes(n: int, nb: int, mixed: bool = False) -> int:
    """Scratch bytes of the full form of the reverse sweep."""
    return lib().tc_adjoint_bytes(n, nb, 1 if mixed else 0)


def adjoint_min_bytes(n: int, nb: int, mixed: bool = False) -> int:
    """Scratch bytes of the memory-short form of the reverse sweep."""
    return lib().tc_adjoint_min_bytes(n, nb, 1 if mixed else 0)


def loglik_seed(ctx: Context, F: Factor, y, Lbar=None) -> float:
    """Eq. 1's log-likelihood from the factor and y (device float64, n);
    fills Lbar (device, packed lower tiles) with dl/dL unless it is None."""
    assert y.is_contiguous() and y.numel() == F.n
    out = ctypes.c_double(0.0)
    _check(lib().tc_loglik_seed(ctx.handle, F.handle, y.data_ptr(),
                                None if Lbar is None else Lbar.data_ptr(), ctypes.byref(out)))
    return out.value


def factor_adjoint(ctx: Context, F: Factor, Lbar, scratch=None, short: bool = False) -> Stats:
    """In place: Lbar (dphi/dL, packed lower tiles) <- dphi/dA (lower
    triangle). Returns the sweep's statistics. Without a scratch buffer one
    is allocated: the full form's size, or the memory-short form's with
    short=True (the library picks the form from the scratch size)."""
    import torch
    nbytes = (adjoint_min_bytes if short else adjoint_bytes)(F.n, F.nb, F.mixed)
    if scratch is None:
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=Lbar.device)
    st = Stats()
    _check(lib().tc_factor_adjoint(ctx.handle, F.handle, Lbar.data_ptr(), scratch.data_ptr(),
                                   scratch.numel() * scratch.element_size(), ctypes.byref(st)))
    return st


def matern_grad(ctx: Context, locs, theta, nb: int, Abar):
    """(sum Abar dSigma/dsigma2, sum Abar dSigma/drange, sum Abar dSigma/dnugget)
    over the lower triangle; theta = (sigma2, range, nu, nugget)."""
    assert locs.is_contiguous() and locs.shape[1] == 2
    th = Matern(*[float(v) for v in theta])
    g = (ctypes.c_double * 3)()
    _check(lib().tc_matern_grad(ctx.handle, locs.shape[0], nb, locs.data_ptr(), ctypes.byref(th),
                                Abar.data_ptr(), g))
    return np.array(list(g))


def _autograd_function():
    import torch

    def make_factor(ctx, locs, full, nb, cm, A=None):
        """Factor of the covariance tiles A (generated when None): binary64
        in place, or mixed under the map cm."""
        n = locs.shape[0]
        if A is None:
            A, _, _ = matern_tiles(ctx, locs, full, nb, norms=False)
        if cm is None:
            return factorize(ctx, A, n, nb, inplace=True)
        return factorize(ctx, A, n, nb, cmap=cm)

    class MaternLogLik(torch.autograd.Function):
        """l(theta) of Eq. 1 for the Matern covariance with nugget, theta =
        (sigma2, range, nugget) as a float64 tensor, nu fixed. Forward:
        covariance tiles, tile Cholesky, log-likelihood and the reverse-mode
        seed. Backward: the blocked reverse sweep and the contraction with
        the covariance derivatives. With eps set, the factorization uses the
        {FP64, FP32} precision map at target accuracy eps (Section IV-C) and
        the gradient is that of the mixed-precision factor.

        memory: "store" keeps the factor and the seed dl/dL (a binary64 copy
        of the lower triangle) from forward to backward and sweeps in the
        full form; "recompute" keeps neither: backward regenerates the
        covariance tiles, factorizes again under the same map, seeds, and
        sweeps in the memory-short form (device memory of about the factor
        plus one triangle plus a few tile columns at its peak, none between
        the passes, for one more factorization); "auto" takes "recompute"
        when the free device memory at forward time cannot hold what
        "store" needs."""

        @staticmethod
        def forward(fctx, theta, locs, y, nu, nb, ctx, eps=None, memory="store"):
            if memory not in ("store", "recompute", "auto"):
                raise ValueError("memory must be 'store', 'recompute' or 'auto'")
            th = [float(v) for v in theta.detach().cpu().tolist()]
            n = locs.shape[0]
            full = (th[0], th[1], float(nu), th[2])
            cm, A = None, None
            if eps is not None:
                A, tf, fro = matern_tiles(ctx, locs, full, nb, norms=True)
                cm = precision_map(n // nb, tf.cpu().numpy(), fro, eps, allowed=(FP64, FP32))
            F = make_factor(ctx, locs, full, nb, cm, A)
            del A
            tri = num_tiles(n, nb) * nb * nb * 8
            if memory == "auto":  # room for the seed and the full sweep's scratch?
                torch.cuda.empty_cache()
                free, _ = torch.cuda.mem_get_info(locs.device)
                memory = "store" if free >= tri + adjoint_bytes(n, nb, F.mixed) else "recompute"
            if memory == "store":
                Lbar = torch.empty(tri // 8, dtype=torch.float64, device=locs.device)
                ll = loglik_seed(ctx, F, y, Lbar)
                fctx.state = (ctx, F, Lbar, locs, y, full, nb, cm)
            else:
                ll = loglik_seed(ctx, F, y, None)
                F.close()
                fctx.state = (ctx, None, None, locs, y, full, nb, cm)
            fctx.memory = memory
            return torch.tensor(ll, dtype=torch.float64, device=theta.device)

        @staticmethod
        def backward(fctx, gout):
            ctx, F, Lbar, locs, y, full, nb, cm = fctx.state
            fctx.state = None
            if F is None:  # recompute: factor and seed again, short sweep
                F = make_factor(ctx, locs, full, nb, cm)
                Lbar = torch.empty(num_tiles(F.n, nb) * nb * nb, dtype=torch.float64,
                                   device=locs.device)
                loglik_seed(ctx, F, y, Lbar)
                factor_adjoint(ctx, F, Lbar, short=True)
            else:
                factor_adjoint(ctx, F, Lbar)
            g = matern_grad(ctx, locs, full, nb, Lbar)
            F.close()
            grad = torch.from_numpy(g).to(device=gout.device, dtype=gout.dtype) * gout
            return grad, None, None, None, None, None, None, None

    return MaternLogLik


_MLL = None


def matern_loglik(theta, locs, y, nu: float, nb: int, ctx: Context, eps=None,
                  memory: str = "store"):
    """Differentiable log-likelihood (torch.autograd): see MaternLogLik."""
    global _MLL
    if _MLL is None:
        _MLL = _autograd_function()
    return _MLL.apply(theta, locs, y, nu, nb, ctx, eps, memory)


def __getattr__(name):
    if name == "MaternLogLik":
        global _MLL
        if _MLL is None:
            _MLL = _autograd_function()
        return _MLL
    raise AttributeError(name)
