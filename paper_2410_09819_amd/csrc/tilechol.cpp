// C ABI of libtilechol (declared in include/tilechol.h) and the host side of
// the static left-looking schedule (Section III-A/III-B, Algorithm 1).
//
// The schedule is fixed before any work is enqueued: for column of tiles
// k = 0..Nt-1,
//   1. panel update   C[k.., k] -= L[k.., 0:k] L[k, 0:k]^T  (one MFMA launch;
//                     SYRK on the diagonal tile, GEMM below it)
//   2. POTRF          of the diagonal tile (recursive halving inside the
//                     tile down to 128 x 128 leaves)
//   3. TRSM           of all tiles below it against L_kk^T (one launch)
// The paper's dependency table (Ready[m, n], busy-waited on by CPU threads)
// becomes stream order on one HIP stream: a step starts when the previous
// one has finished, which is exactly the set of dependencies Algorithm 1
// waits for. Nothing spins.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "tilechol.h"

struct tc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    uint32_t flags = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> gemm_ev;
};

struct tc_factor {
    int64_t n = 0;
    int nb = 0;
    int Nt = 0;
    double* tiles = nullptr;
    int info = 0;
};

namespace {

thread_local std::string g_err;

tc_status fail(tc_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define TC_HIP(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(TC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace regions (all carved from the caller's buffer):
//   info   : one int (failure flag)
//   big    : split-K partial sums of the panel and in-tile updates, and the
//            backward-solve partial sums (used one at a time, stream-ordered)
//   small  : Matern strip sums of squares, log-determinant partials
struct Layout {
    size_t info, big, small, total;
};

size_t big_bytes(int64_t n, int nb) {
    const int Nt = (int)(n / nb);
    size_t mx = 0;
    for (int k = 1; k < Nt; ++k) {
        const int s = tc::panel_splits(Nt, nb, k);
        if (s > 1) mx = std::max(mx, (size_t)s * (size_t)(Nt - k) * nb * nb * sizeof(double));
    }
    for (int m = nb / 2; m >= 128; m /= 2) {
        const int s = tc::syrk_sub_splits(m, m);
        if (s > 1) mx = std::max(mx, (size_t)s * m * m * sizeof(double));
    }
    // in-tile recursion sizes that are not halves (nb not a power of two times 128)
    for (int m = 128; m < nb; m += 128) {
        for (int kd = 128; kd < nb; kd += 128) {
            const int s = tc::syrk_sub_splits(m, kd);
            if (s > 1) mx = std::max(mx, (size_t)s * m * m * sizeof(double));
        }
    }
    mx = std::max(mx, (size_t)64 * nb * 16 * sizeof(double));  // backward-solve partials (<= 64 splits)
    return mx;
}

Layout layout(int64_t n, int nb) {
    const int64_t Nt = n / nb;
    const int64_t ntiles = Nt * (Nt + 1) / 2;
    Layout L;
    L.info = 0;
    L.big = align_up(sizeof(int) * 64);
    const size_t big = align_up(big_bytes(n, nb));
    L.small = L.big + big;
    const size_t small = align_up(std::max<size_t>((size_t)ntiles * tc::matern_strips(nb),
                                                   (size_t)Nt) * sizeof(double));
    L.total = L.small + small;
    return L;
}

bool valid_shape(int64_t n, int nb) {
    return n > 0 && nb >= 128 && nb <= 2048 && nb % 128 == 0 && n % nb == 0 && n / nb <= 65535;
}

tc_status check_shape(int64_t n, int nb) {
    if (!valid_shape(n, nb))
        return fail(TC_EINVAL, "invalid shape: n=" + std::to_string(n) + " nb=" + std::to_string(nb) +
                                   " (need nb in {128,256,...,2048} and n a positive multiple of nb)");
    return TC_OK;
}

tc_status check_ws(tc_ctx* ctx, int64_t n, int nb) {
    const Layout L = layout(n, nb);
    if (ctx->ws == nullptr || ctx->ws_bytes < L.total)
        return fail(TC_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes, have " +
                                   std::to_string(ctx->ws_bytes));
    return TC_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Recursive POTRF of the s x s block at offset o of a diagonal tile.
tc_status potrf_rec(tc_ctx* ctx, double* T, int nb, int o, int s, int64_t col0, int* info,
                    double* big) {
    if (s <= 128) {
        TC_HIP(tc::launch_potrf_leaf(ctx->stream, T + o + (int64_t)o * nb, nb, s, info, col0 + o));
        return TC_OK;
    }
    const int h = ((s / 2 + 127) / 128) * 128;
    tc_status st = potrf_rec(ctx, T, nb, o, h, col0, info, big);
    if (st != TC_OK) return st;
    double* L11 = T + o + (int64_t)o * nb;
    double* A21 = T + (o + h) + (int64_t)o * nb;
    double* A22 = T + (o + h) + (int64_t)(o + h) * nb;
    TC_HIP(tc::launch_trsm(ctx->stream, A21, L11, nb, s - h, h));
    TC_HIP(tc::launch_syrk_sub(ctx->stream, A22, A21, nb, s - h, h, big,
                               tc::syrk_sub_splits(s - h, h)));
    return potrf_rec(ctx, T, nb, o + h, s - h, col0, info, big);
}

}  // namespace

extern "C" {

int64_t tc_tile_offset(int32_t Nt, int32_t i, int32_t j) {
    if (Nt <= 0 || j < 0 || i < j || i >= Nt) return -1;
    return tc::tile_off(Nt, i, j);
}

const char* tc_version(void) { return "tilechol 0.1 (gfx950, FP64 MFMA)"; }

const char* tc_last_error(void) { return g_err.c_str(); }

size_t tc_workspace_bytes(int64_t n, int32_t nb, int32_t nrhs) {
    (void)nrhs;
    if (!valid_shape(n, nb)) return 0;
    return layout(n, nb).total;
}

tc_status tc_ctx_create(tc_ctx** out, int device, void* workspace, size_t workspace_bytes,
                        void* compute_stream, uint32_t flags) {
    if (!out) return fail(TC_EINVAL, "ctx is NULL");
    *out = nullptr;
    int ndev = 0;
    TC_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return fail(TC_EINVAL, "device " + std::to_string(device) + " out of range");
    DeviceGuard g(device);
    tc_ctx* c = new (std::nothrow) tc_ctx();
    if (!c) return fail(TC_ENOMEM, "out of host memory");
    c->device = device;
    c->stream = static_cast<hipStream_t>(compute_stream);
    c->ws = static_cast<char*>(workspace);
    c->ws_bytes = workspace ? workspace_bytes : 0;
    c->flags = flags;
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        delete c;
        return fail(TC_EHIP, "hipEventCreate failed");
    }
    *out = c;
    return TC_OK;
}

tc_status tc_ctx_destroy(tc_ctx* ctx) {
    if (!ctx) return TC_OK;
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    for (hipEvent_t e : ctx->gemm_ev) (void)hipEventDestroy(e);
    delete ctx;
    return TC_OK;
}

tc_status tc_matern_tiles(tc_ctx* ctx, int64_t n, int32_t nb, const double* locs,
                          const tc_matern* th, double* A, double* tile_fro, double* fro_A) {
    if (!ctx || !locs || !th || !A) return fail(TC_EINVAL, "NULL argument");
    if (tc_status s = check_shape(n, nb)) return s;
    if (!(th->sigma2 > 0) || !(th->range > 0) || !(th->nu > 0) || !(th->nugget >= 0))
        return fail(TC_EINVAL, "Matern parameters must satisfy sigma2, range, nu > 0, nugget >= 0");
    if (fro_A && !tile_fro) return fail(TC_EINVAL, "fro_A needs tile_fro");
    if (tc_status s = check_ws(ctx, n, nb)) return s;
    DeviceGuard g(ctx->device);
    const Layout Ly = layout(n, nb);
    double* strip = reinterpret_cast<double*>(ctx->ws + Ly.small);
    int kind = 3;
    if (th->nu == 0.5) kind = 0;
    else if (th->nu == 1.5) kind = 1;
    else if (th->nu == 2.5) kind = 2;
    const double norm_const = th->sigma2 / (std::pow(2.0, th->nu - 1.0) * std::tgamma(th->nu));
    TC_HIP(tc::launch_matern(ctx->stream, n, nb, locs, th->sigma2, 1.0 / th->range, th->nu, kind,
                             norm_const, th->nugget, A, strip));
    const int64_t Nt = n / nb;
    const int64_t ntiles = Nt * (Nt + 1) / 2;
    if (tile_fro) {
        TC_HIP(tc::launch_tile_norms(ctx->stream, ntiles, tc::matern_strips(nb), strip, tile_fro));
    }
    if (fro_A) {
        std::vector<double> h(ntiles);
        TC_HIP(hipMemcpyAsync(h.data(), tile_fro, ntiles * sizeof(double), hipMemcpyDeviceToHost,
                              ctx->stream));
        TC_HIP(hipStreamSynchronize(ctx->stream));
        double s = 0.0;
        for (int64_t j = 0; j < Nt; ++j)
            for (int64_t i = j; i < Nt; ++i) {
                const double v = h[tc::tile_off(Nt, i, j)];
                s += (i == j ? 1.0 : 2.0) * v * v;
            }
        *fro_A = std::sqrt(s);
    } else {
        TC_HIP(hipStreamSynchronize(ctx->stream));
    }
    return TC_OK;
}

size_t tc_factor_bytes(int64_t n, int32_t nb, const uint8_t* map) {
    if (!valid_shape(n, nb)) return 0;
    const int64_t Nt = n / nb;
    const int64_t ntiles = Nt * (Nt + 1) / 2;
    static const size_t bytes_of[5] = {8, 4, 2, 2, 1};
    if (!map) return (size_t)ntiles * nb * nb * sizeof(double);
    size_t tot = 0;
    for (int64_t t = 0; t < ntiles; ++t) {
        if (map[t] > 4) return 0;
        tot += bytes_of[map[t]] * (size_t)nb * nb;
    }
    return tot;
}

tc_status tc_factorize(tc_ctx* ctx, int64_t n, int32_t nb, const double* A, const uint8_t* map,
                       const tc_opts* opts, void* storage, size_t storage_bytes, tc_factor** Lout,
                       tc_stats* stats) {
    (void)opts;
    if (!ctx || !A || !storage || !Lout) return fail(TC_EINVAL, "NULL argument");
    *Lout = nullptr;
    if (tc_status s = check_shape(n, nb)) return s;
    const int Nt = (int)(n / nb);
    const int64_t ntiles = (int64_t)Nt * (Nt + 1) / 2;
    if (map) {
        for (int64_t t = 0; t < ntiles; ++t) {
            if (map[t] > 4) return fail(TC_EINVAL, "bad precision code in map");
            if (map[t] != TC_FP64)
                return fail(TC_EUNSUPPORTED, "mixed-precision maps are not implemented in this build");
        }
    }
    const size_t need = (size_t)ntiles * nb * nb * sizeof(double);
    if (storage_bytes < need)
        return fail(TC_EINVAL, "storage too small: need " + std::to_string(need) + " bytes");
    if (tc_status s = check_ws(ctx, n, nb)) return s;
    DeviceGuard g(ctx->device);
    const Layout Ly = layout(n, nb);
    int* d_info = reinterpret_cast<int*>(ctx->ws + Ly.info);
    double* big = reinterpret_cast<double*>(ctx->ws + Ly.big);
    double* L = static_cast<double*>(storage);
    const int64_t nb2 = (int64_t)nb * nb;
    const bool timed = (ctx->flags & 1u) != 0;
    if (timed && ctx->gemm_ev.size() < (size_t)2 * Nt) {
        while (ctx->gemm_ev.size() < (size_t)2 * Nt) {
            hipEvent_t e;
            TC_HIP(hipEventCreate(&e));
            ctx->gemm_ev.push_back(e);
        }
    }

    TC_HIP(hipEventRecord(ctx->ev0, ctx->stream));
    if (storage != (const void*)A)
        TC_HIP(hipMemcpyAsync(L, A, need, hipMemcpyDeviceToDevice, ctx->stream));
    TC_HIP(tc::launch_zero_info(ctx->stream, d_info));
    double gemm_flops = 0.0;
    int launches = 0;
    for (int k = 0; k < Nt; ++k) {
        if (k > 0) {
            const int sp = tc::panel_splits(Nt, nb, k);
            if (timed) TC_HIP(hipEventRecord(ctx->gemm_ev[2 * launches], ctx->stream));
            TC_HIP(tc::launch_panel_update(ctx->stream, L, Nt, nb, k, sp, big));
            if (timed) TC_HIP(hipEventRecord(ctx->gemm_ev[2 * launches + 1], ctx->stream));
            TC_HIP(tc::launch_panel_reduce(ctx->stream, L, Nt, nb, k, sp, big));
            // algorithmic flops: SYRK nb^2 * K (lower half) + GEMM 2 nb^2 K per tile below
            gemm_flops += (double)nb * nb * ((double)k * nb) * (1.0 + 2.0 * (Nt - k - 1));
            ++launches;
        }
        double* Tkk = L + tc::tile_off(Nt, k, k) * nb2;
        if (tc_status s = potrf_rec(ctx, Tkk, nb, 0, nb, (int64_t)k * nb, d_info, big)) return s;
        if (k + 1 < Nt)
            TC_HIP(tc::launch_trsm(ctx->stream, L + tc::tile_off(Nt, k + 1, k) * nb2, Tkk, nb,
                                   (int64_t)(Nt - k - 1) * nb, nb));
    }
    TC_HIP(hipEventRecord(ctx->ev1, ctx->stream));
    int info = 0;
    TC_HIP(hipMemcpyAsync(&info, d_info, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    TC_HIP(hipStreamSynchronize(ctx->stream));

    tc_factor* f = new (std::nothrow) tc_factor();
    if (!f) return fail(TC_ENOMEM, "out of host memory");
    f->n = n;
    f->nb = nb;
    f->Nt = Nt;
    f->tiles = L;
    f->info = info;
    *Lout = f;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        float ms = 0.f;
        TC_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        stats->ms_total = ms;
        if (timed) {
            double tot = 0.0;
            for (int i = 0; i < launches; ++i) {
                float m = 0.f;
                TC_HIP(hipEventElapsedTime(&m, ctx->gemm_ev[2 * i], ctx->gemm_ev[2 * i + 1]));
                tot += m;
            }
            stats->ms_gemm = tot;
        }
        stats->gemm_flops = gemm_flops;
        stats->gemm_launches = launches;
        stats->info = info;
        const double nd = (double)n;
        stats->flops_total = nd * nd * nd / 3.0;
    }
    if (info > 0) {
        g_err = "matrix is not positive definite (column " + std::to_string(info) + ")";
        return info;
    }
    return TC_OK;
}

tc_status tc_solve(tc_ctx* ctx, const tc_factor* F, double* B, int64_t ldb, int32_t nrhs) {
    if (!ctx || !F || !B) return fail(TC_EINVAL, "NULL argument");
    if (nrhs < 0 || ldb < F->n) return fail(TC_EINVAL, "bad nrhs or ldb");
    if (F->info > 0) return fail(TC_EINVAL, "factor is not valid (factorization failed)");
    if (nrhs == 0) return TC_OK;
    if (tc_status s = check_ws(ctx, F->n, F->nb)) return s;
    DeviceGuard g(ctx->device);
    const Layout Ly = layout(F->n, F->nb);
    double* big = reinterpret_cast<double*>(ctx->ws + Ly.big);
    const int Nt = F->Nt, nb = F->nb;
    const int64_t nb2 = (int64_t)nb * nb;
    const double* L = F->tiles;
    for (int k = 0; k < Nt; ++k) {
        const double* Lkk = L + tc::tile_off(Nt, k, k) * nb2;
        TC_HIP(tc::launch_trsv_diag(ctx->stream, Lkk, nb, B + (int64_t)k * nb, ldb, nrhs, false));
        if (k + 1 < Nt)
            TC_HIP(tc::launch_fwd_update(ctx->stream, L + tc::tile_off(Nt, k + 1, k) * nb2, nb,
                                         (int64_t)(Nt - k - 1) * nb, B + (int64_t)k * nb,
                                         B + (int64_t)(k + 1) * nb, ldb, nrhs));
    }
    for (int k = Nt - 1; k >= 0; --k) {
        if (k + 1 < Nt) {
            const int64_t rows = (int64_t)(Nt - k - 1) * nb;
            TC_HIP(tc::launch_bwd_update(ctx->stream, L + tc::tile_off(Nt, k + 1, k) * nb2, nb, rows,
                                         B + (int64_t)(k + 1) * nb, B + (int64_t)k * nb, ldb, nrhs,
                                         big, tc::bwd_splits(rows)));
        }
        const double* Lkk = L + tc::tile_off(Nt, k, k) * nb2;
        TC_HIP(tc::launch_trsv_diag(ctx->stream, Lkk, nb, B + (int64_t)k * nb, ldb, nrhs, true));
    }
    TC_HIP(hipStreamSynchronize(ctx->stream));
    return TC_OK;
}

tc_status tc_logdet(tc_ctx* ctx, const tc_factor* F, double* out) {
    if (!ctx || !F || !out) return fail(TC_EINVAL, "NULL argument");
    if (F->info > 0) return fail(TC_EINVAL, "factor is not valid (factorization failed)");
    if (tc_status s = check_ws(ctx, F->n, F->nb)) return s;
    DeviceGuard g(ctx->device);
    const Layout Ly = layout(F->n, F->nb);
    double* part = reinterpret_cast<double*>(ctx->ws + Ly.small);
    TC_HIP(tc::launch_logdet_partials(ctx->stream, F->tiles, F->Nt, F->nb, part));
    std::vector<double> h(F->Nt);
    TC_HIP(hipMemcpyAsync(h.data(), part, F->Nt * sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
    TC_HIP(hipStreamSynchronize(ctx->stream));
    double s = 0.0;
    for (double v : h) s += v;
    *out = 2.0 * s;
    return TC_OK;
}

tc_status tc_factor_export(tc_ctx* ctx, const tc_factor* F, double* L64) {
    if (!ctx || !F || !L64) return fail(TC_EINVAL, "NULL argument");
    DeviceGuard g(ctx->device);
    const int64_t ntiles = (int64_t)F->Nt * (F->Nt + 1) / 2;
    if (L64 != F->tiles)
        TC_HIP(hipMemcpyAsync(L64, F->tiles, (size_t)ntiles * F->nb * F->nb * sizeof(double),
                              hipMemcpyDeviceToDevice, ctx->stream));
    TC_HIP(tc::launch_zero_upper(ctx->stream, L64, F->Nt, F->nb));
    TC_HIP(hipStreamSynchronize(ctx->stream));
    return TC_OK;
}

tc_status tc_factor_destroy(tc_factor* F) {
    delete F;
    return TC_OK;
}

}  // extern "C"
