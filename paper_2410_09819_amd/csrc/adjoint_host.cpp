// Reverse sweep of the tile Cholesky and the Matern gradient contraction:
// the host side of adjoint.hip. Column n = Nt-1 ... 0 (left-looking):
//   X = L_nn^{-T}                          (TRSM of an identity tile)
//   PL = transposed tiles of L's column n below the diagonal
//   Lbar_mn -= sum_{k>n} S_mk L_kn          (adj_panel, split-K)
//   Abar_mn = Lbar_mn X^T; kept in place and transposed into Tt
//   Lbar_nn -= tril(Tt_panel PL^T)
//   P = tril(L_nn)^T tril(Lbar_nn), mirrored; H = X P X^T into Tt(n, n);
//   Abar_nn = tril(H), diagonal halved.
// Scratch (caller's device buffer): Tt (packed lower tiles), PL, Tb (one
// column panel each), five nb x nb tiles, and the split-K partial sums.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_common.hpp"

using namespace tc::host;

namespace {

struct AdjLayout {
    size_t tt, pl, tb, sq, part, l64, total;  // offsets in doubles, total in bytes
};

size_t adj_partial_doubles(int Nt, int nb) {
    const int64_t nb2 = (int64_t)nb * nb;
    size_t mx = 0;
    for (int n = 0; n < Nt; ++n) {
        const int64_t R = Nt - n - 1;
        if (R > 0) {
            const int s = tc::adj_panel_splits(Nt, nb, n);
            if (s > 1) mx = std::max(mx, (size_t)s * R * nb2);
            mx = std::max(mx, tc::adj_gemm_plan(R * nb, nb, nb, false).partial_doubles);
            mx = std::max(mx, tc::adj_gemm_plan(nb, nb, R * nb, true).partial_doubles);
        }
    }
    mx = std::max(mx, tc::adj_gemm_plan(nb, nb, nb, false).partial_doubles);
    return mx;
}

AdjLayout adj_layout(int64_t n, int nb, bool mixed) {
    const int64_t Nt = n / nb;
    const int64_t nb2 = (int64_t)nb * nb;
    const int64_t panel = std::max<int64_t>(Nt - 1, 1) * nb2;
    AdjLayout L;
    L.tt = 0;
    L.pl = L.tt + (size_t)(Nt * (Nt + 1) / 2) * nb2;
    L.tb = L.pl + panel;
    L.sq = L.tb + panel;
    L.part = L.sq + 5 * nb2;
    L.l64 = L.part + adj_partial_doubles((int)Nt, nb) + 32;
    // a mixed-precision factor is swept in binary64: room for its upcast tiles
    L.total = (L.l64 + (mixed ? (size_t)(Nt * (Nt + 1) / 2) * nb2 : 0)) * sizeof(double);
    return L;
}

inline tc::AdjMat tiles_mat(double* p, int nb) {  // a column of tiles
    return tc::AdjMat{p, nb, nb, (int64_t)nb * nb};
}
inline tc::AdjMat plain_mat(double* p, int nb) {  // nb rows, column-major, ld nb
    return tc::AdjMat{p, nb, nb, 0};
}

}  // namespace

extern "C" {

size_t tc_adjoint_bytes(int64_t n, int32_t nb, int32_t mixed) {
    if (!valid_shape(n, nb)) return 0;
    return adj_layout(n, nb, mixed != 0).total;
}

tc_status tc_factor_adjoint(tc_ctx* ctx, const tc_factor* F, double* Lbar, void* scratch,
                            size_t scratch_bytes, tc_stats* stats) {
    if (!ctx || !F || !Lbar || !scratch) return fail(TC_EINVAL, "NULL argument");
    if (F->info > 0) return fail(TC_EINVAL, "factor is not valid (factorization failed)");
    const int64_t n = F->n;
    const int nb = F->nb, Nt = F->Nt;
    const AdjLayout Ly = adj_layout(n, nb, F->mixed);
    if (scratch_bytes < Ly.total)
        return fail(TC_ENOMEM, "adjoint scratch too small: need " + std::to_string(Ly.total) +
                                   " bytes, have " + std::to_string(scratch_bytes));
    if (tc_status s = check_ws(ctx, n, nb)) return s;
    DeviceGuard g(ctx->device);
    hipStream_t st = ctx->stream;
    const int64_t nb2 = (int64_t)nb * nb;
    double* S = static_cast<double*>(scratch);
    double* Tt = S + Ly.tt;
    double* PL = S + Ly.pl;
    double* Tb = S + Ly.tb;
    double* X = S + Ly.sq;
    double* W1 = X + nb2;
    double* W2 = W1 + nb2;
    double* P = W2 + nb2;
    double* Y = P + nb2;
    double* part = S + Ly.part;
    const double* L = F->tiles;
    if (F->mixed) {  // sweep the upcast factor
        double* L64 = S + Ly.l64;
        TC_HIP(tc::launch_export(st, factor_view(F), L64));
        L = L64;
    }
    const bool timed = (ctx->flags & 1u) != 0;
    while (timed && ctx->gemm_ev.size() < (size_t)2 * Nt) {
        hipEvent_t e;
        TC_HIP(hipEventCreate(&e));
        ctx->gemm_ev.push_back(e);
    }
    double panel_flops = 0.0, flops = 0.0;
    int launches = 0;
    TC_HIP(hipEventRecord(ctx->ev0, st));
    for (int nn = Nt - 1; nn >= 0; --nn) {
        const int64_t R = Nt - nn - 1;
        const double* Lnn = L + tc::tile_off(Nt, nn, nn) * nb2;
        double* Lbnn = Lbar + tc::tile_off(Nt, nn, nn) * nb2;
        TC_HIP(tc::launch_set_identity(st, X, nb));
        TC_HIP(tc::launch_trsm(st, X, Lnn, nb, nb, nb));  // X = L_nn^{-T}
        flops += (double)nb * nb * nb;
        if (R > 0) {
            const int64_t off = tc::tile_off(Nt, nn + 1, nn) * nb2;
            double* Lbp = Lbar + off;
            double* Ttp = Tt + off;
            TC_HIP(tc::launch_transpose_tiles(st, L + off, PL, nb, R, false));
            const int sp = tc::adj_panel_splits(Nt, nb, nn);
            if (timed) TC_HIP(hipEventRecord(ctx->gemm_ev[2 * launches], st));
            TC_HIP(tc::launch_adj_panel(st, Lbar, Tt, PL, Nt, nb, nn, sp, part));
            if (timed) TC_HIP(hipEventRecord(ctx->gemm_ev[2 * launches + 1], st));
            ++launches;
            const double pf = 2.0 * (double)(R * nb) * nb * (double)(R * nb);
            panel_flops += pf;
            flops += pf;
            // Abar_mn = Lbar_mn L_nn^{-1}
            TC_HIP(tc::launch_adj_gemm(st, tiles_mat(Tb, nb), tiles_mat(Lbp, nb), plain_mat(X, nb),
                                       R * nb, nb, nb, false, false, part));
            flops += 2.0 * (double)(R * nb) * nb * nb;
            TC_HIP(hipMemcpyAsync(Lbp, Tb, (size_t)R * nb2 * sizeof(double),
                                  hipMemcpyDeviceToDevice, st));
            TC_HIP(tc::launch_transpose_tiles(st, Tb, Ttp, nb, R, false));
            // Lbar_nn -= tril(sum_m Abar_mn^T L_mn)
            TC_HIP(tc::launch_adj_gemm(st, plain_mat(Lbnn, nb), plain_mat(Ttp, nb),
                                       plain_mat(PL, nb), nb, nb, R * nb, true, true, part));
            flops += (double)nb * nb * (double)(R * nb);
        }
        // reverse of the diagonal tile's POTRF
        TC_HIP(tc::launch_transpose_tiles(st, Lnn, W1, nb, 1, true));
        TC_HIP(tc::launch_transpose_tiles(st, Lbnn, W2, nb, 1, true));
        TC_HIP(tc::launch_adj_gemm(st, plain_mat(P, nb), plain_mat(W1, nb), plain_mat(W2, nb), nb,
                                   nb, nb, false, false, part));
        TC_HIP(tc::launch_mirror_lower(st, P, nb));
        TC_HIP(tc::launch_adj_gemm(st, plain_mat(Y, nb), plain_mat(X, nb), plain_mat(P, nb), nb,
                                   nb, nb, false, false, part));
        double* H = Tt + tc::tile_off(Nt, nn, nn) * nb2;
        TC_HIP(tc::launch_adj_gemm(st, plain_mat(H, nb), plain_mat(Y, nb), plain_mat(X, nb), nb,
                                   nb, nb, false, false, part));
        TC_HIP(tc::launch_finish_diag(st, H, Lbnn, nb));
        flops += 6.0 * (double)nb * nb * nb;
    }
    TC_HIP(hipEventRecord(ctx->ev1, st));
    TC_HIP(hipStreamSynchronize(st));
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
        stats->gemm_flops = panel_flops;
        stats->gemm_launches = launches;
        stats->flops_total = flops;
        stats->class_flops[TC_FP64] = flops;
    }
    return TC_OK;
}

tc_status tc_matern_grad(tc_ctx* ctx, int64_t n, int32_t nb, const double* locs,
                         const tc_matern* th, const double* Abar, double grad[3]) {
    if (!ctx || !locs || !th || !Abar || !grad) return fail(TC_EINVAL, "NULL argument");
    if (tc_status s = check_shape(n, nb)) return s;
    if (!(th->sigma2 > 0) || !(th->range > 0) || !(th->nu > 0) || !(th->nugget >= 0))
        return fail(TC_EINVAL, "Matern parameters must satisfy sigma2, range, nu > 0, nugget >= 0");
    if (tc_status s = check_ws(ctx, n, nb)) return s;
    DeviceGuard g(ctx->device);
    const Layout Ly = layout(n, nb);
    double* part = reinterpret_cast<double*>(ctx->ws + Ly.small);
    int kind = 3;
    if (th->nu == 0.5) kind = 0;
    else if (th->nu == 1.5) kind = 1;
    else if (th->nu == 2.5) kind = 2;
    const double norm_const = th->sigma2 / (std::pow(2.0, th->nu - 1.0) * std::tgamma(th->nu));
    const int64_t Nt = n / nb;
    const int64_t count = Nt * (Nt + 1) / 2 * tc::matern_strips(nb);
    double* out = part + 3 * count;
    TC_HIP(tc::launch_matern_grad(ctx->stream, n, nb, locs, th->sigma2, 1.0 / th->range, th->nu,
                                  kind, norm_const, Abar, part));
    TC_HIP(tc::launch_sum3(ctx->stream, part, count, out));
    TC_HIP(hipMemcpyAsync(grad, out, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    TC_HIP(hipStreamSynchronize(ctx->stream));
    return TC_OK;
}

}  // extern "C"
