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
//
// Memory-short form, taken when the scratch holds less than the full form
// needs: Abar stays only in Lbar (the panel reads Abar_km^T from there),
// the H_m tiles go to a one-column array instead of Tt's diagonal, and a
// mixed-precision factor is not upcast as a whole: each column's tiles are
// decoded to binary64 again when the sweep reaches that column. Scratch
// shrinks from about one factor (two, for a mixed factor) to about three
// tile columns plus the partial sums; Abar is the same bit for bit.
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
    // offsets in doubles, total in bytes; full form: tt (packed lower
    // tiles) and l64 (mixed upcast); memory-short form: hd (one tile per
    // tile row) and lc (one decoded column, mixed)
    size_t tt, pl, tb, sq, part, l64, total;
    bool short_form;
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

AdjLayout adj_layout(int64_t n, int nb, bool mixed, bool short_form) {
    const int64_t Nt = n / nb;
    const int64_t nb2 = (int64_t)nb * nb;
    const int64_t panel = std::max<int64_t>(Nt - 1, 1) * nb2;
    // full: every Abar tile transposed; short: H_m per tile row
    const size_t tt_tiles = short_form ? (size_t)Nt : (size_t)(Nt * (Nt + 1) / 2);
    // a mixed-precision factor is swept in binary64: its upcast tiles, all
    // of them (full) or one column at a time (short)
    const size_t l64_tiles = !mixed ? 0 : short_form ? (size_t)Nt : (size_t)(Nt * (Nt + 1) / 2);
    AdjLayout L;
    L.short_form = short_form;
    L.tt = 0;
    L.pl = L.tt + tt_tiles * nb2;
    L.tb = L.pl + panel;
    L.sq = L.tb + panel;
    L.part = L.sq + 5 * nb2;
    L.l64 = L.part + adj_partial_doubles((int)Nt, nb) + 32;
    L.total = (L.l64 + l64_tiles * nb2) * sizeof(double);
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
    return adj_layout(n, nb, mixed != 0, false).total;
}

size_t tc_adjoint_min_bytes(int64_t n, int32_t nb, int32_t mixed) {
    if (!valid_shape(n, nb)) return 0;
    return adj_layout(n, nb, mixed != 0, true).total;
}

tc_status tc_factor_adjoint(tc_ctx* ctx, const tc_factor* F, double* Lbar, void* scratch,
                            size_t scratch_bytes, tc_stats* stats) {
    if (!ctx || !F || !Lbar || !scratch) return fail(TC_EINVAL, "NULL argument");
    if (F->info > 0) return fail(TC_EINVAL, "factor is not valid (factorization failed)");
    const int64_t n = F->n;
    const int nb = F->nb, Nt = F->Nt;
    AdjLayout Ly = adj_layout(n, nb, F->mixed, false);
    if (scratch_bytes < Ly.total) Ly = adj_layout(n, nb, F->mixed, true);
    if (scratch_bytes < Ly.total)
        return fail(TC_ENOMEM, "adjoint scratch too small: need " + std::to_string(Ly.total) +
                                   " bytes (memory-short form) or " +
                                   std::to_string(adj_layout(n, nb, F->mixed, false).total) +
                                   ", have " + std::to_string(scratch_bytes));
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
    const bool sf = Ly.short_form;
    double* Tfull = sf ? nullptr : Tt;  // transposed Abar tiles (full form)
    double* Hd = sf ? Tt : nullptr;     // H_m per tile row (memory-short form)
    const double* L = F->tiles;
    double* Lc = S + Ly.l64;  // one decoded column (memory-short form, mixed)
    if (F->mixed && !sf) {    // sweep the upcast factor
        TC_HIP(tc::launch_export(st, factor_view(F), Lc));
        L = Lc;
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
        const int64_t dg = tc::tile_off(Nt, nn, nn);
        const double* Lnn = L + dg * nb2;  // column nn of L from here on
        if (F->mixed && sf) {  // decode the column again (no stored upcast)
            TC_HIP(tc::launch_export_range(st, factor_view(F), dg, R + 1, Lc));
            Lnn = Lc;
        }
        double* Lbnn = Lbar + dg * nb2;
        TC_HIP(tc::launch_set_identity(st, X, nb));
        TC_HIP(tc::launch_trsm(st, X, Lnn, nb, nb, nb));  // X = L_nn^{-T}
        flops += (double)nb * nb * nb;
        if (R > 0) {
            const int64_t off = tc::tile_off(Nt, nn + 1, nn) * nb2;
            double* Lbp = Lbar + off;
            // transposed Abar column: kept in Tt (full) or only for (c) in Tb
            double* Ttp = sf ? Tb : Tt + off;
            TC_HIP(tc::launch_transpose_tiles(st, Lnn + nb2, PL, nb, R, false));
            const int sp = tc::adj_panel_splits(Nt, nb, nn);
            if (timed) TC_HIP(hipEventRecord(ctx->gemm_ev[2 * launches], st));
            TC_HIP(tc::launch_adj_panel(st, Lbar, Tfull, Hd, PL, Nt, nb, nn, sp, part));
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
            TC_HIP(tc::launch_transpose_tiles(st, Lbp, Ttp, nb, R, false));
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
        double* H = sf ? Hd + (int64_t)nn * nb2 : Tt + dg * nb2;
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
