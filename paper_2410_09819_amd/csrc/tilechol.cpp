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
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "formats.hpp"
#include "host_common.hpp"
#include "tilechol.h"

namespace tc {
namespace host {

thread_local std::string g_err;

tc_status fail(tc_status s, const std::string& msg) {
    g_err = msg;
    return s;
}


// Workspace regions (all carved from the caller's buffer):
//   info   : one int (failure flag)
//   big    : split-K partial sums of the panel updates and the
//            backward-solve partial sums (used one at a time, stream-ordered)
//   potrf  : split-K partial sums of the in-tile updates of the recursive
//            POTRF (its own region: POTRF runs concurrently with panel
//            updates under the lookahead schedule)
//   small  : Matern strip sums of squares, log-determinant partials, amax
//            partials of the mixed-precision finalize, column norms
//   panel  : binary64 working columns (mixed precision, out of core)
//   lists  : row-tile lists per column and class (mixed precision)
//   ir     : refinement vectors (b, r) and residual partial sums
size_t big_bytes(int64_t n, int nb) {
    const int Nt = (int)(n / nb);
    size_t mx = 0;
    for (int k = 1; k < Nt; ++k) {
        for (int nc = k - 1; nc <= k; ++nc) {  // lookahead bulk (k-1 columns) or full (k)
            if (nc <= 0) continue;
            const int s = tc::panel_splits(Nt, nb, k, nc);
            if (s > 1) mx = std::max(mx, (size_t)s * (size_t)(Nt - k) * nb * nb * sizeof(double));
        }
    }
    // backward-solve partials (<= 64 splits), one area per solve stream
    mx = std::max(mx, (size_t)2 * tc::bwd_partial_doubles(nb) * sizeof(double));
    // inverted 64 x 64 diagonal blocks of every diagonal tile (mixed factor)
    mx = std::max(mx, (size_t)Nt * nb * 64 * sizeof(double));
    return mx;
}

size_t potrf_bytes(int nb) {
    // also the inverses of a tile's 64 x 64 diagonal blocks (mixed TRSM)
    size_t mx = std::max<size_t>(256, (size_t)nb * 64 * sizeof(double));
    // in-tile recursion (sizes are multiples of 128 below nb)
    for (int m = 128; m < nb; m += 128) {
        for (int kd = 128; kd < nb; kd += 128) {
            const int s = tc::syrk_sub_splits(m, kd);
            if (s > 1) mx = std::max(mx, (size_t)s * m * m * sizeof(double));
        }
    }
    return mx;
}

Layout layout(int64_t n, int nb, int nrhs) {
    const int64_t Nt = n / nb;
    const int64_t ntiles = Nt * (Nt + 1) / 2;
    if (nrhs < 16) nrhs = 16;
    Layout L;
    L.info = 0;
    L.big = align_up(sizeof(int) * 64);
    L.potrf = L.big + align_up(big_bytes(n, nb));
    L.small = L.potrf + align_up(potrf_bytes(nb));
    // Matern strip sums; three per strip for the gradient contraction
    size_t small = std::max<size_t>((size_t)3 * ntiles * tc::matern_strips(nb) + 8, (size_t)Nt * 16);
    small = std::max<size_t>(small, (size_t)2 * nrhs * tc::colnorm_blocks());
    L.panel = L.small + align_up(small * sizeof(double));
    // two working columns (the out-of-core path prefetches the next one)
    L.lists = L.panel + align_up((size_t)2 * Nt * nb * nb * sizeof(double));
    // row lists (mixed precision) or the out-of-core pointer-table ring
    const size_t lists = std::max<size_t>((size_t)5 * Nt * Nt * sizeof(int),
                                          (size_t)64 * ((size_t)Nt * Nt / 4 + Nt) * sizeof(void*));
    L.ir = L.lists + align_up(lists);
    // refinement: b, the residual / correction, the solves' intermediate
    // vector, residual partial sums
    const size_t ir = (size_t)3 * n * nrhs + tc::residual_partial_doubles((int)Nt, nb, nrhs);
    L.total = L.ir + align_up(ir * sizeof(double));
    return L;
}

// The library's own streams: three per device, non-blocking, default
// priority, created once per process and shared by every context on the
// device. HIP runs streams on a small pool of hardware queues (4 unless
// GPU_MAX_HW_QUEUES says otherwise) and lets streams share a queue once the
// pool is used up; work of two streams on one queue runs in submission
// order, so a copy stream that lands on the caller's queue serializes the
// copies with the compute. Three streams plus the caller's fit in four
// queues. Roles: aux[0] and the device-to-host copies share stream 0 (no
// schedule uses both at once except the mixed out-of-core path, whose
// prefetch of A follows the write-back of the column it replaces anyway),
// aux[1] is stream 1, host-to-device copies stream 2.
constexpr int kMaxDevices = 64;
std::mutex g_streams_mu;
hipStream_t g_streams[kMaxDevices][3];

tc_status device_streams(int device, hipStream_t out[3]) {
    if (device < 0 || device >= kMaxDevices)
        return fail(TC_EINVAL, "device " + std::to_string(device) + " out of range");
    std::lock_guard<std::mutex> lock(g_streams_mu);
    for (int i = 0; i < 3; ++i)
        if (!g_streams[device][i])
            TC_HIP(hipStreamCreateWithFlags(&g_streams[device][i], hipStreamNonBlocking));
    for (int i = 0; i < 3; ++i) out[i] = g_streams[device][i];
    return TC_OK;
}

tc_status ctx_ooc_resources(tc_ctx* ctx, size_t bytes) {
    if (ctx->pinned_bytes < bytes) {
        if (ctx->pinned) {
            TC_HIP(hipDeviceSynchronize());
            TC_HIP(hipHostFree(ctx->pinned));
            ctx->pinned = nullptr;
            ctx->pinned_bytes = 0;
        }
        TC_HIP(hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault));
        ctx->pinned_bytes = bytes;
    }
    return TC_OK;
}

tc_status ctx_aux_streams(tc_ctx* ctx) {
    for (int i = 0; i < 3; ++i)
        if (!ctx->aux_ev[i]) TC_HIP(hipEventCreateWithFlags(&ctx->aux_ev[i], hipEventDisableTiming));
    return TC_OK;
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

// Storage plan of a mixed-precision factor. Tiles are stored in their class
// in packed order; then come the operand copies Q_c(Lh_t) for every tile t
// and low class c that the static schedule multiplies it in (as the A
// operand of tile (m, k), class c = class(m, k), n < k < m, or as the B
// operand of the tiles (m', m), m' > m), row-major (k contiguous, the MFMA
// operand order) with a per-copy power-of-two scale: the class's own bits
// for FP16, BF16 and FP8, and for FP32 the binary32 value split into two
// FP16 planes (hi, lo). Then the device tables.
bool make_plan(int64_t n, int nb, const uint8_t* map, Plan& P, int fp64_update) {
    if (fp64_update != TC_FP64 && fp64_update != TC_FP32) return false;
    P.Nt = (int)(n / nb);
    P.nb = nb;
    const int Nt = P.Nt;
    P.ntiles = (int64_t)Nt * (Nt + 1) / 2;
    P.cls.assign(P.ntiles, TC_FP64);
    P.mixed = fp64_update != TC_FP64;
    if (map) {
        for (int64_t t = 0; t < P.ntiles; ++t) {
            if (map[t] > TC_FP8E4M3) return false;
            P.cls[t] = map[t];
            if (map[t] != TC_FP64) P.mixed = true;
        }
        for (int k = 0; k < Nt; ++k)
            if (P.cls[tc::tile_off(Nt, k, k)] != TC_FP64) return false;
    }
    P.diag64 = fp64_update == TC_FP64;
    P.ccls = P.cls;
    for (auto& c : P.ccls)
        if (c == TC_FP64) c = (uint8_t)fp64_update;
    const size_t tb = (size_t)nb * nb;
    P.toff.assign(P.ntiles, 0);
    size_t off = 0;
    for (int64_t t = 0; t < P.ntiles; ++t) {
        P.toff[t] = (int64_t)off;
        off += align_up(tb * tc::fmt_bytes(P.cls[t]));
    }
    // no operand copies until a low class needs them (an all-FP64 plan has
    // none, and the out-of-core mixed path reads this table for it too)
    P.shoff.assign((size_t)P.ntiles * 4, -1);
    if (!P.mixed) {
        P.total = off;
        return true;
    }
    auto C = [&](int i, int j) { return (int)P.ccls[tc::tile_off(Nt, i, j)]; };
    // compute classes present in each row m left of the diagonal and in each
    // column m on and below it (as bit masks; the diagonal's is the SYRK's)
    for (int m = 1; m < Nt; ++m) {
        uint32_t colmask = 0;
        for (int mp = m; mp < Nt; ++mp) colmask |= 1u << C(mp, m);
        // suffix masks of row m: classes of (m, k) for k in (n, m)
        std::vector<uint32_t> suf(m + 1, 0);
        for (int k = m - 1; k >= 0; --k) suf[k] = suf[k + 1] | (1u << C(m, k));
        for (int n2 = 0; n2 < m; ++n2) {
            const uint32_t need = (suf[n2 + 1] | colmask) & ~1u;  // low classes only
            const int64_t t = tc::tile_off(Nt, m, n2);
            for (int c = 1; c <= 4; ++c) {
                if (!(need & (1u << c))) continue;
                P.shoff[t * 4 + c - 1] = (int64_t)off;
                // FP32: two FP16 planes (hi, lo)
                off += align_up(tb * (c == TC_FP32 ? 4 : (size_t)tc::fmt_bytes(c)));
            }
        }
    }
    P.tab_toff = off;
    off += align_up(P.ntiles * sizeof(int64_t));
    P.tab_shoff = off;
    off += align_up(P.ntiles * 4 * sizeof(int64_t));
    P.tab_tscl = off;
    off += align_up(P.ntiles * sizeof(int));
    P.tab_tcls = off;
    off += align_up(P.ntiles);
    P.tab_cscl = off;  // scale exponents of the operand copies, [t * 4 + c - 1]
    off += align_up(P.ntiles * 4 * sizeof(int));
    P.tab_xinv = off;  // inverses of the diagonal tiles (for the solves)
    off += align_up((size_t)Nt * nb * nb * sizeof(double));
    P.total = off;
    return true;
}

void class_lists(const Plan& P, std::vector<int>& lists, std::vector<int>& count,
                 double* cflops, int* ctiles) {
    const int Nt = P.Nt;
    const double nb2 = (double)P.nb * P.nb;
    lists.assign((size_t)5 * Nt * Nt, 0);
    count.assign((size_t)5 * Nt, 0);
    for (int c = 0; c < 5; ++c) {
        cflops[c] = 0.0;
        ctiles[c] = 0;
    }
    for (int64_t t = 0; t < P.ntiles; ++t) ctiles[P.cls[t]]++;
    for (int k = 0; k < Nt; ++k) {
        const double K = (double)k * P.nb;
        // diagonal SYRK (lower half of the flops)
        if (P.diag64) {
            cflops[TC_FP64] += nb2 * K;
        } else {
            lists[((size_t)k * 5 + TC_FP32) * Nt + count[(size_t)k * 5 + TC_FP32]++] = 0;
            cflops[TC_FP32] += nb2 * K;
        }
        for (int r = 1; r < Nt - k; ++r) {
            const int c = P.ccls[tc::tile_off(Nt, k + r, k)];
            lists[((size_t)k * 5 + c) * Nt + count[(size_t)k * 5 + c]++] = r;
            cflops[c] += 2.0 * nb2 * K;
        }
    }
}

// Recursive POTRF of the s x s block at offset o of a diagonal tile.
tc_status potrf_rec(hipStream_t st, double* T, int nb, int o, int s, int64_t col0, int* info,
                    double* big) {
    if (s <= 128) {
        TC_HIP(tc::launch_potrf_leaf(st, T + o + (int64_t)o * nb, nb, s, info, col0 + o));
        return TC_OK;
    }
    const int h = ((s / 2 + 127) / 128) * 128;
    if (tc_status r = potrf_rec(st, T, nb, o, h, col0, info, big)) return r;
    double* L11 = T + o + (int64_t)o * nb;
    double* A21 = T + (o + h) + (int64_t)o * nb;
    double* A22 = T + (o + h) + (int64_t)(o + h) * nb;
    TC_HIP(tc::launch_trsm(st, A21, L11, nb, s - h, h));
    TC_HIP(tc::launch_syrk_sub(st, A22, A21, nb, s - h, h, big, tc::syrk_sub_splits(s - h, h)));
    return potrf_rec(st, T, nb, o + h, s - h, col0, info, big);
}

}  // namespace host
}  // namespace tc

namespace tc {
namespace host {
tc::TileView factor_view(const tc_factor* F) {
    tc::TileView v;
    v.Nt = F->Nt;
    v.nb = F->nb;
    v.base = F->mixed ? F->storage : reinterpret_cast<const char*>(F->tiles);
    v.toff = F->mixed ? F->d_toff : nullptr;
    v.tcls = F->mixed ? F->d_tcls : nullptr;
    v.tscl = F->mixed ? F->d_tscl : nullptr;
    return v;
}
}  // namespace host
}  // namespace tc

using namespace tc::host;

namespace {

tc::TileView view_of(const tc_factor* F) { return factor_view(F); }

const double* diag_tile(const tc_factor* F, int k) {
    const int64_t t = tc::tile_off(F->Nt, k, k);
    if (F->mixed) return reinterpret_cast<const double*>(F->storage + F->toff[t]);
    return F->tiles + t * (int64_t)F->nb * F->nb;
}

// B <- (L L^T)^{-1} B, enqueued on the context stream (no synchronization).
// Both substitutions run a lookahead on a second stream: the long update of
// the rows two or more tiles away from the diagonal solve in progress
// overlaps the chain of diagonal-tile solves, which only waits for the
// adjacent tile's update. ev[k] / ev[Nt + k]: diagonal solve k done (main)
// / side update of column k done.
tc_status solve_events(tc_ctx* ctx, int Nt) {
    if (tc_status s = ctx_aux_streams(ctx)) return s;
    while (ctx->solve_ev.size() < (size_t)2 * Nt) {
        hipEvent_t e;
        TC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->solve_ev.push_back(e);
    }
    return TC_OK;
}

// B <- L^{-1} B (forward substitution by tile rows). big: partial sums of
// the main stream's one-tile updates. With Y (a mixed factor's stored
// diagonal-tile inverses; Y: n x nrhs with the same leading dimension) the
// result goes to Y instead: each diagonal step is then Y_k = L_kk^{-1} B_k,
// a product with the stored inverse, and B keeps the updated right-hand
// sides.
tc_status fwd_enqueue(tc_ctx* ctx, const tc_factor* F, double* B, int64_t ldb, int nrhs,
                      double* big, double* Y) {
    const int Nt = F->Nt, nb = F->nb;
    const tc::TileView V = view_of(F);
    if (tc_status s = solve_events(ctx, Nt)) return s;
    hipStream_t sm = ctx->stream, ss = ctx->aux[0];
    hipEvent_t* ev_t = ctx->solve_ev.data();
    hipEvent_t* ev_s = ev_t + Nt;
    double* part_side = big + tc::bwd_partial_doubles(nb);
    double* X = Y ? Y : B;  // where the solved tile rows go
    const int64_t nb2 = (int64_t)nb * nb;
    for (int k = 0; k < Nt; ++k) {
        if (k >= 1) {  // tile row k from column k-1, after the side's older updates of it
            if (k >= 2) TC_HIP(hipStreamWaitEvent(sm, ev_s[k - 2], 0));
            TC_HIP(tc::launch_tile_update(sm, V, k, k - 1, false, X + (int64_t)(k - 1) * nb,
                                          B + (int64_t)k * nb, ldb, nrhs, big));
        }
        if (Y)
            TC_HIP(tc::launch_tile_inv_apply(sm, F->d_xinv + k * nb2, nb, B + (int64_t)k * nb,
                                             Y + (int64_t)k * nb, ldb, nrhs, false, big));
        else
            TC_HIP(tc::launch_trsv_diag(sm, diag_tile(F, k), nb, B + (int64_t)k * nb, ldb, nrhs,
                                        false));
        if (k + 2 < Nt) {  // rows of tiles k+2.. from column k, on the side stream
            TC_HIP(hipEventRecord(ev_t[k], sm));
            TC_HIP(hipStreamWaitEvent(ss, ev_t[k], 0));
            TC_HIP(tc::launch_fwd_update(ss, V, k, 1, Nt - k - 2, X + (int64_t)k * nb,
                                         B + (int64_t)(k + 2) * nb, ldb, nrhs, part_side));
            TC_HIP(hipEventRecord(ev_s[k], ss));
        }
    }
    return TC_OK;
}

// B <- L^{-T} B (back substitution by tile rows). With Y: the input is Y
// (the forward result, updated in place) and each diagonal step writes
// B_k = L_kk^{-T} Y_k with the stored inverse.
tc_status bwd_enqueue(tc_ctx* ctx, const tc_factor* F, double* B, int64_t ldb, int nrhs,
                      double* big, double* Y) {
    const int Nt = F->Nt, nb = F->nb;
    const tc::TileView V = view_of(F);
    if (tc_status s = solve_events(ctx, Nt)) return s;
    hipStream_t sm = ctx->stream, ss = ctx->aux[0];
    hipEvent_t* ev_t = ctx->solve_ev.data();
    hipEvent_t* ev_s = ev_t + Nt;
    double* part_side = big + tc::bwd_partial_doubles(nb);
    double* R = Y ? Y : B;  // the right-hand sides being reduced
    const int64_t nb2 = (int64_t)nb * nb;
    for (int k = Nt - 1; k >= 0; --k) {
        if (k + 1 < Nt) {  // tile k+1's contribution, after the side's (tiles k+2..)
            if (k + 2 < Nt) TC_HIP(hipStreamWaitEvent(sm, ev_s[k], 0));
            TC_HIP(tc::launch_tile_update(sm, V, k + 1, k, true, B + (int64_t)(k + 1) * nb,
                                          R + (int64_t)k * nb, ldb, nrhs, big));
        }
        if (Y)
            TC_HIP(tc::launch_tile_inv_apply(sm, F->d_xinv + k * nb2, nb, Y + (int64_t)k * nb,
                                             B + (int64_t)k * nb, ldb, nrhs, true, big));
        else
            TC_HIP(tc::launch_trsv_diag(sm, diag_tile(F, k), nb, B + (int64_t)k * nb, ldb, nrhs,
                                        true));
        const int j = k - 2;  // column whose tiles k.. are now final
        if (j >= 0) {
            TC_HIP(hipEventRecord(ev_t[k], sm));
            TC_HIP(hipStreamWaitEvent(ss, ev_t[k], 0));
            TC_HIP(tc::launch_bwd_update(ss, V, j, 1, Nt - j - 2, B + (int64_t)k * nb,
                                         R + (int64_t)j * nb, ldb, nrhs, part_side));
            TC_HIP(hipEventRecord(ev_s[j], ss));
        }
    }
    return TC_OK;
}

// Y: n x nrhs scratch with leading dimension ldb for the inverse-based
// diagonal steps, used when the factor stores its diagonal-tile inverses
// (else NULL: substitution with the diagonal tiles in place).
tc_status solve_enqueue(tc_ctx* ctx, const tc_factor* F, double* B, int64_t ldb, int nrhs,
                        double* big, double* Y) {
    if (!F->d_xinv) Y = nullptr;
    if (tc_status s = fwd_enqueue(ctx, F, B, ldb, nrhs, big, Y)) return s;
    return bwd_enqueue(ctx, F, B, ldb, nrhs, big, Y);
}

// Column norms of X (n x nrhs): ||x_j||_2 into out[j] (synchronizes).
tc_status colnorms(tc_ctx* ctx, const double* X, int64_t ld, int64_t n, int nrhs, double* part,
                   std::vector<double>& out) {
    TC_HIP(tc::launch_colnorm(ctx->stream, X, ld, n, nrhs, part));
    const int nbk = tc::colnorm_blocks();
    std::vector<double> h((size_t)nrhs * nbk);
    TC_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
    TC_HIP(hipStreamSynchronize(ctx->stream));
    out.assign(nrhs, 0.0);
    for (int c = 0; c < nrhs; ++c) {
        double s = 0.0;
        for (int b = 0; b < nbk; ++b) s += h[(size_t)c * nbk + b];
        out[c] = std::sqrt(s);
    }
    return TC_OK;
}

}  // namespace

extern "C" {

int64_t tc_tile_offset(int32_t Nt, int32_t i, int32_t j) {
    if (Nt <= 0 || j < 0 || i < j || i >= Nt) return -1;
    return tc::tile_off(Nt, i, j);
}

tc_status tc_host_alloc(size_t bytes, void** out) {
    if (!out || bytes == 0) return fail(TC_EINVAL, "bad argument");
    *out = nullptr;
    hipError_t e = hipHostMalloc(out, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        *out = nullptr;
        return fail(TC_ENOMEM, "pinned host allocation of " + std::to_string(bytes) +
                                   " bytes failed: " + hipGetErrorString(e));
    }
    return TC_OK;
}

tc_status tc_host_free(void* p) {
    if (!p) return TC_OK;
    TC_HIP(hipHostFree(p));
    return TC_OK;
}

const char* tc_version(void) { return "tilechol 0.3 (gfx950, FP64 MFMA, mixed precision on FP16/BF16/FP8 MFMA)"; }

const char* tc_last_error(void) { return g_err.c_str(); }

size_t tc_workspace_bytes(int64_t n, int32_t nb, int32_t nrhs) {
    if (!valid_shape(n, nb) || nrhs < 0) return 0;
    return layout(n, nb, nrhs).total;
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
        tc_ctx_destroy(c);
        return fail(TC_EHIP, "hipEventCreate failed");
    }
    hipStream_t ds[3];
    if (tc_status s = device_streams(device, ds)) {
        tc_ctx_destroy(c);
        return s;
    }
    c->aux[0] = ds[0];
    c->aux[1] = ds[1];
    c->h2d = ds[2];
    c->d2h = ds[0];
    if (tc_status s = noalloc_scratch_init(device)) {
        tc_ctx_destroy(c);
        return s;
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
    for (hipEvent_t e : ctx->la_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->solve_ev) (void)hipEventDestroy(e);
    // the library's streams are shared, not destroyed: wait for them only
    for (hipStream_t s : {ctx->aux[0], ctx->aux[1], ctx->h2d, ctx->d2h})
        if (s) (void)hipStreamSynchronize(s);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    for (int i = 0; i < 3; ++i)
        if (ctx->aux_ev[i]) (void)hipEventDestroy(ctx->aux_ev[i]);
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

tc_status tc_precision_map(int32_t Nt, const double* tile_fro, double fro_A, double eps,
                           uint32_t allowed_mask, int32_t unit_roundoff, uint8_t* map_out) {
    if (Nt <= 0 || !tile_fro || !map_out) return fail(TC_EINVAL, "NULL argument or Nt <= 0");
    if (!(fro_A > 0) || !(eps > 0)) return fail(TC_EINVAL, "fro_A and eps must be positive");
    if (allowed_mask & ~0x1Fu) return fail(TC_EINVAL, "allowed_mask has unknown classes");
    // candidate low classes, largest epsilon (lowest precision) first
    int order[4], nc = 0;
    const int by_eps[4] = {TC_FP8E4M3, TC_BF16, TC_FP16, TC_FP32};
    for (int c : by_eps)
        if (allowed_mask & (1u << c)) order[nc++] = c;
    for (int32_t j = 0; j < Nt; ++j)
        for (int32_t i = j; i < Nt; ++i) {
            const int64_t t = tc::tile_off(Nt, i, j);
            uint8_t cls = TC_FP64;
            if (i != j) {
                const double lhs = (double)Nt * tile_fro[t] / fro_A;
                for (int q = 0; q < nc; ++q) {
                    const int p = tc::fmt_spec(order[q]).p;
                    const double eps_p = std::ldexp(1.0, unit_roundoff ? -p : 1 - p);
                    if (lhs < eps / eps_p) {
                        cls = (uint8_t)order[q];
                        break;
                    }
                }
            }
            map_out[t] = cls;
        }
    return TC_OK;
}

size_t tc_factor_bytes(int64_t n, int32_t nb, const uint8_t* map, const tc_opts* opts) {
    if (!valid_shape(n, nb)) return 0;
    Plan P;
    if (!make_plan(n, nb, map, P, opts ? opts->fp64_update : TC_FP64)) return 0;
    if (!P.mixed) return (size_t)P.ntiles * nb * nb * sizeof(double);
    return P.total;
}

namespace {

// All-FP64 factorization (storage: packed binary64 tiles, may equal A).
tc_status factorize_fp64(tc_ctx* ctx, int64_t n, int nb, const double* A, double* L,
                         tc_factor** Lout, tc_stats* stats) {
    const int Nt = (int)(n / nb);
    const int64_t ntiles = (int64_t)Nt * (Nt + 1) / 2;
    const size_t need = (size_t)ntiles * nb * nb * sizeof(double);
    const Layout Ly = layout(n, nb);
    int* d_info = reinterpret_cast<int*>(ctx->ws + Ly.info);
    double* big = reinterpret_cast<double*>(ctx->ws + Ly.big);
    double* pot = reinterpret_cast<double*>(ctx->ws + Ly.potrf);
    const int64_t nb2 = (int64_t)nb * nb;
    const bool timed = (ctx->flags & 1u) != 0;
    if (tc_status s = ctx_aux_streams(ctx)) return s;
    while (timed && ctx->gemm_ev.size() < (size_t)2 * Nt) {
        hipEvent_t e;
        TC_HIP(hipEventCreate(&e));
        ctx->gemm_ev.push_back(e);
    }
    while (ctx->la_ev.size() < (size_t)3 * Nt + 1) {
        hipEvent_t e;
        TC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->la_ev.push_back(e);
    }
    // Lookahead schedule on two streams (same column order as Algorithm 1).
    // Column c's update is split by tile columns into three launches:
    //   Pa(c): tile columns [0, c-2)   bulk stream, two columns ahead;
    //   Pb(c): tile column c-2         bulk stream, one column ahead;
    //   P2(c): tile column c-1         main stream, right before POTRF(c).
    // Per column k:
    //   main (stream):   P2(k) (after Pa(k), Pb(k) and TRSM(k-1)), POTRF(k),
    //                    TRSM(k);
    //   bulk (aux[0]):   once P2(k) is done (so after TRSM(k-1)): Pb(k+1),
    //                    then Pa(k+2) -- concurrent with POTRF(k), TRSM(k).
    // The bulk waits for P2(k) instead of starting beside it: launched
    // together, the two share the CUs and P2(k), which the critical path
    // needs first, ends with the longer bulk; POTRF(k) and TRSM(k) then run
    // with the bulk stream idle (measured: every column of the first
    // quarter at n = 131072). Pb(k+1) splits off the tile column that
    // becomes ready last, so Pa(k+2) can run two columns ahead: in the
    // first columns, where the bulk is short, POTRF and TRSM then have more
    // bulk work beside them (n = 65536: 1.527 -> 1.520 s on one box).
    // ev_p[k]: Pa(k) and Pb(k) done (bulk); ev_q[k-1]: P2(k) done (main).
    hipStream_t sm = ctx->stream, sb = ctx->aux[0];
    hipEvent_t* ev_p = ctx->la_ev.data() + Nt;
    hipEvent_t* ev_q = ctx->la_ev.data() + 2 * Nt + 1;
    hipEvent_t ev_go = ctx->la_ev[2 * Nt];
    TC_HIP(hipEventRecord(ctx->ev0, sm));
    if ((const void*)L != (const void*)A)
        TC_HIP(hipMemcpyAsync(L, A, need, hipMemcpyDeviceToDevice, sm));
    TC_HIP(tc::launch_zero_info(sm, d_info));
    TC_HIP(hipEventRecord(ev_go, sm));
    TC_HIP(hipStreamWaitEvent(sb, ev_go, 0));
    double gemm_flops = 0.0, tail_flops = 0.0;
    int launches = 0;
    for (int k = 0; k < Nt; ++k) {
        if (k >= 1) {  // P2(k)
            if (k >= 2) TC_HIP(hipStreamWaitEvent(sm, ev_p[k], 0));
            TC_HIP(tc::launch_panel_update(sm, L, Nt, nb, k, k - 1, k, 1, nullptr, true));
            TC_HIP(hipEventRecord(ev_q[k - 1], sm));
            tail_flops += (double)nb * nb * (double)nb * (1.0 + 2.0 * (Nt - k - 1));
        }
        if (k >= 1 && k + 1 < Nt) {
            TC_HIP(hipStreamWaitEvent(sb, ev_q[k - 1], 0));
            // Pb(k+1): one tile column, launched as a rank-nb update
            TC_HIP(tc::launch_panel_update(sb, L, Nt, nb, k + 1, k - 1, k, 1, nullptr, true));
            tail_flops += (double)nb * nb * (double)nb * (1.0 + 2.0 * (Nt - k - 2));
            TC_HIP(hipEventRecord(ev_p[k + 1], sb));
            if (k + 2 < Nt) {  // Pa(k+2): the bulk launch
                const int c = k + 2;
                const int sp = tc::panel_splits(Nt, nb, c, k);
                if (timed) TC_HIP(hipEventRecord(ctx->gemm_ev[2 * launches], sb));
                TC_HIP(tc::launch_panel_update(sb, L, Nt, nb, c, 0, k, sp, big, false));
                if (timed) TC_HIP(hipEventRecord(ctx->gemm_ev[2 * launches + 1], sb));
                TC_HIP(tc::launch_panel_reduce(sb, L, Nt, nb, c, sp, big));
                gemm_flops += (double)nb * nb * ((double)k * nb) * (1.0 + 2.0 * (Nt - c - 1));
                ++launches;
            }
        }
        double* Tkk = L + tc::tile_off(Nt, k, k) * nb2;
        if (tc_status s = potrf_rec(ctx->stream, Tkk, nb, 0, nb, (int64_t)k * nb, d_info, pot)) return s;
        if (k + 1 < Nt)
            TC_HIP(tc::launch_trsm(sm, L + tc::tile_off(Nt, k + 1, k) * nb2, Tkk, nb,
                                   (int64_t)(Nt - k - 1) * nb, nb, tc::kPanelTrsmLeaf));
    }
    // the bulk stream's last launch, Pb(Nt-1), precedes P2(Nt-1) on the
    // main stream, so the main stream has joined it
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
        stats->class_flops[TC_FP64] = gemm_flops + tail_flops;
        stats->class_tiles[TC_FP64] = (int32_t)ntiles;
    }
    return info > 0 ? info : TC_OK;
}

// Mixed-precision factorization. Column k: copy A's column of tiles into the
// binary64 working column W, subtract the updates class group by class
// group, POTRF the diagonal tile and TRSM the rest in FP64, then store the
// diagonal tile in FP64 and round the others into their classes.
tc_status factorize_mixed(tc_ctx* ctx, int64_t n, int nb, const double* A, const Plan& P,
                          char* storage, int wide, tc_factor** Lout, tc_stats* stats) {
    const int Nt = P.Nt;
    const Layout Ly = layout(n, nb);
    int* d_info = reinterpret_cast<int*>(ctx->ws + Ly.info);
    double* big = reinterpret_cast<double*>(ctx->ws + Ly.big);
    double* part = reinterpret_cast<double*>(ctx->ws + Ly.small);
    double* W = reinterpret_cast<double*>(ctx->ws + Ly.panel);
    int* d_lists = reinterpret_cast<int*>(ctx->ws + Ly.lists);
    const size_t big_cap = Ly.potrf - Ly.big;
    double* pot = reinterpret_cast<double*>(ctx->ws + Ly.potrf);
    const int64_t nb2 = (int64_t)nb * nb;
    int64_t* d_toff = reinterpret_cast<int64_t*>(storage + P.tab_toff);
    int64_t* d_shoff = reinterpret_cast<int64_t*>(storage + P.tab_shoff);
    int* d_tscl = reinterpret_cast<int*>(storage + P.tab_tscl);
    uint8_t* d_tcls = reinterpret_cast<uint8_t*>(storage + P.tab_tcls);
    int* d_cscl = reinterpret_cast<int*>(storage + P.tab_cscl);

    std::vector<int> lists, lcount;
    double cflops[5];
    int ctiles[5];
    class_lists(P, lists, lcount, cflops, ctiles);
    std::vector<int> zeros(P.ntiles, 0);
    if (tc_status s = ctx_aux_streams(ctx)) return s;
    while (ctx->la_ev.size() < (size_t)4 * Nt + 1) {
        hipEvent_t e;
        TC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->la_ev.push_back(e);
    }
    // Lookahead schedule on three streams (same column order as Algorithm 1;
    // the working column of column k is Wb[k % 2]):
    //   aux[0]: column c's A tiles into Wb[c % 2], then its FP64 group over
    //           tile columns [0, c-1), once column c-2 is finalized;
    //   aux[1]: column c's FP32 / FP16 / BF16 / FP8 groups over [0, c-1);
    //   main:   column k's groups over tile column k-1 (after both bulk
    //           parts), POTRF, TRSM, store, finalize.
    // So the bulk of column k+2 overlaps the critical path of column k+1.
    // ev_f[k]: column k finalized (main); ev_c[c]: Wb filled (aux[0]);
    // ev_b64[c], ev_blo[c]: bulk groups of column c done.
    hipStream_t sm = ctx->stream, s64 = ctx->aux[0], slo = ctx->aux[1];
    hipEvent_t* ev_f = ctx->la_ev.data();
    hipEvent_t* ev_c = ev_f + Nt;
    hipEvent_t* ev_b64 = ev_f + 2 * Nt;
    hipEvent_t* ev_blo = ev_f + 3 * Nt;
    hipEvent_t ev_go = ctx->la_ev[4 * Nt];
    double* Wb[2] = {W, W + (int64_t)Nt * nb2};
    auto col_bytes = [&](int c) { return (size_t)(Nt - c) * nb2 * sizeof(double); };
    auto list = [&](int c, int cls) { return d_lists + ((size_t)c * 5 + cls) * Nt; };
    auto count = [&](int c, int cls) { return lcount[(size_t)c * 5 + cls]; };
    // the low-class groups of column c over tile columns [n0, n1) on stream st
    auto low_groups = [&](hipStream_t st, int c, int n0, int n1) -> tc_status {
        double* Wc = Wb[c % 2];
        for (int cls = 1; cls <= 4; ++cls) {
            const int cnt = count(c, cls);
            if (!cnt) continue;
            if (cls == TC_FP32)
                TC_HIP(tc::launch_mxp_gemm_f32(st, Wc, Nt, nb, c, n0, n1, list(c, cls), cnt, storage,
                                               d_shoff, d_cscl, wide));
            else
                TC_HIP(tc::launch_mxp_gemm_narrow(st, Wc, Nt, nb, c, n0, n1, list(c, cls), cnt, cls,
                                                  storage, d_shoff, d_cscl, wide));
        }
        return TC_OK;
    };

    TC_HIP(hipEventRecord(ctx->ev0, sm));
    TC_HIP(hipMemcpyAsync(d_lists, lists.data(), lists.size() * sizeof(int), hipMemcpyHostToDevice,
                          sm));
    TC_HIP(hipMemcpyAsync(d_toff, P.toff.data(), P.toff.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice, sm));
    TC_HIP(hipMemcpyAsync(d_shoff, P.shoff.data(), P.shoff.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice, sm));
    TC_HIP(hipMemcpyAsync(d_tcls, P.cls.data(), P.cls.size(), hipMemcpyHostToDevice, sm));
    TC_HIP(hipMemcpyAsync(d_tscl, zeros.data(), zeros.size() * sizeof(int), hipMemcpyHostToDevice,
                          sm));
    std::vector<int> zeros4((size_t)P.ntiles * 4, 0);
    TC_HIP(hipMemcpyAsync(d_cscl, zeros4.data(), zeros4.size() * sizeof(int), hipMemcpyHostToDevice,
                          sm));
    TC_HIP(tc::launch_zero_info(sm, d_info));
    for (int c = 0; c < 2 && c < Nt; ++c)
        TC_HIP(hipMemcpyAsync(Wb[c], A + tc::tile_off(Nt, c, c) * nb2, col_bytes(c),
                              hipMemcpyDeviceToDevice, sm));
    TC_HIP(hipEventRecord(ev_go, sm));
    TC_HIP(hipStreamWaitEvent(s64, ev_go, 0));
    TC_HIP(hipStreamWaitEvent(slo, ev_go, 0));
    for (int k = 0; k < Nt; ++k) {
        double* Wk = Wb[k % 2];
        if (k >= 2) {
            TC_HIP(hipStreamWaitEvent(sm, ev_b64[k], 0));
            TC_HIP(hipStreamWaitEvent(sm, ev_blo[k], 0));
        }
        if (k >= 1) {  // tile column k-1 (no split-K: the partials belong to aux[0])
            if (P.diag64 || count(k, TC_FP64))
                TC_HIP(tc::launch_mxp_gemm_f64(sm, Wk, Nt, nb, k, k - 1, k, list(k, TC_FP64),
                                               count(k, TC_FP64), P.diag64, storage, d_toff, d_tcls,
                                               d_tscl, nullptr, 0));
            if (tc_status s = low_groups(sm, k, k - 1, k)) return s;
        }
        if (tc_status s = potrf_rec(ctx->stream, Wk, nb, 0, nb, (int64_t)k * nb, d_info, pot)) return s;
        if (k + 1 < Nt)
            TC_HIP(tc::launch_trsm_blockinv(sm, Wk + nb2, Wk, nb, (int64_t)(Nt - k - 1) * nb, pot));
        TC_HIP(hipMemcpyAsync(storage + P.toff[tc::tile_off(Nt, k, k)], Wk, nb2 * sizeof(double),
                              hipMemcpyDeviceToDevice, sm));
        TC_HIP(tc::launch_mxp_finalize(sm, Wk, Nt, nb, k, part, storage, d_toff, d_tcls, d_tscl,
                                       d_shoff, d_cscl));
        TC_HIP(hipEventRecord(ev_f[k], sm));
        const int c = k + 2;  // bulk of column c over tile columns [0, c-1) = [0, k]
        if (c < Nt) {
            TC_HIP(hipStreamWaitEvent(s64, ev_f[k], 0));
            TC_HIP(hipMemcpyAsync(Wb[c % 2], A + tc::tile_off(Nt, c, c) * nb2, col_bytes(c),
                                  hipMemcpyDeviceToDevice, s64));
            TC_HIP(hipEventRecord(ev_c[c], s64));
            // the bulk in launches of at most kBulkChunk tile columns: each
            // workgroup retires after that many, so the critical path's
            // kernels on the main stream are not held out of the CUs for a
            // whole column's K range
            for (int n0 = 0; n0 < c - 1; n0 += kBulkChunk) {
                const int n1 = std::min(c - 1, n0 + kBulkChunk);
                if (P.diag64 || count(c, TC_FP64))
                    TC_HIP(tc::launch_mxp_gemm_f64(s64, Wb[c % 2], Nt, nb, c, n0, n1,
                                                   list(c, TC_FP64), count(c, TC_FP64), P.diag64,
                                                   storage, d_toff, d_tcls, d_tscl, big,
                                                   big_cap / sizeof(double)));
            }
            TC_HIP(hipEventRecord(ev_b64[c], s64));
            TC_HIP(hipStreamWaitEvent(slo, ev_c[c], 0));
            for (int n0 = 0; n0 < c - 1; n0 += kBulkChunk)
                if (tc_status s = low_groups(slo, c, n0, std::min(c - 1, n0 + kBulkChunk))) return s;
            TC_HIP(hipEventRecord(ev_blo[c], slo));
        }
    }
    // L_kk^{-T} of every diagonal tile for the solves (the bulk streams have
    // been joined by the last column, so `big` is free for the inverted
    // 64 x 64 blocks)
    double* xinv = reinterpret_cast<double*>(storage + P.tab_xinv);
    const tc::TileView V{storage, d_toff, d_tcls, d_tscl, Nt, nb};
    TC_HIP(tc::launch_diag_tiles_inv(sm, V, big, xinv));
    TC_HIP(hipEventRecord(ctx->ev1, ctx->stream));
    int info = 0;
    TC_HIP(hipMemcpyAsync(&info, d_info, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    TC_HIP(hipStreamSynchronize(ctx->stream));

    tc_factor* f = new (std::nothrow) tc_factor();
    if (!f) return fail(TC_ENOMEM, "out of host memory");
    f->n = n;
    f->nb = nb;
    f->Nt = Nt;
    f->info = info;
    f->mixed = true;
    f->d_xinv = xinv;
    f->storage = storage;
    f->d_toff = d_toff;
    f->d_tcls = d_tcls;
    f->d_tscl = d_tscl;
    f->toff = P.toff;
    *Lout = f;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        float ms = 0.f;
        TC_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        stats->ms_total = ms;
        stats->info = info;
        const double nd = (double)n;
        stats->flops_total = nd * nd * nd / 3.0;
        for (int c = 0; c < 5; ++c) {
            stats->class_flops[c] = cflops[c];
            stats->class_tiles[c] = ctiles[c];
            stats->gemm_flops += cflops[c];
        }
    }
    return info > 0 ? info : TC_OK;
}

}  // namespace

tc_status tc_factorize(tc_ctx* ctx, int64_t n, int32_t nb, const double* A, const uint8_t* map,
                       const tc_opts* opts, void* storage, size_t storage_bytes, tc_factor** Lout,
                       tc_stats* stats) {
    if (!ctx || !A || !storage || !Lout) return fail(TC_EINVAL, "NULL argument");
    *Lout = nullptr;
    if (tc_status s = check_shape(n, nb)) return s;
    const int fp64_update = opts ? opts->fp64_update : TC_FP64;
    if (fp64_update != TC_FP64 && fp64_update != TC_FP32)
        return fail(TC_EINVAL, "opts->fp64_update must be TC_FP64 or TC_FP32");
    const int wide = opts ? opts->wide_tiles : 0;
    if (wide < -1 || wide > 1) return fail(TC_EINVAL, "opts->wide_tiles must be -1, 0 or 1");
    Plan P;
    if (!make_plan(n, nb, map, P, fp64_update))
        return fail(TC_EINVAL, "bad precision map (codes 0..4, diagonal tiles TC_FP64)");
    const size_t need = P.mixed ? P.total : (size_t)P.ntiles * nb * nb * sizeof(double);
    if (storage_bytes < need)
        return fail(TC_EINVAL, "storage too small: need " + std::to_string(need) + " bytes");
    if (P.mixed && storage == (const void*)A)
        return fail(TC_EINVAL, "a mixed-precision factor cannot overwrite its input");
    if (tc_status s = check_ws(ctx, n, nb)) return s;
    DeviceGuard g(ctx->device);
    tc_status st = P.mixed ? factorize_mixed(ctx, n, nb, A, P, static_cast<char*>(storage), wide,
                                             Lout, stats)
                           : factorize_fp64(ctx, n, nb, A, static_cast<double*>(storage), Lout, stats);
    if (st > 0) g_err = "matrix is not positive definite (column " + std::to_string(st) + ")";
    return st;
}

tc_status tc_solve(tc_ctx* ctx, const tc_factor* F, double* B, int64_t ldb, int32_t nrhs) {
    if (!ctx || !F) return fail(TC_EINVAL, "NULL argument");
    if (nrhs < 0 || ldb < F->n) return fail(TC_EINVAL, "bad nrhs or ldb");
    if (F->info > 0) return fail(TC_EINVAL, "factor is not valid (factorization failed)");
    if (nrhs == 0) return TC_OK;
    if (!B) return fail(TC_EINVAL, "NULL right-hand sides");
    if (tc_status s = check_ws(ctx, F->n, F->nb)) return s;
    DeviceGuard g(ctx->device);
    const Layout Ly = layout(F->n, F->nb);
    double* big = reinterpret_cast<double*>(ctx->ws + Ly.big);
    // the refinement area holds an n x 16 intermediate vector
    double* Y = (ldb == F->n && nrhs <= 16) ? reinterpret_cast<double*>(ctx->ws + Ly.ir) : nullptr;
    if (tc_status s = solve_enqueue(ctx, F, B, ldb, nrhs, big, Y)) return s;
    TC_HIP(hipStreamSynchronize(ctx->stream));
    return TC_OK;
}

tc_status tc_solve_refine(tc_ctx* ctx, const tc_factor* F, const double* A, double* B, int64_t ldb,
                          int32_t nrhs, int32_t max_iter, double tol, tc_ir_stats* stats) {
    if (!ctx || !F || !A || !B) return fail(TC_EINVAL, "NULL argument");
    if (nrhs <= 0 || ldb < F->n || max_iter < 0 || !(tol > 0))
        return fail(TC_EINVAL, "bad nrhs, ldb, max_iter or tol");
    if (F->info > 0) return fail(TC_EINVAL, "factor is not valid (factorization failed)");
    const Layout Ly = layout(F->n, F->nb, nrhs);
    if (ctx->ws == nullptr || ctx->ws_bytes < Ly.total)
        return fail(TC_ENOMEM, "workspace too small for " + std::to_string(nrhs) +
                                   " right-hand sides: need " + std::to_string(Ly.total) + " bytes");
    DeviceGuard g(ctx->device);
    const int64_t n = F->n;
    double* big = reinterpret_cast<double*>(ctx->ws + Ly.big);
    double* part = reinterpret_cast<double*>(ctx->ws + Ly.small);
    double* Bc = reinterpret_cast<double*>(ctx->ws + Ly.ir);  // b
    double* R = Bc + (size_t)n * nrhs;                          // residual / correction
    double* Y = R + (size_t)n * nrhs;                           // the solves' intermediate
    double* rp = Y + (size_t)n * nrhs;                          // residual partial sums
    TC_HIP(hipEventRecord(ctx->ev0, ctx->stream));
    TC_HIP(tc::launch_copy_cols(ctx->stream, Bc, n, B, ldb, n, nrhs));
    std::vector<double> bn, rn;
    if (tc_status s = colnorms(ctx, Bc, n, n, nrhs, part, bn)) return s;
    if (tc_status s = solve_enqueue(ctx, F, B, ldb, nrhs, big, ldb == n ? Y : nullptr)) return s;
    tc_ir_stats st;
    std::memset(&st, 0, sizeof(st));
    double rel = 0.0;
    int it = 0;
    for (;;) {
        TC_HIP(tc::launch_residual(ctx->stream, A, F->Nt, F->nb, B, ldb, Bc, n, nrhs, rp, R, n));
        if (tc_status s = colnorms(ctx, R, n, n, nrhs, part, rn)) return s;
        rel = 0.0;
        for (int c = 0; c < nrhs; ++c) {
            const double r = bn[c] > 0 ? rn[c] / bn[c] : rn[c];
            if (!(r <= rel)) rel = r;  // NaN propagates
        }
        if (it < 32) st.history[it] = rel;
        if (rel <= tol || it >= max_iter) break;
        if (tc_status s = solve_enqueue(ctx, F, R, n, nrhs, big, Y)) return s;
        TC_HIP(tc::launch_axpy(ctx->stream, B, ldb, R, n, n, nrhs));
        ++it;
    }
    TC_HIP(hipEventRecord(ctx->ev1, ctx->stream));
    TC_HIP(hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    TC_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    st.iterations = it;
    st.converged = rel <= tol ? 1 : 0;
    st.rel_residual = rel;
    st.ms_total = ms;
    if (stats) *stats = st;
    if (!st.converged)
        return fail(TC_ENOTCONV, "refinement stopped at relative residual " + std::to_string(rel) +
                                     " after " + std::to_string(it) + " corrections");
    return TC_OK;
}

tc_status tc_logdet(tc_ctx* ctx, const tc_factor* F, double* out) {
    if (!ctx || !F || !out) return fail(TC_EINVAL, "NULL argument");
    if (F->info > 0) return fail(TC_EINVAL, "factor is not valid (factorization failed)");
    if (tc_status s = check_ws(ctx, F->n, F->nb)) return s;
    DeviceGuard g(ctx->device);
    const Layout Ly = layout(F->n, F->nb);
    double* part = reinterpret_cast<double*>(ctx->ws + Ly.small);
    TC_HIP(tc::launch_logdet_partials(ctx->stream, view_of(F), part));
    std::vector<double> h(F->Nt);
    TC_HIP(hipMemcpyAsync(h.data(), part, F->Nt * sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
    TC_HIP(hipStreamSynchronize(ctx->stream));
    double s = 0.0;
    for (double v : h) s += v;
    *out = 2.0 * s;
    return TC_OK;
}

tc_status tc_loglik_seed(tc_ctx* ctx, const tc_factor* F, const double* y, double* Lbar,
                         double* loglik) {
    if (!ctx || !F || !y || !loglik) return fail(TC_EINVAL, "NULL argument");
    if (F->info > 0) return fail(TC_EINVAL, "factor is not valid (factorization failed)");
    if (tc_status s = check_ws(ctx, F->n, F->nb)) return s;
    DeviceGuard g(ctx->device);
    const int64_t n = F->n;
    const Layout Ly = layout(n, F->nb);
    double* big = reinterpret_cast<double*>(ctx->ws + Ly.big);
    double* part = reinterpret_cast<double*>(ctx->ws + Ly.small);
    double* z = reinterpret_cast<double*>(ctx->ws + Ly.ir);
    double* alpha = z + n;
    TC_HIP(tc::launch_copy_cols(ctx->stream, z, n, y, n, n, 1));
    if (tc_status s = fwd_enqueue(ctx, F, z, n, 1, big, nullptr)) return s;
    if (Lbar) {  // alpha = L^{-T} z only for the seed
        TC_HIP(tc::launch_copy_cols(ctx->stream, alpha, n, z, n, n, 1));
        if (tc_status s = bwd_enqueue(ctx, F, alpha, n, 1, big, nullptr)) return s;
        TC_HIP(tc::launch_loglik_seed(ctx->stream, view_of(F), alpha, z, Lbar, F->Nt, F->nb));
    }
    std::vector<double> zn;
    if (tc_status s = colnorms(ctx, z, n, n, 1, part, zn)) return s;
    double ld = 0.0;
    if (tc_status s = tc_logdet(ctx, F, &ld)) return s;
    const double pi = 3.14159265358979323846;
    *loglik = -0.5 * (double)n * std::log(2.0 * pi) - 0.5 * ld - 0.5 * zn[0] * zn[0];
    return TC_OK;
}

tc_status tc_factor_export(tc_ctx* ctx, const tc_factor* F, double* L64) {
    if (!ctx || !F || !L64) return fail(TC_EINVAL, "NULL argument");
    DeviceGuard g(ctx->device);
    if (F->mixed) {
        if ((const void*)L64 == (const void*)F->storage)
            return fail(TC_EINVAL, "export of a mixed-precision factor needs a separate buffer");
        TC_HIP(tc::launch_export(ctx->stream, view_of(F), L64));
    } else {
        const int64_t ntiles = (int64_t)F->Nt * (F->Nt + 1) / 2;
        if (L64 != F->tiles)
            TC_HIP(hipMemcpyAsync(L64, F->tiles, (size_t)ntiles * F->nb * F->nb * sizeof(double),
                                  hipMemcpyDeviceToDevice, ctx->stream));
        TC_HIP(tc::launch_zero_upper(ctx->stream, L64, F->Nt, F->nb));
    }
    TC_HIP(hipStreamSynchronize(ctx->stream));
    return TC_OK;
}

tc_status tc_factor_destroy(tc_factor* F) {
    delete F;
    return TC_OK;
}

}  // extern "C"
