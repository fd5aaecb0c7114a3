// Out-of-core mixed-precision tile Cholesky (Sections III-C, IV-B and IV-C):
// the left-looking schedule of the out-of-core FP64 path with the per-tile
// precision classes of the in-core mixed path.
//
// Host memory: A (binary64 packed lower tiles, read) and the factor image
// (every tile in its class, packed order, followed by the tile scale
// exponents), so each factor tile crosses the link in its class's bytes.
// HBM (the caller's cache buffer): the device tables of the mixed factor,
// staging for new tiles, four binary64 working columns (A's columns are
// prefetched up to three columns ahead, so the link keeps busy while the
// early, short columns compute), and fixed-size cache slots. A slot holds one tile "bundle": the stored
// tile, then the operand copies the tile is multiplied in (the same copies
// the in-core path keeps), rebuilt on the device from the stored bits when
// a tile is loaded. The class-group kernels of the in-core path run
// unchanged: their tile and copy offset tables point into the slots.
//
// Column k: (1) the updates from tile columns n < k stream the operand
// tiles (m, n), m >= k, through the cache in chunks of tile columns
// (loads of missing tiles, table updates, copy rebuilds, then the FP64
// group and the low-class groups of the chunk); (2) POTRF and TRSM on the
// working column; (3) finalize rounds the new tiles into their classes,
// straight into free slots (they are used again in the next column) or into
// a staging area (two halves, alternating by column); (4) the new tiles are
// gathered in their classes' bytes behind the binary64 diagonal tile in the
// working column, which then goes to the host image in one copy. The
// low-class groups of a chunk run on a side stream,
// concurrently with its FP64 group. Eviction is the farthest next use under
// the static schedule, as in the FP64 path; row k's tiles are dead after
// column k.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "formats.hpp"
#include "host_common.hpp"

using namespace tc::host;

namespace {

struct Events {
    std::vector<hipEvent_t> ev;
    int used = 0;
    tc_status get(int& idx) {
        if (used == (int)ev.size()) {
            hipEvent_t e;
            TC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            ev.push_back(e);
        }
        idx = used++;
        return TC_OK;
    }
    ~Events() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

// Bytes of the class-c operand copy of one tile (FP32: two FP16 planes).
size_t copy_bytes(int c, int64_t nb2) {
    return (size_t)nb2 * (c == TC_FP32 ? 4 : (size_t)tc::fmt_bytes(c));
}

// Slot layout: the stored tile (room for binary64), then one copy area per
// copy class any tile needs.
struct Bundle {
    int64_t coff[4] = {0, 0, 0, 0};
    size_t bytes = 0;
};

Bundle bundle_of(const Plan& P) {
    const int64_t nb2 = (int64_t)P.nb * P.nb;
    Bundle B;
    size_t off = align_up((size_t)nb2 * sizeof(double));
    for (int c = 1; c <= 4; ++c) {
        bool used = false;
        for (int64_t t = 0; t < P.ntiles && !used; ++t) used = P.shoff[t * 4 + c - 1] >= 0;
        if (!used) continue;
        B.coff[c - 1] = (int64_t)off;
        off += align_up(copy_bytes(c, nb2));
    }
    B.bytes = off;
    return B;
}

// End of the tile part of the plan (tiles only, packed order).
size_t tiles_end(const Plan& P) {
    const size_t tb = (size_t)P.nb * P.nb;
    size_t end = 0;
    for (int64_t t = 0; t < P.ntiles; ++t)
        end = std::max(end, (size_t)P.toff[t] + align_up(tb * tc::fmt_bytes(P.cls[t])));
    return end;
}

// Device tables at the front of the cache buffer.
struct Tables {
    size_t toff, shoff, tscl, tcls, cscl, need, lists, htoff, ring, total;
};

constexpr int kRing = 16;
constexpr int kWork = 4;  // working columns: A is prefetched up to kWork - 1 columns ahead

Tables tables_of(const Plan& P, size_t ring_entries) {
    Tables T;
    size_t off = 0;
    T.toff = off;
    off += align_up((size_t)P.ntiles * sizeof(int64_t));
    T.shoff = off;
    off += align_up((size_t)P.ntiles * 4 * sizeof(int64_t));
    T.tscl = off;
    off += align_up((size_t)P.ntiles * sizeof(int));
    T.tcls = off;
    off += align_up((size_t)P.ntiles);
    T.cscl = off;
    off += align_up((size_t)P.ntiles * 4 * sizeof(int));
    T.need = off;
    off += align_up((size_t)P.ntiles);
    T.lists = off;
    off += align_up((size_t)5 * P.Nt * P.Nt * sizeof(int));
    T.htoff = off;  // byte offsets of the tiles in the host image
    off += align_up((size_t)P.ntiles * sizeof(int64_t));
    T.ring = off;  // kRing x (ring_entries pairs of int64 + ring_entries int)
    off += (size_t)kRing * align_up(ring_entries * (2 * sizeof(int64_t) + sizeof(int)));
    T.total = off;
    return T;
}

}  // namespace

extern "C" size_t tc_ooc_mixed_host_bytes(int64_t n, int32_t nb, const uint8_t* map) {
    if (!valid_shape(n, nb) || !map) return 0;
    Plan P;
    if (!make_plan(n, nb, map, P)) return 0;
    return align_up(tiles_end(P)) + align_up((size_t)P.ntiles * sizeof(int32_t));
}

extern "C" size_t tc_ooc_mixed_cache_bytes(int64_t n, int32_t nb, const uint8_t* map, int64_t slots,
                                           const tc_opts* opts) {
    if (!valid_shape(n, nb) || !map || slots < 0) return 0;
    Plan P;
    if (!make_plan(n, nb, map, P, opts ? opts->fp64_update : TC_FP64)) return 0;
    const int Nt = P.Nt;
    const Bundle B = bundle_of(P);
    const Tables T = tables_of(P, (size_t)Nt * Nt + 2 * (size_t)Nt);
    const size_t half = (size_t)(Nt > 1 ? Nt - 1 : 1) * B.bytes;
    const size_t colmax = align_up((size_t)Nt * P.nb * P.nb * sizeof(double));
    return T.total + 2 * half + kWork * colmax + (size_t)slots * B.bytes;
}

extern "C" tc_status tc_factorize_ooc_mixed(tc_ctx* ctx, int64_t n, int32_t nb, const double* A_host,
                                            const uint8_t* map, void* L_host, size_t L_host_bytes,
                                            void* cache, size_t cache_bytes, const tc_opts* opts,
                                            tc_ooc_stats* stats) {
    if (!ctx || !A_host || !map || !L_host || !cache) return fail(TC_EINVAL, "NULL argument");
    if (tc_status s = check_shape(n, nb)) return s;
    if (tc_status s = check_ws(ctx, n, nb)) return s;
    const int fp64_update = opts ? opts->fp64_update : TC_FP64;
    if (fp64_update != TC_FP64 && fp64_update != TC_FP32)
        return fail(TC_EINVAL, "opts->fp64_update must be TC_FP64 or TC_FP32");
    const int wide = opts ? opts->wide_tiles : 0;
    if (wide < -1 || wide > 1) return fail(TC_EINVAL, "opts->wide_tiles must be -1, 0 or 1");
    Plan P;
    if (!make_plan(n, nb, map, P, fp64_update)) return fail(TC_EINVAL, "invalid precision map");
    const int Nt = P.Nt;
    const int64_t nb2 = (int64_t)nb * nb;
    const size_t host_tiles = align_up(tiles_end(P));
    if (L_host_bytes < host_tiles + (size_t)P.ntiles * sizeof(int32_t))
        return fail(TC_EINVAL, "L_host too small: need " +
                                   std::to_string(tc_ooc_mixed_host_bytes(n, nb, map)) + " bytes");
    const Bundle B = bundle_of(P);
    // slots: what is left after the tables and the staging of one column
    const size_t ring_entries = (size_t)Nt * Nt + 2 * (size_t)Nt;
    const Tables T = tables_of(P, ring_entries);
    // staging: two halves (columns alternate) of Nt - 1 bundles
    const size_t half = (size_t)(Nt > 1 ? Nt - 1 : 1) * B.bytes;
    const size_t staging = 2 * half;
    const size_t colmax = align_up((size_t)Nt * nb2 * sizeof(double));
    const size_t fixed = T.total + staging + kWork * colmax;
    const int64_t slots = cache_bytes > fixed ? (int64_t)((cache_bytes - fixed) / B.bytes) : 0;
    if (slots < 2 * (int64_t)Nt)
        return fail(TC_ENOMEM, "tile cache too small: need at least " +
                                   std::to_string(fixed + 2 * (size_t)Nt * B.bytes) + " bytes (" +
                                   std::to_string(2 * Nt) + " slots of " + std::to_string(B.bytes) +
                                   " bytes, staging and tables)");
    DeviceGuard g(ctx->device);
    const Layout Ly = layout(n, nb);
    int* d_info = reinterpret_cast<int*>(ctx->ws + Ly.info);
    double* big = reinterpret_cast<double*>(ctx->ws + Ly.big);
    const size_t big_cap = Ly.potrf - Ly.big;
    double* pot = reinterpret_cast<double*>(ctx->ws + Ly.potrf);
    double* part = reinterpret_cast<double*>(ctx->ws + Ly.small);
    char* cbase = static_cast<char*>(cache);
    int64_t* d_toff = reinterpret_cast<int64_t*>(cbase + T.toff);
    int64_t* d_shoff = reinterpret_cast<int64_t*>(cbase + T.shoff);
    int* d_tscl = reinterpret_cast<int*>(cbase + T.tscl);
    uint8_t* d_tcls = reinterpret_cast<uint8_t*>(cbase + T.tcls);
    int* d_cscl = reinterpret_cast<int*>(cbase + T.cscl);
    uint8_t* d_need = reinterpret_cast<uint8_t*>(cbase + T.need);
    int* d_lists = reinterpret_cast<int*>(cbase + T.lists);
    int64_t* d_htoff = reinterpret_cast<int64_t*>(cbase + T.htoff);
    char* d_ring = cbase + T.ring;
    const size_t ring_bytes = align_up(ring_entries * (2 * sizeof(int64_t) + sizeof(int)));
    const size_t stage0 = T.total;          // staging bundles, half h at stage0 + h * half
    const size_t work0 = T.total + staging;  // working column of column k at work0 + (k % kWork) * colmax
    const size_t slot0 = work0 + kWork * colmax;  // slot s at slot0 + s * B.bytes
    auto work = [&](int c) { return reinterpret_cast<double*>(cbase + work0 + (size_t)(c % kWork) * colmax); };
    if (tc_status s = ctx_ooc_resources(ctx, (size_t)kRing * ring_bytes)) return s;
    char* h_ring = static_cast<char*>(ctx->pinned);
    char* Lh = static_cast<char*>(L_host);
    if (tc_status s = ctx_aux_streams(ctx)) return s;
    // sa: prefetch of A's columns (host -> device), apart from the operand
    // reloads on hs so that a column of A never queues ahead of them; it is
    // the write-back stream ds (column k + kWork's prefetch waits for the
    // same event as column k's write-back and follows it)
    hipStream_t cs = ctx->stream, hs = ctx->h2d, ds = ctx->d2h, sl = ctx->aux[1], sa = ctx->d2h;

    std::vector<int> lists, lcount;
    double cflops[5];
    int ctiles[5];
    class_lists(P, lists, lcount, cflops, ctiles);
    auto list = [&](int c, int cls) { return d_lists + ((size_t)c * 5 + cls) * Nt; };
    auto count = [&](int c, int cls) { return lcount[(size_t)c * 5 + cls]; };
    std::vector<uint8_t> need(P.ntiles, 0);
    for (int64_t t = 0; t < P.ntiles; ++t)
        for (int c = 1; c <= 4; ++c)
            if (P.shoff[t * 4 + c - 1] >= 0) need[t] |= (uint8_t)(1u << c);
    auto tile_bytes = [&](int64_t t) { return (size_t)nb2 * tc::fmt_bytes(P.cls[t]); };

    Events E;
    std::vector<int> ring_ev(kRing, -1);
    int ring_next = 0;
    std::vector<int> slot_reader(slots, -1), slot_d2h(slots, -1);
    std::vector<int64_t> tile_slot(P.ntiles, -1);
    std::vector<int> free_slots;
    free_slots.reserve(slots);
    for (int64_t s = slots - 1; s >= 0; --s) free_slots.push_back((int)s);
    std::set<std::pair<int, int>> cached;  // (n, m) of cached tiles
    std::vector<int> col_d2h(Nt, -1), col_done(Nt, -1);
    int stage_last[2] = {-1, -1};  // last column whose new tiles used staging half h
    std::vector<int> evW(Nt, -1);
    tc_ooc_stats st;
    std::memset(&st, 0, sizeof(st));

    auto release = [&](int64_t t, int n2, int m) {
        const int64_t s = tile_slot[t];
        if (s < 0) return;
        tile_slot[t] = -1;
        cached.erase({n2, m});
        free_slots.push_back((int)s);
    };
    auto take_slot = [&](int k, int n0, int n1, int& out) -> tc_status {
        if (!free_slots.empty()) {
            out = free_slots.back();
            free_slots.pop_back();
            return TC_OK;
        }
        auto it = cached.lower_bound({n0, -1});
        std::pair<int, int> victim;
        if (it != cached.begin()) {
            victim = *std::prev(it);  // used already in this column, largest n
        } else {
            victim = *cached.rbegin();  // largest n still to come in this column
            if (victim.first < n1)
                return fail(TC_ENOMEM, "tile cache cannot hold one chunk of column " +
                                           std::to_string(k));
        }
        const int64_t t = tc::tile_off(Nt, victim.second, victim.first);
        out = (int)tile_slot[t];
        tile_slot[t] = -1;
        cached.erase(victim);
        st.evictions++;
        return TC_OK;
    };
    // Table updates (and the tiles whose copies to rebuild) through the ring:
    // staged in pinned memory, copied on the compute stream, applied there.
    auto apply = [&](const std::vector<int64_t>& upd, const std::vector<int>& rebuild) -> tc_status {
        const int cnt = (int)(upd.size() / 2);
        if (cnt == 0) return TC_OK;
        const int j = ring_next;
        ring_next = (ring_next + 1) % kRing;
        if (ring_ev[j] >= 0) TC_HIP(hipEventSynchronize(E.ev[ring_ev[j]]));
        char* hp = h_ring + (size_t)j * ring_bytes;
        char* dp = d_ring + (size_t)j * ring_bytes;
        std::memcpy(hp, upd.data(), upd.size() * sizeof(int64_t));
        std::memcpy(hp + ring_entries * 2 * sizeof(int64_t), rebuild.data(), rebuild.size() * sizeof(int));
        TC_HIP(hipMemcpyAsync(dp, hp, upd.size() * sizeof(int64_t), hipMemcpyHostToDevice, cs));
        if (!rebuild.empty())
            TC_HIP(hipMemcpyAsync(dp + ring_entries * 2 * sizeof(int64_t),
                                  hp + ring_entries * 2 * sizeof(int64_t), rebuild.size() * sizeof(int),
                                  hipMemcpyHostToDevice, cs));
        TC_HIP(tc::launch_slot_tables(cs, reinterpret_cast<const int64_t*>(dp), cnt, d_need, B.coff,
                                      d_toff, d_shoff));
        TC_HIP(tc::launch_mxp_copies(cs, nb, reinterpret_cast<const int*>(dp + ring_entries * 2 * sizeof(int64_t)),
                                     (int)rebuild.size(), cbase, d_toff, d_tcls, d_tscl, d_shoff, d_cscl));
        int e;
        if (tc_status r = E.get(e)) return r;
        TC_HIP(hipEventRecord(E.ev[e], cs));
        ring_ev[j] = e;
        return TC_OK;
    };

    TC_HIP(hipEventRecord(ctx->ev0, cs));
    TC_HIP(tc::launch_zero_info(cs, d_info));
    {
        std::vector<int> zeros((size_t)P.ntiles * 4, 0);
        TC_HIP(hipMemcpyAsync(d_tcls, P.cls.data(), P.cls.size(), hipMemcpyHostToDevice, cs));
        TC_HIP(hipMemcpyAsync(d_need, need.data(), need.size(), hipMemcpyHostToDevice, cs));
        TC_HIP(hipMemcpyAsync(d_tscl, zeros.data(), (size_t)P.ntiles * sizeof(int), hipMemcpyHostToDevice, cs));
        TC_HIP(hipMemcpyAsync(d_cscl, zeros.data(), zeros.size() * sizeof(int), hipMemcpyHostToDevice, cs));
        TC_HIP(hipMemcpyAsync(d_lists, lists.data(), lists.size() * sizeof(int), hipMemcpyHostToDevice, cs));
        TC_HIP(hipMemcpyAsync(d_htoff, P.toff.data(), P.toff.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice, cs));
        TC_HIP(hipStreamSynchronize(cs));  // host vectors go out of scope
    }
    int e0;
    if (tc_status s = E.get(e0)) return s;
    TC_HIP(hipEventRecord(E.ev[e0], cs));
    TC_HIP(hipStreamWaitEvent(hs, E.ev[e0], 0));
    TC_HIP(hipStreamWaitEvent(ds, E.ev[e0], 0));
    TC_HIP(hipStreamWaitEvent(sa, E.ev[e0], 0));
    // A's column c into working column c % kWork (after column c - kWork is finalized)
    auto prefetch = [&](int c) -> tc_status {
        if (c >= kWork) TC_HIP(hipStreamWaitEvent(sa, E.ev[col_done[c - kWork]], 0));
        const size_t bytes = (size_t)(Nt - c) * nb2 * sizeof(double);
        TC_HIP(hipMemcpyAsync(work(c), A_host + tc::tile_off(Nt, c, c) * nb2, bytes, hipMemcpyHostToDevice, sa));
        st.bytes_h2d += bytes;
        if (tc_status s = E.get(evW[c])) return s;
        TC_HIP(hipEventRecord(E.ev[evW[c]], sa));
        return TC_OK;
    };
    for (int c = 0; c < kWork && c < Nt; ++c)
        if (tc_status s = prefetch(c)) return s;

    std::vector<int64_t> upd;
    std::vector<int> rebuild;
    for (int k = 0; k < Nt; ++k) {
        double* W = work(k);
        const int rows = Nt - k;
        TC_HIP(hipStreamWaitEvent(cs, E.ev[evW[k]], 0));
        if (k > 0) {
            int nc = k;
            if ((int64_t)rows * k > slots) nc = (int)std::max<int64_t>(1, slots / (2 * (int64_t)rows));
            for (int n0 = 0; n0 < k; n0 += nc) {
                const int n1 = std::min(k, n0 + nc);
                upd.clear();
                rebuild.clear();
                for (int n2 = n0; n2 < n1; ++n2) {
                    for (int m = k; m < Nt; ++m) {
                        const int64_t t = tc::tile_off(Nt, m, n2);
                        if (tile_slot[t] >= 0) continue;
                        int s;
                        if (tc_status r = take_slot(k, n0, n1, s)) return r;
                        if (slot_reader[s] >= 0) TC_HIP(hipStreamWaitEvent(hs, E.ev[slot_reader[s]], 0));
                        if (slot_d2h[s] >= 0) TC_HIP(hipStreamWaitEvent(hs, E.ev[slot_d2h[s]], 0));
                        TC_HIP(hipStreamWaitEvent(hs, E.ev[col_d2h[n2]], 0));
                        const size_t so = slot0 + (size_t)s * B.bytes;
                        TC_HIP(hipMemcpyAsync(cbase + so, Lh + P.toff[t], tile_bytes(t),
                                              hipMemcpyHostToDevice, hs));
                        tile_slot[t] = s;
                        slot_d2h[s] = -1;
                        cached.insert({n2, m});
                        upd.push_back(t);
                        upd.push_back((int64_t)so);
                        rebuild.push_back((int)t);
                        st.bytes_h2d += tile_bytes(t);
                        st.tiles_reloaded++;
                    }
                }
                if (!upd.empty()) {
                    int el;
                    if (tc_status r = E.get(el)) return r;
                    TC_HIP(hipEventRecord(E.ev[el], hs));
                    TC_HIP(hipStreamWaitEvent(cs, E.ev[el], 0));
                    if (tc_status r = apply(upd, rebuild)) return r;
                }
                // the low-class groups (disjoint tiles of W) run on a side
                // stream, concurrently with the FP64 group; both join here.
                // Launches follow the in-core schedule's pieces: tile
                // columns cut at multiples of kBulkChunk up to column k - 1,
                // then column k - 1 alone (its FP64 group without split-K).
                // The sums are then formed in the in-core order, and with a
                // cache that holds the working set the factor is the in-core
                // one bit for bit.
                bool low = false;
                for (int cls = 1; cls <= 4; ++cls) low = low || count(k, cls) > 0;
                if (low) {
                    int ef;
                    if (tc_status r = E.get(ef)) return r;
                    TC_HIP(hipEventRecord(E.ev[ef], cs));
                    TC_HIP(hipStreamWaitEvent(sl, E.ev[ef], 0));
                }
                for (int p0 = n0; p0 < n1;) {
                    const int p1 = p0 == k - 1
                                       ? k
                                       : std::min({n1, k - 1, (p0 / kBulkChunk + 1) * kBulkChunk});
                    for (int cls = 1; low && cls <= 4; ++cls) {
                        const int cnt = count(k, cls);
                        if (!cnt) continue;
                        if (cls == TC_FP32)
                            TC_HIP(tc::launch_mxp_gemm_f32(sl, W, Nt, nb, k, p0, p1, list(k, cls), cnt, cbase,
                                                           d_shoff, d_cscl, wide));
                        else
                            TC_HIP(tc::launch_mxp_gemm_narrow(sl, W, Nt, nb, k, p0, p1, list(k, cls), cnt,
                                                              cls, cbase, d_shoff, d_cscl, wide));
                    }
                    if (P.diag64 || count(k, TC_FP64)) {
                        const bool last = p0 == k - 1;
                        TC_HIP(tc::launch_mxp_gemm_f64(cs, W, Nt, nb, k, p0, p1, list(k, TC_FP64),
                                                       count(k, TC_FP64), P.diag64, cbase, d_toff, d_tcls,
                                                       d_tscl, last ? nullptr : big,
                                                       last ? 0 : big_cap / sizeof(double)));
                    }
                    p0 = p1;
                }
                if (low) {
                    int ej;
                    if (tc_status r = E.get(ej)) return r;
                    TC_HIP(hipEventRecord(E.ev[ej], sl));
                    TC_HIP(hipStreamWaitEvent(cs, E.ev[ej], 0));
                }
                int er;
                if (tc_status r = E.get(er)) return r;
                TC_HIP(hipEventRecord(E.ev[er], cs));
                for (int m = k; m < Nt; ++m)
                    for (int n2 = n0; n2 < n1; ++n2)
                        slot_reader[tile_slot[tc::tile_off(Nt, m, n2)]] = er;
                // row k's tiles are dead after their use in this column
                for (int n2 = n0; n2 < n1; ++n2) release(tc::tile_off(Nt, k, n2), n2, k);
                st.chunks++;
            }
        }
        if (tc_status s = potrf_rec(ctx->stream, W, nb, 0, nb, (int64_t)k * nb, d_info, pot)) return s;
        if (rows > 1)
            TC_HIP(tc::launch_trsm_blockinv(cs, W + nb2, W, nb, (int64_t)(rows - 1) * nb, pot));
        // new tiles: free slots (used again in the next column) or staging
        // half k & 1, free once the column that last used it is written back
        const int h = k & 1;
        bool staged = false;
        upd.clear();
        rebuild.clear();
        std::vector<int> new_slot(rows, -1);
        for (int m = k + 1; m < Nt; ++m) {
            const int64_t t = tc::tile_off(Nt, m, k);
            size_t o;
            if (!free_slots.empty()) {
                const int s = free_slots.back();
                free_slots.pop_back();
                if (slot_reader[s] >= 0) TC_HIP(hipStreamWaitEvent(cs, E.ev[slot_reader[s]], 0));
                if (slot_d2h[s] >= 0) TC_HIP(hipStreamWaitEvent(cs, E.ev[slot_d2h[s]], 0));
                o = slot0 + (size_t)s * B.bytes;
                tile_slot[t] = s;
                cached.insert({k, m});
                new_slot[m - k] = s;
            } else {
                o = stage0 + (size_t)h * half + (size_t)(m - k - 1) * B.bytes;
                staged = true;
            }
            upd.push_back(t);
            upd.push_back((int64_t)o);
        }
        if (staged && stage_last[h] >= 0) TC_HIP(hipStreamWaitEvent(cs, E.ev[col_d2h[stage_last[h]]], 0));
        if (staged) stage_last[h] = k;
        if (tc_status r = apply(upd, rebuild)) return r;
        TC_HIP(tc::launch_mxp_finalize(cs, W, Nt, nb, k, part, cbase, d_toff, d_tcls, d_tscl, d_shoff,
                                       d_cscl));
        // the column's image in the working column: the binary64 diagonal
        // tile is already at its start, the new tiles follow in their
        // classes' bytes at their host-image offsets (W is free once
        // finalized; the next prefetch into it runs on the write-back stream,
        // after this column's copy)
        TC_HIP(tc::launch_image_gather(cs, cbase, d_toff, d_htoff, d_tcls, Nt, nb, k,
                                       reinterpret_cast<char*>(W)));
        if (tc_status s = E.get(col_done[k])) return s;
        TC_HIP(hipEventRecord(E.ev[col_done[k]], cs));
        // write-back of column k in its classes: one contiguous copy
        TC_HIP(hipStreamWaitEvent(ds, E.ev[col_done[k]], 0));
        const int64_t tkk = tc::tile_off(Nt, k, k), tlast = tc::tile_off(Nt, Nt - 1, k);
        const size_t col_bytes = (size_t)(P.toff[tlast] - P.toff[tkk]) + tile_bytes(tlast);
        TC_HIP(hipMemcpyAsync(Lh + P.toff[tkk], W, col_bytes, hipMemcpyDeviceToHost, ds));
        st.bytes_d2h += col_bytes;
        if (tc_status s = E.get(col_d2h[k])) return s;
        TC_HIP(hipEventRecord(E.ev[col_d2h[k]], ds));
        for (int m = k + 1; m < Nt; ++m)
            if (new_slot[m - k] >= 0) {
                slot_reader[new_slot[m - k]] = col_done[k];
                slot_d2h[new_slot[m - k]] = col_d2h[k];
            }
        // A's column k + kWork into the working column column k just released
        if (k + kWork < Nt)
            if (tc_status s = prefetch(k + kWork)) return s;
    }
    TC_HIP(hipStreamWaitEvent(cs, E.ev[col_d2h[Nt - 1]], 0));
    TC_HIP(hipEventRecord(ctx->ev1, cs));
    TC_HIP(hipMemcpyAsync(Lh + host_tiles, d_tscl, (size_t)P.ntiles * sizeof(int32_t),
                          hipMemcpyDeviceToHost, cs));
    int info = 0;
    TC_HIP(hipMemcpyAsync(&info, d_info, sizeof(int), hipMemcpyDeviceToHost, cs));
    TC_HIP(hipStreamSynchronize(cs));
    TC_HIP(hipStreamSynchronize(hs));
    TC_HIP(hipStreamSynchronize(ds));
    float ms = 0.f;
    TC_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    st.ms_total = ms;
    st.info = info;
    st.flops_total = (double)n * n * n / 3.0;
    st.cache_slots = (int32_t)slots;
    if (stats) *stats = st;
    if (info > 0) {
        g_err = "matrix is not positive definite (column " + std::to_string(info) + ")";
        return info;
    }
    return TC_OK;
}
