// Out-of-core left-looking tile Cholesky (Sections III-C and IV-B).
//
// The matrix A and the factor L live in pinned host memory as packed lower
// tiles. HBM holds two working columns (the accumulators of the column
// being factored and of the next one, which is prefetched: the paper's V1)
// and a fixed-slot tile cache of the caller's size. Everything is decided by
// the static schedule, column k = 0..Nt-1:
//   1. the panel update streams the operand tiles L(m, n), m >= k, n < k,
//      through the cache in chunks of tile columns; a tile already cached is
//      reused (V2), a missing one is loaded from the host copy of L;
//   2. POTRF of the diagonal tile and TRSM of the tiles below run on the
//      working column (the diagonal factor stays in the working column until
//      every TRSM of the column is done: V3; TC_CTX_OOC_NO_V3 instead writes
//      it back after POTRF and reloads it for each tile's TRSM);
//   3. the new column is written back to host memory once (write-through),
//      and its off-diagonal tiles enter the cache when a slot is free (they
//      are needed again in every later column up to their row);
//   4. row k's tiles are dead after column k and free their slots.
// Eviction follows the static future: the victim is the cached tile whose
// next use is farthest (Belady). Within a column tiles are used in order of
// their tile column n, and every live tile is used again in the next column,
// so the farthest next use belongs to the largest n among the tiles already
// used in this column, then to the largest n still to come. A new tile (n =
// k) is used last in the next column, so it only takes a free slot.
//
// Three HIP streams at the default priority: compute (the context's), H2D
// and D2H. Events order: load -> use, last reader -> slot reuse, column done
// -> write-back, write-back -> reload from host and working-column reuse.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "host_common.hpp"

namespace tc {
hipError_t launch_ooc_panel(hipStream_t s, double* W, int rows, int nb, int nc,
                            const double* const* tab, int splits, double* partial);
int64_t ooc_blocks(int rows, int nb);
}  // namespace tc

using namespace tc::host;

namespace {

// Split-K count for one chunk launch: enough workgroups for two rounds of
// two resident workgroups per CU, K per split >= 512.
int ooc_splits(int rows, int nb, int nc, size_t big_bytes) {
    const int64_t W = tc::ooc_blocks(rows, nb);
    const int64_t K = (int64_t)nc * nb;
    int64_t s = (1024 + W - 1) / W;
    if (s > K / 512) s = K / 512;
    if (s > 32) s = 32;
    while (s > 1 && (size_t)s * rows * nb * nb * sizeof(double) > big_bytes) --s;
    return s < 1 ? 1 : (int)s;
}

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

}  // namespace

extern "C" tc_status tc_factorize_ooc(tc_ctx* ctx, int64_t n, int32_t nb, const double* A_host,
                                      double* L_host, void* cache, size_t cache_bytes,
                                      tc_ooc_stats* stats) {
    if (!ctx || !A_host || !L_host || !cache) return fail(TC_EINVAL, "NULL argument");
    if (tc_status s = check_shape(n, nb)) return s;
    if (tc_status s = check_ws(ctx, n, nb)) return s;
    const int Nt = (int)(n / nb);
    const int64_t nb2 = (int64_t)nb * nb;
    const size_t tbytes = (size_t)nb2 * sizeof(double);
    // without V3 two slots stage the reloaded diagonal tile of the TRSMs
    const bool no_v3 = (ctx->flags & TC_CTX_OOC_NO_V3) != 0;
    const int64_t stage_slots = no_v3 ? 2 : 0;
    const int64_t slots = (int64_t)(cache_bytes / tbytes) - stage_slots;
    if (slots < 2 * (int64_t)Nt)
        return fail(TC_ENOMEM, "tile cache too small: need at least " +
                                   std::to_string(2 * Nt + stage_slots) + " tiles of " +
                                   std::to_string(tbytes) + " bytes");
    DeviceGuard g(ctx->device);
    const Layout Ly = layout(n, nb);
    int* d_info = reinterpret_cast<int*>(ctx->ws + Ly.info);
    double* big = reinterpret_cast<double*>(ctx->ws + Ly.big);
    const size_t big_cap = Ly.potrf - Ly.big;
    double* pot = reinterpret_cast<double*>(ctx->ws + Ly.potrf);
    double* Wb[2] = {reinterpret_cast<double*>(ctx->ws + Ly.panel),
                     reinterpret_cast<double*>(ctx->ws + Ly.panel) + (size_t)Nt * nb2};
    // pointer tables: a ring in device workspace, staged through pinned host memory
    const int kRing = 64;
    const size_t tab_entries = (size_t)Nt * Nt / 4 + Nt;
    const double** d_ring = reinterpret_cast<const double**>(ctx->ws + Ly.lists);
    if (tc_status s = ctx_ooc_resources(ctx, (size_t)kRing * tab_entries * sizeof(void*))) return s;
    const double** h_ring = reinterpret_cast<const double**>(ctx->pinned);
    char* cbase = static_cast<char*>(cache);
    // reduced variants for the comparison of strategies: all copies on the
    // compute stream, and/or no reuse of operand tiles across columns
    const bool sync = (ctx->flags & TC_CTX_OOC_SYNC) != 0;
    const bool no_reuse = (ctx->flags & TC_CTX_OOC_NO_REUSE) != 0;
    const bool lru = (ctx->flags & TC_CTX_OOC_EVICT_LRU) != 0;
    hipStream_t cs = ctx->stream;
    hipStream_t hs = sync ? cs : ctx->h2d, ds = sync ? cs : ctx->d2h;

    Events E;
    std::vector<int> ring_ev(kRing, -1);
    int ring_next = 0;
    std::vector<int> slot_tile(slots, -1), slot_reader(slots, -1);
    std::vector<int64_t> tile_slot((size_t)Nt * (Nt + 1) / 2, -1);
    std::vector<int> free_slots;
    free_slots.reserve(slots);
    for (int64_t s = slots - 1; s >= 0; --s) free_slots.push_back((int)s);
    std::set<std::pair<int, int>> cached;  // (n, m) of cached tiles
    std::vector<int> col_d2h(Nt, -1), col_done(Nt, -1);
    int stage_reader[2] = {-1, -1};
    int evW[2] = {-1, -1};
    tc_ooc_stats st;
    std::memset(&st, 0, sizeof(st));

    auto release = [&](int64_t t, int n2, int m) {
        const int64_t s = tile_slot[t];
        if (s < 0) return;
        tile_slot[t] = -1;
        slot_tile[s] = -1;
        cached.erase({n2, m});
        free_slots.push_back((int)s);
    };
    // slot for a tile of chunk [n0, n1) of column k (may evict)
    auto take_slot = [&](int k, int n0, int n1, int& out) -> tc_status {
        if (!free_slots.empty()) {
            out = free_slots.back();
            free_slots.pop_back();
            return TC_OK;
        }
        if (cached.empty())
            return fail(TC_ENOMEM, "tile cache cannot hold one chunk of column " + std::to_string(k));
        std::pair<int, int> victim;
        if (lru) {
            // least recently used: tiles not yet read in this column were last
            // read in column k-1, at the chunk of their tile column n, so the
            // smallest n >= n1 goes first; then the smallest n read in this
            // column (never the chunk being loaded)
            auto later = cached.lower_bound({n1, -1});
            if (later != cached.end()) victim = *later;
            else if (cached.begin()->first < n0) victim = *cached.begin();
            else return fail(TC_ENOMEM, "tile cache cannot hold one chunk of column " + std::to_string(k));
            const int64_t t = tc::tile_off(Nt, victim.second, victim.first);
            out = (int)tile_slot[t];
            tile_slot[t] = -1;
            slot_tile[out] = -1;
            cached.erase(victim);
            st.evictions++;
            return TC_OK;
        }
        auto it = cached.lower_bound({n0, -1});
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
        slot_tile[out] = -1;
        cached.erase(victim);
        st.evictions++;
        return TC_OK;
    };

    TC_HIP(hipEventRecord(ctx->ev0, cs));
    TC_HIP(tc::launch_zero_info(cs, d_info));
    int e0;
    if (tc_status s = E.get(e0)) return s;
    TC_HIP(hipEventRecord(E.ev[e0], cs));
    TC_HIP(hipStreamWaitEvent(hs, E.ev[e0], 0));
    TC_HIP(hipStreamWaitEvent(ds, E.ev[e0], 0));
    // accumulators of column 0
    TC_HIP(hipMemcpyAsync(Wb[0], A_host, (size_t)Nt * tbytes, hipMemcpyHostToDevice, hs));
    st.bytes_h2d += (uint64_t)Nt * tbytes;
    if (tc_status s = E.get(evW[0])) return s;
    TC_HIP(hipEventRecord(E.ev[evW[0]], hs));

    for (int k = 0; k < Nt; ++k) {
        double* W = Wb[k & 1];
        const int rows = Nt - k;
        TC_HIP(hipStreamWaitEvent(cs, E.ev[evW[k & 1]], 0));
        if (k > 0) {
            int nc = k;
            if ((int64_t)rows * k > slots) nc = std::max<int64_t>(1, slots / (2 * (int64_t)rows));
            for (int n0 = 0; n0 < k; n0 += nc) {
                const int n1 = std::min(k, n0 + nc), q = n1 - n0;
                int loads = 0;
                for (int n2 = n0; n2 < n1; ++n2) {
                    for (int m = k; m < Nt; ++m) {
                        const int64_t t = tc::tile_off(Nt, m, n2);
                        if (tile_slot[t] >= 0) continue;
                        int s;
                        if (tc_status r = take_slot(k, n0, n1, s)) return r;
                        if (slot_reader[s] >= 0) TC_HIP(hipStreamWaitEvent(hs, E.ev[slot_reader[s]], 0));
                        TC_HIP(hipStreamWaitEvent(hs, E.ev[col_d2h[n2]], 0));
                        TC_HIP(hipMemcpyAsync(cbase + (size_t)s * tbytes, L_host + t * nb2, tbytes,
                                              hipMemcpyHostToDevice, hs));
                        tile_slot[t] = s;
                        slot_tile[s] = (int)t;
                        cached.insert({n2, m});
                        st.bytes_h2d += tbytes;
                        st.tiles_reloaded++;
                        ++loads;
                    }
                }
                if (loads) {
                    int el;
                    if (tc_status r = E.get(el)) return r;
                    TC_HIP(hipEventRecord(E.ev[el], hs));
                    TC_HIP(hipStreamWaitEvent(cs, E.ev[el], 0));
                }
                // pointer table of this chunk
                const int j = ring_next;
                ring_next = (ring_next + 1) % kRing;
                if (ring_ev[j] >= 0) TC_HIP(hipEventSynchronize(E.ev[ring_ev[j]]));
                const double** hp = h_ring + (size_t)j * tab_entries;
                for (int m = k; m < Nt; ++m)
                    for (int n2 = n0; n2 < n1; ++n2)
                        hp[(size_t)(m - k) * q + (n2 - n0)] = reinterpret_cast<const double*>(
                            cbase + (size_t)tile_slot[tc::tile_off(Nt, m, n2)] * tbytes);
                const double** dp = d_ring + (size_t)j * tab_entries;
                TC_HIP(hipMemcpyAsync(dp, hp, (size_t)rows * q * sizeof(void*), hipMemcpyHostToDevice, cs));
                const int sp = ooc_splits(rows, nb, q, big_cap);
                TC_HIP(tc::launch_ooc_panel(cs, W, rows, nb, q, dp, sp, big));
                int er;
                if (tc_status r = E.get(er)) return r;
                TC_HIP(hipEventRecord(E.ev[er], cs));
                ring_ev[j] = er;
                for (int m = k; m < Nt; ++m)
                    for (int n2 = n0; n2 < n1; ++n2)
                        slot_reader[tile_slot[tc::tile_off(Nt, m, n2)]] = er;
                // row k's tiles are dead after their use in this column
                for (int n2 = n0; n2 < n1; ++n2) release(tc::tile_off(Nt, k, n2), n2, k);
                st.chunks++;
            }
        }
        if (tc_status s = potrf_rec(ctx->stream, W, nb, 0, nb, (int64_t)k * nb, d_info, pot)) return s;
        if (rows > 1 && !no_v3) {
            // V3: the diagonal factor stays in the working column for the
            // one TRSM launch over the tiles below it
            TC_HIP(tc::launch_trsm(cs, W + nb2, W, nb, (int64_t)(rows - 1) * nb, nb,
                                   tc::kPanelTrsmLeaf));
        } else if (rows > 1) {
            // without V3 the diagonal factor goes back to host memory after
            // POTRF and each tile's TRSM loads it again (two staging slots)
            int ep, ed;
            if (tc_status r = E.get(ep)) return r;
            TC_HIP(hipEventRecord(E.ev[ep], cs));
            TC_HIP(hipStreamWaitEvent(ds, E.ev[ep], 0));
            TC_HIP(hipMemcpyAsync(L_host + tc::tile_off(Nt, k, k) * nb2, W, tbytes,
                                  hipMemcpyDeviceToHost, ds));
            st.bytes_d2h += tbytes;
            if (tc_status r = E.get(ed)) return r;
            TC_HIP(hipEventRecord(E.ev[ed], ds));
            for (int m = k + 1; m < Nt; ++m) {
                const int b = (m - k - 1) & 1;
                double* Lkk = reinterpret_cast<double*>(cbase + (size_t)(slots + b) * tbytes);
                TC_HIP(hipStreamWaitEvent(hs, E.ev[ed], 0));
                if (stage_reader[b] >= 0) TC_HIP(hipStreamWaitEvent(hs, E.ev[stage_reader[b]], 0));
                TC_HIP(hipMemcpyAsync(Lkk, L_host + tc::tile_off(Nt, k, k) * nb2, tbytes,
                                      hipMemcpyHostToDevice, hs));
                st.bytes_h2d += tbytes;
                st.tiles_reloaded++;
                int el, er;
                if (tc_status r = E.get(el)) return r;
                TC_HIP(hipEventRecord(E.ev[el], hs));
                TC_HIP(hipStreamWaitEvent(cs, E.ev[el], 0));
                TC_HIP(tc::launch_trsm(cs, W + (size_t)(m - k) * nb2, Lkk, nb, nb, nb));
                if (tc_status r = E.get(er)) return r;
                TC_HIP(hipEventRecord(E.ev[er], cs));
                stage_reader[b] = er;
            }
        }
        if (no_reuse) {  // every operand tile is loaded again in the next column
            std::vector<std::pair<int, int>> all(cached.begin(), cached.end());
            for (const auto& nm : all) release(tc::tile_off(Nt, nm.second, nm.first), nm.first, nm.second);
        }
        // new off-diagonal tiles into free slots (they are used last in the next column)
        int cached_new = 0;
        for (int m = k + 1; m < Nt && !no_reuse && !free_slots.empty(); ++m) {
            const int64_t t = tc::tile_off(Nt, m, k);
            const int s = free_slots.back();
            free_slots.pop_back();
            TC_HIP(hipMemcpyAsync(cbase + (size_t)s * tbytes, W + (size_t)(m - k) * nb2, tbytes,
                                  hipMemcpyDeviceToDevice, cs));
            tile_slot[t] = s;
            slot_tile[s] = (int)t;
            cached.insert({k, m});
            ++cached_new;
        }
        if (tc_status s = E.get(col_done[k])) return s;
        TC_HIP(hipEventRecord(E.ev[col_done[k]], cs));
        for (int m = k + 1; m < k + 1 + cached_new; ++m)
            slot_reader[tile_slot[tc::tile_off(Nt, m, k)]] = col_done[k];
        // write-back of column k (contiguous in packed order; without V3 the
        // diagonal tile went back already)
        TC_HIP(hipStreamWaitEvent(ds, E.ev[col_done[k]], 0));
        const int wb0 = (no_v3 && rows > 1) ? 1 : 0;
        TC_HIP(hipMemcpyAsync(L_host + (tc::tile_off(Nt, k, k) + wb0) * nb2, W + (size_t)wb0 * nb2,
                              (size_t)(rows - wb0) * tbytes, hipMemcpyDeviceToHost, ds));
        st.bytes_d2h += (uint64_t)(rows - wb0) * tbytes;
        if (tc_status s = E.get(col_d2h[k])) return s;
        TC_HIP(hipEventRecord(E.ev[col_d2h[k]], ds));
        // prefetch the accumulators of column k+1 into the other working column
        if (k + 1 < Nt) {
            double* Wn = Wb[(k + 1) & 1];
            if (k >= 1) {
                TC_HIP(hipStreamWaitEvent(hs, E.ev[col_done[k - 1]], 0));
                TC_HIP(hipStreamWaitEvent(hs, E.ev[col_d2h[k - 1]], 0));
            }
            // in place (L_host == A_host): column k+1 of A is still unread there
            TC_HIP(hipMemcpyAsync(Wn, A_host + tc::tile_off(Nt, k + 1, k + 1) * nb2,
                                  (size_t)(rows - 1) * tbytes, hipMemcpyHostToDevice, hs));
            st.bytes_h2d += (uint64_t)(rows - 1) * tbytes;
            if (tc_status s = E.get(evW[(k + 1) & 1])) return s;
            TC_HIP(hipEventRecord(E.ev[evW[(k + 1) & 1]], hs));
        }
    }
    TC_HIP(hipStreamWaitEvent(cs, E.ev[col_d2h[Nt - 1]], 0));
    TC_HIP(hipEventRecord(ctx->ev1, cs));
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
