// Host-side pieces shared by the C-ABI translation units: the context and
// factor objects, error reporting, workspace layout, argument checks and the
// recursive in-tile POTRF driver.
#pragma once

#include <hip/hip_runtime.h>

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
    // the library's per-device streams (device_streams; borrowed, not owned):
    // two more compute streams for the lookahead and class-group schedules,
    // and the copy streams; d2h is the same stream as aux[0]
    hipStream_t aux[2] = {nullptr, nullptr};
    hipEvent_t aux_ev[3] = {nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> la_ev;     // lookahead schedule events
    std::vector<hipEvent_t> solve_ev;  // triangular-solve lookahead events
    hipStream_t h2d = nullptr, d2h = nullptr;
    // out-of-core staging, created on first use
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
};

struct tc_factor {
    int64_t n = 0;
    int nb = 0;
    int Nt = 0;
    double* tiles = nullptr;  // all-FP64 factor: packed binary64 tiles
    int info = 0;
    // mixed-precision factor: tiles per class inside `storage`, tables on the
    // device (also inside `storage`) and the tile offsets on the host
    bool mixed = false;
    char* storage = nullptr;
    const int64_t* d_toff = nullptr;
    const uint8_t* d_tcls = nullptr;
    const int* d_tscl = nullptr;
    std::vector<int64_t> toff;
    // mixed factor: L_kk^{-T} of every diagonal tile (binary64, column-major
    // nb x nb, in tile order) for the solves
    const double* d_xinv = nullptr;
};

namespace tc {
namespace host {

// Records msg as the calling thread's last error and returns s.
tc_status fail(tc_status s, const std::string& msg);
extern thread_local std::string g_err;

inline size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

struct Layout {
    size_t info, big, potrf, small, panel, lists, ir, total;
};

Layout layout(int64_t n, int nb, int nrhs = 16);
bool valid_shape(int64_t n, int nb);
tc_status check_shape(int64_t n, int nb);
tc_status check_ws(tc_ctx* ctx, int64_t n, int nb);
// The library's three streams on `device` (created on first call, shared by
// all contexts on the device, kept until the process ends).
tc_status device_streams(int device, hipStream_t out[3]);
// A pinned staging buffer of at least `bytes` bytes in the context (grown
// on demand).
tc_status ctx_ooc_resources(tc_ctx* ctx, size_t bytes);
// The events that order the auxiliary streams in the context (once).
tc_status ctx_aux_streams(tc_ctx* ctx);
// Storage plan of a mixed-precision factor (tiles per class in packed order,
// then the operand copies, then the device tables); see make_plan.
struct Plan {
    int Nt = 0, nb = 0;
    int64_t ntiles = 0;
    std::vector<uint8_t> cls;
    // class whose arithmetic computes the updates into each tile: cls, or
    // TC_FP32 for the FP64 tiles when their updates run in FP32
    std::vector<uint8_t> ccls;
    bool diag64 = true;  // the diagonal SYRK runs in binary64
    std::vector<int64_t> toff, shoff;  // shoff[t * 4 + c - 1], -1 if absent
    size_t tab_toff = 0, tab_shoff = 0, tab_tscl = 0, tab_tcls = 0, tab_cscl = 0, tab_xinv = 0,
           total = 0;
    bool mixed = false;
};
// Fills P for map (NULL: all FP64); false if the map is invalid.
// fp64_update: arithmetic of the updates into FP64-class tiles, diagonal
// SYRK included (TC_FP64, or TC_FP32: the split-FP16 FP32 class; the plan
// is then mixed even for an all-FP64 map).
bool make_plan(int64_t n, int nb, const uint8_t* map, Plan& P, int fp64_update = 0);
// Tile columns per bulk group launch of the mixed schedule (16: measured
// against 8, 32 and whole columns at n = 131072, nb = 1024). The out-of-core
// mixed schedule cuts its group launches at the same multiples.
constexpr int kBulkChunk = 16;
// Row lists of a mixed factorization: for column k and compute class c, the
// rows r (tile k + r; r = 0, the diagonal, only in the FP32 list when the
// diagonal SYRK runs in FP32) at lists[(k * 5 + c) * Nt + i], i < count[k *
// 5 + c]; flops per compute class.
void class_lists(const Plan& P, std::vector<int>& lists, std::vector<int>& count,
                 double* cflops, int* ctiles);
// Read-only device view of a factor's tiles (any precision layout).
tc::TileView factor_view(const tc_factor* F);
// POTRF of the s x s block at offset o of a diagonal tile (leading dim nb),
// recursive halving down to 128 x 128 leaves; failures set *info.
tc_status potrf_rec(hipStream_t st, double* T, int nb, int o, int s, int64_t col0, int* info,
                    double* big);

// Device address of `device`'s fixed scratch array of tc_factorize_noalloc,
// taken once per device with the device current (context creation).
tc_status noalloc_scratch_init(int device);

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

}  // namespace host
}  // namespace tc

#define TC_HIP(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::tc::host::fail(TC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)
