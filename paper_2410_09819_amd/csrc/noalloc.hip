// The binary64 tile Cholesky of tc_factorize for callers that cannot
// allocate device memory: every scratch buffer its kernels use (the failure
// flag, the split-K partial sums of the panel updates, those of the in-tile
// updates of the recursive POTRF) lives in one fixed device array per GPU,
// and the whole factorization runs in stream order on the context's compute
// stream (no lookahead stream, so no events either).
//
// The array is a file-scope __device__ variable: each GPU the library runs on
// holds its own copy from the module's load until the process ends. Host code
// never uses its name as an address (on the host it is only a stand-in for
// the symbol); its device address comes from hipGetSymbolAddress, taken once
// per device with that device current (at context creation) and kept in
// g_scratch_ptr.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "host_common.hpp"

namespace {

constexpr size_t kScratchBytes = TC_NOALLOC_SCRATCH_BYTES;
constexpr size_t kInfoBytes = 256;
// in-tile POTRF partial sums: the largest need over nb <= 2048 is 30.25 MiB
// (nb = 2048: two splits of a 1408 x 1408 block)
constexpr size_t kPotrfBytes = (size_t)31 << 20;
constexpr size_t kPanelBytes = kScratchBytes - kInfoBytes - kPotrfBytes;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace tc {
namespace host {

// Device address of this GPU's scratch array (device must be current).
tc_status noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(TC_EINVAL, "device index too large");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return TC_OK;
    void* p = nullptr;
    TC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = static_cast<char*>(p);
    return TC_OK;
}

}  // namespace host
}  // namespace tc

using namespace tc::host;

extern "C" tc_status tc_factorize_noalloc(tc_ctx* ctx, int64_t n, int32_t nb, const double* A,
                                          double* L, int32_t* info) {
    if (!ctx || !A || !L || !info) return fail(TC_EINVAL, "NULL argument");
    *info = 0;
    if (tc_status s = check_shape(n, nb)) return s;
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch_ptr[ctx->device];
    }
    if (!base) return fail(TC_EINVAL, "fixed scratch of the context's device not set up");
    // the in-tile POTRF's partial sums must fit their fixed region (they do
    // for every nb <= 2048; the check guards the constant)
    int64_t pneed = 0;
    for (int m = 128; m < nb; m += 128)
        for (int kd = 128; kd < nb; kd += 128) {
            const int s = tc::syrk_sub_splits(m, kd);
            if (s > 1) pneed = std::max<int64_t>(pneed, (int64_t)s * m * m * (int64_t)sizeof(double));
        }
    if ((size_t)pneed > kPotrfBytes)
        return fail(TC_ENOMEM, "tile size too large for the fixed scratch of tc_factorize_noalloc");
    DeviceGuard g(ctx->device);
    int* d_info = reinterpret_cast<int*>(base);
    double* pot = reinterpret_cast<double*>(base + kInfoBytes);
    double* big = reinterpret_cast<double*>(base + kInfoBytes + kPotrfBytes);
    const int Nt = (int)(n / nb);
    const int64_t nb2 = (int64_t)nb * nb;
    hipStream_t sm = ctx->stream;
    if ((const void*)L != (const void*)A)
        TC_HIP(hipMemcpyAsync(L, A, (size_t)Nt * (Nt + 1) / 2 * nb2 * sizeof(double),
                              hipMemcpyDeviceToDevice, sm));
    TC_HIP(tc::launch_zero_info(sm, d_info));  // the array keeps the previous call's flag
    // Algorithm 1's column order on one stream: column k's panel update over
    // tile columns [0, k), POTRF of the diagonal tile, TRSM of the tiles below
    for (int k = 0; k < Nt; ++k) {
        if (k >= 1) {
            const int sp = tc::panel_splits(Nt, nb, k, k, kPanelBytes);
            TC_HIP(tc::launch_panel_update(sm, L, Nt, nb, k, 0, k, sp, big, false));
            TC_HIP(tc::launch_panel_reduce(sm, L, Nt, nb, k, sp, big));
        }
        double* Tkk = L + tc::tile_off(Nt, k, k) * nb2;
        if (tc_status s = potrf_rec(sm, Tkk, nb, 0, nb, (int64_t)k * nb, d_info, pot)) return s;
        if (k + 1 < Nt)
            TC_HIP(tc::launch_trsm(sm, L + tc::tile_off(Nt, k + 1, k) * nb2, Tkk, nb,
                                   (int64_t)(Nt - k - 1) * nb, nb, tc::kPanelTrsmLeaf));
    }
    int h_info = 0;
    TC_HIP(hipMemcpyAsync(&h_info, d_info, sizeof(int), hipMemcpyDeviceToHost, sm));
    TC_HIP(hipStreamSynchronize(sm));
    *info = h_info;
    if (h_info > 0) return fail(h_info, "matrix is not positive definite");
    return TC_OK;
}
