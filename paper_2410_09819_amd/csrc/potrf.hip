// POTRF of a small diagonal block (the leaf of the recursive in-tile
// factorization; Section III-A, the POTRF task of Algorithm 1).
//
// One workgroup loads the lower triangle of an s x s block (s <= 128) into
// LDS and runs the right-looking column algorithm there: pivot square root,
// column scaling, rank-1 update of the trailing lower triangle. A pivot that
// is not strictly positive (or NaN) stops the block and records LAPACK's
// info (1-based global column) if no earlier failure was recorded.
#include "common.hpp"

namespace tc {
namespace {

constexpr int kLeafMax = 128;
constexpr int kLeafThreads = 256;
constexpr int kPW = 16;          // panel width
constexpr int kPP = kPW + 1;     // LDS row pitch of the panel

// Blocked right-looking POTRF of an s x s block (s <= 128, a multiple of 16)
// by one workgroup. 256 threads as a 16 x 16 grid: thread (tx, ty) owns the
// 8 x 8 elements (tx + 16p, ty + 16q) in registers. For each 16-column panel:
//   1. the owners publish the panel's lower part in LDS;
//   2. wave 0 factors the panel with one or two rows per lane: pivot square
//      root, column scaling and the in-panel updates, values exchanged with
//      lane shuffles (no barriers);
//   3. every thread takes the factored panel back and applies the rank-16
//      update to the trailing elements it owns.
// Every loop is unrolled with compile-time indices (the panel loop too), so
// the tile stays in plain registers; a failed pivot turns the remaining
// work off through uniform predicates.
template <int pb>
__device__ __forceinline__ void leaf_panel(double (&a)[8][8], double* P, int* fail, int* info,
                                           int64_t col0, int s) {
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int j0 = pb * kPW;
    // 1. publish the panel (column j0 + ty, rows >= that column)
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int i = tx + 16 * p;
        if (p >= pb && i >= j0 + ty && i < s) P[i * kPP + ty] = a[p][pb];
    }
    __syncthreads();
    // 2. wave 0 factors rows j0..s-1 of the panel
    if (tid < 64) {
        const int lane = tid;
        const int r0 = j0 + lane, r1 = j0 + lane + 64;
        const bool v0 = r0 < s, v1 = r1 < s;
        double x0[kPW], x1[kPW];
#pragma unroll
        for (int l = 0; l < kPW; ++l) {
            x0[l] = v0 ? P[r0 * kPP + l] : 0.0;
            x1[l] = v1 ? P[r1 * kPP + l] : 0.0;
        }
        bool ok = true;
#pragma unroll
        for (int jj = 0; jj < kPW; ++jj) {
            const double d = readlane_d(x0[jj], jj);  // uniform across the wave
            if (ok && !(d > 0.0)) {
                ok = false;
                if (lane == 0) {
                    *fail = 1;
                    atomicCAS(info, 0, (int)(col0 + j0 + jj + 1));
                }
            }
            if (ok) {
                const double sd = sqrt(d);
                const double rd = 1.0 / sd;
                if (lane == jj) x0[jj] = sd;
                if (lane > jj) x0[jj] *= rd;
                x1[jj] *= rd;
#pragma unroll
                for (int cc = jj + 1; cc < kPW; ++cc) {
                    const double lc = readlane_d(x0[jj], cc);  // L[j0 + cc][j0 + jj]
                    if (lane >= cc) x0[cc] -= x0[jj] * lc;
                    x1[cc] -= x1[jj] * lc;
                }
            }
        }
        if (ok) {
#pragma unroll
            for (int l = 0; l < kPW; ++l) {
                if (v0) P[r0 * kPP + l] = x0[l];
                if (v1) P[r1 * kPP + l] = x1[l];
            }
        }
    }
    __syncthreads();
    if (*fail) return;  // uniform
    // 3a. panel owners take the factored panel back
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int i = tx + 16 * p;
        if (p >= pb && i >= j0 + ty && i < s) a[p][pb] = P[i * kPP + ty];
    }
    // 3b. rank-16 update of the trailing elements (rows and columns >= j0 + 16)
    if (pb < 7) {
#pragma unroll 2
        for (int l = 0; l < kPW; ++l) {
            double li[8], lc[8];
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                li[p] = (p > pb && tx + 16 * p < s) ? P[(tx + 16 * p) * kPP + l] : 0.0;
                lc[p] = (p > pb && ty + 16 * p < s) ? P[(ty + 16 * p) * kPP + l] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (q <= pb) continue;
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                    if (p < q) continue;
                    a[p][q] -= li[p] * lc[q];
                }
            }
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kLeafThreads) void potrf_leaf_kernel(double* __restrict__ T, int ld,
                                                                  int s, int* __restrict__ info,
                                                                  int64_t col0) {
    __shared__ double P[kLeafMax * kPP];  // P[i * kPP + l] = element (i, j0 + l)
    __shared__ int fail;
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    double a[8][8];
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = tx + 16 * p, c = ty + 16 * q;
            a[p][q] = (i < s && c < s && i >= c) ? T[(int64_t)c * ld + i] : 0.0;
        }
    if (tid == 0) fail = 0;
    __syncthreads();
    const int npan = s / kPW;
    // one instantiation per panel: every register index is a constant
    if (npan > 0 && !fail) leaf_panel<0>(a, P, &fail, info, col0, s);
    if (npan > 1 && !fail) leaf_panel<1>(a, P, &fail, info, col0, s);
    if (npan > 2 && !fail) leaf_panel<2>(a, P, &fail, info, col0, s);
    if (npan > 3 && !fail) leaf_panel<3>(a, P, &fail, info, col0, s);
    if (npan > 4 && !fail) leaf_panel<4>(a, P, &fail, info, col0, s);
    if (npan > 5 && !fail) leaf_panel<5>(a, P, &fail, info, col0, s);
    if (npan > 6 && !fail) leaf_panel<6>(a, P, &fail, info, col0, s);
    if (npan > 7 && !fail) leaf_panel<7>(a, P, &fail, info, col0, s);

#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = tx + 16 * p, c = ty + 16 * q;
            if (i < s && c < s && i >= c) T[(int64_t)c * ld + i] = a[p][q];
        }
}

__global__ void zero_info_kernel(int* info) {
    if (threadIdx.x == 0) *info = 0;
}

__global__ void zero_upper_kernel(double* __restrict__ L, int Nt, int nb) {
    const int k = blockIdx.y;
    double* t = L + tile_off(Nt, k, k) * (int64_t)nb * nb;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nb * nb) return;
    const int64_t c = e / nb, r = e - c * nb;
    if (r < c) t[e] = 0.0;
}

}  // namespace

hipError_t launch_potrf_leaf(hipStream_t s, double* T, int ld, int size, int* info, int64_t col0) {
    if (size > kLeafMax || size % kPW != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(potrf_leaf_kernel, dim3(1), dim3(kLeafThreads), 0, s, T, ld, size, info,
                       col0);
    return hipGetLastError();
}

hipError_t launch_zero_info(hipStream_t s, int* info) {
    hipLaunchKernelGGL(zero_info_kernel, dim3(1), dim3(64), 0, s, info);
    return hipGetLastError();
}

hipError_t launch_zero_upper(hipStream_t s, double* L, int Nt, int nb) {
    const int64_t e = (int64_t)nb * nb;
    hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)((e + 255) / 256), Nt), dim3(256), 0, s,
                       L, Nt, nb);
    return hipGetLastError();
}

}  // namespace tc
