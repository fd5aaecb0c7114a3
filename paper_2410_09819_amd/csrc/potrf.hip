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
constexpr int kLeafP = kLeafMax + 1;
constexpr int kLeafThreads = 512;

__global__ __launch_bounds__(kLeafThreads) void potrf_leaf_kernel(double* __restrict__ T, int ld,
                                                                  int s, int* __restrict__ info,
                                                                  int64_t col0) {
    __shared__ double a[kLeafMax * kLeafP];  // a[c * kLeafP + r], column-major
    __shared__ int fail;
    const int tid = threadIdx.x;
    for (int e = tid; e < s * s; e += kLeafThreads) {
        const int c = e / s, r = e % s;
        if (r >= c) a[c * kLeafP + r] = T[(int64_t)c * ld + r];
    }
    if (tid == 0) fail = 0;
    __syncthreads();

    for (int j = 0; j < s; ++j) {
        if (tid == 0) {
            const double d = a[j * kLeafP + j];
            if (!(d > 0.0)) {
                fail = 1;
                atomicCAS(info, 0, (int)(col0 + j + 1));
            } else {
                a[j * kLeafP + j] = sqrt(d);
            }
        }
        __syncthreads();
        if (fail) break;
        const double dj = a[j * kLeafP + j];
        for (int i = j + 1 + tid; i < s; i += kLeafThreads) a[j * kLeafP + i] /= dj;
        __syncthreads();
        const int m = s - j - 1;
        for (int e = tid; e < m * m; e += kLeafThreads) {
            const int c = j + 1 + e / m, i = j + 1 + e % m;
            if (i >= c) a[c * kLeafP + i] -= a[j * kLeafP + i] * a[j * kLeafP + c];
        }
        __syncthreads();
    }

    for (int e = tid; e < s * s; e += kLeafThreads) {
        const int c = e / s, r = e % s;
        if (r >= c) T[(int64_t)c * ld + r] = a[c * kLeafP + r];
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
    if (size > kLeafMax) return hipErrorInvalidValue;
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
