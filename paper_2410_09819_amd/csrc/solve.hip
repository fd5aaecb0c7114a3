// Solves with the tile factor (Section III-D: Sigma^{-1} y and log|Sigma|
// for the likelihood of Eq. 1).
//
// Forward  L Y = B  : for each tile row k, solve with the diagonal tile, then
//                     subtract L_mk Y_k from every block below (the tile
//                     column k is contiguous in packed storage, so each L
//                     tile is read once, coalesced).
// Backward L^T X = Y: for each k from the bottom, subtract
//                     sum_{m>k} L_mk^T X_m (split over rows, partial sums
//                     reduced in a fixed order), then solve with L_kk^T.
// B is column-major (ldb), up to 16 right-hand sides per workgroup; more
// right-hand sides use more workgroups.
#include "common.hpp"

namespace tc {
namespace {

constexpr int kNR = 16;   // right-hand sides per workgroup
constexpr int kDB = 32;   // diagonal sub-block of the in-tile solve
constexpr int kDBP = kDB + 1;

// One workgroup per group of 16 right-hand sides: blocked substitution with
// L_kk (or L_kk^T), sub-blocks of 32 rows staged in LDS.
__global__ __launch_bounds__(256) void trsv_diag_kernel(const double* __restrict__ Lkk, int nb,
                                                        double* __restrict__ B, int64_t ldb,
                                                        int nrhs, int transpose) {
    __shared__ double Ls[kDB * kDBP];  // Ls[r * kDBP + c] = L[jb + r][jb + c]
    __shared__ double Ys[kDB * kNR];   // Ys[r * kNR + c]
    const int tid = threadIdx.x;
    const int c0 = blockIdx.x * kNR;
    const int nr = nrhs - c0 < kNR ? nrhs - c0 : kNR;
    double* Bc = B + (int64_t)c0 * ldb;
    const int nblk = nb / kDB;
    for (int bi = 0; bi < nblk; ++bi) {
        const int jb = transpose ? (nblk - 1 - bi) * kDB : bi * kDB;
        for (int e = tid; e < kDB * kDB; e += 256) {
            const int c = e / kDB, r = e % kDB;
            Ls[r * kDBP + c] = (r >= c) ? Lkk[(int64_t)(jb + c) * nb + jb + r] : 0.0;
        }
        for (int e = tid; e < kDB * kNR; e += 256) {
            const int c = e / kDB, r = e % kDB;
            if (c < nr) Ys[r * kNR + c] = Bc[(int64_t)c * ldb + jb + r];
        }
        __syncthreads();
        if (tid < nr) {
            const int c = tid;
            if (!transpose) {
                for (int j = 0; j < kDB; ++j) {
                    double y = Ys[j * kNR + c];
                    for (int l = 0; l < j; ++l) y -= Ls[j * kDBP + l] * Ys[l * kNR + c];
                    Ys[j * kNR + c] = y / Ls[j * kDBP + j];
                }
            } else {
                for (int j = kDB - 1; j >= 0; --j) {
                    double y = Ys[j * kNR + c];
                    for (int l = j + 1; l < kDB; ++l) y -= Ls[l * kDBP + j] * Ys[l * kNR + c];
                    Ys[j * kNR + c] = y / Ls[j * kDBP + j];
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < kDB * kNR; e += 256) {
            const int c = e / kDB, r = e % kDB;
            if (c < nr) Bc[(int64_t)c * ldb + jb + r] = Ys[r * kNR + c];
        }
        // update the rest of the tile's rows with this block
        if (!transpose) {
            const int rows = nb - jb - kDB;
            for (int e = tid; e < rows * nr; e += 256) {
                const int c = e / rows, i = jb + kDB + e % rows;
                double s = 0.0;
                for (int l = 0; l < kDB; ++l) s += Lkk[(int64_t)(jb + l) * nb + i] * Ys[l * kNR + c];
                Bc[(int64_t)c * ldb + i] -= s;
            }
        } else {
            const int rows = jb;
            for (int e = tid; e < rows * nr; e += 256) {
                const int c = e / rows, i = e % rows;
                const double* li = Lkk + (int64_t)i * nb + jb;  // L[jb + l][i] = li[l]
                double s = 0.0;
                for (int l = 0; l < kDB; ++l) s += li[l] * Ys[l * kNR + c];
                Bc[(int64_t)c * ldb + i] -= s;
            }
        }
        __threadfence_block();
        __syncthreads();
    }
}

// B_below[r][c] -= sum_j Lpanel[r][j] Y[j][c]; one thread per row.
constexpr int kFwdRows = 256;
constexpr int kFwdChunk = 128;
__global__ __launch_bounds__(kFwdRows) void fwd_update_kernel(const double* __restrict__ Lcol,
                                                              int nb, int64_t rows,
                                                              const double* __restrict__ Y,
                                                              double* __restrict__ Bb,
                                                              int64_t ldb, int nrhs) {
    __shared__ double Ys[kFwdChunk * kNR];
    const int tid = threadIdx.x;
    const int c0 = blockIdx.y * kNR;
    const int nr = nrhs - c0 < kNR ? nrhs - c0 : kNR;
    const int64_t r = (int64_t)blockIdx.x * kFwdRows + tid;
    const int64_t nb2 = (int64_t)nb * nb;
    const double* lrow = Lcol + (r / nb) * nb2 + (r % nb);
    double acc[kNR];
#pragma unroll
    for (int c = 0; c < kNR; ++c) acc[c] = 0.0;
    for (int j0 = 0; j0 < nb; j0 += kFwdChunk) {
        __syncthreads();
        for (int e = tid; e < kFwdChunk * kNR; e += kFwdRows) {
            const int c = e / kFwdChunk, j = e % kFwdChunk;
            Ys[j * kNR + c] = (c < nr) ? Y[(int64_t)(c0 + c) * ldb + j0 + j] : 0.0;
        }
        __syncthreads();
        if (r < rows) {
            for (int j = 0; j < kFwdChunk; ++j) {
                const double lv = lrow[(int64_t)(j0 + j) * nb];
#pragma unroll
                for (int c = 0; c < kNR; ++c) acc[c] += lv * Ys[j * kNR + c];
            }
        }
    }
    if (r < rows)
        for (int c = 0; c < nr; ++c) Bb[(int64_t)(c0 + c) * ldb + r] -= acc[c];
}

// partial[split][j][c] = sum over the split's rows r of Lpanel[r][j] X[r][c]
// for the 64 columns j of this workgroup's strip.
constexpr int kBwdStrip = 64;
constexpr int kBwdSub = 64;
__global__ __launch_bounds__(256) void bwd_partial_kernel(const double* __restrict__ Lcol, int nb,
                                                          int64_t rows_per_split,
                                                          const double* __restrict__ X,
                                                          int64_t ldb, int nrhs, int rhs0,
                                                          double* __restrict__ partial) {
    __shared__ double Ls[kBwdStrip * (kBwdSub + 1)];  // Ls[j * 65 + r]
    __shared__ double Xs[kBwdSub * kNR];
    const int tid = threadIdx.x;
    const int j0 = blockIdx.x * kBwdStrip;
    const int split = blockIdx.y;
    const int nr = nrhs - rhs0 < kNR ? nrhs - rhs0 : kNR;
    const int jj = tid & 63, cg = tid >> 6;  // column of the strip, group of 4 RHS
    const int64_t nb2 = (int64_t)nb * nb;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t rbeg = (int64_t)split * rows_per_split;
    for (int64_t rb = rbeg; rb < rbeg + rows_per_split; rb += kBwdSub) {
        __syncthreads();
        const double* lt = Lcol + (rb / nb) * nb2 + (rb % nb);
        for (int e = tid; e < kBwdStrip * kBwdSub; e += 256) {
            const int j = e / kBwdSub, r = e % kBwdSub;
            Ls[j * (kBwdSub + 1) + r] = lt[(int64_t)(j0 + j) * nb + r];
        }
        for (int e = tid; e < kBwdSub * kNR; e += 256) {
            const int c = e / kBwdSub, r = e % kBwdSub;
            Xs[r * kNR + c] = (c < nr) ? X[(int64_t)(rhs0 + c) * ldb + rb + r] : 0.0;
        }
        __syncthreads();
        for (int r = 0; r < kBwdSub; ++r) {
            const double lv = Ls[jj * (kBwdSub + 1) + r];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += lv * Xs[r * kNR + cg * 4 + q];
        }
    }
    double* p = partial + (int64_t)split * nb * kNR;
#pragma unroll
    for (int q = 0; q < 4; ++q) p[(int64_t)(j0 + jj) * kNR + cg * 4 + q] = acc[q];
}

__global__ void bwd_reduce_kernel(double* __restrict__ Y, int nb, int64_t ldb, int nrhs, int rhs0,
                                  int splits, const double* __restrict__ partial) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nb * kNR) return;
    const int j = e / kNR, c = e % kNR;
    if (rhs0 + c >= nrhs) return;
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += partial[(int64_t)sp * nb * kNR + e];
    Y[(int64_t)(rhs0 + c) * ldb + j] -= s;
}

__global__ __launch_bounds__(256) void logdet_kernel(const double* __restrict__ L, int Nt, int nb,
                                                     double* __restrict__ partial) {
    __shared__ double red[4];
    const int k = blockIdx.x;
    const double* t = L + tile_off(Nt, k, k) * (int64_t)nb * nb;
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) s += log(t[(int64_t)i * nb + i]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[k] = (red[0] + red[1]) + (red[2] + red[3]);
}

}  // namespace

hipError_t launch_trsv_diag(hipStream_t s, const double* Lkk, int nb, double* B, int64_t ldb,
                            int nrhs, bool transpose) {
    hipLaunchKernelGGL(trsv_diag_kernel, dim3((nrhs + kNR - 1) / kNR), dim3(256), 0, s, Lkk, nb, B,
                       ldb, nrhs, transpose ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_fwd_update(hipStream_t s, const double* Lcol, int nb, int64_t rows,
                             const double* Yk, double* Bbelow, int64_t ldb, int nrhs) {
    dim3 grid((unsigned)((rows + kFwdRows - 1) / kFwdRows), (nrhs + kNR - 1) / kNR);
    hipLaunchKernelGGL(fwd_update_kernel, grid, dim3(kFwdRows), 0, s, Lcol, nb, rows, Yk, Bbelow,
                       ldb, nrhs);
    return hipGetLastError();
}

int bwd_splits(int64_t rows) {
    // rows is a multiple of nb >= 128; aim for >= 512 workgroups with at least
    // 256 rows each
    int64_t s = rows / 256;
    if (s > 64) s = 64;
    while (s > 1 && rows % (s * kBwdSub) != 0) --s;
    return s < 1 ? 1 : (int)s;
}

hipError_t launch_bwd_update(hipStream_t s, const double* Lcol, int nb, int64_t rows,
                             const double* Xbelow, double* Yk, int64_t ldb, int nrhs,
                             double* partial, int splits) {
    for (int rhs0 = 0; rhs0 < nrhs; rhs0 += kNR) {
        dim3 grid(nb / kBwdStrip, splits);
        hipLaunchKernelGGL(bwd_partial_kernel, grid, dim3(256), 0, s, Lcol, nb, rows / splits,
                           Xbelow, ldb, nrhs, rhs0, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(bwd_reduce_kernel, dim3((nb * kNR + 255) / 256), dim3(256), 0, s, Yk, nb,
                           ldb, nrhs, rhs0, splits, partial);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_logdet_partials(hipStream_t s, const double* L, int Nt, int nb,
                                  double* partial) {
    hipLaunchKernelGGL(logdet_kernel, dim3(Nt), dim3(256), 0, s, L, Nt, nb, partial);
    return hipGetLastError();
}

}  // namespace tc
