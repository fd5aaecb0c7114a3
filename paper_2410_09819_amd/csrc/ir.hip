// Residual of the FP64 iterative-refinement solve: R = B - A X with A the
// symmetric matrix given by its packed lower tiles (binary64; the strict
// upper triangle of diagonal tiles is not read), X and B column-major
// (ldb), up to 16 right-hand sides per workgroup.
//
//   lower kernel: P_L[g][r] = sum over tile columns j of chunk g, j <= i(r),
//                 of row r of A_ij (lower part on the diagonal tile) times X_j
//   upper kernel: P_U[g][c] = sum over tile rows i of chunk g, i >= j(c), of
//                 column c of A_ij (strictly lower part on the diagonal tile)
//                 transposed times X_i
//   reduce:       R = B - sum_g P_L[g] - sum_g P_U[g]  (fixed order)
// Chunks of kChunk tiles keep the work per workgroup bounded; every partial
// slot is written (zeros when a chunk has no tiles), so the reduce reads
// defined data only.
#include "common.hpp"

namespace tc {
namespace {

constexpr int kNR = 16;
constexpr int kRowsL = 64;
constexpr int kStripU = 64;
constexpr int kSubU = 64;

__global__ __launch_bounds__(256) void symv_lower_kernel(const double* __restrict__ A, int Nt, int nb,
                                                         const double* __restrict__ X, int64_t ldb,
                                                         int nrhs, int chunk,
                                                         double* __restrict__ PL) {
    __shared__ double red[4 * kRowsL * kNR];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t n = (int64_t)Nt * nb;
    const int64_t r = (int64_t)blockIdx.x * kRowsL + lane;  // global row
    const int i = (int)(((int64_t)blockIdx.x * kRowsL) / nb);
    const int rr = (int)(r % nb);
    const int g = blockIdx.y;
    const int c0 = blockIdx.z * kNR;
    const int nr = nrhs - c0 < kNR ? nrhs - c0 : kNR;
    const int jbeg = g * chunk;
    int jend = jbeg + chunk;
    if (jend > i + 1) jend = i + 1;
    double acc[kNR];
#pragma unroll
    for (int c = 0; c < kNR; ++c) acc[c] = 0.0;
    // waves split the columns of each tile
    const int cq = nb / 4;
    for (int j = jbeg; j < jend; ++j) {
        const double* t = A + tile_off(Nt, i, j) * (int64_t)nb * nb + rr;
        const double* xj = X + (int64_t)c0 * ldb + (int64_t)j * nb;
        const int cb = wave * cq;
        int ce = cb + cq;
        if (j == i && ce > rr + 1) ce = rr + 1 > cb ? rr + 1 : cb;  // lower part only (divergent bound)
        for (int cc = cb; cc < cb + cq; ++cc) {
            if (cc >= ce) break;
            const double a = t[(int64_t)cc * nb];
#pragma unroll
            for (int c = 0; c < kNR; ++c)
                if (c < nr) acc[c] += a * xj[(int64_t)c * ldb + cc];
        }
    }
#pragma unroll
    for (int c = 0; c < kNR; ++c) red[(wave * kRowsL + lane) * kNR + c] = acc[c];
    __syncthreads();
    for (int e = tid; e < kRowsL * kNR; e += 256) {
        const int row = e % kRowsL, c = e / kRowsL;
        if (c < nr) {
            const double s = (red[(0 * kRowsL + row) * kNR + c] + red[(1 * kRowsL + row) * kNR + c]) +
                             (red[(2 * kRowsL + row) * kNR + c] + red[(3 * kRowsL + row) * kNR + c]);
            PL[((int64_t)g * nrhs + c0 + c) * n + (int64_t)blockIdx.x * kRowsL + row] = s;
        }
    }
}

__global__ __launch_bounds__(256) void symv_upper_kernel(const double* __restrict__ A, int Nt, int nb,
                                                         const double* __restrict__ X, int64_t ldb,
                                                         int nrhs, int chunk,
                                                         double* __restrict__ PU) {
    __shared__ double Ls[kStripU * (kSubU + 1)];  // Ls[c * 65 + r]
    __shared__ double Xs[kSubU * kNR];
    const int tid = threadIdx.x;
    const int64_t n = (int64_t)Nt * nb;
    const int strips = nb / kStripU;
    const int j = blockIdx.x / strips;
    const int c0 = (blockIdx.x % strips) * kStripU;  // column strip within tile column j
    const int g = blockIdx.y;
    const int rhs0 = blockIdx.z * kNR;
    const int nr = nrhs - rhs0 < kNR ? nrhs - rhs0 : kNR;
    const int jj = tid & 63, cg = tid >> 6;  // column of the strip, group of 4 RHS
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int ibeg = g * chunk, iend = ibeg + chunk;
    if (ibeg < j) ibeg = j;
    if (iend > Nt) iend = Nt;
    for (int i = ibeg; i < iend; ++i) {
        const double* t = A + tile_off(Nt, i, j) * (int64_t)nb * nb;
        for (int rb = 0; rb < nb; rb += kSubU) {
            if (i == j && rb + kSubU <= c0) continue;  // rows above the strip: upper part
            __syncthreads();
            for (int e = tid; e < kStripU * kSubU; e += 256) {
                const int c = e / kSubU, r = e % kSubU;
                const bool keep = i != j || rb + r > c0 + c;  // strictly lower on the diagonal tile
                Ls[c * (kSubU + 1) + r] = keep ? t[(int64_t)(c0 + c) * nb + rb + r] : 0.0;
            }
            for (int e = tid; e < kSubU * kNR; e += 256) {
                const int c = e / kSubU, r = e % kSubU;
                Xs[r * kNR + c] = (c < nr) ? X[(int64_t)(rhs0 + c) * ldb + (int64_t)i * nb + rb + r] : 0.0;
            }
            __syncthreads();
            for (int r = 0; r < kSubU; ++r) {
                const double lv = Ls[jj * (kSubU + 1) + r];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] += lv * Xs[r * kNR + cg * 4 + q];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = cg * 4 + q;
        if (c < nr)
            PU[((int64_t)g * nrhs + rhs0 + c) * n + (int64_t)j * nb + c0 + jj] = acc[q];
    }
}

__global__ void residual_reduce_kernel(const double* __restrict__ B, int64_t ldb, int64_t n,
                                       int nrhs, int groups, const double* __restrict__ PL,
                                       const double* __restrict__ PU, double* __restrict__ R,
                                       int64_t ldr) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nrhs) return;
    const int c = (int)(e / n);
    const int64_t row = e - (int64_t)c * n;
    double s = 0.0;
    for (int g = 0; g < groups; ++g) s += PL[((int64_t)g * nrhs + c) * n + row];
    for (int g = 0; g < groups; ++g) s += PU[((int64_t)g * nrhs + c) * n + row];
    R[(int64_t)c * ldr + row] = B[(int64_t)c * ldb + row] - s;
}

// sum of squares of each column of X (n x nrhs, ld) into part[block][c]
constexpr int kNormThreads = 256;
__global__ __launch_bounds__(kNormThreads) void colnorm_kernel(const double* __restrict__ X,
                                                               int64_t ld, int64_t n,
                                                               double* __restrict__ part) {
    __shared__ double red[kNormThreads / 64];
    const int c = blockIdx.y;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t b = (int64_t)blockIdx.x * per;
    int64_t e = b + per;
    if (e > n) e = n;
    double s = 0.0;
    for (int64_t i = b + threadIdx.x; i < e; i += kNormThreads) {
        const double v = X[(int64_t)c * ld + i];
        s += v * v;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[(int64_t)c * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void axpy_kernel(double* __restrict__ Y, int64_t ldy, const double* __restrict__ D,
                            int64_t ldd, int64_t n, int nrhs) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nrhs) return;
    const int c = (int)(e / n);
    const int64_t row = e - (int64_t)c * n;
    Y[(int64_t)c * ldy + row] += D[(int64_t)c * ldd + row];
}

__global__ void copy_cols_kernel(double* __restrict__ Y, int64_t ldy, const double* __restrict__ X,
                                 int64_t ldx, int64_t n, int nrhs) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nrhs) return;
    const int c = (int)(e / n);
    const int64_t row = e - (int64_t)c * n;
    Y[(int64_t)c * ldy + row] = X[(int64_t)c * ldx + row];
}

}  // namespace

int symv_chunk() { return 16; }

size_t residual_partial_doubles(int Nt, int nb, int nrhs) {
    const int groups = (Nt + symv_chunk() - 1) / symv_chunk();
    return (size_t)2 * groups * nrhs * (size_t)Nt * nb;
}

hipError_t launch_residual(hipStream_t s, const double* A, int Nt, int nb, const double* X,
                           int64_t ldx, const double* B, int64_t ldb, int nrhs, double* partial,
                           double* R, int64_t ldr) {
    const int chunk = symv_chunk();
    const int groups = (Nt + chunk - 1) / chunk;
    const int64_t n = (int64_t)Nt * nb;
    double* PL = partial;
    double* PU = partial + (size_t)groups * nrhs * n;
    const int zc = (nrhs + kNR - 1) / kNR;
    hipLaunchKernelGGL(symv_lower_kernel, dim3((unsigned)(n / kRowsL), groups, zc), dim3(256), 0, s,
                       A, Nt, nb, X, ldx, nrhs, chunk, PL);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(symv_upper_kernel, dim3((unsigned)(Nt * (nb / kStripU)), groups, zc),
                       dim3(256), 0, s, A, Nt, nb, X, ldx, nrhs, chunk, PU);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t tot = n * nrhs;
    hipLaunchKernelGGL(residual_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, B,
                       ldb, n, nrhs, groups, PL, PU, R, ldr);
    return hipGetLastError();
}

int colnorm_blocks() { return 64; }

hipError_t launch_colnorm(hipStream_t s, const double* X, int64_t ld, int64_t n, int nrhs,
                          double* part) {
    hipLaunchKernelGGL(colnorm_kernel, dim3(colnorm_blocks(), nrhs), dim3(kNormThreads), 0, s, X, ld,
                       n, part);
    return hipGetLastError();
}

hipError_t launch_axpy(hipStream_t s, double* Y, int64_t ldy, const double* D, int64_t ldd,
                       int64_t n, int nrhs) {
    const int64_t tot = n * nrhs;
    hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Y, ldy, D,
                       ldd, n, nrhs);
    return hipGetLastError();
}

hipError_t launch_copy_cols(hipStream_t s, double* Y, int64_t ldy, const double* X, int64_t ldx,
                            int64_t n, int nrhs) {
    const int64_t tot = n * nrhs;
    hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Y,
                       ldy, X, ldx, n, nrhs);
    return hipGetLastError();
}

}  // namespace tc
