// Triangular solve X L^T = C for the tiles below a diagonal tile (the TRSM
// task of Section III-A / Algorithm 1: L_mk = A_mk L_kk^{-T}), as one launch
// over the whole column of tiles.
//
// Each workgroup owns 64 rows of the panel and walks the w columns in
// 64-wide blocks, left to right (blocked forward substitution, no explicit
// inverse, so the solve stays backward stable):
//   1. R = C[:, jb] - X[:, 0:jb] L[jb, 0:jb]^T   (FP64 MFMA, K = jb)
//   2. X[:, jb] = R L[jb, jb]^{-T}               (substitution, one thread
//                                                  per row, L block in LDS)
// X overwrites C. Rows of the workgroup are re-read from global memory by
// the same workgroup in later blocks; a workgroup-scope fence and barrier
// order those accesses.
#include "gemm_f64.hpp"

namespace tc {
namespace {

constexpr int kRows = 64;
constexpr int kCol = 64;
constexpr int kP = kCol + 1;  // LDS row pitch (bank spread)

struct ColOp {
    const double* base;
    int64_t ld;
    __device__ const double* operator()(int64_t kk) const { return base + kk * ld; }
};

__global__ __launch_bounds__(kGemmThreads) void trsm_kernel(double* __restrict__ C,
                                                            const double* __restrict__ L, int nb,
                                                            int w) {
    using Tl = MfmaTile<kRows, kCol>;
    __shared__ double lds[Tl::LDS_DOUBLES];
    __shared__ double S[kRows * kP];  // S[r * kP + c]: the block being solved, row-major
    __shared__ double Ld[kCol * kP];  // Ld[j * kP + l] = L[jb + j][jb + l], l <= j
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kRows;
    const int64_t nb2 = (int64_t)nb * nb;
    double* Cb = C + (r0 / nb) * nb2 + (r0 % nb);  // row 0 of this block; column c at + c*nb

    for (int jb = 0; jb < w; jb += kCol) {
        d4 acc[Tl::MI][Tl::NI];
#pragma unroll
        for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < Tl::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
        const ColOp aop{Cb, nb};
        const ColOp bop{L + jb, nb};
        mfma_mainloop<kRows, kCol>(acc, aop, bop, nb, 0, jb, lds);

        // R = C[:, jb block] - acc  -> S (row-major)
#pragma unroll
        for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < Tl::NI; ++ni)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = acc_row<kRows, kCol>(mi);
                    const int col = acc_col<kRows, kCol>(ni, v);
                    S[row * kP + col] = Cb[(int64_t)(jb + col) * nb + row] - acc[mi][ni][v];
                }
        // diagonal block of L, lower part
        for (int e = tid; e < kCol * kCol; e += kGemmThreads) {
            const int l = e / kCol, j = e % kCol;  // column l, row j: coalesced in j
            if (j >= l) Ld[j * kP + l] = L[(int64_t)(jb + l) * nb + jb + j];
        }
        __syncthreads();

        if (tid < kRows) {
            double* s = S + tid * kP;
            for (int j = 0; j < kCol; ++j) {
                const double* lj = Ld + j * kP;
                double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
                int l = 0;
                for (; l + 4 <= j; l += 4) {
                    p0 += s[l] * lj[l];
                    p1 += s[l + 1] * lj[l + 1];
                    p2 += s[l + 2] * lj[l + 2];
                    p3 += s[l + 3] * lj[l + 3];
                }
                for (; l < j; ++l) p0 += s[l] * lj[l];
                s[j] = (s[j] - ((p0 + p1) + (p2 + p3))) / lj[j];
            }
        }
        __syncthreads();

        // X block -> global, coalesced along rows
        for (int e = tid; e < kRows * kCol; e += kGemmThreads) {
            const int c = e / kRows, r = e % kRows;
            Cb[(int64_t)(jb + c) * nb + r] = S[r * kP + c];
        }
        __threadfence_block();
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_trsm(hipStream_t s, double* C, const double* L, int nb, int64_t M, int w) {
    hipLaunchKernelGGL(trsm_kernel, dim3((unsigned)(M / kRows)), dim3(kGemmThreads), 0, s, C, L,
                       nb, w);
    return hipGetLastError();
}

}  // namespace tc
