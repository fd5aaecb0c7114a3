// Triangular solve X L^T = C for the tiles below a diagonal tile (the TRSM
// task of Section III-A / Algorithm 1: L_mk = A_mk L_kk^{-T}), over the whole
// column of tiles at once.
//
// Recursive on the width w of L (no explicit inverse anywhere, so the solve
// stays backward stable):
//   X1 = C1 L11^{-T};  C2 -= X1 L21^T;  X2 = C2 L22^{-T}
// The middle step is a large MFMA GEMM (M x w/2 x w/2). Widths up to the
// caller's leaf width (128 by default) are solved by a fused leaf kernel:
// each workgroup owns 64 rows and walks the columns in 64-wide blocks
// (MFMA update with the columns already solved, then substitution against
// the 64 x 64 diagonal block of L in LDS, four threads per row). With
// 128-column leaves the GEMMs carry 7/8 of the flops for w = 1024; wider
// leaves mean fewer launches and more of the work in the leaves.
//
// C rows are "tile-strided": row r of the panel lives at
// C + (r / nb) * nb^2 + (r % nb), column c at + c * nb (rows of consecutive
// tiles of a tile column, or rows of one tile when M <= nb).
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

__global__ __launch_bounds__(kGemmThreads) void trsm_leaf_kernel(double* __restrict__ C,
                                                                 const double* __restrict__ L,
                                                                 int nb, int w) {
    using Tl = MfmaTile<kRows, kCol>;
    static_assert(kRows * kP <= Tl::LDS_DOUBLES, "solve block must fit the GEMM staging area");
    __shared__ double lds[Tl::LDS_DOUBLES];
    // S[r * kP + c]: the block being solved, row-major. It reuses the GEMM
    // staging area, which the main loop has finished with (its last step ends
    // with a barrier) before S is written.
    double* S = lds;
    __shared__ double Ld[kCol * kP];  // Ld[l * kP + j] = L[jb + l][jb + j], l >= j (column j contiguous in l)
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kRows;
    const int64_t nb2 = (int64_t)nb * nb;
    double* Cb = C + (r0 / nb) * nb2 + (r0 % nb);  // row 0 of this block; column c at + c*nb
    // substitution layout: 4 threads per row; thread owns columns q + 4u
    const int sr = tid >> 2, sq = tid & 3;

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
        for (int e = tid; e < kCol * kCol; e += kGemmThreads) {
            const int j = e / kCol, l = e % kCol;  // column j, row l: coalesced in l
            if (l >= j) Ld[l * kP + j] = L[(int64_t)(jb + j) * nb + jb + l];
        }
        __syncthreads();

        // right-looking substitution on row sr: for j: x_j = y_j / L_jj, then
        // y_l -= x_j L[l][j] for l > j. Thread sq holds y_l for l = sq + 4u.
        double y[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) y[u] = S[sr * kP + sq + 4 * u];
#pragma unroll
        for (int j = 0; j < kCol; ++j) {
            const int ju = j >> 2, jq = j & 3;
            double xj = 0.0;
            if (sq == jq) {
                y[ju] = y[ju] / Ld[j * kP + j];
                xj = y[ju];
            }
            xj = __shfl(xj, (threadIdx.x & 63 & ~3) | jq, 64);
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                if (4 * u + 3 <= j) continue;  // all four columns done (compile time)
                const int l = sq + 4 * u;
                if (l > j) y[u] -= xj * Ld[l * kP + j];
            }
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) S[sr * kP + sq + 4 * u] = y[u];
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

// C (M x N, tile-strided rows) -= A (M x K, tile-strided rows) B^T, B N x K
// inside one tile (leading dimension nb). 128 x 128 blocks; M, N multiples
// of 128, K a multiple of 16.
constexpr int kGB = 128;

struct StridedOp {
    const double* base;  // row 0 of the block
    int64_t ld;
    __device__ const double* operator()(int64_t kk) const { return base + kk * ld; }
};

__global__ __launch_bounds__(kGemmThreads, 2) void strided_gemm_kernel(
    double* __restrict__ C, const double* __restrict__ A, const double* __restrict__ B, int nb,
    int64_t M, int N, int K) {
    using Tl = MfmaTile<kGB, kGB>;
    __shared__ double lds[Tl::LDS_DOUBLES];
    const int nbc = N / kGB;
    const int64_t total = (M / kGB) * nbc;
    const int64_t logical = xcd_remap(blockIdx.x, total);
    const int64_t br = logical / nbc;
    const int bc = (int)(logical - br * nbc);
    const int64_t r0 = br * kGB;
    const int64_t nb2 = (int64_t)nb * nb;
    const int64_t roff = (r0 / nb) * nb2 + (r0 % nb);

    d4 acc[Tl::MI][Tl::NI];
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
    const StridedOp aop{A + roff, nb};
    const StridedOp bop{B + (int64_t)bc * kGB, nb};
    mfma_mainloop<kGB, kGB>(acc, aop, bop, nb, 0, K, lds);

    double* out = C + roff + (int64_t)bc * kGB * nb;
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = acc_row<kGB, kGB>(mi);
                const int col = acc_col<kGB, kGB>(ni, v);
                out[(int64_t)col * nb + row] -= acc[mi][ni][v];
            }
}

// Inverses of the 64 x 64 diagonal blocks of a lower-triangular tile L
// (leading dimension nb), for trsm_blockinv_kernel: element (i, j) of
// block b's inverse goes to Dinv + j * nb + 64 b + i (so block b is a
// 64 x 64 column-major matrix with leading dimension nb). Thread j of
// workgroup b solves D x = e_j by forward substitution with IEEE division
// (x_i = 0 for i < j, so those terms drop out).
__global__ __launch_bounds__(kCol) void diag_inv_kernel(const double* __restrict__ L, int nb,
                                                        double* __restrict__ Dinv) {
    __shared__ double D[kCol * kP];  // D[i * kP + l] = L[64b + i][64b + l]
    const int b = blockIdx.x, j = threadIdx.x;
    const double* Lb = L + (int64_t)b * kCol * nb + b * kCol;
    for (int l = 0; l < kCol; ++l) D[j * kP + l] = Lb[(int64_t)l * nb + j];  // coalesced in j
    __syncthreads();
    double x[kCol];
#pragma unroll
    for (int i = 0; i < kCol; ++i) {
        double t = i == j ? 1.0 : 0.0;
#pragma unroll
        for (int l = 0; l < i; ++l) t -= D[i * kP + l] * x[l];
        x[i] = i < j ? 0.0 : t / D[i * kP + i];
    }
    double* out = Dinv + (int64_t)j * nb + b * kCol;
#pragma unroll
    for (int i = 0; i < kCol; ++i) out[i] = x[i];
}

// X L^T = C over the whole width w (a multiple of 64) in one launch, with
// the diagonal blocks' inverses from diag_inv_kernel. Each workgroup owns
// 64 rows and walks the 64-wide column blocks jb:
//   R = C_jb - X_[0,jb) L[jb, 0:jb]^T  (MFMA, written over C_jb),
//   X_jb = R D_jb^{-T}                 (MFMA, written over C_jb).
// The product with the inverse of each 64 x 64 diagonal block replaces the
// serial substitution (its error grows with the condition number of that
// block only).
// X L^T = C for the 64 rows of C at Cb (tile-strided rows, column c at
// + c * nb), walking the 64-wide column blocks jb of the width w:
//   R = C_jb - X_[0,jb) L[jb, 0:jb]^T  (MFMA, written over C_jb),
//   X_jb = R D_jb^{-T}                 (MFMA, written over C_jb),
// with D_jb^{-1} from diag_inv_kernel at Dinv + jb (leading dimension nb).
// The product with the inverse of each 64 x 64 diagonal block replaces the
// serial substitution (its error grows with the condition number of that
// block only).
__device__ __forceinline__ void blockinv_rows(double* Cb, const double* L, const double* Dinv,
                                              int nb, int w, double* lds) {
    using Tl = MfmaTile<kRows, kCol>;
    for (int jb = 0; jb < w; jb += kCol) {
        d4 acc[Tl::MI][Tl::NI];
#pragma unroll
        for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < Tl::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
        mfma_mainloop<kRows, kCol>(acc, ColOp{Cb, nb}, ColOp{L + jb, nb}, nb, 0, jb, lds);
#pragma unroll
        for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < Tl::NI; ++ni)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double* p = Cb + (int64_t)(jb + acc_col<kRows, kCol>(ni, v)) * nb +
                                acc_row<kRows, kCol>(mi);
                    *p -= acc[mi][ni][v];
                    acc[mi][ni][v] = 0.0;
                }
        __threadfence_block();
        __syncthreads();
        mfma_mainloop<kRows, kCol>(acc, ColOp{Cb + (int64_t)jb * nb, nb}, ColOp{Dinv + jb, nb}, nb, 0,
                                   kCol, lds);
        // the main loop ends with a barrier: every read of R is done
#pragma unroll
        for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < Tl::NI; ++ni)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Cb[(int64_t)(jb + acc_col<kRows, kCol>(ni, v)) * nb + acc_row<kRows, kCol>(mi)] =
                        acc[mi][ni][v];
        __threadfence_block();
        __syncthreads();
    }
}

// X L^T = C over the whole width w (a multiple of 64) in one launch; each
// workgroup owns 64 rows of C.
__global__ __launch_bounds__(kGemmThreads) void trsm_blockinv_kernel(double* __restrict__ C,
                                                                     const double* __restrict__ L,
                                                                     const double* __restrict__ Dinv,
                                                                     int nb, int w) {
    __shared__ double lds[MfmaTile<kRows, kCol>::LDS_DOUBLES];
    const int64_t r0 = (int64_t)blockIdx.x * kRows;
    double* Cb = C + (r0 / nb) * ((int64_t)nb * nb) + (r0 % nb);
    blockinv_rows(Cb, L, Dinv, nb, w, lds);
}

// The diagonal tiles of a factor (binary64 in every precision layout).
__device__ __forceinline__ const double* diag_of(const TileView& V, int k) {
    const int64_t t = tile_off(V.Nt, k, k);
    const int64_t nb2 = (int64_t)V.nb * V.nb;
    return reinterpret_cast<const double*>(V.base + (V.toff ? V.toff[t] : t * nb2 * 8));
}

// diag_inv_kernel for every diagonal tile k = blockIdx.y of a factor, into
// Dinv + k * nb * 64.
__global__ __launch_bounds__(kCol) void diag_tiles_inv_kernel(TileView V, double* __restrict__ Dinv) {
    __shared__ double D[kCol * kP];
    const int b = blockIdx.x, j = threadIdx.x, k = blockIdx.y, nb = V.nb;
    const double* Lb = diag_of(V, k) + (int64_t)b * kCol * nb + b * kCol;
    for (int l = 0; l < kCol; ++l) D[j * kP + l] = Lb[(int64_t)l * nb + j];
    __syncthreads();
    double x[kCol];
#pragma unroll
    for (int i = 0; i < kCol; ++i) {
        double t = i == j ? 1.0 : 0.0;
#pragma unroll
        for (int l = 0; l < i; ++l) t -= D[i * kP + l] * x[l];
        x[i] = i < j ? 0.0 : t / D[i * kP + i];
    }
    double* out = Dinv + (int64_t)k * nb * kCol + (int64_t)j * nb + b * kCol;
#pragma unroll
    for (int i = 0; i < kCol; ++i) out[i] = x[i];
}

// Xinv_k = L_kk^{-T} (solution of X L_kk^T = I; upper triangular,
// column-major nb x nb at Xinv + k * nb^2) for every diagonal tile k =
// blockIdx.y; workgroup blockIdx.x owns 64 rows.
__global__ __launch_bounds__(kGemmThreads) void tiles_inv_kernel(TileView V,
                                                                 const double* __restrict__ Dinv,
                                                                 double* __restrict__ Xinv) {
    __shared__ double lds[MfmaTile<kRows, kCol>::LDS_DOUBLES];
    const int k = blockIdx.y, nb = V.nb;
    const int64_t r0 = (int64_t)blockIdx.x * kRows;
    double* Cb = Xinv + (int64_t)k * nb * nb + r0;
    for (int e = threadIdx.x; e < kRows * nb; e += kGemmThreads) {  // identity rows r0 ..
        const int c = e / kRows, r = e % kRows;
        Cb[(int64_t)c * nb + r] = (r0 + r == c) ? 1.0 : 0.0;
    }
    __threadfence_block();
    __syncthreads();
    blockinv_rows(Cb, diag_of(V, k), Dinv + (int64_t)k * nb * kCol, nb, nb, lds);
}

hipError_t trsm_rec(hipStream_t s, double* C, const double* L, int nb, int64_t M, int w, int leaf) {
    if (w <= leaf) {
        hipLaunchKernelGGL(trsm_leaf_kernel, dim3((unsigned)(M / kRows)), dim3(kGemmThreads), 0, s,
                           C, L, nb, w);
        return hipGetLastError();
    }
    const int h = ((w / 2 + 127) / 128) * 128;
    hipError_t e = trsm_rec(s, C, L, nb, M, h, leaf);
    if (e != hipSuccess) return e;
    // C2 -= X1 L21^T: C2 = columns [h, w), X1 = columns [0, h), L21 = L[h:w, 0:h]
    const int64_t blocks = (M / kGB) * ((w - h) / kGB);
    hipLaunchKernelGGL(strided_gemm_kernel, dim3((unsigned)blocks), dim3(kGemmThreads), 0, s,
                       C + (int64_t)h * nb, C, L + h, nb, M, w - h, h);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return trsm_rec(s, C + (int64_t)h * nb, L + h + (int64_t)h * nb, nb, M, w - h, leaf);
}

}  // namespace

hipError_t launch_trsm(hipStream_t s, double* C, const double* L, int nb, int64_t M, int w,
                       int leaf) {
    if (M % kGB != 0 || w % kGB != 0 || leaf < 128 || leaf % kGB != 0) return hipErrorInvalidValue;
    return trsm_rec(s, C, L, nb, M, w, leaf);
}

hipError_t launch_diag_tiles_inv(hipStream_t s, const TileView& V, double* dinv, double* xinv) {
    if (V.nb % kCol != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(diag_tiles_inv_kernel, dim3((unsigned)(V.nb / kCol), (unsigned)V.Nt), dim3(kCol), 0,
                       s, V, dinv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tiles_inv_kernel, dim3((unsigned)(V.nb / kRows), (unsigned)V.Nt),
                       dim3(kGemmThreads), 0, s, V, dinv, xinv);
    return hipGetLastError();
}

hipError_t launch_trsm_blockinv(hipStream_t s, double* C, const double* L, int nb, int64_t M,
                                double* dinv) {
    if (M % kRows != 0 || nb % kCol != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(diag_inv_kernel, dim3((unsigned)(nb / kCol)), dim3(kCol), 0, s, L, nb, dinv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || M == 0) return e;
    hipLaunchKernelGGL(trsm_blockinv_kernel, dim3((unsigned)(M / kRows)), dim3(kGemmThreads), 0, s,
                       C, L, dinv, nb, nb);
    return hipGetLastError();
}

}  // namespace tc
