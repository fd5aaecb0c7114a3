// FP64 MFMA main loop shared by the GEMM/SYRK and TRSM kernels.
//
// Computes acc += A_blk * B_blk^T where A_blk is BM x K and B_blk is BN x K,
// both read column by column (consecutive rows contiguous, column stride
// `ld`): exactly how an nb x nb column-major tile stores a block of rows.
// The K range is walked in steps of BK = 16; each step is staged through a
// double-buffered LDS tile (stored k-major so a 16-lane group reads 16
// consecutive doubles) while the next step's global loads are in flight.
//
// 256 threads = 4 waves in a 2 x 2 arrangement; each wave owns a
// (BM/2) x (BN/2) sub-tile made of 16 x 16 blocks of
// v_mfma_f64_16x16x4_f64. For D = X Y (X 16x4, Y 4x16) lane l supplies
// X[l%16][l/16] and Y[l/16][l%16], and accumulator element v of lane l is
// D[l/16 + 4v][l%16] (checked on the device). The blocks are computed
// transposed, D = B_blk A_blk^T = C^T, so that element v of lane l is
// C[l%16][l/16 + 4v]: for each v, 16 lanes hold 16 consecutive rows of one
// column, and stores to column-major tiles are 128-byte contiguous runs.
#pragma once

#include "common.hpp"

namespace tc {

constexpr int kGemmThreads = 256;

template <int BM, int BN>
struct MfmaTile {
    static constexpr int BK = 16;
    static constexpr int PAD = 16;  // doubles of padding per LDS k-row (bank spread)
    static constexpr int LDA = BM + PAD;
    static constexpr int LDB = BN + PAD;
    static constexpr int MI = BM / 32;  // 16x16 blocks per wave along M
    static constexpr int NI = BN / 32;  // ... along N
    static constexpr int A_LOADS = BM * BK / 2 / kGemmThreads;  // double2 loads per thread
    static constexpr int B_LOADS = BN * BK / 2 / kGemmThreads;
    static constexpr int LDS_DOUBLES = 2 * BK * (LDA + LDB);
    static_assert(A_LOADS >= 1 && B_LOADS >= 1, "tile too small for 256 threads");
};

// Operand providers return the address of element (row 0 of the block,
// column kk); column kk+q is at ptr + q * ld for q < BK.
template <int BM, int BN, class AOp, class BOp>
__device__ __forceinline__ void mfma_mainloop(d4 (&acc)[BM / 32][BN / 32], const AOp& aop,
                                              const BOp& bop, int64_t ld, int64_t kbeg,
                                              int64_t kend, double* lds) {
    using T = MfmaTile<BM, BN>;
    if (kbeg >= kend) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    double* As = lds;                     // [2][BK][LDA]
    double* Bs = lds + 2 * T::BK * T::LDA;  // [2][BK][LDB]

    int64_t a_goff[T::A_LOADS];
    int a_soff[T::A_LOADS];
#pragma unroll
    for (int q = 0; q < T::A_LOADS; ++q) {
        const int e = (q * kGemmThreads + tid) * 2;
        const int col = e / BM, row = e % BM;
        a_goff[q] = (int64_t)col * ld + row;
        a_soff[q] = col * T::LDA + row;
    }
    int64_t b_goff[T::B_LOADS];
    int b_soff[T::B_LOADS];
#pragma unroll
    for (int q = 0; q < T::B_LOADS; ++q) {
        const int e = (q * kGemmThreads + tid) * 2;
        const int col = e / BN, row = e % BN;
        b_goff[q] = (int64_t)col * ld + row;
        b_soff[q] = col * T::LDB + row;
    }

    d2 ra[T::A_LOADS], rb[T::B_LOADS];
    auto gload = [&](int64_t kk) {
        const double* pa = aop(kk);
        const double* pb = bop(kk);
#pragma unroll
        for (int q = 0; q < T::A_LOADS; ++q) ra[q] = *reinterpret_cast<const d2*>(pa + a_goff[q]);
#pragma unroll
        for (int q = 0; q < T::B_LOADS; ++q) rb[q] = *reinterpret_cast<const d2*>(pb + b_goff[q]);
    };
    auto sstore = [&](int buf) {
        double* as = As + buf * T::BK * T::LDA;
        double* bs = Bs + buf * T::BK * T::LDB;
#pragma unroll
        for (int q = 0; q < T::A_LOADS; ++q) *reinterpret_cast<d2*>(as + a_soff[q]) = ra[q];
#pragma unroll
        for (int q = 0; q < T::B_LOADS; ++q) *reinterpret_cast<d2*>(bs + b_soff[q]) = rb[q];
    };

    gload(kbeg);
    sstore(0);
    __syncthreads();
    int buf = 0;
    const int li = lane & 15, lk = lane >> 4;
    for (int64_t kk = kbeg; kk < kend; kk += T::BK) {
        const bool more = kk + T::BK < kend;
        if (more) gload(kk + T::BK);
        const double* as = As + buf * T::BK * T::LDA + wm * (BM / 2) + li;
        const double* bs = Bs + buf * T::BK * T::LDB + wn * (BN / 2) + li;
#pragma unroll
        for (int ks = 0; ks < T::BK / 4; ++ks) {
            const int k = ks * 4 + lk;
            double a[T::MI], b[T::NI];
#pragma unroll
            for (int mi = 0; mi < T::MI; ++mi) a[mi] = as[k * T::LDA + mi * 16];
#pragma unroll
            for (int ni = 0; ni < T::NI; ++ni) b[ni] = bs[k * T::LDB + ni * 16];
#pragma unroll
            for (int mi = 0; mi < T::MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < T::NI; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[ni], a[mi], acc[mi][ni],
                                                                      0, 0, 0);
        }
        if (more) sstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
}

// Row / column (within the BM x BN block) of accumulator element v of
// block (mi, ni) for the calling lane.
template <int BM, int BN>
__device__ __forceinline__ int acc_row(int mi) {
    const int lane = threadIdx.x & 63, wm = (threadIdx.x >> 6) & 1;
    return wm * (BM / 2) + mi * 16 + (lane & 15);
}
template <int BM, int BN>
__device__ __forceinline__ int acc_col(int ni, int v) {
    const int lane = threadIdx.x & 63, wn = threadIdx.x >> 7;
    return wn * (BN / 2) + ni * 16 + (lane >> 4) + 4 * v;
}

}  // namespace tc
