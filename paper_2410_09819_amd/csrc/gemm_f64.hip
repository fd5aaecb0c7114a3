// Panel update of the left-looking tile Cholesky (Section III-A,
// Algorithm 1): for column of tiles k, every tile (m, k), m >= k, receives
//   A_mk -= sum_{n<k} L_mn L_kn^T
// (SYRK for m = k, GEMM for m > k). All of column k's updates are one
// launch: a GEMM whose M dimension runs over tiles k..Nt-1 of the column,
// N = nb, K = k*nb running over the tiles to the left. The accumulator of
// every output block stays in registers for the whole K loop (the paper's
// "V1" accumulator reuse, Section IV-B, at register level), and in the
// diagonal tile only blocks on or below the diagonal are computed (SYRK).
//
// When the panel has too few output blocks to fill 256 CUs (late columns),
// K is split: each split writes its partial sum to workspace and a reduce
// kernel subtracts the splits' sum from the tile in a fixed order.
//
// Workgroup -> block mapping is XCD-aware: hardware workgroup ids are dealt
// round-robin to the 8 XCDs, so ids are remapped so that each XCD works on a
// contiguous run of logical blocks; consecutive logical blocks share their
// A rows, which then stay in that XCD's L2.
#include "gemm_f64.hpp"

namespace tc {
namespace {

constexpr int kPanelBM = 128;
constexpr int kSubB = 64;

// Decode logical block b of a panel into (global block-row gb, block-col bc).
// Blocks of the diagonal tile come first, lower triangle only, row by row.
__device__ __forceinline__ void panel_block(int64_t b, int T, int64_t& gb, int& bc) {
    const int64_t tri = (int64_t)T * (T + 1) / 2;
    if (b < tri) {
        int br = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
        while ((int64_t)(br + 1) * (br + 2) / 2 <= b) ++br;
        while ((int64_t)br * (br + 1) / 2 > b) --br;
        gb = br;
        bc = (int)(b - (int64_t)br * (br + 1) / 2);
    } else {
        const int64_t b2 = b - tri;
        gb = T + b2 / T;
        bc = (int)(b2 % T);
    }
}

struct PanelA {
    const double* L;
    int64_t Nt, nb, nb2, rowtile, r0;
    __device__ const double* operator()(int64_t kk) const {
        const int64_t n = kk / nb;
        return L + tile_off(Nt, rowtile, n) * nb2 + (kk - n * nb) * nb + r0;
    }
};

// TAIL only separates the rank-nb launches of the lookahead schedule (K =
// one tile column) from the bulk launches in kernel traces.
template <bool TAIL>
__global__ __launch_bounds__(kGemmThreads, 2) void panel_update_kernel(
    double* __restrict__ L, int Nt, int nb, int k, int nbeg, int nend, int splits, int64_t nblocks,
    int64_t kchunk, double* __restrict__ partial) {
    using Tl = MfmaTile<kPanelBM, kPanelBM>;
    __shared__ double lds[Tl::LDS_DOUBLES];
    const int64_t logical = xcd_remap(blockIdx.x, nblocks * splits);
    const int split = (int)(logical / nblocks);
    const int64_t b = logical - (int64_t)split * nblocks;
    const int T = nb / kPanelBM;
    int64_t gb;
    int bc;
    panel_block(b, T, gb, bc);
    const int64_t rt = gb / T;                    // tile row within the panel (0 = diagonal)
    const int64_t r0 = (gb % T) * kPanelBM;       // first row inside that tile
    const int64_t nb2 = (int64_t)nb * nb;

    // K range: tile columns [nbeg, nend), as absolute column indices of row k
    const int64_t Kend = (int64_t)nend * nb;
    const int64_t kbeg = (int64_t)nbeg * nb + (int64_t)split * kchunk;
    const int64_t kend = kbeg + kchunk < Kend ? kbeg + kchunk : Kend;

    d4 acc[Tl::MI][Tl::NI];
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};

    const PanelA aop{L, Nt, nb, nb2, k + rt, r0};
    const PanelA bop{L, Nt, nb, nb2, k, (int64_t)bc * kPanelBM};
    mfma_mainloop<kPanelBM, kPanelBM>(acc, aop, bop, nb, kbeg, kend, lds);

    double* out;
    if (splits == 1)
        out = L + tile_off(Nt, k + rt, k) * nb2;
    else
        out = partial + ((int64_t)split * (Nt - k) + rt) * nb2;
    out += (int64_t)bc * kPanelBM * nb + r0;
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = acc_row<kPanelBM, kPanelBM>(mi);
                const int col = acc_col<kPanelBM, kPanelBM>(ni, v);
                double* p = out + (int64_t)col * nb + row;
                if (splits == 1)
                    *p -= acc[mi][ni][v];
                else
                    *p = acc[mi][ni][v];
            }
}

// C_tile -= sum_s partial_s over the computed blocks of the panel.
__global__ void panel_reduce_kernel(double* __restrict__ L, int Nt, int nb, int k, int splits,
                                    const double* __restrict__ partial) {
    const int64_t nb2 = (int64_t)nb * nb;
    const int64_t R = Nt - k;
    const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2;
    if (e >= R * nb2) return;
    const int64_t rt = e / nb2, w = e - rt * nb2;
    const int64_t col = w / nb, row = w - col * nb;
    if (rt == 0 && row / kPanelBM < col / kPanelBM) return;  // block above the diagonal
    d2 s = *reinterpret_cast<const d2*>(partial + e);
    for (int sp = 1; sp < splits; ++sp)
        s += *reinterpret_cast<const d2*>(partial + (int64_t)sp * R * nb2 + e);
    d2* c = reinterpret_cast<d2*>(L + tile_off(Nt, k + rt, k) * nb2 + w);
    *c = *c - s;
}

struct SubOp {
    const double* base;
    int64_t ld;
    __device__ const double* operator()(int64_t kk) const { return base + kk * ld; }
};

// In-tile SYRK: C (m x m, lower 64x64 blocks) -= A A^T, A m x kdim, all
// column-major with leading dimension ld.
__global__ __launch_bounds__(kGemmThreads) void syrk_sub_kernel(double* __restrict__ C,
                                                                const double* __restrict__ A,
                                                                int ld, int m, int kdim, int splits,
                                                                int64_t nblocks,
                                                                double* __restrict__ partial) {
    using Tl = MfmaTile<kSubB, kSubB>;
    __shared__ double lds[Tl::LDS_DOUBLES];
    const int64_t logical = blockIdx.x;
    const int split = (int)(logical / nblocks);
    const int64_t b = logical - (int64_t)split * nblocks;
    int br = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((int64_t)(br + 1) * (br + 2) / 2 <= b) ++br;
    while ((int64_t)br * (br + 1) / 2 > b) --br;
    const int bc = (int)(b - (int64_t)br * (br + 1) / 2);
    const int64_t kchunk = (((kdim + splits - 1) / splits + 15) / 16) * 16;
    const int64_t kbeg = (int64_t)split * kchunk;
    const int64_t kend = kbeg + kchunk < kdim ? kbeg + kchunk : kdim;

    d4 acc[Tl::MI][Tl::NI];
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
    const SubOp aop{A + br * kSubB, ld};
    const SubOp bop{A + bc * kSubB, ld};
    mfma_mainloop<kSubB, kSubB>(acc, aop, bop, ld, kbeg, kend, lds);

    double* out;
    int64_t ldo;
    if (splits == 1) {
        out = C;
        ldo = ld;
    } else {
        out = partial + (int64_t)split * m * m;
        ldo = m;
    }
    out += (int64_t)bc * kSubB * ldo + br * kSubB;
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = acc_row<kSubB, kSubB>(mi);
                const int col = acc_col<kSubB, kSubB>(ni, v);
                double* p = out + (int64_t)col * ldo + row;
                if (splits == 1)
                    *p -= acc[mi][ni][v];
                else
                    *p = acc[mi][ni][v];
            }
}

__global__ void syrk_sub_reduce_kernel(double* __restrict__ C, int ld, int m, int splits,
                                       const double* __restrict__ partial) {
    const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2;
    if (e >= (int64_t)m * m) return;
    const int col = (int)(e / m), row = (int)(e - (int64_t)col * m);
    if (row / kSubB < col / kSubB) return;
    d2 s = *reinterpret_cast<const d2*>(partial + e);
    for (int sp = 1; sp < splits; ++sp)
        s += *reinterpret_cast<const d2*>(partial + (int64_t)sp * m * m + e);
    d2* c = reinterpret_cast<d2*>(C + (int64_t)col * ld + row);
    *c = *c - s;
}

}  // namespace

int64_t panel_blocks(int Nt, int nb, int k) {
    const int64_t T = nb / kPanelBM;
    return T * (T + 1) / 2 + (int64_t)(Nt - k - 1) * T * T;
}

// Split K for columns whose panel has few output blocks. Each split keeps
// >= 512 of K and the partial sums stay under cap_bytes. The count minimises
// an estimate of the column's time: rounds of 512 resident workgroups
// (2 per CU) times one workgroup's K/S share at the FP64 MFMA rate, plus
// writing and re-reading the partial sums at HBM speed; fewer splits win
// unless clearly faster.
int panel_splits(int Nt, int nb, int k, int ncols, size_t cap_bytes) {
    const int64_t W = panel_blocks(Nt, nb, k);
    const int64_t K = (int64_t)ncols * nb;
    const double panel_bytes = (double)(Nt - k) * nb * nb * sizeof(double);
    int64_t smax = K / 512;
    if (smax > 32) smax = 32;
    while (smax > 1 && smax * panel_bytes > (double)cap_bytes) --smax;
    if (smax < 1) return 1;
    const int64_t slots = 512;
    const double slot_flops = 78.6e12 / slots;
    double best = 1e300;
    int bests = 1;
    for (int64_t s = 1; s <= smax; ++s) {
        const double rounds = (double)((W * s + slots - 1) / slots);
        double t = rounds * (2.0 * 128 * 128 * ((double)K / s)) / slot_flops;
        if (s > 1) t += 2.0 * s * panel_bytes / 5e12;
        if (t < best * 0.97) {
            best = t;
            bests = (int)s;
        }
    }
    return bests;
}

hipError_t launch_panel_update(hipStream_t s, double* L, int Nt, int nb, int k, int nbeg, int nend,
                               int splits, double* partial, bool tail) {
    const int64_t W = panel_blocks(Nt, nb, k);
    const int64_t K = (int64_t)(nend - nbeg) * nb;
    if (K <= 0) return hipSuccess;
    const int64_t kchunk = (((K + splits - 1) / splits + 15) / 16) * 16;  // covers K
    if (tail)
        hipLaunchKernelGGL(panel_update_kernel<true>, dim3((unsigned)(W * splits)), dim3(kGemmThreads),
                           0, s, L, Nt, nb, k, nbeg, nend, splits, W, kchunk, partial);
    else
        hipLaunchKernelGGL(panel_update_kernel<false>, dim3((unsigned)(W * splits)), dim3(kGemmThreads),
                           0, s, L, Nt, nb, k, nbeg, nend, splits, W, kchunk, partial);
    return hipGetLastError();
}

hipError_t launch_panel_reduce(hipStream_t s, double* L, int Nt, int nb, int k, int splits,
                               const double* partial) {
    if (splits == 1) return hipSuccess;
    const int64_t elems = (int64_t)(Nt - k) * nb * nb / 2;
    hipLaunchKernelGGL(panel_reduce_kernel, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0, s,
                       L, Nt, nb, k, splits, partial);
    return hipGetLastError();
}

int syrk_sub_splits(int m, int kdim) {
    const int64_t T = m / kSubB;
    const int64_t W = T * (T + 1) / 2;
    int64_t s = (256 + W - 1) / W;
    const int64_t smax = kdim / 128;
    if (s > smax) s = smax;
    return s < 1 ? 1 : (int)s;
}

hipError_t launch_syrk_sub(hipStream_t s, double* C, const double* A, int ld, int m, int kdim,
                           double* partial, int splits) {
    const int64_t T = m / kSubB;
    const int64_t W = T * (T + 1) / 2;
    hipLaunchKernelGGL(syrk_sub_kernel, dim3((unsigned)(W * splits)), dim3(kGemmThreads), 0, s, C,
                       A, ld, m, kdim, splits, W, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    const int64_t elems = (int64_t)m * m / 2;
    hipLaunchKernelGGL(syrk_sub_reduce_kernel, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0,
                       s, C, ld, m, splits, partial);
    return hipGetLastError();
}

}  // namespace tc
