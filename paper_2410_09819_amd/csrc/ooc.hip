// Panel update for the out-of-core factorization (Sections III-C, IV-B).
//
// The column being updated (the accumulator, the paper's "V1") is resident
// in HBM as a contiguous working column W: tile k+rt of column k at
// W + rt * nb^2. The operand tiles L(m, n), m >= k, n in [n0, n0 + nc),
// live wherever the tile cache put them; the host passes one device pointer
// per (row rt, chunk column q) in `tab` (row 0 = tile (k, n), the B operand).
// One launch applies one chunk of K:
//   W[rt] -= sum_{q < nc} L(k + rt, n0 + q) L(k, n0 + q)^T
// with the FP64 MFMA main loop of the in-core kernel, lower blocks only in
// the diagonal tile, and optional split-K (partials reduced in fixed order).
#include "formats.hpp"
#include "gemm_f64.hpp"

namespace tc {
namespace {

constexpr int kB = 128;

struct TabOp {
    const double* const* tab;
    int64_t nb, nc, row, r0;
    __device__ const double* operator()(int64_t kk) const {
        const int64_t q = kk / nb;
        return tab[row * nc + q] + (kk - q * nb) * nb + r0;
    }
};

__global__ __launch_bounds__(kGemmThreads, 2) void ooc_panel_kernel(
    double* __restrict__ W, int rows, int nb, int nc, const double* const* __restrict__ tab,
    int splits, int64_t kchunk, double* __restrict__ partial) {
    using Tl = MfmaTile<kB, kB>;
    __shared__ double lds[Tl::LDS_DOUBLES];
    const int T = nb / kB;
    const int64_t tri = (int64_t)T * (T + 1) / 2;
    const int64_t nblocks = tri + (int64_t)(rows - 1) * T * T;
    const int64_t logical = xcd_remap(blockIdx.x, nblocks * splits);
    const int split = (int)(logical / nblocks);
    const int64_t b = logical - (int64_t)split * nblocks;
    int64_t rt;
    int br, bc;
    if (b < tri) {
        int r = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
        while ((int64_t)(r + 1) * (r + 2) / 2 <= b) ++r;
        while ((int64_t)r * (r + 1) / 2 > b) --r;
        rt = 0;
        br = r;
        bc = (int)(b - (int64_t)r * (r + 1) / 2);
    } else {
        const int64_t b2 = b - tri;
        rt = 1 + b2 / ((int64_t)T * T);
        const int w = (int)(b2 % ((int64_t)T * T));
        br = w / T;
        bc = w % T;
    }
    const int64_t K = (int64_t)nc * nb;
    const int64_t kbeg = (int64_t)split * kchunk;
    const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
    d4 acc[Tl::MI][Tl::NI];
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
    const TabOp aop{tab, nb, nc, rt, (int64_t)br * kB};
    const TabOp bop{tab, nb, nc, 0, (int64_t)bc * kB};
    mfma_mainloop<kB, kB>(acc, aop, bop, nb, kbeg, kend, lds);
    const int64_t nb2 = (int64_t)nb * nb;
    double* out = splits == 1 ? W + rt * nb2 : partial + ((int64_t)split * rows + rt) * nb2;
    out += (int64_t)bc * kB * nb + br * kB;
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double* p = out + (int64_t)acc_col<kB, kB>(ni, v) * nb + acc_row<kB, kB>(mi);
                if (splits == 1)
                    *p -= acc[mi][ni][v];
                else
                    *p = acc[mi][ni][v];
            }
}

__global__ void ooc_reduce_kernel(double* __restrict__ W, int rows, int nb, int splits,
                                  const double* __restrict__ partial) {
    const int64_t nb2 = (int64_t)nb * nb;
    const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2;
    if (e >= rows * nb2) return;
    const int64_t rt = e / nb2, w = e - rt * nb2;
    const int64_t col = w / nb, row = w - col * nb;
    if (rt == 0 && row / kB < col / kB) return;  // upper blocks of the diagonal tile
    d2 s = *reinterpret_cast<const d2*>(partial + e);
    for (int sp = 1; sp < splits; ++sp)
        s += *reinterpret_cast<const d2*>(partial + (int64_t)sp * rows * nb2 + e);
    d2* c = reinterpret_cast<d2*>(W + e);
    *c = *c - s;
}

// One row of blocks per new tile; 16 bytes per thread and step (tile sizes
// in every class are multiples of 16 bytes, offsets multiples of 256).
__global__ __launch_bounds__(256) void image_gather_kernel(const char* __restrict__ cache,
                                                          const int64_t* __restrict__ toff,
                                                          const int64_t* __restrict__ htoff,
                                                          const uint8_t* __restrict__ tcls, int Nt,
                                                          int nb, int k, char* __restrict__ dst) {
    const int m = k + 1 + (int)blockIdx.y;
    const int64_t t = tile_off(Nt, m, k), tkk = tile_off(Nt, k, k);
    const int64_t chunks = (int64_t)nb * nb * fmt_bytes(tcls[t]) / 16;
    const uint4* src = reinterpret_cast<const uint4*>(cache + toff[t]);
    uint4* out = reinterpret_cast<uint4*>(dst + (htoff[t] - htoff[tkk]));
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < chunks; i += (int64_t)gridDim.x * 256)
        out[i] = src[i];
}

}  // namespace

hipError_t launch_image_gather(hipStream_t s, const char* cache, const int64_t* toff,
                               const int64_t* htoff, const uint8_t* tcls, int Nt, int nb, int k,
                               char* dst) {
    const int rows = Nt - k - 1;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(image_gather_kernel, dim3(64, rows), dim3(256), 0, s, cache, toff, htoff, tcls,
                       Nt, nb, k, dst);
    return hipGetLastError();
}

int64_t ooc_blocks(int rows, int nb) {
    const int64_t T = nb / kB;
    return T * (T + 1) / 2 + (int64_t)(rows - 1) * T * T;
}

hipError_t launch_ooc_panel(hipStream_t s, double* W, int rows, int nb, int nc,
                            const double* const* tab, int splits, double* partial) {
    const int64_t K = (int64_t)nc * nb;
    const int64_t kchunk = (((K + splits - 1) / splits + 15) / 16) * 16;
    const int64_t blocks = ooc_blocks(rows, nb) * splits;
    hipLaunchKernelGGL(ooc_panel_kernel, dim3((unsigned)blocks), dim3(kGemmThreads), 0, s, W, rows,
                       nb, nc, tab, splits, kchunk, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    const int64_t elems = (int64_t)rows * nb * nb / 2;
    hipLaunchKernelGGL(ooc_reduce_kernel, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0, s, W,
                       rows, nb, splits, partial);
    return hipGetLastError();
}

}  // namespace tc
