// Mixed-precision panel update and tile finalization (Section IV-C).
//
// Each off-diagonal tile has a class (FP64, FP32, FP16, BF16 or FP8 e4m3)
// that decides how it is stored and how the updates into it are computed:
//   C_mk = A_mk - sum_{n<k} Q_p(Lh_mn) Q_p(Lh_kn)^T,   p = class(m, k)
// where Lh are the stored factor tiles and Q_p rounds a stored tile to class
// p with its per-tile scale. Diagonal tiles and FP64-class tiles use FP64
// MFMA on the stored operands, upcast exactly while they are staged into LDS.
// The low classes use FP32 MFMA with FP32 accumulation on "operand copies":
// for every tile and every low class it will be multiplied in (known from
// the static schedule), the finalize step writes Q_p(Lh) in binary32. For
// FP16, BF16 and FP8 operands every product of two operands is exact in
// binary32 (barring underflow), so this computes what a narrow-format MFMA with FP32
// accumulation computes (same rounded operands, exact products, binary32
// sums; only the summation order may differ). For FP32-class tiles the
// products are rounded to binary32 as usual. POTRF and TRSM run in FP64 on a working
// copy of the column; finalize rounds each new tile to its class (with its
// scale) into the factor storage and writes its operand copies.
#include "formats.hpp"
#include "gemm_f64.hpp"

namespace tc {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kB = 128;       // output block
constexpr int kStrips = 16;   // strips per tile for amax / cast
constexpr int kThreads = 256;

__device__ __forceinline__ int64_t xcd_remap_m(int64_t hw, int64_t total) {
    const int64_t xcd = hw % 8, idx = hw / 8;
    const int64_t q = total / 8, r = total % 8;
    return xcd * q + (xcd < r ? xcd : r) + idx;
}

// ---------------------------------------------------------------------------
// FP64 main loop over operands stored in any class (upcast while staging).
// ---------------------------------------------------------------------------
struct MixedTile {
    const char* base;  // tile start
    int cls;
    int scale;
};

template <class AOp, class BOp>
__device__ __forceinline__ void mixed_mainloop(d4 (&acc)[kB / 32][kB / 32], const AOp& aop,
                                               const BOp& bop, int64_t nb, int64_t kbeg,
                                               int64_t kend, double* lds) {
    using T = MfmaTile<kB, kB>;
    if (kbeg >= kend) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    double* As = lds;
    double* Bs = lds + 2 * T::BK * T::LDA;
    int ecol[T::A_LOADS], erow[T::A_LOADS];
#pragma unroll
    for (int q = 0; q < T::A_LOADS; ++q) {
        const int e = (q * kGemmThreads + tid) * 2;
        ecol[q] = e / kB;
        erow[q] = e % kB;
    }
    d2 ra[T::A_LOADS], rb[T::B_LOADS];
    auto load2 = [&](const MixedTile& t, int64_t idx) -> d2 {
        if (t.cls == kFP64) return *reinterpret_cast<const d2*>(reinterpret_cast<const double*>(t.base) + idx);
        return d2{load_elem(t.base, idx, t.cls, t.scale), load_elem(t.base, idx + 1, t.cls, t.scale)};
    };
    auto gload = [&](int64_t kk) {
        int64_t ia, ib;
        const MixedTile ta = aop(kk, ia), tb = bop(kk, ib);
#pragma unroll
        for (int q = 0; q < T::A_LOADS; ++q) ra[q] = load2(ta, ia + (int64_t)ecol[q] * nb + erow[q]);
#pragma unroll
        for (int q = 0; q < T::B_LOADS; ++q) rb[q] = load2(tb, ib + (int64_t)ecol[q] * nb + erow[q]);
    };
    auto sstore = [&](int buf) {
        double* as = As + buf * T::BK * T::LDA;
        double* bs = Bs + buf * T::BK * T::LDB;
#pragma unroll
        for (int q = 0; q < T::A_LOADS; ++q)
            *reinterpret_cast<d2*>(as + ecol[q] * T::LDA + erow[q]) = ra[q];
#pragma unroll
        for (int q = 0; q < T::B_LOADS; ++q)
            *reinterpret_cast<d2*>(bs + ecol[q] * T::LDB + erow[q]) = rb[q];
    };
    gload(kbeg);
    sstore(0);
    __syncthreads();
    int buf = 0;
    const int li = lane & 15, lk = lane >> 4;
    for (int64_t kk = kbeg; kk < kend; kk += T::BK) {
        const bool more = kk + T::BK < kend;
        if (more) gload(kk + T::BK);
        const double* as = As + buf * T::BK * T::LDA + wm * (kB / 2) + li;
        const double* bs = Bs + buf * T::BK * T::LDB + wn * (kB / 2) + li;
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

// Stored tile (m, n) as a MixedTile; idx = element offset of column kk % nb
// plus the first row r0.
struct StoredOp {
    const char* storage;
    const int64_t* toff;
    const uint8_t* tcls;
    const int* tscl;
    int64_t Nt, nb, row_tile, r0;
    __device__ MixedTile operator()(int64_t kk, int64_t& idx) const {
        const int64_t n = kk / nb;
        const int64_t t = tile_off(Nt, row_tile, n);
        idx = (kk - n * nb) * nb + r0;
        return MixedTile{storage + toff[t], (int)tcls[t], tscl[t]};
    }
};

// Decode logical block b of a class group: the diagonal tile's lower
// blocks first (when the group includes it), then T x T blocks per listed
// row tile.
__device__ __forceinline__ void group_block(int64_t b, int T, bool diag, const int* rows,
                                            int64_t& rt, int& br, int& bc) {
    const int64_t tri = diag ? (int64_t)T * (T + 1) / 2 : 0;
    if (b < tri) {
        int r = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
        while ((int64_t)(r + 1) * (r + 2) / 2 <= b) ++r;
        while ((int64_t)r * (r + 1) / 2 > b) --r;
        rt = 0;
        br = r;
        bc = (int)(b - (int64_t)r * (r + 1) / 2);
    } else {
        const int64_t b2 = b - tri;
        rt = rows[b2 / ((int64_t)T * T)];
        const int w = (int)(b2 % ((int64_t)T * T));
        br = w / T;
        bc = w % T;
    }
}

// FP64 group of column k: W[rt] -= sum_n Lh(k+rt, n) Lh(k, n)^T for rt in
// the diagonal tile (lower blocks, when diag) and the listed row tiles.
__global__ __launch_bounds__(kGemmThreads, 2) void mxp_gemm_f64_kernel(
    double* __restrict__ W, int Nt, int nb, int k, const int* __restrict__ rows, int nrows, int diag,
    const char* __restrict__ storage, const int64_t* __restrict__ toff,
    const uint8_t* __restrict__ tcls, const int* __restrict__ tscl) {
    using Tl = MfmaTile<kB, kB>;
    __shared__ double lds[Tl::LDS_DOUBLES];
    const int T = nb / kB;
    const int64_t total = (diag ? (int64_t)T * (T + 1) / 2 : 0) + (int64_t)nrows * T * T;
    const int64_t b = xcd_remap_m(blockIdx.x, total);
    int64_t rt;
    int br, bc;
    group_block(b, T, diag != 0, rows, rt, br, bc);
    d4 acc[Tl::MI][Tl::NI];
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
    const StoredOp aop{storage, toff, tcls, tscl, Nt, nb, k + rt, (int64_t)br * kB};
    const StoredOp bop{storage, toff, tcls, tscl, Nt, nb, k, (int64_t)bc * kB};
    mixed_mainloop(acc, aop, bop, nb, 0, (int64_t)k * nb, lds);
    double* out = W + rt * (int64_t)nb * nb + (int64_t)bc * kB * nb + br * kB;
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                out[(int64_t)acc_col<kB, kB>(ni, v) * nb + acc_row<kB, kB>(mi)] -= acc[mi][ni][v];
}

// ---------------------------------------------------------------------------
// FP32 MFMA main loop over binary32 operand copies (column-major tiles).
// v_mfma_f32_16x16x4_f32: lane l supplies X[l%16][l/16], Y[l/16][l%16];
// accumulator element v of lane l is D[4(l/16) + v][l%16] (checked on the
// device). Blocks are computed as C^T = B A^T so element v of lane l is
// C[l%16][4(l/16) + v].
// ---------------------------------------------------------------------------
constexpr int kBK32 = 16;
constexpr int kPad32 = 16;
constexpr int kLD32 = kB + kPad32;
constexpr int kLoads32 = kB * kBK32 / 4 / kGemmThreads;  // float4 loads per thread per operand

struct CopyOp {
    const char* storage;
    const int64_t* shoff;
    int cls;
    int64_t Nt, nb, row_tile, r0;
    __device__ const float* operator()(int64_t kk) const {
        const int64_t n = kk / nb;
        const int64_t t = tile_off(Nt, row_tile, n);
        return reinterpret_cast<const float*>(storage + shoff[t * 4 + (cls - 1)]) +
               (kk - n * nb) * nb + r0;
    }
};

__global__ __launch_bounds__(kGemmThreads, 2) void mxp_gemm_f32_kernel(
    double* __restrict__ W, int Nt, int nb, int k, const int* __restrict__ rows, int nrows, int cls,
    const char* __restrict__ storage, const int64_t* __restrict__ shoff) {
    __shared__ float As[2 * kBK32 * kLD32];
    __shared__ float Bs[2 * kBK32 * kLD32];
    const int T = nb / kB;
    const int64_t total = (int64_t)nrows * T * T;
    const int64_t b = xcd_remap_m(blockIdx.x, total);
    int64_t rt;
    int br, bc;
    group_block(b, T, false, rows, rt, br, bc);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const CopyOp aop{storage, shoff, cls, Nt, nb, k + rt, (int64_t)br * kB};
    const CopyOp bop{storage, shoff, cls, Nt, nb, k, (int64_t)bc * kB};
    int ecol[kLoads32], erow[kLoads32];
#pragma unroll
    for (int q = 0; q < kLoads32; ++q) {
        const int e = (q * kGemmThreads + tid) * 4;
        ecol[q] = e / kB;
        erow[q] = e % kB;
    }
    f4 acc[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = f4{0.f, 0.f, 0.f, 0.f};
    f4 ra[kLoads32], rb[kLoads32];
    auto gload = [&](int64_t kk) {
        const float* pa = aop(kk);
        const float* pb = bop(kk);
#pragma unroll
        for (int q = 0; q < kLoads32; ++q) {
            ra[q] = *reinterpret_cast<const f4*>(pa + (int64_t)ecol[q] * nb + erow[q]);
            rb[q] = *reinterpret_cast<const f4*>(pb + (int64_t)ecol[q] * nb + erow[q]);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < kLoads32; ++q) {
            *reinterpret_cast<f4*>(As + buf * kBK32 * kLD32 + ecol[q] * kLD32 + erow[q]) = ra[q];
            *reinterpret_cast<f4*>(Bs + buf * kBK32 * kLD32 + ecol[q] * kLD32 + erow[q]) = rb[q];
        }
    };
    const int64_t K = (int64_t)k * nb;
    if (K > 0) {
        gload(0);
        sstore(0);
        __syncthreads();
        int buf = 0;
        const int li = lane & 15, lk = lane >> 4;
        for (int64_t kk = 0; kk < K; kk += kBK32) {
            const bool more = kk + kBK32 < K;
            if (more) gload(kk + kBK32);
            const float* as = As + buf * kBK32 * kLD32 + wm * (kB / 2) + li;
            const float* bs = Bs + buf * kBK32 * kLD32 + wn * (kB / 2) + li;
#pragma unroll
            for (int ks = 0; ks < kBK32 / 4; ++ks) {
                const int kq = ks * 4 + lk;
                float a[4], bq[4];
#pragma unroll
                for (int mi = 0; mi < 4; ++mi) a[mi] = as[kq * kLD32 + mi * 16];
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) bq[ni] = bs[kq * kLD32 + ni * 16];
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 4; ++ni)
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(bq[ni], a[mi], acc[mi][ni],
                                                                          0, 0, 0);
            }
            if (more) sstore(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }
    double* out = W + rt * (int64_t)nb * nb + (int64_t)bc * kB * nb + br * kB;
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wm * (kB / 2) + mi * 16 + (lane & 15);
                const int col = wn * (kB / 2) + ni * 16 + 4 * (lane >> 4) + v;
                out[(int64_t)col * nb + row] -= (double)acc[mi][ni][v];
            }
}

// ---------------------------------------------------------------------------
// Finalize the tiles below the diagonal of column k: amax, then rounding to
// the tile's class with its scale, and the operand copies.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void tile_amax_kernel(const double* __restrict__ W, int nb,
                                                             double* __restrict__ part) {
    __shared__ double red[kThreads / 64];
    const int rt = blockIdx.y, strip = blockIdx.x;
    const int64_t per = (int64_t)nb * nb / kStrips;
    const double* p = W + (int64_t)rt * nb * nb + strip * per;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < per; i += kThreads) m = fmax(m, fabs(p[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int w = 1; w < kThreads / 64; ++w) t = fmax(t, red[w]);
        part[rt * kStrips + strip] = t;
    }
}

__global__ __launch_bounds__(kThreads) void tile_cast_kernel(
    const double* __restrict__ W, int Nt, int nb, int k, const double* __restrict__ part,
    char* __restrict__ storage, const int64_t* __restrict__ toff, const uint8_t* __restrict__ tcls,
    int* __restrict__ tscl, const int64_t* __restrict__ shoff) {
    const int rt = blockIdx.y, strip = blockIdx.x;  // rt: tile k + 1 + rt of column k
    const int64_t t = tile_off(Nt, k + 1 + rt, k);
    double amax = 0.0;
    for (int s = 0; s < kStrips; ++s) amax = fmax(amax, part[rt * kStrips + s]);
    const int c = tcls[t];
    const int e = class_scale(amax, c);
    // largest stored value (rounding is monotone): decides the copies' scales
    const double amax_h = ldexp(fabs(round_to_class(ldexp(amax, -e), c)), e);
    int ce[5];
    float* copy[5];
#pragma unroll
    for (int c2 = 1; c2 <= 4; ++c2) {
        const int64_t o = shoff[t * 4 + (c2 - 1)];
        copy[c2] = (o >= 0 && !(c2 == kFP32 && c == kFP32)) ? reinterpret_cast<float*>(storage + o)
                                                            : nullptr;
        ce[c2] = class_scale(amax_h, c2);
    }
    if (strip == 0 && threadIdx.x == 0) tscl[t] = e;
    const int64_t per = (int64_t)nb * nb / kStrips;
    const double* src = W + (int64_t)(1 + rt) * nb * nb;
    void* dst = storage + toff[t];
    for (int64_t i = strip * per + threadIdx.x; i < (strip + 1) * per; i += kThreads) {
        const double r = round_to_class(ldexp(src[i], -e), c);
        store_elem(dst, i, c, r);
        const double v = ldexp(r, e);  // the stored factor value
#pragma unroll
        for (int c2 = 1; c2 <= 4; ++c2)
            if (copy[c2]) copy[c2][i] = (float)ldexp(round_to_class(ldexp(v, -ce[c2]), c2), ce[c2]);
    }
}

}  // namespace

hipError_t launch_mxp_gemm_f64(hipStream_t s, double* W, int Nt, int nb, int k, const int* rows,
                               int nrows, bool diag, const char* storage, const int64_t* toff,
                               const uint8_t* tcls, const int* tscl) {
    const int64_t T = nb / kB;
    const int64_t total = (diag ? T * (T + 1) / 2 : 0) + (int64_t)nrows * T * T;
    if (total == 0 || k == 0) return hipSuccess;
    hipLaunchKernelGGL(mxp_gemm_f64_kernel, dim3((unsigned)total), dim3(kGemmThreads), 0, s, W, Nt,
                       nb, k, rows, nrows, diag ? 1 : 0, storage, toff, tcls, tscl);
    return hipGetLastError();
}

hipError_t launch_mxp_gemm_f32(hipStream_t s, double* W, int Nt, int nb, int k, const int* rows,
                               int nrows, int cls, const char* storage, const int64_t* shoff) {
    const int64_t T = nb / kB;
    const int64_t total = (int64_t)nrows * T * T;
    if (total == 0 || k == 0) return hipSuccess;
    hipLaunchKernelGGL(mxp_gemm_f32_kernel, dim3((unsigned)total), dim3(kGemmThreads), 0, s, W, Nt,
                       nb, k, rows, nrows, cls, storage, shoff);
    return hipGetLastError();
}

hipError_t launch_mxp_finalize(hipStream_t s, const double* W, int Nt, int nb, int k, double* part,
                               char* storage, const int64_t* toff, const uint8_t* tcls, int* tscl,
                               const int64_t* shoff) {
    const int rows = Nt - k - 1;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(tile_amax_kernel, dim3(kStrips, rows), dim3(kThreads), 0, s,
                       W + (int64_t)nb * nb, nb, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tile_cast_kernel, dim3(kStrips, rows), dim3(kThreads), 0, s, W, Nt, nb, k,
                       part, storage, toff, tcls, tscl, shoff);
    return hipGetLastError();
}

}  // namespace tc
