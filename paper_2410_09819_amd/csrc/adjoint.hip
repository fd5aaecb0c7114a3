// Reverse mode of the tile Cholesky (the log-likelihood gradient of Eq. 1).
//
// The blocked reverse sweep of Murray (2016, "Differentiation of the
// Cholesky decomposition"), reordered to be left-looking over tile columns
// n = Nt-1 ... 0. With S = Abar + Abar^T (tile (m,k) of S is Abar_mk below
// the diagonal, Abar_km^T above it and H_m = Abar_mm + Abar_mm^T on it),
// column n takes
//   (a) Lbar_mn -= sum_{k>n} S_mk L_kn          for m > n  (one panel GEMM)
//   (b) Abar_mn  = Lbar_mn L_nn^{-1}             for m > n
//   (c) Lbar_nn -= tril(sum_{m>n} Abar_mn^T L_mn)
//   (d) Abar_nn from the unblocked reverse of the diagonal tile:
//       P = L_nn^T tril(Lbar_nn), M = P with its lower triangle mirrored,
//       H = L_nn^{-T} M L_nn^{-1}, Abar_nn = tril(H) with the diagonal halved.
// Every contraction is the FP64 MFMA "A B^T" main loop: transposed copies
// of L's column panel and of Abar's columns (kept for the later panels)
// make all operands column-major with unit row stride.
//
// Memory-short form: no transposed copy of Abar is kept. The panel (a)
// reads the chunks of S_mk with k > m as Abar_km transposed straight from
// Lbar (each 16-column K chunk of the operand loaded row by row and written
// transposed into LDS, the same LDS image as the copy gives), and H_m
// lives in a one-tile-column array. Its products equal those of the full
// form bit for bit: same operand values, same chunking and MFMA order.
#include "gemm_f64.hpp"

namespace tc {
namespace {

constexpr int kPB = 128;  // output block of the panel kernel

// Row block r0 of tile row m of S, K index kk counted from tile column n+1.
struct SymOp {
    const double* Ab;  // Abar (lower packed tiles)
    const double* Tt;  // Abar^T tiles (tile (k, m) holds Abar_km^T; diagonal: H_m)
    int64_t Nt, nb, nb2, m, n, r0;
    __device__ const double* operator()(int64_t kk) const {
        const int64_t q = kk / nb;
        const int64_t k = n + 1 + q;
        const double* t = k < m ? Ab + tile_off(Nt, m, k) * nb2 : Tt + tile_off(Nt, k, m) * nb2;
        return t + (kk - q * nb) * nb + r0;
    }
};

struct ColOp {
    const double* p;
    int64_t ld;
    __device__ const double* operator()(int64_t kk) const { return p + kk * ld; }
};

// Memory-short operand of (a): chunk (row block r0 of tile row m, K index
// kk). Sets `tr` when the chunk is Abar_km with k > m, read transposed:
// element (row, col) at p + row * nb + col; otherwise p + col * nb + row.
struct SymOpShort {
    const double* Ab;  // Abar (lower packed tiles, in place in Lbar)
    const double* Hd;  // H_m for tile row m at Hd + m * nb^2
    int64_t Nt, nb, nb2, m, n, r0;
    __device__ const double* operator()(int64_t kk, bool& tr) const {
        const int64_t q = kk / nb;
        const int64_t k = n + 1 + q;
        const int64_t j = kk - q * nb;
        tr = k > m;
        if (k < m) return Ab + tile_off(Nt, m, k) * nb2 + j * nb + r0;
        if (k == m) return Hd + m * nb2 + j * nb + r0;
        return Ab + tile_off(Nt, k, m) * nb2 + r0 * nb + j;
    }
};

// mfma_mainloop<kPB, kPB> with the A operand of SymOpShort: a chunk read
// transposed is loaded as 128 rows of 16 consecutive K values (eight
// threads per 128-byte row run) and stored column by column into the
// k-major LDS tile, so the MFMA reads are those of the natural chunks.
__device__ __forceinline__ void sym_short_mainloop(d4 (&acc)[kPB / 32][kPB / 32],
                                                   const SymOpShort& aop, const ColOp& bop,
                                                   int64_t ld, int64_t kbeg, int64_t kend,
                                                   double* lds) {
    using T = MfmaTile<kPB, kPB>;
    if (kbeg >= kend) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    double* As = lds;
    double* Bs = lds + 2 * T::BK * T::LDA;

    int64_t a_goff[T::A_LOADS], t_goff[T::A_LOADS];
    int a_soff[T::A_LOADS], t_soff[T::A_LOADS];
#pragma unroll
    for (int q = 0; q < T::A_LOADS; ++q) {
        const int e = (q * kGemmThreads + tid) * 2;
        const int col = e / kPB, row = e % kPB;
        a_goff[q] = (int64_t)col * ld + row;
        a_soff[q] = col * T::LDA + row;
        const int e2 = q * kGemmThreads + tid;  // d2 index: row e2 / 8, columns 2 (e2 % 8) + {0, 1}
        const int trow = e2 >> 3, tcol = (e2 & 7) * 2;
        t_goff[q] = (int64_t)trow * ld + tcol;
        t_soff[q] = tcol * T::LDA + trow;
    }
    int64_t b_goff[T::B_LOADS];
    int b_soff[T::B_LOADS];
#pragma unroll
    for (int q = 0; q < T::B_LOADS; ++q) {
        const int e = (q * kGemmThreads + tid) * 2;
        const int col = e / kPB, row = e % kPB;
        b_goff[q] = (int64_t)col * ld + row;
        b_soff[q] = col * T::LDB + row;
    }

    d2 ra[T::A_LOADS], rb[T::B_LOADS];
    bool rtr = false;  // the chunk in ra was read transposed
    auto gload = [&](int64_t kk) {
        bool tr;
        const double* pa = aop(kk, tr);
        const double* pb = bop(kk);
        rtr = tr;
        if (tr) {
#pragma unroll
            for (int q = 0; q < T::A_LOADS; ++q)
                ra[q] = *reinterpret_cast<const d2*>(pa + t_goff[q]);
        } else {
#pragma unroll
            for (int q = 0; q < T::A_LOADS; ++q)
                ra[q] = *reinterpret_cast<const d2*>(pa + a_goff[q]);
        }
#pragma unroll
        for (int q = 0; q < T::B_LOADS; ++q) rb[q] = *reinterpret_cast<const d2*>(pb + b_goff[q]);
    };
    auto sstore = [&](int buf) {
        double* as = As + buf * T::BK * T::LDA;
        double* bs = Bs + buf * T::BK * T::LDB;
        if (rtr) {
#pragma unroll
            for (int q = 0; q < T::A_LOADS; ++q) {
                as[t_soff[q]] = ra[q].x;
                as[t_soff[q] + T::LDA] = ra[q].y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < T::A_LOADS; ++q) *reinterpret_cast<d2*>(as + a_soff[q]) = ra[q];
        }
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
        const double* as = As + buf * T::BK * T::LDA + wm * (kPB / 2) + li;
        const double* bs = Bs + buf * T::BK * T::LDB + wn * (kPB / 2) + li;
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

// Output block of (a): subtract into Lbar (one split) or store the split's
// partial sums.
__device__ __forceinline__ void panel_store(const d4 (&acc)[kPB / 32][kPB / 32],
                                            double* __restrict__ Lb, double* __restrict__ partial,
                                            int Nt, int nb, int n, int splits, int split,
                                            int64_t rt, int br, int bc) {
    using Tl = MfmaTile<kPB, kPB>;
    const int64_t R = Nt - n - 1;
    const int64_t nb2 = (int64_t)nb * nb;
    double* out = splits == 1 ? Lb + tile_off(Nt, n + 1 + rt, n) * nb2
                              : partial + ((int64_t)split * R + rt) * nb2;
    out += (int64_t)bc * kPB * nb + br * kPB;
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double* p = out + (int64_t)acc_col<kPB, kPB>(ni, v) * nb + acc_row<kPB, kPB>(mi);
                if (splits == 1)
                    *p -= acc[mi][ni][v];
                else
                    *p = acc[mi][ni][v];
            }
}

// (a): output tiles (n+1+rt, n), rt < R = Nt-n-1, all nb/128 x nb/128 blocks.
// PL: nb x R*nb column-major (ld nb), PL(c, kk) = L_{n+1+kk/nb, n}(kk % nb, c).
__global__ __launch_bounds__(kGemmThreads, 2) void adj_panel_kernel(
    double* __restrict__ Lb, const double* __restrict__ Tt, const double* __restrict__ PL, int Nt,
    int nb, int n, int splits, int64_t nblocks, int64_t kchunk, double* __restrict__ partial) {
    using Tl = MfmaTile<kPB, kPB>;
    __shared__ double lds[Tl::LDS_DOUBLES];
    const int64_t logical = xcd_remap(blockIdx.x, nblocks * splits);
    const int split = (int)(logical / nblocks);
    const int64_t b = logical - (int64_t)split * nblocks;
    const int T = nb / kPB;
    const int64_t rt = b / (T * T);
    const int w = (int)(b - rt * T * T);
    const int br = w / T, bc = w % T;
    const int64_t R = Nt - n - 1;
    const int64_t nb2 = (int64_t)nb * nb;
    const int64_t K = R * nb;
    const int64_t kbeg = (int64_t)split * kchunk;
    const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;

    d4 acc[Tl::MI][Tl::NI];
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
    const SymOp aop{Lb, Tt, Nt, nb, nb2, n + 1 + rt, n, (int64_t)br * kPB};
    const ColOp bop{PL + (int64_t)bc * kPB, nb};
    mfma_mainloop<kPB, kPB>(acc, aop, bop, nb, kbeg, kend, lds);
    panel_store(acc, Lb, partial, Nt, nb, n, splits, split, rt, br, bc);
}

// (a) in the memory-short form: Hd holds H_m per tile row, Abar_km^T is
// read from Lbar itself. Same blocks, splits and output as adj_panel_kernel.
__global__ __launch_bounds__(kGemmThreads, 2) void adj_panel_short_kernel(
    double* __restrict__ Lb, const double* __restrict__ Hd, const double* __restrict__ PL, int Nt,
    int nb, int n, int splits, int64_t nblocks, int64_t kchunk, double* __restrict__ partial) {
    using Tl = MfmaTile<kPB, kPB>;
    __shared__ double lds[Tl::LDS_DOUBLES];
    const int64_t logical = xcd_remap(blockIdx.x, nblocks * splits);
    const int split = (int)(logical / nblocks);
    const int64_t b = logical - (int64_t)split * nblocks;
    const int T = nb / kPB;
    const int64_t rt = b / (T * T);
    const int w = (int)(b - rt * T * T);
    const int br = w / T, bc = w % T;
    const int64_t R = Nt - n - 1;
    const int64_t nb2 = (int64_t)nb * nb;
    const int64_t K = R * nb;
    const int64_t kbeg = (int64_t)split * kchunk;
    const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;

    d4 acc[Tl::MI][Tl::NI];
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
    const SymOpShort aop{Lb, Hd, Nt, nb, nb2, n + 1 + rt, n, (int64_t)br * kPB};
    const ColOp bop{PL + (int64_t)bc * kPB, nb};
    sym_short_mainloop(acc, aop, bop, nb, kbeg, kend, lds);
    panel_store(acc, Lb, partial, Nt, nb, n, splits, split, rt, br, bc);
}

__global__ void adj_panel_reduce_kernel(double* __restrict__ Lb, int Nt, int nb, int n, int splits,
                                        const double* __restrict__ partial) {
    const int64_t nb2 = (int64_t)nb * nb;
    const int64_t R = Nt - n - 1;
    const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2;
    if (e >= R * nb2) return;
    d2 s = *reinterpret_cast<const d2*>(partial + e);
    for (int sp = 1; sp < splits; ++sp)
        s += *reinterpret_cast<const d2*>(partial + (int64_t)sp * R * nb2 + e);
    d2* c = reinterpret_cast<d2*>(Lb + tile_off(Nt, n + 1, n) * nb2 + e);
    *c = *c - s;
}

// C (M x N) = or -= A B^T for the matrices of AdjMat form; blocks of B x B,
// lower != 0: only blocks on or below the block diagonal (M == N).
template <int B>
__global__ __launch_bounds__(kGemmThreads, 2) void adj_gemm_kernel(
    AdjMat C, AdjMat A, AdjMat Bm, int64_t M, int64_t N, int64_t K, int sub, int lower,
    int splits, int64_t kchunk, int64_t nbm, int64_t nblocks, double* __restrict__ partial) {
    using Tl = MfmaTile<B, B>;
    __shared__ double lds[Tl::LDS_DOUBLES];
    const int64_t logical = xcd_remap(blockIdx.x, nblocks * splits);
    const int split = (int)(logical / nblocks);
    const int64_t b = logical - (int64_t)split * nblocks;
    int64_t br, bc;
    if (lower) {
        int64_t r = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
        while ((r + 1) * (r + 2) / 2 <= b) ++r;
        while (r * (r + 1) / 2 > b) --r;
        br = r;
        bc = b - r * (r + 1) / 2;
    } else {
        br = b % nbm;
        bc = b / nbm;
    }
    const int64_t r0 = br * B, c0 = bc * B;
    const int64_t kbeg = (int64_t)split * kchunk;
    const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
    d4 acc[Tl::MI][Tl::NI];
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
    const ColOp aop{A.p + A.off(r0, 0), A.ld};
    const ColOp bop{Bm.p + Bm.off(c0, 0), Bm.ld};
    mfma_mainloop<B, B>(acc, aop, bop, A.ld, kbeg, kend, lds);

    double* out;
    int64_t ldo;
    if (splits == 1) {
        out = C.p + C.off(r0, c0);
        ldo = C.ld;
    } else {
        out = partial + (int64_t)split * M * N + c0 * M + r0;
        ldo = M;
    }
#pragma unroll
    for (int mi = 0; mi < Tl::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < Tl::NI; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double* p = out + (int64_t)acc_col<B, B>(ni, v) * ldo + acc_row<B, B>(mi);
                if (splits == 1 && sub)
                    *p -= acc[mi][ni][v];
                else
                    *p = acc[mi][ni][v];
            }
}

__global__ void adj_gemm_reduce_kernel(AdjMat C, int64_t M, int64_t N, int sub, int lower, int B,
                                       int splits, const double* __restrict__ partial) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M * N) return;
    const int64_t c = e / M, r = e - c * M;
    if (lower && r / B < c / B) return;
    double s = partial[e];
    for (int sp = 1; sp < splits; ++sp) s += partial[(int64_t)sp * M * N + e];
    double* p = C.p + C.off(r, c);
    *p = sub ? *p - s : s;
}

// dst tile t = src tile t transposed (nb x nb, column-major), for `count`
// consecutive tiles; tril != 0 reads the source as its lower triangle.
constexpr int kTB = 64;
__global__ __launch_bounds__(256) void transpose_tiles_kernel(const double* __restrict__ src,
                                                              double* __restrict__ dst, int nb,
                                                              int tril) {
    __shared__ double t[kTB][kTB + 1];
    const int64_t nb2 = (int64_t)nb * nb;
    const double* s = src + (int64_t)blockIdx.z * nb2;
    double* d = dst + (int64_t)blockIdx.z * nb2;
    const int r0 = blockIdx.x * kTB, c0 = blockIdx.y * kTB;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int j = ty; j < kTB; j += 4) {
        const int r = r0 + tx, c = c0 + j;
        double v = s[(int64_t)c * nb + r];
        if (tril && r < c) v = 0.0;
        t[j][tx] = v;  // t[col][row]
    }
    __syncthreads();
    // dst(c, r) = src(r, c): dst column r0 + j, rows c0 + tx
    for (int j = ty; j < kTB; j += 4) d[(int64_t)(r0 + j) * nb + c0 + tx] = t[tx][j];
}

__global__ void set_identity_kernel(double* __restrict__ X, int nb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nb * nb) return;
    const int64_t c = e / nb, r = e - c * nb;
    X[e] = r == c ? 1.0 : 0.0;
}

// Upper triangle := lower triangle mirrored (in place).
__global__ void mirror_lower_kernel(double* __restrict__ P, int nb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nb * nb) return;
    const int64_t c = e / nb, r = e - c * nb;
    if (r < c) P[e] = P[r * nb + c];
}

// Abar_nn = tril(H) with the diagonal halved; strict upper triangle zero.
__global__ void finish_diag_kernel(const double* __restrict__ H, double* __restrict__ D, int nb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nb * nb) return;
    const int64_t c = e / nb, r = e - c * nb;
    D[e] = r > c ? H[e] : (r == c ? 0.5 * H[e] : 0.0);
}

// Seed of the log-likelihood: Lbar = tril(alpha z^T) - diag(1 / L_ii).
__global__ void loglik_seed_kernel(TileView L, const double* __restrict__ alpha,
                                   const double* __restrict__ z, double* __restrict__ Lb,
                                   int64_t Nt, int nb) {
    const int64_t t = blockIdx.y;
    int64_t j = 0;
    while (tile_off(Nt, Nt - 1, j) < t) ++j;
    const int64_t i = j + (t - tile_off(Nt, j, j));
    const int64_t nb2 = (int64_t)nb * nb;
    const int c = blockIdx.x;  // one column of the tile per workgroup
    const double zc = z[j * nb + c];
    double* out = Lb + t * nb2 + (int64_t)c * nb;
    // diagonal tiles are binary64 in every factor layout
    const double* Lt = reinterpret_cast<const double*>(
                           L.toff ? L.base + L.toff[t] : L.base + t * nb2 * (int64_t)sizeof(double)) +
                       (int64_t)c * nb;
    for (int r = threadIdx.x; r < nb; r += blockDim.x) {
        double v = alpha[i * nb + r] * zc;
        if (i == j) {
            if (r < c) v = 0.0;
            else if (r == c) v -= 1.0 / Lt[r];
        }
        out[r] = v;
    }
}

}  // namespace

int64_t adj_panel_blocks(int Nt, int nb, int n) {
    const int64_t T = nb / kPB;
    return (int64_t)(Nt - n - 1) * T * T;
}

// Split-K for the panel of column n: the time model of the forward panel
// (rounds of 512 resident workgroups at the FP64 MFMA rate, plus the
// partial sums at HBM speed), each split keeping >= 512 of K and the
// partials under 512 MiB.
int adj_panel_splits(int Nt, int nb, int n) {
    const int64_t W = adj_panel_blocks(Nt, nb, n);
    const int64_t K = (int64_t)(Nt - n - 1) * nb;
    const double panel_bytes = (double)(Nt - n - 1) * nb * nb * sizeof(double);
    int64_t smax = K / 512;
    if (smax > 32) smax = 32;
    while (smax > 1 && smax * panel_bytes > 512.0 * 1024 * 1024) --smax;
    if (smax < 1) return 1;
    const int64_t slots = 512;
    const double slot_flops = 78.6e12 / slots;
    double best = 1e300;
    int bests = 1;
    for (int64_t s = 1; s <= smax; ++s) {
        const double rounds = (double)((W * s + slots - 1) / slots);
        double t = rounds * (2.0 * kPB * kPB * ((double)K / s)) / slot_flops;
        if (s > 1) t += 2.0 * s * panel_bytes / 5e12;
        if (t < best * 0.97) {
            best = t;
            bests = (int)s;
        }
    }
    return bests;
}

hipError_t launch_adj_panel(hipStream_t s, double* Lb, const double* Tt, const double* Hd,
                            const double* PL, int Nt, int nb, int n, int splits, double* partial) {
    const int64_t W = adj_panel_blocks(Nt, nb, n);
    if (W == 0) return hipSuccess;
    if ((Tt == nullptr) == (Hd == nullptr)) return hipErrorInvalidValue;
    const int64_t K = (int64_t)(Nt - n - 1) * nb;
    const int64_t kchunk = (((K + splits - 1) / splits + 15) / 16) * 16;
    if (Tt)
        hipLaunchKernelGGL(adj_panel_kernel, dim3((unsigned)(W * splits)), dim3(kGemmThreads), 0, s,
                           Lb, Tt, PL, Nt, nb, n, splits, W, kchunk, partial);
    else
        hipLaunchKernelGGL(adj_panel_short_kernel, dim3((unsigned)(W * splits)), dim3(kGemmThreads),
                           0, s, Lb, Hd, PL, Nt, nb, n, splits, W, kchunk, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    const int64_t elems = (int64_t)(Nt - n - 1) * nb * nb / 2;
    hipLaunchKernelGGL(adj_panel_reduce_kernel, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0,
                       s, Lb, Nt, nb, n, splits, partial);
    return hipGetLastError();
}

// Block size, split count and partial-sum doubles of an adj_gemm launch.
AdjGemmPlan adj_gemm_plan(int64_t M, int64_t N, int64_t K, bool lower) {
    AdjGemmPlan p;
    const int64_t b128 = (M / 128) * (N / 128);
    p.block = (M % 128 == 0 && N % 128 == 0 && b128 >= 256) ? 128 : 64;
    const int64_t bm = M / p.block, bn = N / p.block;
    p.nblocks = lower ? bm * (bm + 1) / 2 : bm * bn;
    int64_t s = (512 + p.nblocks - 1) / p.nblocks;
    const int64_t smax = K / 128;
    if (s > smax) s = smax;
    if (s > 64) s = 64;
    p.splits = s < 1 ? 1 : (int)s;
    p.partial_doubles = p.splits > 1 ? (size_t)p.splits * M * N : 0;
    return p;
}

hipError_t launch_adj_gemm(hipStream_t s, const AdjMat& C, const AdjMat& A, const AdjMat& B,
                           int64_t M, int64_t N, int64_t K, bool sub, bool lower,
                           double* partial) {
    const AdjGemmPlan p = adj_gemm_plan(M, N, K, lower);
    const int64_t kchunk = (((K + p.splits - 1) / p.splits + 15) / 16) * 16;
    const int64_t nbm = M / p.block;
    const dim3 grid((unsigned)(p.nblocks * p.splits));
    if (p.block == 128)
        hipLaunchKernelGGL(adj_gemm_kernel<128>, grid, dim3(kGemmThreads), 0, s, C, A, B, M, N, K,
                           (int)sub, (int)lower, p.splits, kchunk, nbm, p.nblocks, partial);
    else
        hipLaunchKernelGGL(adj_gemm_kernel<64>, grid, dim3(kGemmThreads), 0, s, C, A, B, M, N, K,
                           (int)sub, (int)lower, p.splits, kchunk, nbm, p.nblocks, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p.splits == 1) return e;
    const int64_t elems = M * N;
    hipLaunchKernelGGL(adj_gemm_reduce_kernel, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0,
                       s, C, M, N, (int)sub, (int)lower, p.block, p.splits, partial);
    return hipGetLastError();
}

hipError_t launch_transpose_tiles(hipStream_t s, const double* src, double* dst, int nb,
                                  int64_t count, bool tril) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(transpose_tiles_kernel, dim3(nb / kTB, nb / kTB, (unsigned)count), dim3(256),
                       0, s, src, dst, nb, (int)tril);
    return hipGetLastError();
}

hipError_t launch_set_identity(hipStream_t s, double* X, int nb) {
    const int64_t e = (int64_t)nb * nb;
    hipLaunchKernelGGL(set_identity_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, X,
                       nb);
    return hipGetLastError();
}

hipError_t launch_mirror_lower(hipStream_t s, double* P, int nb) {
    const int64_t e = (int64_t)nb * nb;
    hipLaunchKernelGGL(mirror_lower_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, P,
                       nb);
    return hipGetLastError();
}

hipError_t launch_finish_diag(hipStream_t s, const double* H, double* D, int nb) {
    const int64_t e = (int64_t)nb * nb;
    hipLaunchKernelGGL(finish_diag_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, H, D,
                       nb);
    return hipGetLastError();
}

hipError_t launch_loglik_seed(hipStream_t s, const TileView& L, const double* alpha, const double* z,
                              double* Lb, int Nt, int nb) {
    const int64_t ntiles = (int64_t)Nt * (Nt + 1) / 2;
    hipLaunchKernelGGL(loglik_seed_kernel, dim3(nb, (unsigned)ntiles), dim3(256), 0, s, L, alpha, z,
                       Lb, (int64_t)Nt, nb);
    return hipGetLastError();
}

}  // namespace tc
