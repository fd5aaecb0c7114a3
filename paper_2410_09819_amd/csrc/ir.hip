// Residual of the FP64 iterative-refinement solve: R = B - A X with A the
// symmetric matrix given by its packed lower tiles (binary64; the strict
// upper triangle of diagonal tiles is not read), X and B column-major.
//
// One pass over A. X is first copied into Xt, 16 right-hand sides
// interleaved per row (zero padded), so that an MFMA operand is one
// coalesced 512-byte read. A workgroup takes a run of up to kRunT tiles
// (i, j) down tile column j and one segment of NS 64-wide column strips of
// those tiles; each 64 x 64 block of A is staged once through LDS and used
// twice with v_mfma_f64_16x16x4_f64:
//   lower: Y_i[rows of the block] += A_blk X_j[cols of the block]
//          (kept per tile and segment in PL),
//   upper: Y_j[cols of the block] += A_blk^T X_i[rows of the block]
//          (accumulated in registers over the run, then stored in PU),
// with the lower triangle (lower) or strict lower triangle (upper) of
// diagonal tiles. A reduce kernel then forms R = B - sum PL - sum PU in a
// fixed order.
#include "common.hpp"

namespace tc {
namespace {

constexpr int kNR = 16;    // right-hand sides per pass
constexpr int kSB = 64;    // block edge
constexpr int kRunT = 4;   // tiles per run down a tile column
constexpr int kAP = kSB + 1;  // LDS column pitch (doubles)

__host__ __device__ inline int runs_in_col(int Nt, int j) { return (Nt - j + kRunT - 1) / kRunT; }

__host__ __device__ inline int seg_strips(int nb) {
    const int s = nb / kSB;
    if (s % 8 == 0) return 8;
    if (s % 6 == 0) return 6;
    if (s % 4 == 0) return 4;
    return 2;
}

// Xt[(z * n + row) * 16 + c] = X[(16 z + c) * ldx + row] (0 beyond nrhs)
__global__ void interleave_rhs_kernel(const double* __restrict__ X, int64_t ldx, int64_t n, int nrhs,
                                      int zc, double* __restrict__ Xt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)zc * n * kNR) return;
    const int c = (int)(e % kNR);
    const int64_t rowz = e / kNR;
    const int z = (int)(rowz / n);
    const int64_t row = rowz - (int64_t)z * n;
    const int col = z * kNR + c;
    Xt[e] = col < nrhs ? X[(int64_t)col * ldx + row] : 0.0;
}

struct Blk16 {
    d4 v0, v1, v2, v3;  // 16 consecutive doubles of one column
};

__device__ __forceinline__ void load_blk(const double* p, Blk16& r) {
    r.v0 = *reinterpret_cast<const d4*>(p);
    r.v1 = *reinterpret_cast<const d4*>(p + 4);
    r.v2 = *reinterpret_cast<const d4*>(p + 8);
    r.v3 = *reinterpret_cast<const d4*>(p + 12);
}

__device__ __forceinline__ void store_blk(double* d, const Blk16& r) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        d[q] = r.v0[q];
        d[4 + q] = r.v1[q];
        d[8 + q] = r.v2[q];
        d[12 + q] = r.v3[q];
    }
}

// 16 MFMA steps over one 64 x 64 block (see the file comment).
__device__ __forceinline__ d4 lower_steps(const double* as, const double* xj, int w, int la, int lb,
                                          bool mask, int rdiag, d4 acc) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        double a = as[(4 * s + lb) * kAP + 16 * w + la];
        if (mask && rdiag < 4 * s + lb) a = 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, xj[(4 * s + lb) * kNR + la], acc, 0, 0, 0);
    }
    return acc;
}

__device__ __forceinline__ d4 upper_steps(const double* as, const double* xi, int w, int la, int lb,
                                          bool mask, int cdiag, d4 acc) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        double a = as[(16 * w + la) * kAP + 4 * s + lb];
        if (mask && 4 * s + lb <= cdiag) a = 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, xi[(4 * s + lb) * kNR + la], acc, 0, 0, 0);
    }
    return acc;
}

template <int NS>
__global__ __launch_bounds__(256, 2) void symv_tile_kernel(const double* __restrict__ A, int Nt,
                                                           int nb, const double* __restrict__ Xt,
                                                           double* __restrict__ PL,
                                                           double* __restrict__ PU, int nseg,
                                                           int64_t nruns) {
    __shared__ double As[2][kSB * kAP];  // [buf][col * kAP + row]
    __shared__ int sh[2];
    const int seg = blockIdx.y, z = blockIdx.z;
    if (threadIdx.x == 0) {
        int64_t b = blockIdx.x;
        int j = 0;
        for (;;) {
            const int rc = runs_in_col(Nt, j);
            if (b < rc) break;
            b -= rc;
            ++j;
        }
        sh[0] = j;
        sh[1] = (int)b;
    }
    __syncthreads();
    const int j = sh[0], g = sh[1];
    const int i0 = j + g * kRunT;
    const int i1 = i0 + kRunT < Nt ? i0 + kRunT : Nt;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int la = lane & 15, lb = lane >> 4;
    const int64_t n = (int64_t)Nt * nb;
    const int64_t nb2 = (int64_t)nb * nb;
    const double* X = Xt + (int64_t)z * n * kNR;
    const int nrb = nb / kSB;
    const int cs0 = seg * NS;  // first 64-wide strip of this segment
    // A block loads: thread t moves column t / 4, rows 16 (t % 4) .. +15
    const int lcol = tid >> 2, lrow = (tid & 3) * 16;
    double* const sdst0 = &As[0][lcol * kAP + lrow];
    double* const sdst1 = &As[1][lcol * kAP + lrow];

    d4 up[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) up[q] = d4{0.0, 0.0, 0.0, 0.0};
    d4 lo = d4{0.0, 0.0, 0.0, 0.0};
    Blk16 ra;

    load_blk(A + tile_off(Nt, i0, j) * nb2 + (int64_t)(cs0 * kSB + lcol) * nb + lrow, ra);
    store_blk(sdst0, ra);
    __syncthreads();
    int buf = 0;
    for (int i = i0; i < i1; ++i) {
        const bool diag = i == j;
        const double* tile = A + tile_off(Nt, i, j) * nb2;
        for (int rb = 0; rb < nrb; ++rb) {
            const double* xi = X + ((int64_t)i * nb + rb * kSB) * kNR;
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                // keep each strip's loads in its own step (no hoisting of the
                // next strips' X loads into this one)
                __builtin_amdgcn_sched_barrier(0);
                const int cs = cs0 + q;
                // next block in (i, rb, q) order
                const double* nxt = nullptr;
                if (q + 1 < NS)
                    nxt = tile + (int64_t)((cs + 1) * kSB + lcol) * nb + rb * kSB + lrow;
                else if (rb + 1 < nrb)
                    nxt = tile + (int64_t)(cs0 * kSB + lcol) * nb + (rb + 1) * kSB + lrow;
                else if (i + 1 < i1)
                    nxt = A + tile_off(Nt, i + 1, j) * nb2 + (int64_t)(cs0 * kSB + lcol) * nb + lrow;
                if (nxt) load_blk(nxt, ra);
                const double* as = As[buf];
                const bool mask = diag && rb <= cs;
                // X_j depends on the strip only; an opaque per-step offset keeps
                // its loads inside the step (hoisted out of the block loops they
                // would hold NS x 16 values in registers)
                int xo = 0;
                asm volatile("" : "+v"(xo));
                const double* xj = X + ((int64_t)j * nb + cs * kSB) * kNR + xo;
                lo = lower_steps(as, xj, w, la, lb, mask, (rb - cs) * kSB + 16 * w + la, lo);
                up[q] = upper_steps(as, xi + xo, w, la, lb, mask, (cs - rb) * kSB + 16 * w + la, up[q]);
                if (nxt) store_blk(buf ? sdst0 : sdst1, ra);
                __syncthreads();
                buf ^= 1;
            }
            // lane holds rows 16w + lb + 4v of this block row, right-hand side la
            double* pl = PL + ((((int64_t)z * Nt * (Nt + 1) / 2 + tile_off(Nt, i, j)) * nseg + seg) * kNR + la) * nb +
                         rb * kSB + 16 * w + lb;
#pragma unroll
            for (int v = 0; v < 4; ++v) pl[4 * v] = lo[v];
            lo = d4{0.0, 0.0, 0.0, 0.0};
        }
    }
    // Y_j partial over this run: columns (cs0 + q) * 64 + 16w + lb + 4v
    const int sw = NS * kSB;
    int64_t run = g;
    for (int jj = 0; jj < j; ++jj) run += runs_in_col(Nt, jj);
    double* pu = PU + ((((int64_t)z * nruns + run) * nseg + seg) * kNR + la) * sw + 16 * w + lb;
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) pu[q * kSB + 4 * v] = up[q][v];
}

// R[c][row] = B[c][row] - sum_{j <= i} PL[(i, j), seg][c][row]
//                       - sum over runs of column i of PU[run, seg][c][row]
__global__ void residual_reduce_kernel(const double* __restrict__ B, int64_t ldb, int Nt, int nb,
                                       int nrhs, int nseg, int sw, int64_t nruns,
                                       const double* __restrict__ PL, const double* __restrict__ PU,
                                       double* __restrict__ R, int64_t ldr) {
    const int64_t n = (int64_t)Nt * nb;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nrhs) return;
    const int col = (int)(e / n);
    const int64_t row = e - (int64_t)col * n;
    const int z = col / kNR, c = col % kNR;
    const int i = (int)(row / nb), rr = (int)(row % nb);
    const int64_t ntiles = (int64_t)Nt * (Nt + 1) / 2;
    double s = 0.0;
    for (int j = 0; j <= i; ++j)
        for (int sg = 0; sg < nseg; ++sg)
            s += PL[((((int64_t)z * ntiles + tile_off(Nt, i, j)) * nseg + sg) * kNR + c) * nb + rr];
    int64_t run0 = 0;
    for (int jj = 0; jj < i; ++jj) run0 += runs_in_col(Nt, jj);
    const int sg = rr / sw, rs = rr % sw;
    const int rc = runs_in_col(Nt, i);
    for (int g = 0; g < rc; ++g)
        s += PU[((((int64_t)z * nruns + run0 + g) * nseg + sg) * kNR + c) * sw + rs];
    R[(int64_t)col * ldr + row] = B[(int64_t)col * ldb + row] - s;
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

static int64_t total_runs(int Nt) {
    int64_t r = 0;
    for (int j = 0; j < Nt; ++j) r += runs_in_col(Nt, j);
    return r;
}

size_t residual_partial_doubles(int Nt, int nb, int nrhs) {
    const int64_t n = (int64_t)Nt * nb;
    const int zc = (nrhs + kNR - 1) / kNR;
    const int nseg = nb / (seg_strips(nb) * kSB);
    const int64_t ntiles = (int64_t)Nt * (Nt + 1) / 2;
    const size_t xt = (size_t)zc * n * kNR;
    const size_t pl = (size_t)zc * ntiles * nseg * kNR * nb;
    const size_t pu = (size_t)zc * total_runs(Nt) * nseg * kNR * (seg_strips(nb) * kSB);
    return xt + pl + pu;
}

hipError_t launch_residual(hipStream_t s, const double* A, int Nt, int nb, const double* X,
                           int64_t ldx, const double* B, int64_t ldb, int nrhs, double* partial,
                           double* R, int64_t ldr) {
    const int64_t n = (int64_t)Nt * nb;
    const int zc = (nrhs + kNR - 1) / kNR;
    const int NS = seg_strips(nb);
    const int sw = NS * kSB;
    const int nseg = nb / sw;
    const int64_t ntiles = (int64_t)Nt * (Nt + 1) / 2;
    const int64_t nruns = total_runs(Nt);
    double* Xt = partial;
    double* PL = Xt + (size_t)zc * n * kNR;
    double* PU = PL + (size_t)zc * ntiles * nseg * kNR * nb;
    const int64_t xe = (int64_t)zc * n * kNR;
    hipLaunchKernelGGL(interleave_rhs_kernel, dim3((unsigned)((xe + 255) / 256)), dim3(256), 0, s, X,
                       ldx, n, nrhs, zc, Xt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)nruns, nseg, zc), block(256);
    switch (NS) {
        case 8: hipLaunchKernelGGL(symv_tile_kernel<8>, grid, block, 0, s, A, Nt, nb, Xt, PL, PU, nseg, nruns); break;
        case 6: hipLaunchKernelGGL(symv_tile_kernel<6>, grid, block, 0, s, A, Nt, nb, Xt, PL, PU, nseg, nruns); break;
        case 4: hipLaunchKernelGGL(symv_tile_kernel<4>, grid, block, 0, s, A, Nt, nb, Xt, PL, PU, nseg, nruns); break;
        default: hipLaunchKernelGGL(symv_tile_kernel<2>, grid, block, 0, s, A, Nt, nb, Xt, PL, PU, nseg, nruns); break;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t tot = n * nrhs;
    hipLaunchKernelGGL(residual_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, B,
                       ldb, Nt, nb, nrhs, nseg, sw, nruns, PL, PU, R, ldr);
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
