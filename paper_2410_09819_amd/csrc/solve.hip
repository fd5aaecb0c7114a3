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
#include "formats.hpp"

namespace tc {
namespace {

constexpr int kNR = 16;   // right-hand sides per workgroup of the update kernels
// right-hand sides per workgroup of the diagonal solve: one (16 workgroups
// for 16 right-hand sides: the 16-RHS solve at n = 65536 took 35.5 ms
// against 42.7 ms with four per workgroup, same results)
constexpr int kDR = 1;
constexpr int kDB = 64;   // diagonal sub-block of the in-tile solve
constexpr int kDBP = kDB + 1;

// Solve with the diagonal tile L_kk (or L_kk^T) for kDR right-hand sides per
// workgroup, in 64-row sub-blocks. Wave w solves right-hand side w of the
// sub-block by substitution across its 64 lanes (one row per lane, the
// solved value broadcast with v_readlane); then all 1024 threads apply
// the sub-block to the remaining rows of the tile.
__global__ __launch_bounds__(1024) void trsv_diag_kernel(const double* __restrict__ Lkk, int nb,
                                                        double* __restrict__ B, int64_t ldb,
                                                        int nrhs, int transpose) {
    __shared__ double Ls[kDB * kDBP];  // Ls[l * kDBP + j] = L[jb + l][jb + j], l >= j
    __shared__ double Rd[kDB];         // 1 / L[jb + j][jb + j]
    __shared__ double X[kDB * kDR];    // X[l * kDR + c]: solved sub-block
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int c0 = blockIdx.x * kDR;
    const int nr = nrhs - c0 < kDR ? nrhs - c0 : kDR;
    const int nblk = nb / kDB;
    for (int bi = 0; bi < nblk; ++bi) {
        const int jb = transpose ? (nblk - 1 - bi) * kDB : bi * kDB;
        for (int e = tid; e < kDB * kDB; e += 1024) {
            const int j = e / kDB, l = e % kDB;
            if (l >= j) {
                const double v = Lkk[(int64_t)(jb + j) * nb + jb + l];
                Ls[l * kDBP + j] = v;
                if (l == j) Rd[j] = 1.0 / v;
            }
        }
        __syncthreads();
        if (wave < nr) {
            double* bcol = B + (int64_t)(c0 + wave) * ldb + jb;
            double y = bcol[lane];
            const double rd = Rd[lane];
            if (!transpose) {
                for (int j = 0; j < kDB; ++j) {
                    const double xj = readlane_d(y, j) * readlane_d(rd, j);
                    if (lane == j) y = xj;
                    if (lane > j) y -= xj * Ls[lane * kDBP + j];
                }
            } else {
                for (int j = kDB - 1; j >= 0; --j) {
                    const double xj = readlane_d(y, j) * readlane_d(rd, j);
                    if (lane == j) y = xj;
                    if (lane < j) y -= xj * Ls[j * kDBP + lane];
                }
            }
            X[lane * kDR + wave] = y;
            bcol[lane] = y;
        }
        __syncthreads();
        // apply the solved sub-block to the rest of the tile's rows (one row
        // per thread; loads issued 32 at a time)
        if (!transpose) {
            for (int i = jb + kDB + tid; i < nb; i += 1024) {
                double s[kDR] = {};
#pragma unroll 1
                for (int l0 = 0; l0 < kDB; l0 += 32) {
                    double lv[32];
#pragma unroll
                    for (int u = 0; u < 32; ++u) lv[u] = Lkk[(int64_t)(jb + l0 + u) * nb + i];
#pragma unroll
                    for (int u = 0; u < 32; ++u)
#pragma unroll
                        for (int c = 0; c < kDR; ++c) s[c] += lv[u] * X[(l0 + u) * kDR + c];
                }
#pragma unroll
                for (int c = 0; c < kDR; ++c)
                    if (c < nr) B[(int64_t)(c0 + c) * ldb + i] -= s[c];
            }
        } else {
            for (int i = tid; i < jb; i += 1024) {
                const d2* li = reinterpret_cast<const d2*>(Lkk + (int64_t)i * nb + jb);  // L[jb + l][i]
                double s[kDR] = {};
#pragma unroll 1
                for (int l0 = 0; l0 < kDB / 2; l0 += 16) {
                    d2 lv[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) lv[u] = li[l0 + u];
#pragma unroll
                    for (int u = 0; u < 16; ++u)
#pragma unroll
                        for (int c = 0; c < kDR; ++c)
                            s[c] += lv[u].x * X[(2 * (l0 + u)) * kDR + c] +
                                    lv[u].y * X[(2 * (l0 + u) + 1) * kDR + c];
                }
#pragma unroll
                for (int c = 0; c < kDR; ++c)
                    if (c < nr) B[(int64_t)(c0 + c) * ldb + i] -= s[c];
            }
        }
        __threadfence_block();
        __syncthreads();
    }
}

// Tile (m, k) of a factor view: its first element, class and scale.
__device__ __forceinline__ const char* view_tile(const TileView& L, int m, int k, int& cls,
                                                 int& scale) {
    const int64_t t = tile_off(L.Nt, m, k);
    if (!L.toff) {
        cls = kFP64;
        scale = 0;
        return L.base + t * (int64_t)L.nb * L.nb * sizeof(double);
    }
    cls = L.tcls[t];
    scale = L.tscl[t];
    return L.base + L.toff[t];
}

template <int C>
__device__ __forceinline__ double ld_cls(const char* base, int64_t i) {
    if (C == kFP64) return reinterpret_cast<const double*>(base)[i];
    if (C == kFP32) return reinterpret_cast<const float*>(base)[i];
    if (C == kFP16) return dec_fp16(reinterpret_cast<const uint16_t*>(base)[i]);
    if (C == kBF16) return dec_bf16(reinterpret_cast<const uint16_t*>(base)[i]);
    return dec_fp8(reinterpret_cast<const uint8_t*>(base)[i]);
}

// One 64 x 64 block of a tile stored in class C (unscaled values) and the
// matching 64 x 16 block of right-hand sides into registers: thread t takes
// L elements (row t % 64 + 64-row offset, column j0 + t / 64 + 4u), read
// along contiguous rows, and right-hand-side elements (row t % 64, column
// t / 64 + 4u). The caller stores them to LDS.
template <int C>
__device__ __forceinline__ void fetch_block(const char* tile, int nb, int64_t col0, int row0,
                                            const double* X, int64_t ldb, int64_t xrow0, int c0,
                                            int nr, double (&lr)[16], double (&xr)[4]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * u;
        lr[u] = ld_cls<C>(tile, (col0 + e / 64) * nb + row0 + e % 64);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + 256 * u, c = e / 64;
        xr[u] = c < nr ? X[(int64_t)(c0 + c) * ldb + xrow0 + e % 64] : 0.0;
    }
}
__device__ __forceinline__ void fetch_block_cls(int cls, const char* tile, int nb, int64_t col0,
                                                int row0, const double* X, int64_t ldb,
                                                int64_t xrow0, int c0, int nr, double (&lr)[16],
                                                double (&xr)[4]) {
    switch (cls) {
        case kFP64: fetch_block<kFP64>(tile, nb, col0, row0, X, ldb, xrow0, c0, nr, lr, xr); break;
        case kFP32: fetch_block<kFP32>(tile, nb, col0, row0, X, ldb, xrow0, c0, nr, lr, xr); break;
        case kFP16: fetch_block<kFP16>(tile, nb, col0, row0, X, ldb, xrow0, c0, nr, lr, xr); break;
        case kBF16: fetch_block<kBF16>(tile, nb, col0, row0, X, ldb, xrow0, c0, nr, lr, xr); break;
        default: fetch_block<kFP8>(tile, nb, col0, row0, X, ldb, xrow0, c0, nr, lr, xr); break;
    }
}

// B_below[r][c] -= sum_j L[k+1+r/nb, k][r%nb][j] Y[j][c], on the FP64 matrix
// cores, straight from HBM into the MFMA operands (no LDS, no barriers). A wave owns 64 rows of one tile
// and 16 right-hand sides and runs v_mfma_f64_16x16x4f64 with A = Y^T
// (16 RHS x 4 k) and B = L^T (4 k x 16 rows). The order of rows and of k
// inside the MFMA blocks is free, and is chosen so that every load is a
// short vector: row block mi of lane i is tile row 4 i + mi (the lane's
// four rows are adjacent in a column), and in k-step t of a 32-column
// group j0, lane group g takes column j0 + 8 g + t (its eight Y rows are
// adjacent). The next group is loaded while the current one is multiplied. A wave covers the columns of its K split; with more than one
// split, each writes its (scaled) partial sums and fwd_reduce subtracts
// them in split order.
template <int C>
__device__ __forceinline__ void ld4_cls(const char* base, int64_t i, double (&v)[4]) {
    if (C == kFP64) {
        const d2 a = *reinterpret_cast<const d2*>(reinterpret_cast<const double*>(base) + i);
        const d2 b = *reinterpret_cast<const d2*>(reinterpret_cast<const double*>(base) + i + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else if (C == kFP32) {
        const float4 a = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(base) + i);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else if (C == kFP16 || C == kBF16) {
        const uint2 a = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(base) + i);
        const uint16_t h[4] = {(uint16_t)(a.x & 0xFFFFu), (uint16_t)(a.x >> 16),
                               (uint16_t)(a.y & 0xFFFFu), (uint16_t)(a.y >> 16)};
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = C == kFP16 ? dec_fp16(h[u]) : dec_bf16(h[u]);
    } else {
        const uint32_t a = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint8_t*>(base) + i);
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = dec_fp8((uint8_t)(a >> (8 * u)));
    }
}

template <int C>
__device__ __forceinline__ void fwd_mfma_wave(const char* tile, int nb, int rr0, int jbeg, int jend,
                                              const double* __restrict__ Y, int64_t ldb, int c0,
                                              int nr, d4 (&acc)[4]) {
    const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
    const int64_t lofs = (int64_t)rr0 + 4 * i;
    const bool yok = i < nr;
    const double* yp = Y + (int64_t)(c0 + (yok ? i : 0)) * ldb + 8 * g;
    double lv[8][4], yv[8], ln[8][4], yn[8];
    auto fetch = [&](int j0, double (&l)[8][4], double (&y)[8]) {
#pragma unroll
        for (int t = 0; t < 8; ++t) ld4_cls<C>(tile, (int64_t)(j0 + 8 * g + t) * nb + lofs, l[t]);
#pragma unroll
        for (int t = 0; t < 8; ++t) y[t] = yok ? yp[j0 + t] : 0.0;
    };
    fetch(jbeg, lv, yv);
    for (int j0 = jbeg; j0 < jend; j0 += 32) {
        if (j0 + 32 < jend) fetch(j0 + 32, ln, yn);
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
                acc[mi] = __builtin_amdgcn_mfma_f64_16x16x4f64(yv[t], lv[t][mi], acc[mi], 0, 0, 0);
        if (j0 + 32 < jend) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                yv[t] = yn[t];
#pragma unroll
                for (int mi = 0; mi < 4; ++mi) lv[t][mi] = ln[t][mi];
            }
        }
    }
}

constexpr int kFwdWaveRows = 64;
__global__ __launch_bounds__(256) void fwd_update_mfma_kernel(TileView L, int k, int t0, int64_t rows,
                                                              int splits,
                                                              const double* __restrict__ Y,
                                                              double* __restrict__ Bb, int64_t ldb,
                                                              int nrhs, int cbase,
                                                              double* __restrict__ part) {
    const int nb = L.nb;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);  // wave: rows 64 w ..
    const int64_t row0 = w * kFwdWaveRows;
    if (row0 >= rows) return;
    const int split = blockIdx.y, c0 = cbase + blockIdx.z * kNR;
    const int nr = nrhs - c0 < kNR ? nrhs - c0 : kNR;
    const int kc = nb / splits;
    const int jbeg = split * kc, jend = jbeg + kc;
    int cls, scale;
    const char* tile = view_tile(L, k + 1 + t0 + (int)(row0 / nb), k, cls, scale);
    const int rr0 = (int)(row0 % nb);
    d4 acc[4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) acc[mi] = d4{0.0, 0.0, 0.0, 0.0};
    switch (cls) {
        case kFP64: fwd_mfma_wave<kFP64>(tile, nb, rr0, jbeg, jend, Y, ldb, c0, nr, acc); break;
        case kFP32: fwd_mfma_wave<kFP32>(tile, nb, rr0, jbeg, jend, Y, ldb, c0, nr, acc); break;
        case kFP16: fwd_mfma_wave<kFP16>(tile, nb, rr0, jbeg, jend, Y, ldb, c0, nr, acc); break;
        case kBF16: fwd_mfma_wave<kBF16>(tile, nb, rr0, jbeg, jend, Y, ldb, c0, nr, acc); break;
        default: fwd_mfma_wave<kFP8>(tile, nb, rr0, jbeg, jend, Y, ldb, c0, nr, acc); break;
    }
    // lane l, value v of block mi: row 4 (l % 16) + mi, right-hand side l / 16 + 4 v
    const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int c = g + 4 * v;
        if (c >= nr) continue;
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
            const int64_t r = row0 + 4 * i + mi;
            const double a = scale ? ldexp(acc[mi][v], scale) : acc[mi][v];
            if (splits == 1)
                Bb[(int64_t)(c0 + c) * ldb + r] -= a;
            else
                part[((int64_t)split * rows + r) * kNR + c] = a;
        }
    }
}

__global__ void fwd_reduce_kernel(double* __restrict__ Bb, int64_t rows, int64_t ldb, int nrhs,
                                  int c0, int splits, const double* __restrict__ part) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * kNR) return;
    const int64_t r = e / kNR;
    const int c = (int)(e % kNR);
    if (c0 + c >= nrhs) return;
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += part[(int64_t)sp * rows * kNR + e];
    Bb[(int64_t)(c0 + c) * ldb + r] -= s;
}

// partial[split][j][c] = sum over the split's rows r of L[k+1+r/nb, k][r%nb][j]
// X[r][c] for the columns j of the tile column k, on the FP64 matrix cores,
// straight from HBM into the
// MFMA operands. A wave owns 32 columns j of the tile column (two MFMA
// blocks sharing the X operand) and the rows of its split, and runs
// v_mfma_f64_16x16x4f64 with A = X^T (16 RHS x 4 k) and B = L (4 k x 16
// columns). Rows go in 32-row groups (never across a
// tile, as nb and the split length are multiples of 64); in k-step t of a
// group at row rb, lane group g takes row rb + 8 g + t, so each lane reads
// 8 adjacent rows of its column of L and of its right-hand side of X. The
// next group is loaded while the current one is multiplied; each tile's
// power-of-two scale is applied to its loaded values (exact).
template <int C>
__device__ __forceinline__ void bwd_mfma_range(const char* tile, int nb, int scale, int col,
                                               int64_t rr, int64_t xr0, int ngroups,
                                               const double* __restrict__ xp, bool xok,
                                               d4 (&acc)[2]) {
    const int g = (threadIdx.x & 63) >> 4;
    double lv[2][8], xv[8], ln[2][8], xn[8];
    auto fetch = [&](int q, double (&l)[2][8], double (&x)[8]) {
        const int64_t o = (int64_t)32 * q + 8 * g;
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                double v4[4];
                ld4_cls<C>(tile, (int64_t)(col + 16 * ni) * nb + rr + o + 4 * u, v4);
#pragma unroll
                for (int t = 0; t < 4; ++t) l[ni][4 * u + t] = v4[t];
            }
        if (C != kFP64 && scale != 0) {
#pragma unroll
            for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                for (int t = 0; t < 8; ++t) l[ni][t] = ldexp(l[ni][t], scale);
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) x[t] = xok ? xp[xr0 + o + t] : 0.0;
    };
    fetch(0, lv, xv);
    for (int q = 0; q < ngroups; ++q) {
        if (q + 1 < ngroups) fetch(q + 1, ln, xn);
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int ni = 0; ni < 2; ++ni)
                acc[ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[t], lv[ni][t], acc[ni], 0, 0, 0);
        if (q + 1 < ngroups) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                xv[t] = xn[t];
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) lv[ni][t] = ln[ni][t];
            }
        }
    }
}

constexpr int kBwdWaveCols = 32;
__global__ __launch_bounds__(256) void bwd_partial_mfma_kernel(TileView L, int k, int t0,
                                                               int64_t rows, int64_t rows_per_split,
                                                               const double* __restrict__ X,
                                                               int64_t ldb, int nrhs, int rhs0,
                                                               double* __restrict__ partial) {
    const int nb = L.nb;
    const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
    const int cbase = (blockIdx.x * 4 + (threadIdx.x >> 6)) * kBwdWaveCols;  // the wave's columns
    if (cbase >= nb) return;
    const int col = cbase + i;  // this lane's columns: col, col + 16
    const int split = blockIdx.y;
    const int nr = nrhs - rhs0 < kNR ? nrhs - rhs0 : kNR;
    const bool xok = i < nr;
    const double* xp = X + (int64_t)(rhs0 + (xok ? i : 0)) * ldb;
    const int64_t rbeg = (int64_t)split * rows_per_split;
    const int64_t rend = rbeg + rows_per_split < rows ? rbeg + rows_per_split : rows;
    d4 acc[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};
    for (int64_t ra = rbeg; ra < rend;) {
        const int m = (int)(ra / nb);
        const int64_t tend = (int64_t)(m + 1) * nb < rend ? (int64_t)(m + 1) * nb : rend;
        int cls, scale;
        const char* tile = view_tile(L, k + 1 + t0 + m, k, cls, scale);
        const int64_t rr = ra - (int64_t)m * nb;
        const int ng = (int)((tend - ra) / 32);
        switch (cls) {
            case kFP64: bwd_mfma_range<kFP64>(tile, nb, scale, col, rr, ra, ng, xp, xok, acc); break;
            case kFP32: bwd_mfma_range<kFP32>(tile, nb, scale, col, rr, ra, ng, xp, xok, acc); break;
            case kFP16: bwd_mfma_range<kFP16>(tile, nb, scale, col, rr, ra, ng, xp, xok, acc); break;
            case kBF16: bwd_mfma_range<kBF16>(tile, nb, scale, col, rr, ra, ng, xp, xok, acc); break;
            default: bwd_mfma_range<kFP8>(tile, nb, scale, col, rr, ra, ng, xp, xok, acc); break;
        }
        ra = tend;
    }
    // block ni, lane l, value v: right-hand side l / 16 + 4 v, column col + 16 ni
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
        double* p = partial + ((int64_t)split * nb + col + 16 * ni) * kNR;
#pragma unroll
        for (int v = 0; v < 4; ++v) p[g + 4 * v] = acc[ni][v];
    }
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

// One tile's contribution to a block of right-hand sides, split for
// parallelism: Y (nb x nr) -= op(T) X, op(T) = T (forward, T = L_{k+1,k}
// ... any tile of a factor view) or T^T (backward), X = nb rows of B.
// Workgroup (i, s) takes output rows 64 i .. 64 i + 63 and the 64 inner
// indices 64 s .. 64 s + 63: the 64 x 64 block of op(T) (decoded from its
// class, all 16 loads of a thread issued together) and the X rows go
// through LDS, each thread forms 4 (row, rhs) sums, and writes its partial
// to part[s][row][rhs]; tile_update_reduce adds up the nb / 64 partials in
// a fixed order. With dense != NULL, T is that binary64 nb x nb matrix
// (column-major) instead of a factor tile, and tri names the blocks of
// op(T) known to be zero (1: op(T) lower triangular, 2: upper); their
// workgroups write zero partials without reading T.
constexpr int kTU = 64;
__global__ __launch_bounds__(256) void tile_update_kernel(TileView L, int ti, int tj,
                                                          const double* __restrict__ dense, int tri,
                                                          int transpose,
                                                          const double* __restrict__ X, int64_t ldb,
                                                          int nrhs, int rhs0,
                                                          double* __restrict__ part) {
    __shared__ double Ts[kTU * (kTU + 1)];  // Ts[q * 65 + r] = op(T)[r0 + r][q0 + q]
    __shared__ double Xs[kTU * kNR];
    const int nb = L.nb;
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * kTU, q0 = blockIdx.y * kTU;
    const int nr = nrhs - rhs0 < kNR ? nrhs - rhs0 : kNR;
    const int r = tid & 63, cg = tid >> 6;  // row, group of 4 right-hand sides
    double* p = part + ((int64_t)blockIdx.y * nb + r0 + r) * kNR + cg * 4;
    if ((tri == 1 && q0 > r0) || (tri == 2 && q0 < r0)) {
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] = 0.0;
        return;
    }
    int cls = kFP64, scale = 0;
    const char* tile = dense ? reinterpret_cast<const char*>(dense) : view_tile(L, ti, tj, cls, scale);
    double lr[16], xr[4];
    // the stored block: rows r0.., columns q0.. (op(T) = T) or rows q0..,
    // columns r0.. (op(T) = T^T); lr[u] = element (row e % 64, column e / 64)
    // of it, e = tid + 256 u
    if (!transpose)
        fetch_block_cls(cls, tile, nb, q0, r0, X, ldb, q0, rhs0, nr, lr, xr);
    else
        fetch_block_cls(cls, tile, nb, r0, q0, X, ldb, q0, rhs0, nr, lr, xr);
    if (scale != 0 && cls != kFP64) {
#pragma unroll
        for (int u = 0; u < 16; ++u) lr[u] = ldexp(lr[u], scale);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * u, a = e % kTU, b = e / kTU;
        if (!transpose) Ts[b * (kTU + 1) + a] = lr[u];  // op(T)[r0 + a][q0 + b]
        else Ts[a * (kTU + 1) + b] = lr[u];             // op(T)[r0 + b][q0 + a]
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + 256 * u;
        Xs[(e % kTU) * kNR + e / kTU] = xr[u];
    }
    __syncthreads();
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (int q = 0; q < kTU; ++q) {
        const double t = Ts[q * (kTU + 1) + r];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += t * Xs[q * kNR + cg * 4 + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) p[u] = acc[u];
}

// Y -= (assign: Y =) the sum of the nb / 64 partials, in split order.
__global__ void tile_update_reduce_kernel(double* __restrict__ Y, int nb, int64_t ldb, int nrhs,
                                          int rhs0, const double* __restrict__ part, int assign) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nb * kNR) return;
    const int row = e / kNR, c = e % kNR;
    if (rhs0 + c >= nrhs) return;
    const int splits = nb / kTU;
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += part[(int64_t)sp * nb * kNR + e];
    double* y = Y + (int64_t)(rhs0 + c) * ldb + row;
    if (assign) *y = s;
    else *y -= s;
}

__global__ __launch_bounds__(256) void logdet_kernel(TileView L, double* __restrict__ partial) {
    __shared__ double red[4];
    const int k = blockIdx.x;
    const int nb = L.nb;
    int cls, scale;
    const double* t = reinterpret_cast<const double*>(view_tile(L, k, k, cls, scale));
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) s += log(t[(int64_t)i * nb + i]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[k] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Factor tiles as binary64 (packed lower order), strict upper triangle of
// diagonal tiles zero.
constexpr int kExpStrips = 16;
__global__ __launch_bounds__(256) void export_kernel(TileView L, int64_t t0,
                                                     double* __restrict__ out) {
    const int nb = L.nb, Nt = L.Nt;
    const int64_t t = t0 + blockIdx.y;
    int64_t j = 0;
    while (tile_off(Nt, Nt - 1, j) < t) ++j;
    const int64_t i = j + (t - tile_off(Nt, j, j));
    int cls, scale;
    const char* tile = view_tile(L, (int)i, (int)j, cls, scale);
    const int64_t per = (int64_t)nb * nb / kExpStrips;
    double* o = out + (int64_t)blockIdx.y * nb * nb;
    for (int64_t e = blockIdx.x * per + threadIdx.x; e < (blockIdx.x + 1) * per; e += 256) {
        const int64_t c = e / nb, r = e - c * nb;
        o[e] = (i == j && r < c) ? 0.0 : load_elem(tile, e, cls, scale);
    }
}

}  // namespace

hipError_t launch_trsv_diag(hipStream_t s, const double* Lkk, int nb, double* B, int64_t ldb,
                            int nrhs, bool transpose) {
    hipLaunchKernelGGL(trsv_diag_kernel, dim3((nrhs + kDR - 1) / kDR), dim3(1024), 0, s, Lkk, nb, B,
                       ldb, nrhs, transpose ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_fwd_update(hipStream_t s, const TileView& L, int k, int t0, int tcount,
                             const double* Yk, double* Bbelow, int64_t ldb, int nrhs,
                             double* partial) {
    if (tcount <= 0) return hipSuccess;
    if (t0 < 0 || k + 1 + t0 + tcount > L.Nt) return hipErrorInvalidValue;
    const int64_t rows = (int64_t)tcount * L.nb;
    if (L.nb % kFwdWaveRows != 0 || L.nb % 32 != 0 || nrhs <= 0) return hipErrorInvalidValue;
    // K splits while the launch has few tiles: tcount * splits <= 64 keeps
    // the partials within bwd_partial_doubles(nb), and each split keeps a
    // whole number of 32-column groups
    int splits = 1;
    while (splits < 8 && tcount * splits * 2 <= 64 && L.nb % (32 * splits * 2) == 0) splits *= 2;
    const int64_t waves = rows / kFwdWaveRows;
    const unsigned wgs = (unsigned)((waves + 3) / 4);
    const int groups = (nrhs + kNR - 1) / kNR;
    if (splits == 1) {
        hipLaunchKernelGGL(fwd_update_mfma_kernel, dim3(wgs, 1, (unsigned)groups), dim3(256), 0, s, L,
                           k, t0, rows, 1, Yk, Bbelow, ldb, nrhs, 0, partial);
        return hipGetLastError();
    }
    // split: the partials hold one group of 16 right-hand sides at a time
    for (int c0 = 0; c0 < nrhs; c0 += kNR) {
        hipLaunchKernelGGL(fwd_update_mfma_kernel, dim3(wgs, (unsigned)splits, 1), dim3(256), 0, s, L,
                           k, t0, rows, splits, Yk, Bbelow, ldb, nrhs, c0, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(fwd_reduce_kernel, dim3((unsigned)((rows * kNR + 255) / 256)), dim3(256), 0,
                           s, Bbelow, rows, ldb, nrhs, c0, splits, partial);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
// Split of a backward update's rows: up to 64 splits, each a multiple of 64
// rows long (the last one may be shorter), at least 128 rows where possible.
int64_t bwd_split_rows(int64_t rows) {
    int64_t s = rows / 128;
    if (s > 64) s = 64;
    if (s < 1) s = 1;
    const int64_t per = (rows + s - 1) / s;
    return (per + 63) / 64 * 64;
}

hipError_t launch_bwd_update(hipStream_t s, const TileView& L, int k, int t0, int tcount,
                             const double* Xbelow, double* Yk, int64_t ldb, int nrhs,
                             double* partial) {
    if (tcount <= 0) return hipSuccess;
    if (t0 < 0 || k + 1 + t0 + tcount > L.Nt) return hipErrorInvalidValue;
    const int64_t rows = (int64_t)tcount * L.nb;
    if (L.nb % 64 != 0 || nrhs <= 0) return hipErrorInvalidValue;
    const int64_t per = bwd_split_rows(rows);
    const int splits = (int)((rows + per - 1) / per);
    for (int rhs0 = 0; rhs0 < nrhs; rhs0 += kNR) {
        dim3 grid((L.nb + 4 * kBwdWaveCols - 1) / (4 * kBwdWaveCols), splits);
        hipLaunchKernelGGL(bwd_partial_mfma_kernel, grid, dim3(256), 0, s, L, k, t0, rows, per,
                           Xbelow, ldb, nrhs, rhs0, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(bwd_reduce_kernel, dim3((L.nb * kNR + 255) / 256), dim3(256), 0, s, Yk,
                           L.nb, ldb, nrhs, rhs0, splits, partial);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {
hipError_t tile_product(hipStream_t s, const TileView& L, int ti, int tj, const double* dense,
                        int tri, bool transpose, const double* X, double* Y, int64_t ldb,
                        int nrhs, double* partial, int assign) {
    if (L.nb % kTU != 0 || nrhs <= 0) return hipErrorInvalidValue;
    for (int rhs0 = 0; rhs0 < nrhs; rhs0 += kNR) {
        hipLaunchKernelGGL(tile_update_kernel, dim3(L.nb / kTU, L.nb / kTU), dim3(256), 0, s, L, ti, tj,
                           dense, tri, transpose ? 1 : 0, X, ldb, nrhs, rhs0, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(tile_update_reduce_kernel, dim3((L.nb * kNR + 255) / 256), dim3(256), 0, s, Y,
                           L.nb, ldb, nrhs, rhs0, partial, assign);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

hipError_t launch_tile_update(hipStream_t s, const TileView& L, int ti, int tj, bool transpose,
                              const double* X, double* Y, int64_t ldb, int nrhs, double* partial) {
    return tile_product(s, L, ti, tj, nullptr, 0, transpose, X, Y, ldb, nrhs, partial, 0);
}

hipError_t launch_tile_inv_apply(hipStream_t s, const double* xinv, int nb, const double* in,
                                 double* out, int64_t ldb, int nrhs, bool transpose,
                                 double* partial) {
    // M = Xinv^T (lower) is op(T) = T^T with T = Xinv; M = Xinv (upper) is op(T) = T
    TileView D{nullptr, nullptr, nullptr, nullptr, 1, nb};
    return tile_product(s, D, 0, 0, xinv, transpose ? 2 : 1, !transpose, in, out, ldb, nrhs,
                        partial, 1);
}

hipError_t launch_logdet_partials(hipStream_t s, const TileView& L, double* partial) {
    hipLaunchKernelGGL(logdet_kernel, dim3(L.Nt), dim3(256), 0, s, L, partial);
    return hipGetLastError();
}

hipError_t launch_export_range(hipStream_t s, const TileView& L, int64_t t0, int64_t count,
                               double* out) {
    const int64_t ntiles = (int64_t)L.Nt * (L.Nt + 1) / 2;
    if (t0 < 0 || count < 0 || t0 + count > ntiles) return hipErrorInvalidValue;
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(export_kernel, dim3(kExpStrips, (unsigned)count), dim3(256), 0, s, L, t0,
                       out);
    return hipGetLastError();
}

hipError_t launch_export(hipStream_t s, const TileView& L, double* out) {
    return launch_export_range(s, L, 0, (int64_t)L.Nt * (L.Nt + 1) / 2, out);
}

}  // namespace tc
