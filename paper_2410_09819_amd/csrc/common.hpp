// Internal declarations shared by the kernel files and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

// Tiles stored before lower tile (i, j) in packed column-of-tiles order.
__host__ __device__ inline int64_t tile_off(int64_t Nt, int64_t i, int64_t j) {
    return j * Nt - j * (j - 1) / 2 + (i - j);
}

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));

// Value of v in lane `lane` of the wave (lane must be wave-uniform): two
// v_readlane_b32 into scalar registers, no LDS round trip.
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// ---- launchers (all enqueue on `s`, return hipGetLastError()) -------------

// Matern tiles + per-tile sum of squares partials (matern.hip).
// nu_kind: 0 -> nu = 1/2, 1 -> 3/2, 2 -> 5/2, 3 -> general nu (quadrature).
hipError_t launch_matern(hipStream_t s, int64_t n, int nb, const double* locs, double sigma2,
                         double inv_range, double nu, int nu_kind, double norm_const, double nugget,
                         double* A, double* strip_ss);
hipError_t launch_tile_norms(hipStream_t s, int64_t ntiles, int strips, const double* strip_ss,
                             double* tile_fro);
// Number of column strips per tile used by launch_matern's partial sums.
int matern_strips(int nb);

// Panel update for column k (gemm_f64.hip):
//   C[k.., k] -= L[k.., 0:k] L[k, 0:k]^T, lower blocks only in the diagonal
// tile. splits > 1 writes partial sums to `partial`; launch_panel_reduce
// then subtracts their sum (no-op for splits == 1).
hipError_t launch_panel_update(hipStream_t s, double* L, int Nt, int nb, int k, int splits,
                               double* partial);
hipError_t launch_panel_reduce(hipStream_t s, double* L, int Nt, int nb, int k, int splits,
                               const double* partial);
// Number of workgroups of one panel launch (before split-K).
int64_t panel_blocks(int Nt, int nb, int k);
int panel_splits(int Nt, int nb, int k);

// In-tile update for the recursive POTRF (column-major sub-blocks, ld):
//   C (m x m, lower blocks) -= A A^T, A is m x kdim.
hipError_t launch_syrk_sub(hipStream_t s, double* C, const double* A, int ld, int m, int kdim,
                           double* partial, int splits);
int syrk_sub_splits(int m, int kdim);

// TRSM X = C L^{-T} (trsm_f64.hip). C: M rows (a multiple of 64), w columns;
// row r at C + (r / nb) * nb * nb + (r % nb) + c * nb (rows of consecutive
// tiles of a tile column, or a sub-block of one tile when M <= nb).
// L: w x w lower, column-major with leading dimension nb.
hipError_t launch_trsm(hipStream_t s, double* C, const double* L, int nb, int64_t M, int w);

// Leaf POTRF of an s x s block (s <= 128) at T (leading dimension ld), in
// place; on failure sets *info = col0 + j + 1 if *info was 0 (potrf.hip).
hipError_t launch_potrf_leaf(hipStream_t s, double* T, int ld, int size, int* info, int64_t col0);
hipError_t launch_zero_info(hipStream_t s, int* info);
// Strict upper triangle of every diagonal tile to zero (export).
hipError_t launch_zero_upper(hipStream_t s, double* L, int Nt, int nb);

// Solves with the factor (solve.hip).
hipError_t launch_trsv_diag(hipStream_t s, const double* Lkk, int nb, double* B, int64_t ldb,
                            int nrhs, bool transpose);
hipError_t launch_fwd_update(hipStream_t s, const double* Lcol, int nb, int64_t rows,
                             const double* Yk, double* Bbelow, int64_t ldb, int nrhs);
hipError_t launch_bwd_update(hipStream_t s, const double* Lcol, int nb, int64_t rows,
                             const double* Xbelow, double* Yk, int64_t ldb, int nrhs,
                             double* partial, int splits);
int bwd_splits(int64_t rows);
hipError_t launch_logdet_partials(hipStream_t s, const double* L, int Nt, int nb, double* partial);

}  // namespace tc
