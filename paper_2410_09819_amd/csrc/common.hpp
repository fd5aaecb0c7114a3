// Internal declarations shared by the kernel files and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

// Tiles stored before lower tile (i, j) in packed column-of-tiles order.
__host__ __device__ inline int64_t tile_off(int64_t Nt, int64_t i, int64_t j) {
    return j * Nt - j * (j - 1) / 2 + (i - j);
}

// Workgroup ids are dealt round-robin to the 8 XCDs (each with its own L2).
// Logical block of hardware id hw out of `total`: each XCD takes a contiguous
// run of logical blocks, so neighbouring blocks (which share operand rows)
// run under one L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t hw, int64_t total) {
    const int64_t xcd = hw % 8, idx = hw / 8;
    const int64_t q = total / 8, r = total % 8;
    return xcd * q + (xcd < r ? xcd : r) + idx;
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

// Read-only view of a factor's tiles. Without tables (toff == nullptr) the
// tiles are binary64 in packed lower order at `base`; otherwise tile t is
// stored in class tcls[t] at base + toff[t] bytes, scaled by 2^tscl[t].
struct TileView {
    const char* base;
    const int64_t* toff;
    const uint8_t* tcls;
    const int* tscl;
    int Nt;
    int nb;
};

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
//   C[k.., k] -= L[k.., nbeg:nend] L[k, nbeg:nend]^T (tile columns), lower
// blocks only in the diagonal tile. splits > 1 writes partial sums to
// `partial`; launch_panel_reduce then subtracts their sum (no-op for
// splits == 1). `tail` selects the kernel instance used for the rank-nb
// updates of the lookahead schedule (same code, separate trace name).
hipError_t launch_panel_update(hipStream_t s, double* L, int Nt, int nb, int k, int nbeg, int nend,
                               int splits, double* partial, bool tail);
hipError_t launch_panel_reduce(hipStream_t s, double* L, int Nt, int nb, int k, int splits,
                               const double* partial);
// Number of workgroups of one panel launch (before split-K).
int64_t panel_blocks(int Nt, int nb, int k);
// Split count for column k's update over ncols tile columns, with the
// partial sums held to cap_bytes.
int panel_splits(int Nt, int nb, int k, int ncols, size_t cap_bytes = (size_t)512 << 20);

// In-tile update for the recursive POTRF (column-major sub-blocks, ld):
//   C (m x m, lower blocks) -= A A^T, A is m x kdim.
hipError_t launch_syrk_sub(hipStream_t s, double* C, const double* A, int ld, int m, int kdim,
                           double* partial, int splits);
int syrk_sub_splits(int m, int kdim);

// TRSM X = C L^{-T} (trsm_f64.hip). C: M rows (a multiple of 64), w columns;
// row r at C + (r / nb) * nb * nb + (r % nb) + c * nb (rows of consecutive
// tiles of a tile column, or a sub-block of one tile when M <= nb).
// L: w x w lower, column-major with leading dimension nb. leaf: widest
// column block solved by one leaf launch (a multiple of 128).
hipError_t launch_trsm(hipStream_t s, double* C, const double* L, int nb, int64_t M, int w,
                       int leaf = 128);
// Leaf width of the FP64 factorizations' panel TRSM (the tiles below a
// diagonal tile). While a bulk panel update holds the chip, a kernel on
// another stream gets workgroup slots mostly after the bulk's last
// workgroups are dispatched, so the TRSM waits once per launch: 512-column
// leaves (a leaf, a GEMM, a leaf for nb = 1024) instead of 128-column ones
// (fifteen launches) let it finish earlier, and alone it is faster too.
// The n = 65536, nb = 1024 factorization, alternating runs on one box:
// 1.528 s (128), 1.520 s (256), 1.516 s (512), 1.520 s (1024: one launch,
// whose workgroups then walk all 16 column blocks alone).
constexpr int kPanelTrsmLeaf = 512;
// The same solve for a whole nb x nb factor tile (w = nb) in two launches:
// inverses of L's 64 x 64 diagonal blocks into dinv (nb * 64 doubles), then
// one pass in which each workgroup walks its 64 rows' column blocks with
// MFMA products (the substitution inside a block becomes a product with the
// block's inverse). M a multiple of 64. Used where binary64 substitution
// order is not required (the mixed-precision factorizations).
hipError_t launch_trsm_blockinv(hipStream_t s, double* C, const double* L, int nb, int64_t M,
                                double* dinv);
// xinv + k nb^2 <- L_kk^{-T} (upper triangular, column-major) for every
// diagonal tile k of the factor view, in two launches (dinv: Nt * nb * 64
// doubles of scratch for the inverted 64 x 64 diagonal blocks).
hipError_t launch_diag_tiles_inv(hipStream_t s, const TileView& V, double* dinv, double* xinv);
// out = M in for one diagonal tile's inverse Xinv = L_kk^{-T}: M = Xinv^T
// (= L_kk^{-1}, transpose false) or Xinv (= L_kk^{-T}, transpose true).
// in and out: nb rows x nrhs, column-major with leading dimension ldb, not
// overlapping. Split over the nonzero 64 x 64 blocks of M like
// launch_tile_update (partial: the same workspace).
hipError_t launch_tile_inv_apply(hipStream_t s, const double* xinv, int nb, const double* in,
                                 double* out, int64_t ldb, int nrhs, bool transpose,
                                 double* partial);

// Leaf POTRF of an s x s block (s <= 128) at T (leading dimension ld), in
// place; on failure sets *info = col0 + j + 1 if *info was 0 (potrf.hip).
hipError_t launch_potrf_leaf(hipStream_t s, double* T, int ld, int size, int* info, int64_t col0);
hipError_t launch_zero_info(hipStream_t s, int* info);
// Strict upper triangle of every diagonal tile to zero (export).
hipError_t launch_zero_upper(hipStream_t s, double* L, int Nt, int nb);

// Solves with the factor (solve.hip). Lkk is the (binary64) diagonal tile.
hipError_t launch_trsv_diag(hipStream_t s, const double* Lkk, int nb, double* B, int64_t ldb,
                            int nrhs, bool transpose);
// B rows of tiles m = k+1+t0 .. k+t0+tcount -= L[m, k] Y_k (Y_k = B rows of
// tile k; Bbelow = B rows of tile k+1+t0). partial: bwd_partial_doubles(nb)
// doubles of workspace (launches with few tiles are split over K).
hipError_t launch_fwd_update(hipStream_t s, const TileView& L, int k, int t0, int tcount,
                             const double* Yk, double* Bbelow, int64_t ldb, int nrhs,
                             double* partial);
// Y_k -= sum L_mk^T X_m over m = k+1+t0 .. k+t0+tcount (Xbelow = B rows of
// tile k+1+t0); partial: bwd_partial_doubles(nb) doubles of workspace.
hipError_t launch_bwd_update(hipStream_t s, const TileView& L, int k, int t0, int tcount,
                             const double* Xbelow, double* Yk, int64_t ldb, int nrhs,
                             double* partial);
int64_t bwd_split_rows(int64_t rows);
inline int64_t bwd_partial_doubles(int nb) { return (int64_t)64 * nb * 16; }
// Y -= op(T) X for the single tile T = (ti, tj) of a factor view (op = T or
// T^T), split over nb / 64 inner blocks (partial: nb / 64 * nb * 16 doubles,
// <= bwd_partial_doubles(nb)) and reduced in a fixed order.
hipError_t launch_tile_update(hipStream_t s, const TileView& L, int ti, int tj, bool transpose,
                              const double* X, double* Y, int64_t ldb, int nrhs, double* partial);
hipError_t launch_logdet_partials(hipStream_t s, const TileView& L, double* partial);

// Mixed precision (mxp.hip): class-group panel updates into the working
// column W (binary64, tile-strided rows, W[0] = diagonal tile) over the
// tile columns n in [nbeg, nend) of column k, and the finalize step that
// rounds column k's new tiles into storage.
hipError_t launch_mxp_gemm_f64(hipStream_t s, double* W, int Nt, int nb, int k, int nbeg, int nend,
                               const int* rows, int nrows, bool diag, const char* storage,
                               const int64_t* toff, const uint8_t* tcls, const int* tscl,
                               double* partial, size_t partial_cap);
// FP32 group: FP16 MFMA over the two-plane (hi, lo) split copies.
// wide: 256 x 256 blocks (1: whenever nb allows, 0: when the launch has at
// least 256 of them, -1: never) or 128 x 128 blocks.
hipError_t launch_mxp_gemm_f32(hipStream_t s, double* W, int Nt, int nb, int k, int nbeg, int nend,
                               const int* rows, int nrows, const char* storage,
                               const int64_t* shoff, const int* cscl, int wide);
// FP16 / BF16 / FP8 group: narrow-format MFMA over the class's operand
// copies (row-major bits, per-copy scale cscl), FP32 accumulation.
hipError_t launch_mxp_gemm_narrow(hipStream_t s, double* W, int Nt, int nb, int k, int nbeg,
                                  int nend, const int* rows, int nrows, int cls,
                                  const char* storage, const int64_t* shoff, const int* cscl,
                                  int wide);
// Operand copies of the stored tiles list[0..count) (out of core: tiles
// loaded into cache slots), from their stored bits and recorded scales.
hipError_t launch_mxp_copies(hipStream_t s, int nb, const int* list, int count, char* storage,
                             const int64_t* toff, const uint8_t* tcls, const int* tscl,
                             const int64_t* shoff, const int* cscl);
// Point the tile and copy offset tables of tiles upd[2i] at slot offsets
// upd[2i + 1] (copy class c at + coff[c - 1] when bit c of need[t] is set).
hipError_t launch_slot_tables(hipStream_t s, const int64_t* upd, int count, const uint8_t* need,
                              const int64_t* coff, int64_t* toff, int64_t* shoff);
// Host image of column k of an out-of-core mixed factor in dst: the new
// tiles (k+1.., k), read at cache offsets toff[t] in their classes (tcls),
// written at dst + htoff[t] - htoff[(k, k)] (their host-image offsets
// relative to the diagonal tile, which is already at dst).
hipError_t launch_image_gather(hipStream_t s, const char* cache, const int64_t* toff,
                               const int64_t* htoff, const uint8_t* tcls, int Nt, int nb, int k,
                               char* dst);
hipError_t launch_mxp_finalize(hipStream_t s, const double* W, int Nt, int nb, int k, double* part,
                               char* storage, const int64_t* toff, const uint8_t* tcls, int* tscl,
                               const int64_t* shoff, int* cscl);
hipError_t launch_export(hipStream_t s, const TileView& L, double* out);
// Tiles [t0, t0 + count) of the packed lower order as binary64 into out.
hipError_t launch_export_range(hipStream_t s, const TileView& L, int64_t t0, int64_t count,
                               double* out);

// Refinement (ir.hip).
size_t residual_partial_doubles(int Nt, int nb, int nrhs);
hipError_t launch_residual(hipStream_t s, const double* A, int Nt, int nb, const double* X,
                           int64_t ldx, const double* B, int64_t ldb, int nrhs, double* partial,
                           double* R, int64_t ldr);
int colnorm_blocks();
hipError_t launch_colnorm(hipStream_t s, const double* X, int64_t ld, int64_t n, int nrhs,
                          double* part);
hipError_t launch_axpy(hipStream_t s, double* Y, int64_t ldy, const double* D, int64_t ldd,
                       int64_t n, int nrhs);
hipError_t launch_copy_cols(hipStream_t s, double* Y, int64_t ldy, const double* X, int64_t ldx,
                            int64_t n, int nrhs);

// Reverse mode (adjoint.hip). AdjMat: element (r, c) of a matrix whose rows
// come in chunks of `rt` rows placed `rs` doubles apart, each chunk
// column-major with leading dimension `ld` (rt = nb, rs = nb^2 for a column
// of tiles; rs = 0 and rt >= rows for a plain column-major matrix).
struct AdjMat {
    double* p;
    int64_t ld, rt, rs;
    __host__ __device__ int64_t off(int64_t r, int64_t c) const {
        return (r / rt) * rs + (r % rt) + c * ld;
    }
};
struct AdjGemmPlan {
    int block;
    int splits;
    int64_t nblocks;
    size_t partial_doubles;
};
// Lbar_mn -= sum_{k>n} S_mk L_kn for the tiles below (n, n) (see adjoint.hip).
// Exactly one of Tt (transposed copies of Abar, H_m on the diagonal) and Hd
// (memory-short form: H_m per tile row; Abar_km^T read from Lb) is non-null.
hipError_t launch_adj_panel(hipStream_t s, double* Lb, const double* Tt, const double* Hd,
                            const double* PL, int Nt, int nb, int n, int splits, double* partial);
int64_t adj_panel_blocks(int Nt, int nb, int n);
int adj_panel_splits(int Nt, int nb, int n);
// C = A B^T (sub: C -= A B^T); A: M x K, B: N x K, all AdjMat with the same
// ld; block rows must not straddle chunks. lower: only blocks on or below
// the diagonal (M == N).
AdjGemmPlan adj_gemm_plan(int64_t M, int64_t N, int64_t K, bool lower);
hipError_t launch_adj_gemm(hipStream_t s, const AdjMat& C, const AdjMat& A, const AdjMat& B,
                           int64_t M, int64_t N, int64_t K, bool sub, bool lower, double* partial);
hipError_t launch_transpose_tiles(hipStream_t s, const double* src, double* dst, int nb,
                                  int64_t count, bool tril);
hipError_t launch_set_identity(hipStream_t s, double* X, int nb);
hipError_t launch_mirror_lower(hipStream_t s, double* P, int nb);
hipError_t launch_finish_diag(hipStream_t s, const double* H, double* D, int nb);
hipError_t launch_loglik_seed(hipStream_t s, const TileView& L, const double* alpha, const double* z,
                              double* Lb, int Nt, int nb);
// sum_{i>=j} Abar_ij (C_ij / sigma2, dC_ij/drange) and sum_i Abar_ii, as 3
// partial sums per (tile, strip) in `part` (matern.hip).
hipError_t launch_matern_grad(hipStream_t s, int64_t n, int nb, const double* locs, double sigma2,
                              double inv_range, double nu, int nu_kind, double norm_const,
                              const double* Abar, double* part);
hipError_t launch_sum3(hipStream_t s, const double* part, int64_t count, double* out);

}  // namespace tc
