/*
 * tilechol.h - C ABI of libtilechol, a tile-based left-looking Cholesky
 * factorization A = L L^T of dense symmetric positive-definite matrices on
 * one AMD Instinct MI355X (gfx950), with hand-written HIP kernels.
 *
 * Method: arXiv 2410.09819, "Accelerating Mixed-Precision Out-of-Core
 * Cholesky Factorization with Static Task Scheduling".
 *   - Section III-A / Algorithm 1: the matrix is cut into Nt x Nt tiles of
 *     size nb; column of tiles k is produced by SYRK-updating the diagonal
 *     tile with every tile to its left and factorizing it (POTRF), then
 *     GEMM-updating each tile below it with the tiles to its left and solving
 *     it against the transposed diagonal factor (TRSM).
 *   - Section III-B: a static schedule; the order of all tasks is fixed
 *     before the factorization starts.
 *   - Section III-D, Eq. 1 and Eq. 2: the matrix is a Matern covariance over
 *     spatial locations; its factor gives log|Sigma| and Sigma^{-1} y.
 *
 * Conventions for every entry point:
 *   - Returns tc_status and never throws. 0 is success. A positive value
 *     from tc_factorize is LAPACK's "info": the 1-based global index of the
 *     first column whose pivot was not strictly positive (or was NaN).
 *     Negative values are errors; tc_last_error() then describes them.
 *   - Tiled storage ("packed lower tiles"): only the Nt(Nt+1)/2 tiles (i,j)
 *     with i >= j are stored, each nb x nb and column-major (leading
 *     dimension nb), listed column of tiles by column of tiles, top to
 *     bottom: tile (i,j) starts at element tc_tile_offset(Nt,i,j) * nb * nb.
 *     Diagonal tiles are stored in full; their strict upper triangle is
 *     ignored on input and undefined in a factor (tc_factor_export writes
 *     zeros there).
 *   - Device pointers are plain HIP device addresses on the context's
 *     device; the caller owns and frees every buffer it passes in. Work is
 *     enqueued on the context's compute stream; each call returns after its
 *     work has completed unless stated otherwise.
 *   - n must be a positive multiple of nb, and nb a multiple of 128 with
 *     nb <= 2048.
 */
#ifndef TILECHOL_H
#define TILECHOL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tc_status;
#define TC_OK 0
#define TC_EINVAL (-1)        /* bad argument (null pointer, bad size, ...) */
#define TC_ENOMEM (-2)        /* workspace or budget too small */
#define TC_EHIP (-3)          /* a HIP runtime call failed */
#define TC_ENOTCONV (-4)      /* refinement did not reach the tolerance */
#define TC_EUNSUPPORTED (-5)  /* valid request the library does not implement */

/* Storage classes of a tile (Section IV-C: one precision per tile). */
typedef enum { TC_FP64 = 0, TC_FP32 = 1, TC_FP16 = 2, TC_BF16 = 3, TC_FP8E4M3 = 4 } tc_prec;

typedef struct tc_ctx tc_ctx;       /* device, streams, workspace */
typedef struct tc_factor tc_factor; /* a computed factor (metadata; tiles live in caller memory) */

/* Matern parameters of Eq. 2 plus a nugget added on the diagonal:
 * Sigma_ij = sigma2 / (2^(nu-1) Gamma(nu)) x^nu K_nu(x) + nugget [i==j],
 * x = ||s_i - s_j|| / range. */
typedef struct {
    double sigma2;
    double range;
    double nu;
    double nugget;
} tc_matern;

typedef struct {
    int32_t inplace;     /* 1: the factor overwrites the input tiles (storage == A) */
    /* Arithmetic of the GEMM/SYRK updates into FP64-class tiles, the
     * diagonal tiles' SYRK included: TC_FP64 (0, default; the paper's
     * four-precision scheme, Section IV-C) or TC_FP32 (the FP32 class's
     * arithmetic: binary32-rounded operands split into two FP16 terms, FP32
     * accumulation). With TC_FP32 binary64 arithmetic is left to POTRF,
     * TRSM, the rounding of new tiles and the refinement residuals; FP64
     * tiles stay stored in binary64. The factor is then a mixed factor
     * even for an all-FP64 map, and its storage grows by the FP32 operand
     * copies of the FP64 tiles (tc_factor_bytes with the same opts).
     * Refined solves reach binary64 accuracy with such a factor; its
     * log-determinant carries the FP32-class error of the updates. */
    int32_t fp64_update;
    /* Block shape of the FP32 / FP16 / BF16 / FP8 update kernels: 0
     * (default) takes 256 x 256 blocks when nb is a multiple of 256 and a
     * group launch has at least 128 of them, else 128 x 128; 1 takes
     * 256 x 256 whenever nb is a multiple of 256; -1 always 128 x 128. The
     * two shapes round the binary32 sums in a different order and are
     * otherwise the same arithmetic. */
    int32_t wide_tiles;
    int32_t reserved[5];
} tc_opts;

typedef struct {
    double ms_total;        /* factorization wall time, HIP events on the compute stream */
    double ms_gemm;         /* summed duration of the bulk panel GEMM/SYRK launches (if timed);
                               in the FP64 factorization these are the updates of column k+1
                               from tile columns < k that run ahead of column k's POTRF/TRSM */
    double gemm_flops;      /* algorithmic flops of those launches */
    int32_t gemm_launches;  /* number of those launches */
    int32_t info;           /* same as the positive return value, or 0 */
    double flops_total;     /* n^3/3, the count the throughput metric uses */
    double class_flops[5];  /* panel-update flops executed per class (tc_prec order) */
    int32_t class_tiles[5]; /* stored tiles per class */
    int32_t reserved;
} tc_stats;

typedef struct {
    int32_t iterations;     /* refinement corrections applied */
    int32_t converged;      /* 1 if max_j ||b_j - A x_j|| / ||b_j|| <= tol */
    double rel_residual;    /* final max_j ||b_j - A x_j||_2 / ||b_j||_2 (binary64) */
    double history[32];     /* the same quantity after the first solve and each correction */
    double ms_total;        /* wall time of the whole solve, HIP events */
} tc_ir_stats;

typedef struct {
    uint64_t bytes_h2d;      /* host -> HBM bytes (accumulators and reloaded operand tiles) */
    uint64_t bytes_d2h;      /* HBM -> host bytes (write-back of the factor) */
    int32_t tiles_reloaded;  /* operand tiles loaded from the host copy of L */
    int32_t evictions;       /* cached tiles evicted to make room */
    int32_t chunks;          /* panel-update launches (K chunks) */
    int32_t cache_slots;     /* tiles the cache holds */
    double ms_total;         /* wall time, HIP events */
    double flops_total;      /* n^3/3 */
    int32_t info;            /* LAPACK info or 0 */
    int32_t reserved;
} tc_ooc_stats;

/* Tiles stored before lower tile (i,j), i >= j, in packed lower order:
 * j*Nt - j*(j-1)/2 + (i-j) (Section III-A: the matrix as tiles A_ij, of
 * which the left-looking factorization reads and writes the lower
 * triangle, column of tiles by column of tiles). Returns -1 if the indices
 * are out of range. */
int64_t tc_tile_offset(int32_t Nt, int32_t i, int32_t j);

/* Pinned (page-locked) host memory of exactly `bytes` bytes for the
 * out-of-core entry points' host buffers (hipHostMalloc); *out = NULL and
 * TC_ENOMEM when the system refuses. Free with tc_host_free. */
tc_status tc_host_alloc(size_t bytes, void **out);
tc_status tc_host_free(void *p);

/* Library version string (static storage). */
const char *tc_version(void);

/* Text of the last error on the calling thread (static thread-local
 * storage, valid until the next call on that thread). */
const char *tc_last_error(void);

/* Bytes of device workspace a context needs for matrices up to order n with
 * tile size nb and up to nrhs right-hand sides per refined solve. */
size_t tc_workspace_bytes(int64_t n, int32_t nb, int32_t nrhs);

/* Create a context on HIP device `device`. `workspace` is a device buffer of
 * `workspace_bytes` bytes that the context uses for scratch (split-K
 * partial sums, failure flag, reduction partials); it must stay allocated
 * until tc_ctx_destroy. `compute_stream` is a hipStream_t (NULL: the null
 * stream). `flags` bit 0 (TC_CTX_TIMED) times each panel GEMM launch with
 * HIP events (filled into tc_stats). Bits 1 and 2 select reduced variants
 * of tc_factorize_ooc for the paper's comparison of out-of-core strategies
 * (Section IV-B): TC_CTX_OOC_SYNC issues every host transfer on the compute
 * stream (no overlap of copies with compute); TC_CTX_OOC_NO_REUSE drops
 * every cached operand tile after each column (the accumulator still stays
 * resident, V1, but operands are not reused across columns, no V2).
 * Bit 3 (TC_CTX_OOC_EVICT_LRU) replaces the next-use eviction of
 * tc_factorize_ooc by least-recently-used eviction (the paper's "least
 * utilized" tiles, Section IV-B), for the same comparison. Bit 4
 * (TC_CTX_OOC_NO_V3) drops V3 (Section IV-B: the diagonal tile kept in HBM
 * through its column's TRSMs): tc_factorize_ooc writes the diagonal factor
 * back after POTRF and loads it again from host memory for each tile's
 * TRSM, through two extra cache slots (so the cache needs 2 * Nt + 2).
 *
 * Besides the caller's stream the library uses three streams of its own per
 * device (non-blocking, default priority), created by the first context on
 * the device, shared by all contexts there and kept until the process ends.
 * HIP places streams on a small pool of hardware queues (GPU_MAX_HW_QUEUES,
 * 4 by default) and shares a queue between streams once the pool is used
 * up; two streams on one queue run in submission order, which serializes
 * the overlap of copies (and of the lookahead) with compute. A process that
 * holds more streams than the pool has queues may therefore see slower
 * out-of-core and lookahead schedules (results unchanged); raising
 * GPU_MAX_HW_QUEUES avoids it. tc_ctx_destroy waits for the library's
 * streams on the device. Errors: TC_EINVAL (device out of range),
 * TC_EHIP (event or stream creation). */
#define TC_CTX_TIMED 1u
#define TC_CTX_OOC_SYNC 2u
#define TC_CTX_OOC_NO_REUSE 4u
#define TC_CTX_OOC_EVICT_LRU 8u
#define TC_CTX_OOC_NO_V3 16u
tc_status tc_ctx_create(tc_ctx **ctx, int device, void *workspace, size_t workspace_bytes,
                        void *compute_stream, uint32_t flags);
tc_status tc_ctx_destroy(tc_ctx *ctx);

/* Matern covariance tiles (Section III-D, Eq. 2) for n locations.
 * locs: device, n x 2 binary64, row-major (x0, y0, x1, y1, ...).
 * A: device, packed lower tiles of Nt = n/nb tiles per side (written; both
 *    triangles of the diagonal tiles are filled).
 * tile_fro: device, Nt(Nt+1)/2 binary64 or NULL: Frobenius norm of every
 *    stored tile (diagonal tiles in full), in packed order.
 * fro_A: host, 1 binary64 or NULL: ||Sigma||_F of the full symmetric matrix
 *    (requires tile_fro).
 * Smoothness nu = 0.5, 1.5 and 2.5 use closed forms; other nu > 0 use the
 * integral K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt by the
 * trapezoid rule. */
tc_status tc_matern_tiles(tc_ctx *ctx, int64_t n, int32_t nb, const double *locs,
                          const tc_matern *theta, double *A, double *tile_fro, double *fro_A);

/* Per-tile precision map (Section IV-C): tile (i,j), i > j, takes the lowest
 * class p in allowed_mask (bit c set = class c allowed) for which
 *   Nt * tile_fro[t] / fro_A < eps / eps_p
 * holds, eps_p being the class's machine epsilon 2^(1-p_bits) (or its unit
 * roundoff 2^-p_bits when unit_roundoff != 0); otherwise, and on the
 * diagonal, TC_FP64. tile_fro: host, Nt(Nt+1)/2 Frobenius norms in packed
 * order; fro_A: ||A||_F of the full symmetric matrix; map_out: host,
 * Nt(Nt+1)/2 bytes. Host-only computation. */
tc_status tc_precision_map(int32_t Nt, const double *tile_fro, double fro_A, double eps,
                           uint32_t allowed_mask, int32_t unit_roundoff, uint8_t *map_out);

/* Tile Cholesky factorization (Algorithm 1 under a static schedule).
 * A: device packed lower tiles (n, nb), binary64, read only unless
 *    storage == A (allowed for all-FP64 maps only).
 * map: host, Nt(Nt+1)/2 tc_prec codes in packed order, or NULL for all
 *    TC_FP64. Diagonal tiles must be TC_FP64. With low-precision tiles the
 *    factor is stored per tile in its class (FP16 and FP8 tiles with a
 *    power-of-two scale), each update into a tile of class p is computed
 *    from operands rounded to p with FP32 accumulation, POTRF and TRSM run
 *    in FP64 and each new tile is rounded to its class. FP32-class updates
 *    run on the FP16 matrix cores with each binary32 operand split into two
 *    FP16 terms (three products; at most 3 * 2^-22 relative error per
 *    product for entries within 2^18 of their tile's largest, before the
 *    FP32 accumulation).
 * opts: NULL for the defaults, or see tc_opts. TC_EINVAL for an
 *    fp64_update other than TC_FP64 or TC_FP32.
 * storage: device buffer of tc_factor_bytes(n, nb, map, opts) bytes that
 *    receives the factor (tiles, operand copies for the low-precision
 *    updates, the factor's own tables and, for a mixed factor, L_kk^{-T} of
 *    every diagonal tile for the solves). It must outlive *L.
 * L: receives a new factor handle (free with tc_factor_destroy), also when
 *    the return value is positive (the factor is then partial).
 * stats: NULL or filled. */
size_t tc_factor_bytes(int64_t n, int32_t nb, const uint8_t *map, const tc_opts *opts);
tc_status tc_factorize(tc_ctx *ctx, int64_t n, int32_t nb, const double *A, const uint8_t *map,
                       const tc_opts *opts, void *storage, size_t storage_bytes,
                       tc_factor **L, tc_stats *stats);

/* Solve Sigma X = B with the factor: B <- L^{-T} L^{-1} B (tiles used as
 * stored, upcast to binary64). Section III-D: applying Sigma^{-1}, the
 * y^T Sigma^{-1} y term of Eq. 1, through the Cholesky factor. For a mixed factor with ldb == n and
 * nrhs <= 16 the diagonal steps multiply by the stored L_kk^{-1} and
 * L_kk^{-T} (through an intermediate vector in the workspace); otherwise
 * they substitute with the diagonal tiles.
 * B: device, n x nrhs binary64, column-major with leading dimension ldb >= n
 *    (may be NULL when nrhs == 0, which does nothing). */
tc_status tc_solve(tc_ctx *ctx, const tc_factor *L, double *B, int64_t ldb, int32_t nrhs);

/* Iterative refinement in binary64 (not in the paper; the classic scheme it
 * cites): x = (L L^T)^{-1} b, then repeat r = b - A x (binary64, A from its
 * packed lower tiles), x += (L L^T)^{-1} r until max_j ||r_j|| / ||b_j|| <= tol
 * or max_iter corrections. A: the matrix that was factored (device packed
 * lower tiles). B: on input b, on output x (device, column-major, ldb).
 * Returns TC_ENOTCONV (with stats filled) if tol is not reached. The
 * workspace must be sized with tc_workspace_bytes(n, nb, nrhs') for some
 * nrhs' >= nrhs. */
tc_status tc_solve_refine(tc_ctx *ctx, const tc_factor *L, const double *A, double *B,
                          int64_t ldb, int32_t nrhs, int32_t max_iter, double tol,
                          tc_ir_stats *stats);

/* log|Sigma| = 2 sum_i log L_ii (Eq. 1's log-determinant), into *out (host). */
tc_status tc_logdet(tc_ctx *ctx, const tc_factor *L, double *out);

/* Out-of-core FP64 tile Cholesky (Sections III-C and IV-B): the matrix and
 * the factor stay in host memory and stream through HBM under the static
 * left-looking schedule.
 * A_host: pinned host memory (hipHostMalloc or equivalent), packed lower
 *    tiles (n, nb), binary64, read.
 * L_host: pinned host memory of the same size receiving the factor; it may
 *    equal A_host (in place: column k of A is read before column k of L is
 *    written back).
 * cache: device buffer of cache_bytes bytes used as a fixed-slot tile cache
 *    (at least 2 * Nt tiles of nb*nb binary64); the two working columns come
 *    from the context workspace.
 * Operand tiles are streamed through the cache in chunks of tile columns
 * when it cannot hold a column's whole working set; evictions take the tile
 * with the farthest next use under the static schedule. The work runs on
 * the compute stream and two library streams (host->device, device->host),
 * all at the default priority. Returns after everything has completed; the
 * factor is L_host (no tc_factor handle). */
tc_status tc_factorize_ooc(tc_ctx *ctx, int64_t n, int32_t nb, const double *A_host,
                           double *L_host, void *cache, size_t cache_bytes, tc_ooc_stats *stats);

/* Bytes of host memory receiving an out-of-core mixed-precision factor:
 * every tile in its class (8/4/2/2/1 bytes per entry; FP16 and FP8 tiles
 * hold x * 2^-e), packed lower order, each tile starting on a 256-byte
 * boundary (tile t at the sum of the rounded-up sizes of the tiles before
 * it), then one int32 scale exponent e per tile in packed order (value =
 * stored value * 2^e). 0 if the shape or the map is invalid. */
size_t tc_ooc_mixed_host_bytes(int64_t n, int32_t nb, const uint8_t *map);

/* Device cache bytes tc_factorize_ooc_mixed needs to hold `slots` tile
 * slots (plus its tables and the staging of new tiles) with the same opts
 * (NULL: defaults; fp64_update = TC_FP32 adds FP32 operand copies of the
 * FP64 tiles to each slot); at least 2 * Nt slots are required. 0 if the
 * shape, the map or the opts are invalid. */
size_t tc_ooc_mixed_cache_bytes(int64_t n, int32_t nb, const uint8_t *map, int64_t slots,
                                const tc_opts *opts);

/* Out-of-core mixed-precision tile Cholesky (Sections III-C, IV-B, IV-C):
 * the schedule of tc_factorize_ooc with the precision map of tc_factorize,
 * the factor crossing the link in its classes' bytes.
 * A_host: pinned host memory, packed lower tiles (n, nb), binary64, read.
 * map: host, Nt(Nt+1)/2 tc_prec codes, diagonal tiles TC_FP64.
 * L_host: pinned host memory of L_host_bytes >= tc_ooc_mixed_host_bytes
 *    bytes receiving the factor image described there.
 * cache: device buffer of cache_bytes bytes holding the device tables, a
 *    staging area for new tiles (two columns' worth), four binary64
 *    working columns (A is prefetched up to three columns ahead) and
 *    fixed-size slots (one tile in its class plus the operand copies it is
 *    multiplied in, rebuilt on the device when the tile is loaded); at
 *    least 2 * Nt slots, else TC_ENOMEM with the required size in
 *    tc_last_error().
 * opts: NULL for the defaults; fp64_update as in tc_factorize (the cache
 *    must then be sized with the same opts). TC_EINVAL for other codes.
 * Updates into a tile of class p are computed as in tc_factorize (same
 * kernels; the summation is split at the chunk boundaries, so results
 * agree with the in-core factor up to rounding). Runs on the compute stream
 * and the library's streams, default priority; returns after everything
 * has completed (no tc_factor handle). */
tc_status tc_factorize_ooc_mixed(tc_ctx *ctx, int64_t n, int32_t nb, const double *A_host,
                                 const uint8_t *map, void *L_host, size_t L_host_bytes,
                                 void *cache, size_t cache_bytes, const tc_opts *opts,
                                 tc_ooc_stats *stats);

/* Copy the factor into L64 (device, packed lower tiles, binary64; each tile
 * upcast from its class, Section IV-C: one precision per tile, stored with
 * its power-of-two scale) with the strict upper triangle of every diagonal
 * tile set to zero. For an all-FP64 factor L64 may be the factor's own
 * storage; otherwise it must be a separate buffer. */
tc_status tc_factor_export(tc_ctx *ctx, const tc_factor *L, double *L64);

/* ---- Gradient of the Gaussian log-likelihood (Eq. 1) ------------------
 * The log-likelihood l(theta) = -n/2 log(2 pi) - 1/2 log|Sigma| - 1/2 y^T
 * Sigma^{-1} y of Eq. 1 is differentiated by reverse mode through the tile
 * Cholesky: seed dl/dL, run the blocked reverse sweep of the factorization
 * (Murray, "Differentiation of the Cholesky decomposition", 2016) to get
 * dl/dA for the lower triangle, then contract it with the derivatives of
 * the Matern covariance (Eq. 2 plus the nugget). */

/* With z = L^{-1} y and alpha = L^{-T} z: *loglik = -n/2 log(2 pi) -
 * sum_i log L_ii - 1/2 z^T z (host), and Lbar (device, packed lower tiles
 * (n, nb), binary64, overwritten, strict upper triangle of the diagonal
 * tiles zero) receives dl/dL = tril(alpha z^T) - diag(1 / L_ii); Lbar NULL:
 * only *loglik (no seed written).
 * y: device, n binary64. L: any factor (the solves read mixed-precision
 * tiles upcast to binary64). */
tc_status tc_loglik_seed(tc_ctx *ctx, const tc_factor *L, const double *y, double *Lbar,
                         double *loglik);

/* Bytes of device scratch tc_factor_adjoint needs in its full form (about
 * the size of the factor plus two tile columns; mixed != 0 adds room for
 * the binary64 upcast of a mixed-precision factor); 0 for an invalid shape. */
size_t tc_adjoint_bytes(int64_t n, int32_t nb, int32_t mixed);

/* Bytes of device scratch for the memory-short form of tc_factor_adjoint
 * (three tile columns plus the split-K partial sums, which the panel
 * products cap at 512 MiB; mixed != 0 adds one decoded tile column); 0 for
 * an invalid shape. */
size_t tc_adjoint_min_bytes(int64_t n, int32_t nb, int32_t mixed);

/* Reverse sweep of the tile Cholesky. On input Lbar (device, packed lower
 * tiles, binary64) holds d(phi)/dL for a scalar phi of the factor (lower
 * triangle; the strict upper triangle of diagonal tiles is ignored). On
 * output it holds Abar = d(phi)/dA for the lower triangle of A, the only
 * part the factorization reads: phi changes by sum_{i>=j} Abar_ij dA_ij when
 * A_ij and A_ji change by dA_ij (strict upper triangle of diagonal tiles set
 * to zero). L: the factor of A; a mixed-precision factor is upcast to
 * binary64 and the sweep is the exact reverse of the binary64 Cholesky at
 * that factor (an approximation of the gradient at the accuracy of the
 * precision map).
 * scratch: device buffer, mixed = whether L is a mixed-precision factor.
 * With at least tc_adjoint_bytes(n, nb, mixed) bytes the sweep keeps a
 * transposed copy of every Abar tile for the later panel products (and the
 * binary64 upcast of a mixed factor). With less, but at least
 * tc_adjoint_min_bytes(n, nb, mixed), it runs in its memory-short form:
 * the panel products read Abar's transposed tiles from Lbar itself, and a
 * mixed factor's tiles are decoded to binary64 again, one tile column at a
 * time, when the sweep reaches that column (recomputed, not stored).
 * Both forms give the same Abar bit for bit; the short form is slower
 * (strided reads of the transposed tiles). Fewer bytes: TC_ENOMEM.
 * stats: NULL or filled (ms_total, flops_total; ms_gemm, gemm_flops and
 * gemm_launches for the panel GEMMs when the context is timed). */
tc_status tc_factor_adjoint(tc_ctx *ctx, const tc_factor *L, double *Lbar, void *scratch,
                            size_t scratch_bytes, tc_stats *stats);

/* Contraction of Abar (device, packed lower tiles (n, nb), binary64, lower
 * triangle read) with the Matern derivatives, entries regenerated from the
 * locations (device, n x 2 row-major) and th:
 *   grad[0] = sum_{i>=j} Abar_ij dSigma_ij/dsigma2   (= C_ij / sigma2),
 *   grad[1] = sum_{i>=j} Abar_ij dSigma_ij/drange,
 *   grad[2] = sum_i Abar_ii                           (dSigma/dnugget = I).
 * grad: host, 3 doubles. Deterministic (fixed reduction order). */
tc_status tc_matern_grad(tc_ctx *ctx, int64_t n, int32_t nb, const double *locs,
                         const tc_matern *th, const double *Abar, double grad[3]);

/* ---- Factorization without device allocation --------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The FP64
 * factorization of tc_factorize (NULL map, default opts) with its scratch
 * (failure flag, split-K partial sums of the panel updates and of the
 * in-tile POTRF) in one fixed device array of TC_NOALLOC_SCRATCH_BYTES per
 * GPU, which the library holds from the first context on that GPU until the
 * process ends; the context's workspace is not used. Every column runs in
 * Algorithm 1's order on the context's compute stream (no lookahead stream,
 * no events); when the partial sums of a late column's split-K would not
 * fit, fewer splits are used, so any n, nb that tc_factorize accepts is
 * accepted (TC_ENOMEM if a tile size ever needed more in-tile scratch than
 * the array holds). Calls no allocating routine on the device or host
 * (except to format an error message).
 * A: device packed lower tiles (n, nb), binary64, read (may equal L).
 * L: device packed lower tiles receiving the factor (diagonal tiles' strict
 *    upper triangles undefined, as with tc_factorize).
 * info: host, receives 0 or LAPACK's info (also returned).
 * All calls on one GPU share its array, which keeps the last call's
 * contents (the failure flag is cleared at the start of each call): calls
 * that overlap on one GPU, from any thread or stream, race and must not be
 * made. Returns after the factorization has completed. */
#define TC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
tc_status tc_factorize_noalloc(tc_ctx *ctx, int64_t n, int32_t nb, const double *A, double *L,
                               int32_t *info);

/* Free the handle (not the caller's storage). NULL is accepted. */
tc_status tc_factor_destroy(tc_factor *L);

#ifdef __cplusplus
}
#endif
#endif /* TILECHOL_H */
