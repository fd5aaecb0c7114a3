/*
 * CPU oracle for the tile Cholesky path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it. It shares no code, header, table or helper
 * with the GPU library.
 *
 * Everything is binary64, plain loops, no BLAS. Matrices are dense n x n,
 * column-major (element (i,j) at a[i + j*lda]); only the lower triangle is
 * read or written by the factorizations.
 *
 * Paper: "Accelerating Mixed-Precision Out-of-Core Cholesky Factorization
 * with Static Task Scheduling" (arXiv 2410.09819).
 *   - tile_cholesky follows the left-looking tile algorithm of Section III-A
 *     (Algorithm 1): column of tiles k = 0..Nt-1; the diagonal tile gets the
 *     SYRK updates from every tile to its left and is factorized (POTRF);
 *     each tile below it gets the GEMM updates from the tiles to its left and
 *     is solved against the transposed diagonal factor (TRSM). The GEMM sum
 *     runs over the column index n < k, and the TRSM is L_mk = A_mk L_kk^-T.
 *   - cholesky_unblocked is a different code path (row-by-row Cholesky-
 *     Banachiewicz on the whole matrix), used only to cross-check.
 *   - forward/back substitution give Sigma^{-1} y for the likelihood of
 *     Eq. 1 (Section III-D).
 *
 * Failure convention (the paper is silent): LAPACK's. A pivot that is not
 * strictly positive (or NaN) stops the factorization and the return value
 * is the 1-based global index of that column.
 *
 * ORACLE_MUTANT (compile-time, 0 = none) plants one deliberate mistake per
 * value. It exists only so that the tests can show that the pins catch each
 * of those mistakes; the oracle used everywhere else is built with 0.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

#define AT(p, ld, i, j) ((p)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

/* POTRF of one nb x nb diagonal tile stored at t with leading dimension ld:
 * Cholesky-Crout, column by column. Returns 0, or the 1-based local column
 * of the first pivot that is not > 0. */
static int64_t potrf_tile(double *t, int64_t ld, int64_t nb)
{
    for (int64_t j = 0; j < nb; ++j) {
        double d = AT(t, ld, j, j);
        for (int64_t l = 0; l < j; ++l)
            d -= AT(t, ld, j, l) * AT(t, ld, j, l);
        if (!(d > 0.0))
            return j + 1;
        d = sqrt(d);
        AT(t, ld, j, j) = d;
        for (int64_t i = j + 1; i < nb; ++i) {
            double s = AT(t, ld, i, j);
#if ORACLE_MUTANT == 4
            for (int64_t l = 0; l + 1 < j; ++l) /* drops the last term */
#else
            for (int64_t l = 0; l < j; ++l)
#endif
                s -= AT(t, ld, i, l) * AT(t, ld, j, l);
            AT(t, ld, i, j) = s / d;
        }
    }
    return 0;
}

/* SYRK on a diagonal tile: C -= A A^T, lower triangle of C only.
 * C and A are nb x nb tiles with leading dimension ld. */
static void syrk_tile(double *c, const double *a, int64_t ld, int64_t nb)
{
    for (int64_t j = 0; j < nb; ++j)
        for (int64_t l = 0; l < nb; ++l) {
            const double b = AT(a, ld, j, l);
            for (int64_t i = j; i < nb; ++i)
                AT(c, ld, i, j) -= AT(a, ld, i, l) * b;
        }
}

/* GEMM on an off-diagonal tile: C -= A B^T (all nb x nb, leading dim ld). */
static void gemm_tile(double *c, const double *a, const double *b, int64_t ld, int64_t nb)
{
    for (int64_t j = 0; j < nb; ++j)
        for (int64_t l = 0; l < nb; ++l) {
#if ORACLE_MUTANT == 2
            const double bj = AT(b, ld, l, j); /* transposed operand */
#else
            const double bj = AT(b, ld, j, l);
#endif
            for (int64_t i = 0; i < nb; ++i)
                AT(c, ld, i, j) -= AT(a, ld, i, l) * bj;
        }
}

/* TRSM on an off-diagonal tile: overwrite C with X solving X L^T = C, L the
 * lower-triangular factor of the diagonal tile. Column j of X:
 *   x_j = (c_j - sum_{l<j} x_l L[j,l]) / L[j,j]. */
static void trsm_tile(double *c, const double *L, int64_t ld, int64_t nb)
{
    for (int64_t j = 0; j < nb; ++j) {
        for (int64_t l = 0; l < j; ++l) {
#if ORACLE_MUTANT == 3
            const double f = AT(L, ld, l, j); /* wrong index: upper entry */
#else
            const double f = AT(L, ld, j, l);
#endif
            for (int64_t i = 0; i < nb; ++i)
                AT(c, ld, i, j) -= AT(c, ld, i, l) * f;
        }
        const double d = AT(L, ld, j, j);
        for (int64_t i = 0; i < nb; ++i)
            AT(c, ld, i, j) /= d;
    }
}

/* Left-looking tile Cholesky (Algorithm 1) of the n x n matrix a (lda >= n),
 * tile size nb (n % nb == 0). Overwrites the lower triangle with L; the
 * strict upper triangle of each diagonal tile is left as it was.
 * Returns 0 on success, the 1-based global failing column otherwise, or -1
 * on bad arguments. `threads` > 1 runs the independent tiles of one column
 * concurrently with OpenMP (each tile's arithmetic is sequential, so the
 * result does not depend on the thread count). */
int64_t oracle_tile_cholesky(int64_t n, int64_t nb, double *a, int64_t lda, int threads)
{
    if (n < 0 || nb <= 0 || n % nb != 0 || lda < n)
        return -1;
    const int64_t Nt = n / nb;
#define TILE(m, k) (&AT(a, lda, (m) * nb, (k) * nb))
    for (int64_t k = 0; k < Nt; ++k) {
        /* diagonal task: SYRK updates from every tile to the left, POTRF */
#if ORACLE_MUTANT == 1
        for (int64_t n2 = 1; n2 < k; ++n2) /* drops the first update */
#else
        for (int64_t n2 = 0; n2 < k; ++n2)
#endif
            syrk_tile(TILE(k, k), TILE(k, n2), lda, nb);
        int64_t info = potrf_tile(TILE(k, k), lda, nb);
        if (info)
            return k * nb + info;
        /* off-diagonal tasks of column k: GEMM updates, then TRSM */
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads > 0 ? threads : 1)
        for (int64_t m = k + 1; m < Nt; ++m) {
            for (int64_t n2 = 0; n2 < k; ++n2)
#if ORACLE_MUTANT == 5
                gemm_tile(TILE(m, k), TILE(k, n2), TILE(m, n2), lda, nb); /* operands swapped */
#else
                gemm_tile(TILE(m, k), TILE(m, n2), TILE(k, n2), lda, nb);
#endif
            trsm_tile(TILE(m, k), TILE(k, k), lda, nb);
        }
    }
#undef TILE
    return 0;
}

/* Unblocked Cholesky-Banachiewicz (row by row) on the whole matrix: a
 * different code path from the tile algorithm, used to cross-check it.
 * Same return convention. */
int64_t oracle_cholesky_unblocked(int64_t n, double *a, int64_t lda)
{
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j <= i; ++j) {
            double s = 0.0;
            for (int64_t l = 0; l < j; ++l)
                s += AT(a, lda, i, l) * AT(a, lda, j, l);
            if (i == j) {
                const double d = AT(a, lda, i, i) - s;
                if (!(d > 0.0))
                    return i + 1;
                AT(a, lda, i, i) = sqrt(d);
            } else {
                AT(a, lda, i, j) = (AT(a, lda, i, j) - s) / AT(a, lda, j, j);
            }
        }
    }
    return 0;
}

/* In place: B <- L^{-1} B (forward substitution), B is n x nrhs, ldb >= n. */
void oracle_forward_solve(int64_t n, const double *L, int64_t ldl, double *B, int64_t ldb, int64_t nrhs)
{
    for (int64_t r = 0; r < nrhs; ++r) {
        double *b = B + (size_t)r * (size_t)ldb;
        for (int64_t j = 0; j < n; ++j) {
            b[j] /= AT(L, ldl, j, j);
            const double bj = b[j];
            for (int64_t i = j + 1; i < n; ++i)
                b[i] -= AT(L, ldl, i, j) * bj;
        }
    }
}

/* In place: B <- L^{-T} B (back substitution with the transpose). */
void oracle_back_solve(int64_t n, const double *L, int64_t ldl, double *B, int64_t ldb, int64_t nrhs)
{
    for (int64_t r = 0; r < nrhs; ++r) {
        double *b = B + (size_t)r * (size_t)ldb;
        for (int64_t j = n - 1; j >= 0; --j) {
            double s = b[j];
            for (int64_t i = j + 1; i < n; ++i)
                s -= AT(L, ldl, i, j) * b[i];
            b[j] = s / AT(L, ldl, j, j);
        }
    }
}

int oracle_mutant_id(void) { return ORACLE_MUTANT; }
