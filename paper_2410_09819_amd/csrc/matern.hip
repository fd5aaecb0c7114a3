// Matern covariance tiles (Section III-D, Eq. 2) with a nugget on the
// diagonal, written straight into packed lower tile storage, plus the
// per-tile Frobenius norms that the precision criterion of Section IV-C
// needs.
//
// One workgroup fills a strip of STRIP_COLS columns of one tile; threads
// walk down the rows so the column-major tile is written contiguously. The
// strip's sum of squares goes to its own slot, and a second kernel adds the
// strips of each tile in a fixed order (deterministic norms).
#include "common.hpp"

namespace tc {
namespace {

constexpr int kThreads = 256;
constexpr int kStripCols = 16;
// Trapezoid rule for K_nu: step and a bound on the number of nodes. The
// integrand exp(-x (cosh t - 1)) cosh(nu t) is analytic in |Im t| < pi/2,
// so the rule's error falls like exp(-pi^2 / (2 h)); h = 0.1 makes it far
// below binary64 rounding. Nodes stop once x (cosh t - 1) > 745, where the
// exponential underflows.
constexpr double kQuadStep = 0.1;
constexpr int kQuadMax = 320;

__device__ inline double matern_value(double x, int nu_kind, double sigma2, double nu,
                                      double norm_const, const double* qc, const double* qe,
                                      int nq) {
    switch (nu_kind) {
        case 0: return sigma2 * exp(-x);
        case 1: return sigma2 * (1.0 + x) * exp(-x);
        case 2: return sigma2 * (1.0 + x + x * x * (1.0 / 3.0)) * exp(-x);
        default: {
            if (x == 0.0) return sigma2;
            // K_nu(x) = e^{-x} * h * [1/2 + sum_k exp(-x (cosh t_k - 1)) cosh(nu t_k)]
            double s = 0.5;
            for (int k = 0; k < nq; ++k) {
                const double a = x * qe[k];
                if (a > 745.0) break;
                s += exp(-a) * qc[k];
            }
            const double K = exp(-x) * kQuadStep * s;
            return norm_const * pow(x, nu) * K;
        }
    }
}

__global__ __launch_bounds__(kThreads) void matern_tiles_kernel(
    int64_t Nt, int nb, const double* __restrict__ locs, double sigma2, double inv_range, double nu,
    int nu_kind, double norm_const, double nugget, double* __restrict__ A,
    double* __restrict__ strip_ss) {
    __shared__ double qc[kQuadMax];
    __shared__ double qe[kQuadMax];
    __shared__ double red[kThreads / 64];
    const int strips = nb / kStripCols;
    const int64_t t = blockIdx.y;
    const int strip = blockIdx.x;
    // tile column j: the last tile of column j has index tile_off(Nt, Nt-1, j)
    int64_t j = 0;
    while (tile_off(Nt, Nt - 1, j) < t) ++j;
    const int64_t i = j + (t - tile_off(Nt, j, j));

    int nq = 0;
    if (nu_kind == 3) {
        nq = kQuadMax;
        for (int k = threadIdx.x; k < kQuadMax; k += kThreads) {
            const double tk = (k + 1) * kQuadStep;
            const double sh = sinh(0.5 * tk);
            qe[k] = 2.0 * sh * sh;  // cosh(t) - 1 without cancellation
            qc[k] = cosh(nu * tk);
        }
        __syncthreads();
    }

    double* tile = A + t * (int64_t)nb * nb;
    double ss = 0.0;
    const int c0 = strip * kStripCols;
    for (int cc = 0; cc < kStripCols; ++cc) {
        const int c = c0 + cc;
        const int64_t gj = j * nb + c;
        const double xj = locs[2 * gj], yj = locs[2 * gj + 1];
        for (int r = threadIdx.x; r < nb; r += kThreads) {
            const int64_t gi = i * nb + r;
            const double dx = locs[2 * gi] - xj;
            const double dy = locs[2 * gi + 1] - yj;
            const double h = sqrt(dx * dx + dy * dy);
            double v = matern_value(h * inv_range, nu_kind, sigma2, nu, norm_const, qc, qe, nq);
            if (gi == gj) v += nugget;
            tile[(int64_t)c * nb + r] = v;
            ss += v * v;
        }
    }
    // workgroup sum of squares (fixed order: wave shuffles, then waves)
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_down(ss, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) tot += red[w];
        strip_ss[t * strips + strip] = tot;
    }
}

__global__ void tile_norms_kernel(int64_t ntiles, int strips, const double* __restrict__ ss,
                                  double* __restrict__ fro) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    double s = 0.0;
    for (int k = 0; k < strips; ++k) s += ss[t * strips + k];
    fro[t] = sqrt(s);
}

}  // namespace

int matern_strips(int nb) { return nb / kStripCols; }

hipError_t launch_matern(hipStream_t s, int64_t n, int nb, const double* locs, double sigma2,
                         double inv_range, double nu, int nu_kind, double norm_const, double nugget,
                         double* A, double* strip_ss) {
    const int64_t Nt = n / nb;
    const int64_t ntiles = Nt * (Nt + 1) / 2;
    dim3 grid(nb / kStripCols, (unsigned)ntiles);
    hipLaunchKernelGGL(matern_tiles_kernel, grid, dim3(kThreads), 0, s, Nt, nb, locs, sigma2,
                       inv_range, nu, nu_kind, norm_const, nugget, A, strip_ss);
    return hipGetLastError();
}

hipError_t launch_tile_norms(hipStream_t s, int64_t ntiles, int strips, const double* strip_ss,
                             double* tile_fro) {
    const int th = 256;
    hipLaunchKernelGGL(tile_norms_kernel, dim3((unsigned)((ntiles + th - 1) / th)), dim3(th), 0, s,
                       ntiles, strips, strip_ss, tile_fro);
    return hipGetLastError();
}

}  // namespace tc
