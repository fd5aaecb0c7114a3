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

// Derivatives of Eq. 2 for the likelihood gradient, with x = h / a:
//   dC/dsigma2 = C / sigma2,
//   dC/da = sigma2 / (2^(nu-1) Gamma(nu)) x^(nu+1) K_(nu-1)(x) / a,
// from d/dx[x^nu K_nu(x)] = -x^nu K_(nu-1)(x) and dx/da = -x / a; both are
// taken at x = 0 as their limits 1 and 0. K_(nu-1) = K_|nu-1| comes from the
// same quadrature nodes as K_nu (second table qc2).
__device__ inline void matern_derivs(double x, int nu_kind, double sigma2, double inv_range,
                                     double nu, double norm_const, const double* qc,
                                     const double* qc2, const double* qe, double& c_s2,
                                     double& d_a) {
    if (x == 0.0) {
        c_s2 = 1.0;
        d_a = 0.0;
        return;
    }
    const double ex = exp(-x);
    switch (nu_kind) {
        case 0:
            c_s2 = ex;
            d_a = sigma2 * inv_range * x * ex;
            return;
        case 1:
            c_s2 = (1.0 + x) * ex;
            d_a = sigma2 * inv_range * x * x * ex;
            return;
        case 2:
            c_s2 = (1.0 + x + x * x * (1.0 / 3.0)) * ex;
            d_a = sigma2 * inv_range * (1.0 / 3.0) * x * x * (1.0 + x) * ex;
            return;
        default: {
            double s1 = 0.5, s2 = 0.5;
            for (int k = 0; k < kQuadMax; ++k) {
                const double a = x * qe[k];
                if (a > 745.0) break;
                const double e = exp(-a);
                s1 += e * qc[k];
                s2 += e * qc2[k];
            }
            const double Knu = ex * kQuadStep * s1;
            const double Knm1 = ex * kQuadStep * s2;
            const double xn = pow(x, nu);
            c_s2 = norm_const / sigma2 * xn * Knu;
            d_a = norm_const * inv_range * xn * x * Knm1;
            return;
        }
    }
}

// One workgroup per (tile, strip of columns): partial sums over the lower
// entries of
//   Abar_ij dC_ij/dsigma2,  Abar_ij dC_ij/da,  and Abar_ii (the nugget).
__global__ __launch_bounds__(kThreads) void matern_grad_kernel(
    int64_t Nt, int nb, const double* __restrict__ locs, double sigma2, double inv_range,
    double nu, int nu_kind, double norm_const, const double* __restrict__ Abar,
    double* __restrict__ part) {
    __shared__ double qc[kQuadMax];
    __shared__ double qc2[kQuadMax];
    __shared__ double qe[kQuadMax];
    __shared__ double red[3][kThreads / 64];
    const int strips = nb / kStripCols;
    const int64_t t = blockIdx.y;
    const int strip = blockIdx.x;
    int64_t j = 0;
    while (tile_off(Nt, Nt - 1, j) < t) ++j;
    const int64_t i = j + (t - tile_off(Nt, j, j));
    if (nu_kind == 3) {
        const double nu2 = fabs(nu - 1.0);
        for (int k = threadIdx.x; k < kQuadMax; k += kThreads) {
            const double tk = (k + 1) * kQuadStep;
            const double sh = sinh(0.5 * tk);
            qe[k] = 2.0 * sh * sh;
            qc[k] = cosh(nu * tk);
            qc2[k] = cosh(nu2 * tk);
        }
        __syncthreads();
    }
    const double* tile = Abar + t * (int64_t)nb * nb;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    const int c0 = strip * kStripCols;
    for (int cc = 0; cc < kStripCols; ++cc) {
        const int c = c0 + cc;
        const int64_t gj = j * nb + c;
        const double xj = locs[2 * gj], yj = locs[2 * gj + 1];
        const int rbeg = i == j ? c : 0;
        for (int r = rbeg + threadIdx.x; r < nb; r += kThreads) {
            const int64_t gi = i * nb + r;
            const double dx = locs[2 * gi] - xj;
            const double dy = locs[2 * gi + 1] - yj;
            const double h = sqrt(dx * dx + dy * dy);
            const double ab = tile[(int64_t)c * nb + r];
            double cs, da;
            matern_derivs(h * inv_range, nu_kind, sigma2, inv_range, nu, norm_const, qc, qc2, qe,
                          cs, da);
            g0 += ab * cs;
            g1 += ab * da;
            if (gi == gj) g2 += ab;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        g0 += __shfl_down(g0, off, 64);
        g1 += __shfl_down(g1, off, 64);
        g2 += __shfl_down(g2, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = g0;
        red[1][threadIdx.x >> 6] = g1;
        red[2][threadIdx.x >> 6] = g2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double tot = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) tot += red[threadIdx.x][w];
        part[(t * strips + strip) * 3 + threadIdx.x] = tot;
    }
}

// out[q] = sum_e part[3 e + q] over e < count, in a fixed order.
__global__ __launch_bounds__(256) void sum3_kernel(const double* __restrict__ part, int64_t count,
                                                   double* __restrict__ out) {
    __shared__ double red[3][256];
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t e = threadIdx.x; e < count; e += 256)
        for (int q = 0; q < 3; ++q) s[q] += part[3 * e + q];
    for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
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

hipError_t launch_matern_grad(hipStream_t s, int64_t n, int nb, const double* locs, double sigma2,
                              double inv_range, double nu, int nu_kind, double norm_const,
                              const double* Abar, double* part) {
    const int64_t Nt = n / nb;
    const int64_t ntiles = Nt * (Nt + 1) / 2;
    dim3 grid(nb / kStripCols, (unsigned)ntiles);
    hipLaunchKernelGGL(matern_grad_kernel, grid, dim3(kThreads), 0, s, Nt, nb, locs, sigma2,
                       inv_range, nu, nu_kind, norm_const, Abar, part);
    return hipGetLastError();
}

hipError_t launch_sum3(hipStream_t s, const double* part, int64_t count, double* out) {
    hipLaunchKernelGGL(sum3_kernel, dim3(1), dim3(256), 0, s, part, count, out);
    return hipGetLastError();
}

}  // namespace tc
