// HIP device code for gfx950 (MI355X): sigma_min(zI - A) for matrices whose bandwidth exceeds
// what the banded kernels hold in registers (kl or ku > 4), at small n (n <= 64): the matrix is
// dense for the purpose, as in the paper's Jordan example of Sec. 2 (a Jordan block with one
// corner entry).  sigma_min is s_n of the SVD of zI - A (Sec. 2.1).
//
// One wavefront per shift.  M = zI - A sits in LDS (64 x 64 complex doubles, column-major
// with an XOR swizzle so that both a lane per row and a lane per column read distinct banks).
// Householder reflections from the left and the right reduce M to an upper bidiagonal B
// (U^H M V = B, unitary U, V): each reflection is one wavefront-wide reduction and one
// rank-one update in which every lane updates its own column (left) or row (right).  The
// entries of B are made real and non-negative by unitary diagonal scalings, which leave the
// singular values unchanged: the diagonal is |beta_k|, the superdiagonal |gamma_k|.  The
// reduction is backward stable: the singular values of B are those of M + E with
// |E| ~ n eps |M|, which is far below the absolute part of the stopping target.
//
// The singular values of B are the non-negative eigenvalues of the Golub-Kahan matrix, the
// symmetric tridiagonal T of order 2n with zero diagonal and off-diagonal
// d_0, e_0, d_1, e_1, ..., d_{n-1}; T - tI has n + #{s_i < t} negative pivots in its
// L D L^T (Sylvester), computed by the Sturm recurrence q_1 = -t, q_k = -t - b_{k-1}^2 / q_{k-1}.
// The 64 lanes each count at one point of the bracket: a round splits it into 65 parts, until
// hi - lo <= tol_norm ||A||_F + tol_rel lo; sigma = the midpoint.
#include "ps_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ps {

namespace {

constexpr int kDN = kDenseMaxN;   // 64

__device__ __forceinline__ int sw(int i, int j) { return j * kDN + (i ^ j); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double grid_x(double lo, double hi, int64_t k, int64_t n) {
    return n > 1 ? __dadd_rn(lo, __ddiv_rn(__dmul_rn(hi - lo, (double)k), (double)(n - 1))) : lo;
}

// #{singular values of B below t} for t > 0: the negative pivots of T - tI, minus n.  A zero
// pivot is replaced by a tiny negative number (the count for t nudged upward by that amount).
__device__ int count_below(const double *b2, int m, double t, double pivmin) {
    double q = -t;
    int neg = 0;
    for (int k = 0; k < m; ++k) {
        if (k > 0) q = -t - b2[k - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        neg += q < 0.0 ? 1 : 0;
    }
    return neg;
}

__global__ void __launch_bounds__(64) k_dense_sigma(EvalArgs a) {
    __shared__ double2 M[kDN * kDN];
    __shared__ double2 vec[kDN];
    __shared__ double b2[2 * kDN];      // squared off-diagonal of T: d_0^2, e_0^2, d_1^2, ...
    const int64_t p = blockIdx.x;
    if (p >= *a.count_dev) return;
    const int lane = (int)threadIdx.x;
    const int n = (int)a.n;
    double zx, zy;
    if (a.mode == kShiftList) {
        zx = a.z[p].x;
        zy = a.z[p].y;
    } else {
        const int64_t flat = a.idx ? a.idx[p] : p;
        const int64_t gi = flat / a.nx, gj = flat - gi * a.nx;
        zx = grid_x(a.ga, a.gb, gj, a.nx);
        zy = grid_x(a.gc, a.gd, gi, a.ny);
    }
    // M = zI - A: lane j builds column j from the row band (A[i][j] at row i, i - kl + d = j)
    const int w = a.kl + a.ku + 1;
    if (lane < n) {
        const int j = lane;
        for (int i = 0; i < n; ++i) {
            const int d = j - i + a.kl;
            double2 e = make_double2(0.0, 0.0);
            if (d >= 0 && d < w) {
                const double2 t = a.arow[(int64_t)i * w + d];
                e = make_double2(-t.x, -t.y);
            }
            if (i == j) {
                e.x += zx;
                e.y += zy;
            }
            M[sw(i, j)] = e;
        }
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        // left reflection of column k, rows k .. n-1: H x = beta e_k, |beta| = |x|
        double2 x = lane >= k && lane < n ? M[sw(lane, k)] : make_double2(0.0, 0.0);
        const double alpha = sqrt(wave_sum(x.x * x.x + x.y * x.y));
        const double2 x0 = M[sw(k, k)];
        const double a0 = hypot(x0.x, x0.y);
        b2[2 * k] = alpha * alpha;
        if (alpha > 0.0) {
            // beta = -phase(x0) alpha; v = x - beta e_k, v^H v = 2 alpha (alpha + |x0|)
            const double px = a0 > 0.0 ? x0.x / a0 : 1.0, py = a0 > 0.0 ? x0.y / a0 : 0.0;
            if (lane == k) x = make_double2(x0.x + px * alpha, x0.y + py * alpha);
            if (lane < n) vec[lane] = x;
            const double s = 1.0 / (alpha * (alpha + a0));   // 2 / v^H v
            __syncthreads();
            if (lane > k && lane < n) {   // column j = lane: M[:, j] -= v (s v^H M[:, j])
                const int j = lane;
                double cr = 0.0, ci = 0.0;
                for (int i = k; i < n; ++i) {
                    const double2 vi = vec[i], mij = M[sw(i, j)];
                    cr += vi.x * mij.x + vi.y * mij.y;
                    ci += vi.x * mij.y - vi.y * mij.x;
                }
                cr *= s;
                ci *= s;
                for (int i = k; i < n; ++i) {
                    const double2 vi = vec[i];
                    double2 mij = M[sw(i, j)];
                    mij.x -= vi.x * cr - vi.y * ci;
                    mij.y -= vi.x * ci + vi.y * cr;
                    M[sw(i, j)] = mij;
                }
            }
            __syncthreads();
        }
        if (k + 1 >= n) break;
        // right reflection of row k, columns k+1 .. n-1: y H_R = gamma e_{k+1}, |gamma| = |y|,
        // from the Householder vector of conj(y)
        double2 y = lane > k && lane < n ? M[sw(k, lane)] : make_double2(0.0, 0.0);
        const double g = sqrt(wave_sum(y.x * y.x + y.y * y.y));
        const double2 y0 = M[sw(k, k + 1)];
        const double g0 = hypot(y0.x, y0.y);
        b2[2 * k + 1] = g * g;
        if (g > 0.0) {
            // u = conj(y) - beta' e_{k+1}, beta' = -phase(conj y0) g; u^H u = 2 g (g + |y0|)
            double2 u = make_double2(y.x, -y.y);
            const double px = g0 > 0.0 ? y0.x / g0 : 1.0, py = g0 > 0.0 ? -y0.y / g0 : 0.0;
            if (lane == k + 1) u = make_double2(y0.x + px * g, -y0.y + py * g);
            if (lane < n) vec[lane] = u;
            const double s = 1.0 / (g * (g + g0));
            __syncthreads();
            if (lane > k && lane < n) {   // row i = lane: M[i, :] -= (s M[i, :] u) u^H
                const int i = lane;
                double cr = 0.0, ci = 0.0;
                for (int j = k + 1; j < n; ++j) {
                    const double2 uj = vec[j], mij = M[sw(i, j)];
                    cr += mij.x * uj.x - mij.y * uj.y;
                    ci += mij.x * uj.y + mij.y * uj.x;
                }
                cr *= s;
                ci *= s;
                for (int j = k + 1; j < n; ++j) {
                    const double2 uj = vec[j];
                    double2 mij = M[sw(i, j)];
                    mij.x -= cr * uj.x + ci * uj.y;
                    mij.y -= ci * uj.x - cr * uj.y;
                    M[sw(i, j)] = mij;
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
    // multisection on the Golub-Kahan matrix: lane l counts at lo + (hi - lo) (l + 1) / 65
    const int m = 2 * n - 1;            // order 2n; its m = 2n - 1 squared off-diagonal entries
    double bmax = 0.0;
    for (int k = 0; k < m; ++k) bmax = fmax(bmax, b2[k]);
    double lo = 0.0, hi = 2.0 * sqrt(bmax) + 1e-300;   // |T| <= 2 max |b|
    const double pivmin = fmax(bmax, 1.0) * 0x1p-1000;
    const double target_abs = a.tol_norm * a.normA;
    int rounds = 0;
    while (hi - lo > target_abs + a.tol_rel * lo && rounds < 64) {
        const double t = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        const int c = count_below(b2, 2 * n, t, pivmin) - n;
        // lowest point with at least one singular value below it
        const unsigned long long below = __ballot(c >= 1);
        const int first = below ? __ffsll(below) - 1 : 64;
        const double nhi = first < 64 ? lo + (hi - lo) * (double)(first + 1) / 65.0 : hi;
        const double nlo = first > 0 ? lo + (hi - lo) * (double)first / 65.0 : lo;
        if (!(nhi - nlo < hi - lo)) break;   // no progress at the resolution of doubles
        lo = nlo;
        hi = nhi;
        ++rounds;
    }
    if (lane == 0) {
        const double sigma = 0.5 * (lo + hi);
        a.sigma[p] = sigma;
        if (a.info) a.info[p] = PS_PT_CONVERGED;
        if (a.iters) a.iters[p] = rounds;
        if (a.sens) a.sens[p] = (uint8_t)(sigma <= a.eps);
    }
}

}  // namespace

hipError_t launch_dense(const EvalArgs &a, int64_t npts_max, hipStream_t st) {
    if (a.n > kDenseMaxN) return hipErrorInvalidValue;
    if (npts_max < 1) return hipSuccess;
    hipLaunchKernelGGL(k_dense_sigma, dim3((unsigned)npts_max), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace ps
