/*
 * CPU oracle for sigma_min(zI - A): dense one-sided (Hestenes) Jacobi SVD in
 * complex double precision, one shift at a time.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or calls
 * this file; only the test suite, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no source with the GPU library.
 *
 * What it computes (the plain definition the GPU path must reproduce):
 *   - Sec. 2 (Pseudospectrum definition, third form): z is in the
 *     eps-pseudospectrum iff sigma_min(zI - A) <= eps.
 *   - Sec. 2.1 (Singular Value Decomposition): with zI - A = U S V^*,
 *     S = diag(s_1 >= ... >= s_n >= 0), sigma_min(z) = s_n.
 * The paper obtains s_n from a full SVD at each grid point; this oracle does the
 * same with the one-sided Jacobi method, which needs no library and whose every
 * step can be checked by eye:
 *   1. M = zI - A, dense, column-major; V = I when vectors are wanted.
 *   2. Sweep over column pairs (p, q), p < q (cyclic by rows, or a round-robin
 *      order whose rounds hold disjoint pairs and may run in parallel).  For each
 *      pair: alpha = |m_p|^2, beta = |m_q|^2, gamma = m_p^H m_q.  If
 *      |gamma| <= tau * sqrt(alpha * beta) (tau = n * 2^-53) the pair is left
 *      alone.  Otherwise, with e = gamma/|gamma|, zeta = (beta - alpha)/(2|gamma|),
 *      t = sign(zeta)/(|zeta| + sqrt(1 + zeta^2)) (sign(0) = +1),
 *      c = 1/sqrt(1 + t^2), s = c t, the columns become
 *          m_p <- c m_p - s conj(e) m_q,   m_q <- s e m_p + c m_q
 *      (same rotation on the columns of V).  This makes m_p and m_q orthogonal.
 *   3. Stop after a sweep that rotates nothing (error after 60 sweeps).
 *   4. The columns are now M V = U S: s_i = |m_i|.  sigma_min = min_i s_i (first
 *      index on ties); u = m_imin / sigma_min, v = V[:, imin]; u and v are then
 *      rotated by one common unit scalar so that the first entry of v of largest
 *      modulus is real and positive.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORACLE_MAX_SWEEPS 60

/* One Jacobi rotation on columns p and q of M (and V).  Returns 1 if applied. */
static int rotate_pair(int64_t n, cplx *mp, cplx *mq, cplx *vp, cplx *vq, double tau)
{
    double alpha = 0.0, beta = 0.0;
    cplx gamma = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        alpha += creal(mp[i]) * creal(mp[i]) + cimag(mp[i]) * cimag(mp[i]);
        beta += creal(mq[i]) * creal(mq[i]) + cimag(mq[i]) * cimag(mq[i]);
        gamma += conj(mp[i]) * mq[i];
    }
    double g = cabs(gamma);
    if (g == 0.0 || g <= tau * sqrt(alpha) * sqrt(beta))
        return 0;
    cplx e = gamma / g;
    double zeta = (beta - alpha) / (2.0 * g);
    double sgn = (zeta >= 0.0) ? 1.0 : -1.0;
    double t = sgn / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    double c = 1.0 / sqrt(1.0 + t * t);
    double s = c * t;
    cplx se = s * e, sec = s * conj(e);
    for (int64_t i = 0; i < n; ++i) {
        cplx a = mp[i], b = mq[i];
        mp[i] = c * a - sec * b;
        mq[i] = se * a + c * b;
    }
    if (vp) {
        for (int64_t i = 0; i < n; ++i) {
            cplx a = vp[i], b = vq[i];
            vp[i] = c * a - sec * b;
            vq[i] = se * a + c * b;
        }
    }
    return 1;
}

/* Round-robin (tournament) pairing: m players (m even), round r in [0, m-1),
 * slot k in [0, m/2): players (a, b).  Player 0 stays fixed, the rest rotate. */
static void rr_pair(int64_t m, int64_t r, int64_t k, int64_t *a, int64_t *b)
{
    int64_t x, y;
    if (k == 0) {
        x = 0;
        y = 1 + (r % (m - 1));
    } else {
        x = 1 + ((r + k) % (m - 1));
        y = 1 + ((r + m - 1 - k) % (m - 1));
    }
    *a = x < y ? x : y;
    *b = x < y ? y : x;
}

/* Dense one-sided Jacobi on M (n x n, column-major).  V may be NULL.
 * Returns the number of sweeps, or -1 if it did not converge. */
static int jacobi(int64_t n, cplx *M, cplx *V, int parallel_pairs, int nthreads)
{
    double tau = (double)n * ldexp(1.0, -53);
    (void)nthreads;
    for (int sweep = 1; sweep <= ORACLE_MAX_SWEEPS; ++sweep) {
        int64_t rotations = 0;
        if (!parallel_pairs) {
            for (int64_t p = 0; p < n - 1; ++p)
                for (int64_t q = p + 1; q < n; ++q)
                    rotations += rotate_pair(n, M + p * n, M + q * n,
                                             V ? V + p * n : NULL, V ? V + q * n : NULL, tau);
        } else {
            int64_t m = n + (n & 1); /* odd n: one dummy player never paired with a real one */
            for (int64_t r = 0; r < m - 1; ++r) {
                int64_t rot_r = 0;
#pragma omp parallel for schedule(static) reduction(+ : rot_r) num_threads(nthreads)
                for (int64_t k = 0; k < m / 2; ++k) {
                    int64_t a, b;
                    rr_pair(m, r, k, &a, &b);
                    if (b >= n)
                        continue;
                    rot_r += rotate_pair(n, M + a * n, M + b * n,
                                         V ? V + a * n : NULL, V ? V + b * n : NULL, tau);
                }
                rotations += rot_r;
            }
        }
        if (rotations == 0)
            return sweep;
    }
    return -1;
}

/* Build M = zI - A (column-major) from the LAPACK GB band: AB[ku + i - j + j*ldab] = A[i, j]. */
static void build_shifted(int64_t n, int64_t kl, int64_t ku, const cplx *ab, int64_t ldab, cplx z, cplx *M)
{
    memset(M, 0, sizeof(cplx) * (size_t)(n * n));
    for (int64_t j = 0; j < n; ++j) {
        int64_t i0 = j - ku > 0 ? j - ku : 0;
        int64_t i1 = j + kl < n - 1 ? j + kl : n - 1;
        for (int64_t i = i0; i <= i1; ++i)
            M[i + j * n] = -ab[ku + i - j + j * ldab];
        M[j + j * n] += z;
    }
}

/* sigma_min and (optionally) all singular values and the singular pair for one shift. */
static int one_point(int64_t n, int64_t kl, int64_t ku, const cplx *ab, int64_t ldab, cplx z,
                     double *sigma, double *sall, cplx *u, cplx *v, int32_t *sweeps,
                     int parallel_pairs, int nthreads)
{
    int want_vec = (u != NULL) || (v != NULL);
    cplx *M = (cplx *)malloc(sizeof(cplx) * (size_t)(n * n));
    cplx *V = want_vec ? (cplx *)malloc(sizeof(cplx) * (size_t)(n * n)) : NULL;
    if (!M || (want_vec && !V)) {
        free(M);
        free(V);
        return 2;
    }
    build_shifted(n, kl, ku, ab, ldab, z, M);
    if (V) {
        memset(V, 0, sizeof(cplx) * (size_t)(n * n));
        for (int64_t i = 0; i < n; ++i)
            V[i + i * n] = 1.0;
    }
    int sw = jacobi(n, M, V, parallel_pairs, nthreads);
    if (sweeps)
        *sweeps = sw;
    int64_t imin = 0;
    double smin = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double s2 = 0.0;
        for (int64_t r = 0; r < n; ++r)
            s2 += creal(M[r + i * n]) * creal(M[r + i * n]) + cimag(M[r + i * n]) * cimag(M[r + i * n]);
        double s = sqrt(s2);
        if (sall)
            sall[i] = s;
        if (s < smin) {
            smin = s;
            imin = i;
        }
    }
    *sigma = smin;
    if (want_vec) {
        /* phase: first entry of v of largest modulus made real positive */
        const cplx *vc = V + imin * n;
        int64_t kmax = 0;
        double amax = -1.0;
        for (int64_t r = 0; r < n; ++r) {
            double a = cabs(vc[r]);
            if (a > amax) {
                amax = a;
                kmax = r;
            }
        }
        cplx ph = (amax > 0.0) ? conj(vc[kmax]) / amax : 1.0;
        for (int64_t r = 0; r < n; ++r) {
            if (v)
                v[r] = vc[r] * ph;
            if (u)
                u[r] = (smin > 0.0) ? M[r + imin * n] * ph / smin : 0.0;
        }
    }
    free(M);
    free(V);
    return sw < 0 ? 1 : 0;
}

/*
 * Public entry (ctypes).  ab: GB band, column-major with leading dimension ldab.
 * z[npts]: shifts.  Outputs: sigma[npts]; optional sigma_all[npts*n] (unsorted,
 * column order), u[npts*n], v[npts*n], sweeps[npts].  nthreads > 0 sets the
 * OpenMP thread count.  parallel_pairs = 1: points one after another, each
 * using the round-robin order with the pairs of a round spread over threads;
 * 0: cyclic order, points spread over threads.
 * Returns 0, or 1 if some point did not converge in 60 sweeps, 2 on allocation failure.
 */
int oracle_sigma_min(int64_t n, int64_t kl, int64_t ku, const cplx *ab, int64_t ldab, int64_t npts,
                     const cplx *z, double *sigma, double *sigma_all, cplx *u, cplx *v, int32_t *sweeps,
                     int nthreads, int parallel_pairs)
{
    int status = 0;
    if (nthreads <= 0)
        nthreads = 1;
    if (parallel_pairs) {
        for (int64_t p = 0; p < npts; ++p) {
            int st = one_point(n, kl, ku, ab, ldab, z[p], sigma + p, sigma_all ? sigma_all + p * n : NULL,
                               u ? u + p * n : NULL, v ? v + p * n : NULL, sweeps ? sweeps + p : NULL, 1,
                               nthreads);
            if (st > status)
                status = st;
        }
    } else {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
        for (int64_t p = 0; p < npts; ++p) {
            int st = one_point(n, kl, ku, ab, ldab, z[p], sigma + p, sigma_all ? sigma_all + p * n : NULL,
                               u ? u + p * n : NULL, v ? v + p * n : NULL, sweeps ? sweeps + p : NULL, 0, 1);
            if (st) {
#pragma omp critical
                if (st > status)
                    status = st;
            }
        }
    }
    return status;
}

/* Dense entry for tests: M given directly (column-major n x n), no shift. */
int oracle_svd_dense(int64_t n, const cplx *Min, double *sall, cplx *Uout, cplx *Vout, int32_t *sweeps)
{
    cplx *M = (cplx *)malloc(sizeof(cplx) * (size_t)(n * n));
    cplx *V = (cplx *)malloc(sizeof(cplx) * (size_t)(n * n));
    if (!M || !V) {
        free(M);
        free(V);
        return 2;
    }
    memcpy(M, Min, sizeof(cplx) * (size_t)(n * n));
    memset(V, 0, sizeof(cplx) * (size_t)(n * n));
    for (int64_t i = 0; i < n; ++i)
        V[i + i * n] = 1.0;
    int sw = jacobi(n, M, V, 0, 1);
    if (sweeps)
        *sweeps = sw;
    for (int64_t i = 0; i < n; ++i) {
        double s2 = 0.0;
        for (int64_t r = 0; r < n; ++r)
            s2 += creal(M[r + i * n]) * creal(M[r + i * n]) + cimag(M[r + i * n]) * cimag(M[r + i * n]);
        sall[i] = sqrt(s2);
        for (int64_t r = 0; r < n; ++r) {
            if (Uout)
                Uout[r + i * n] = sall[i] > 0.0 ? M[r + i * n] / sall[i] : 0.0;
            if (Vout)
                Vout[r + i * n] = V[r + i * n];
        }
    }
    free(M);
    free(V);
    return sw < 0 ? 1 : 0;
}
