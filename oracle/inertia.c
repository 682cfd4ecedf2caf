/*
 * CPU oracle: how many singular values of M = zI - A lie below a threshold t > 0.
 *
 * TEST INFRASTRUCTURE ONLY (like jacobi.c): used by the test suite to certify GPU
 * values of sigma_min at sizes where a dense SVD per shift is out of reach.  It shares
 * no source with the GPU library.
 *
 * Mathematics (not from the paper, which computes sigma_min by a full SVD, Sec. 2.1):
 *   The Hermitian matrix H(t) = [[-t I, M], [M^H, -t I]] has the eigenvalues
 *   s_i - t and -s_i - t (s_i the singular values of M).  For t > 0 the second group is
 *   negative, so the number of negative eigenvalues of H(t) is n + #{i : s_i < t}.
 *   By Sylvester's law of inertia that number equals the number of negative pivots of a
 *   factorisation H(t) = L D L^H (L unit lower triangular, D real diagonal).
 *   Interleaving the unknowns (x_0, y_0, x_1, y_1, ...) makes H(t) banded with
 *   half-bandwidth b = 2 max(kl, ku) + 1, so the factorisation costs O(n b^2).
 *   sigma_min(M) lies in [t0, t1) exactly when count(t0) = 0 and count(t1) >= 1.
 * The factorisation takes no pivots; a pivot that is exactly zero makes the count
 * undefined and is reported (-1).  Large pivot growth (t far below the other singular
 * values of M) can spoil the count; callers use thresholds away from that regime.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Entry of M = zI - A from the LAPACK GB band (AB[ku + i - j + j*ldab] = A[i, j]). */
static cplx m_entry(int64_t kl, int64_t ku, const cplx *ab, int64_t ldab, cplx z, int64_t i, int64_t j)
{
    cplx v = 0.0;
    if (i - j <= kl && j - i <= ku)
        v = -ab[ku + i - j + j * ldab];
    if (i == j)
        v += z;
    return v;
}

static int64_t count_one(int64_t n, int64_t kl, int64_t ku, const cplx *ab, int64_t ldab, cplx z, double t)
{
    const int64_t N = 2 * n;
    const int64_t b = 2 * (kl > ku ? kl : ku) + 1;
    const int64_t w = b + 1;
    /* lower band of H(t): W[r * w + d] = H[r][r - d], d = 0..b */
    cplx *W = calloc((size_t)(N * w), sizeof(cplx));
    if (!W)
        return -2;
    for (int64_t r = 0; r < N; ++r)
        W[r * w] = -t;
    /* H[2i][2j+1] = M[i][j], H[2j+1][2i] = conj(M[i][j]) */
    for (int64_t i = 0; i < n; ++i) {
        int64_t j0 = i - kl > 0 ? i - kl : 0;
        int64_t j1 = i + ku < n - 1 ? i + ku : n - 1;
        for (int64_t j = j0; j <= j1; ++j) {
            cplx m = m_entry(kl, ku, ab, ldab, z, i, j);
            int64_t rx = 2 * i, cy = 2 * j + 1;
            if (cy > rx)
                W[cy * w + (cy - rx)] = conj(m);   /* row y_j, column x_i */
            else
                W[rx * w + (rx - cy)] = m;         /* row x_i, column y_j */
        }
    }
    int64_t neg = 0;
    for (int64_t k = 0; k < N; ++k) {
        double dk = creal(W[k * w]);
        if (dk == 0.0) {
            free(W);
            return -1;
        }
        if (dk < 0.0)
            ++neg;
        int64_t iend = k + b < N - 1 ? k + b : N - 1;
        /* Schur complement: H[i][j] -= H[i][k] conj(H[j][k]) / d_k for k < j <= i */
        for (int64_t i = k + 1; i <= iend; ++i) {
            cplx hik = W[i * w + (i - k)];
            if (hik == 0.0)
                continue;
            cplx f = hik / dk;
            for (int64_t j = k + 1; j <= i; ++j)
                W[i * w + (i - j)] -= f * conj(W[j * w + (j - k)]);
        }
    }
    free(W);
    return neg - n;
}

/* counts[p] = #{singular values of z_p I - A below t[p]} (or -1 for an exactly zero pivot).
 * Returns 0, or -1 if any point failed. */
int oracle_count_below(int64_t n, int64_t kl, int64_t ku, const cplx *ab, int64_t ldab, int64_t npts,
                       const cplx *z, const double *t, int64_t *counts, int nthreads)
{
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
#endif
    for (int64_t p = 0; p < npts; ++p) {
        counts[p] = count_one(n, kl, ku, ab, ldab, z[p], t[p]);
        if (counts[p] < 0)
            bad |= 1;
    }
    (void)nthreads;
    return bad ? -1 : 0;
}
