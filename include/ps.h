/*
 * ps.h -- C ABI of the MI355X (gfx950) library for sigma_min(zI - A) of a banded
 * non-normal matrix A at many complex shifts z.
 *
 * What is computed.  Sec. 2 (definition of the pseudospectrum, third form) and
 * Sec. 2.1 (Singular Value Decomposition): for each shift z, sigma_min(z) is the
 * smallest singular value s_n of zI - A; z lies in the eps-pseudospectrum iff
 * sigma_min(z) <= eps, and the sensitive zone is S_eps = {z in G : sigma_min(z) <= eps}
 * (Sec. 2.1, eq. (sensitive_zone)).  The shifts are either the full grid
 * G = {x_j + i y_i} of Sec. 2.1 (plain method) or a subset R of it (Sec. 4: the
 * restricted region; values on R are exact, errors are only omissions).
 *
 * How it is computed (not the paper's dense SVD): per shift a complex banded LU with
 * partial pivoting of zI - A, then Golub-Kahan (inverse Lanczos) bidiagonalisation of
 * (zI - A)^{-1} through banded triangular solves; sigma_min = 1 / sigma_max of the
 * bidiagonal.  Solves are overflow-safe (per-row binary exponents), so sigma_min far
 * below the double range is reported as 0 with PS_PT_UNDERFLOW.
 *
 * Conventions shared by every call:
 *  - Complex numbers are ps_c128 = {re, im} doubles (same bytes as
 *    hipDoubleComplex and torch.complex128).
 *  - Pointers named *_dev or documented "device" must be device (HBM) pointers on the
 *    current HIP device; all other pointers are host pointers.
 *  - "stream" is a hipStream_t (NULL = the default stream).  Calls that take a stream
 *    only enqueue work on it and return; results are valid after the stream is
 *    synchronised.  Calls without a stream argument are synchronous.
 *  - Ownership: ps_create_banded copies the band into library-owned device memory
 *    (freed by ps_destroy).  Everything else (shifts, masks, outputs, workspace) is
 *    owned by the caller; the library keeps no pointer after a call returns.
 *  - Errors: every call validates its arguments before launching anything and returns
 *    a ps_status; no exception or process exit crosses the ABI.  ps_last_error()
 *    returns a thread-local message describing the last failure on this thread.
 *    Per-shift outcomes are reported in the optional info[] output (PS_PT_* bits).
 */
#ifndef PS_H_
#define PS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double re, im;
} ps_c128;

typedef struct ps_matrix_s *ps_matrix;

typedef enum {
    PS_OK = 0,
    PS_ERR_INVALID = 1,     /* bad argument (sizes, NULL where required, ...)            */
    PS_ERR_NONFINITE = 2,   /* NaN or Inf in the band or in the grid parameters          */
    PS_ERR_WORKSPACE = 3,   /* workspace NULL or smaller than the minimum for the call   */
    PS_ERR_HIP = 4,         /* a HIP runtime call failed (message in ps_last_error)      */
    PS_ERR_UNSUPPORTED = 5  /* bandwidths outside the compiled range, ...                */
} ps_status;

/* Per-shift info bits (info[p]).  0 means converged to the requested tolerance. */
enum {
    PS_PT_CONVERGED = 0,
    PS_PT_SINGULAR = 1,   /* the LU met an exactly zero (or negligible) pivot: sigma_min = 0 */
    PS_PT_MAXITER = 2,    /* iteration cap reached: sigma is the best (upper) estimate        */
    PS_PT_UNDERFLOW = 4,  /* sigma_min below the smallest normal double: reported as 0, with
                             -floor(log2 sigma_min) in bits 8..31 of info                   */
    PS_PT_BISECT = 8      /* sigma came from the inertia bisection (sigma only, kl + ku >= 1):
                             sigma_min^2 is the smallest eigenvalue of (zI-A)^H (zI-A), so
                             t < sigma_min exactly when (zI-A)^H (zI-A) - t^2 I has a Cholesky
                             factor; bits 8..31 of info hold the number of passes over
                             the band (a pass makes one or more such tests: lanes per shift
                             x tests per lane), and no Golub-Kahan step was taken          */
};

/* Flags of ps_create_banded. */
enum {
    PS_DEVICE_PTR = 1,    /* ab is a device pointer (default: host pointer)                  */
    PS_REAL_A = 2         /* A is real: ps_backward returns the real part of the band gradient */
};

/* Grid of Sec. 2.1: x_j = a + (b - a) j / (nx - 1), y_i = c + (d - c) i / (ny - 1)
 * (inclusive ends; a single point sits at a, resp. c); z_ij = x_j + i y_i; flat index
 * i * nx + j (row index <-> y).  Requires nx, ny >= 1 and finite a, b, c, d. */
typedef struct {
    double a, b, c, d;
    int64_t nx, ny;
} ps_grid;

/* Options.  tol_norm and tol_rel set the stopping target
 * |sigma - sigma_min| <= tol_norm * ||A||_F + tol_rel * sigma_min.
 * max_iter caps the Lanczos steps per shift (1 .. 4096).  slots: number of shifts
 * processed concurrently (0 = library default; rounded down to a multiple of 256). */
typedef struct {
    double tol_norm;      /* default 1e-10 */
    double tol_rel;       /* default 1e-8  */
    int32_t max_iter;     /* default 3000  */
    int32_t want_vectors; /* 1: also return u, v (sizes [npts][n])          */
    int32_t slots;        /* 0: default                                       */
    int32_t check_shift;  /* Ritz-value checks every max(1, k >> check_shift)
                             Lanczos steps (0: default 5); set by ps_autotune  */
    int32_t bisect;       /* 0 (default): a shift where the rounding of (zI-A)^H (zI-A),
                             about 32 eps (|z| + ||A||)^2 / sigma in sigma, stays below an
                             eighth of the target gets sigma_min by bisection on Cholesky
                             tests instead of Lanczos steps (kl + ku >= 1);
                             -1: every shift takes the Golub-Kahan path                  */
    int32_t lanes;        /* sigma only: lanes of a wavefront that share one shift's
                             bisection (0 = default 1; 1, 2, 4, or 64 = one wavefront per
                             shift, the plain per-shift form; 64 is refused in batch mode) */
    int32_t tests;        /* sigma only: tests per lane and bisection pass (0 = default 2;
                             1: one; 2: three for kl + ku <= 2, two for <= 5, one above;
                             3: two for kl + ku <= 6, one above).  A pass splits the bracket
                             into lanes * tests + 1 parts.  Set by ps_autotune.            */
} ps_opts;

/* Fills *o with the defaults listed above. */
void ps_opts_default(ps_opts *o);

/*
 * ps_create_banded -- register a banded matrix A (n x n, kl sub- and ku superdiagonals).
 * Passage: the problem input A in C^{n x n} (Sec. 2; banded class of Sec. 3.3, eq. (matrix)).
 *   ab    LAPACK general-band storage, column-major: A[i][j] = ab[(ku + i - j) + j * ldab]
 *         for max(0, j - ku) <= i <= min(n - 1, j + kl); other entries are ignored.
 *         Host pointer unless flags has PS_DEVICE_PTR.
 *   ldab  >= kl + ku + 1.   n >= 1.   0 <= kl, ku <= n - 1.
 *         kl, ku <= 4: the banded kernels (every entry point).  kl or ku > 4 with n <= 64:
 *         the matrix is taken as dense (as the Jordan example of Sec. 2, a Jordan block with a
 *         corner entry): ps_eval_points and ps_eval_grid compute sigma only, one wavefront
 *         per shift (Householder bidiagonalisation in LDS, then bisection by Sturm counts on
 *         the Golub-Kahan tridiagonal; info 0, iters = bisection rounds); vectors, the adjoint,
 *         labels, contours, batches and the allocation-free call return PS_ERR_UNSUPPORTED.
 *   flags PS_DEVICE_PTR | PS_REAL_A.   stream: used for the upload (the call waits for it).
 *   out   receives a handle that owns a device copy of the band (plus ||A||_F).
 * Errors: PS_ERR_INVALID (sizes, NULL), PS_ERR_NONFINITE (NaN/Inf in the band),
 *         PS_ERR_UNSUPPORTED (kl or ku > 4 with n > 64), PS_ERR_HIP.
 */
ps_status ps_create_banded(const ps_c128 *ab, int64_t ldab, int64_t n, int32_t kl, int32_t ku,
                           uint32_t flags, void *stream, ps_matrix *out);

/* ps_destroy -- free the handle and its device memory (NULL is accepted). */
ps_status ps_destroy(ps_matrix m);

/* ps_matrix_info -- n, kl, ku and ||A||_F of a handle (any output may be NULL). */
ps_status ps_matrix_info(ps_matrix m, int64_t *n, int32_t *kl, int32_t *ku, double *fro);

/*
 * ps_workspace_size -- bytes of device workspace needed by ps_eval_points / ps_eval_grid
 * for npts shifts with options o (NULL = defaults).  The result depends on n, kl, ku, the
 * number of slots and whether vectors are wanted, not on the shift values.  With vectors it
 * includes room for Lanczos vectors of each slot (up to 64 of them, at most 16 GiB in all),
 * from which the Ritz vector is formed instead of replaying the Lanczos steps.  A smaller
 * workspace is accepted: the call keeps fewer Lanczos vectors (a shift that needs more steps
 * than are kept replays them), and below what the slots themselves need it runs on fewer slots.
 */
ps_status ps_workspace_size(ps_matrix m, int64_t npts, const ps_opts *o, size_t *bytes);

/*
 * ps_eval_points -- sigma_min(z_p I - A) for an explicit list of shifts (the restricted
 * set R of Sec. 4 given as a list, or any points).
 *   z_dev      device ps_c128[npts].   npts >= 0 (0: nothing is launched).
 *   ws_dev     device workspace of ws_bytes >= ps_workspace_size(m, npts, o).
 *   sigma_dev  device double[npts] (required).
 *   u_dev, v_dev  device ps_c128[npts][n] or NULL; required when o->want_vectors.
 *              Unit singular vectors with (zI - A) v = sigma u; the joint phase makes the
 *              first entry of v of largest modulus real and positive.  For a shift that took
 *              the inertia bisection (PS_PT_BISECT in info; the bisection kernel runs first
 *              over all shifts of a call with vectors and saves each bracket), v comes from
 *              four steps of inverse iteration with L D L^H of (zI - A)^H (zI - A) - lo^2 I
 *              (lo the bracket's lower end, where the bisection found it positive definite),
 *              and u = (zI - A) v / |(zI - A) v|.  For the other shifts v is the Ritz vector
 *              of the converged Lanczos process, formed from the Lanczos vectors the first
 *              pass kept (see ps_workspace_size) or, where they were not kept, by a second pass
 *              that replays its steps exactly (then vectors cost about twice the steps of
 *              sigma alone), and u one inverse-iteration step from it,
 *              u = (zI - A)^{-H} v / |(zI - A)^{-H} v|.
 *   info_dev   device int32[npts] or NULL (PS_PT_* bits).  iters_dev: int32[npts] or NULL:
 *              Golub-Kahan (inverse Lanczos) steps (0 for a shift flagged PS_PT_BISECT,
 *              whose number of Cholesky tests is in info).
 * Errors: PS_ERR_INVALID, PS_ERR_WORKSPACE, PS_ERR_HIP.
 */
ps_status ps_eval_points(ps_matrix m, const ps_c128 *z_dev, int64_t npts, const ps_opts *o, void *ws_dev,
                         size_t ws_bytes, double *sigma_dev, ps_c128 *u_dev, ps_c128 *v_dev, int32_t *info_dev,
                         int32_t *iters_dev, void *stream);

/*
 * ps_eval_grid -- sigma_min on the grid G of Sec. 2.1, or on the masked subset of it.
 *   g          grid parameters (host struct).
 *   mask_dev   device uint8[ny][nx] or NULL.  NULL: every grid point (the plain method).
 *              Otherwise the points with mask != 0 (the restricted region R of Sec. 4).
 *   idx_dev    device int64[nx*ny] (required): on return idx_dev[p] is the flat grid index
 *              of the p-th evaluated point, ascending; entries past the count are untouched.
 *   count_dev  device int64[1] (required): number of evaluated points.
 *   The outputs sigma_dev, u_dev, v_dev, info_dev, iters_dev are indexed by p (compacted,
 *   like idx_dev) and must hold nx*ny entries (rows of n for u, v).
 *   ws_dev / ws_bytes: as for ps_eval_points with npts = nx*ny.
 *   eps, sens_dev: if sens_dev != NULL, sens_dev[p] = (sigma_dev[p] <= eps) (uint8), the
 *              sensitive zone of Sec. 2.1 eq. (sensitive_zone) restricted to the points.
 * Errors: PS_ERR_INVALID, PS_ERR_NONFINITE (grid bounds), PS_ERR_WORKSPACE, PS_ERR_HIP.
 */
ps_status ps_eval_grid(ps_matrix m, const ps_grid *g, const uint8_t *mask_dev, const ps_opts *o, void *ws_dev,
                       size_t ws_bytes, int64_t *idx_dev, int64_t *count_dev, double *sigma_dev, ps_c128 *u_dev,
                       ps_c128 *v_dev, int32_t *info_dev, int32_t *iters_dev, double eps, uint8_t *sens_dev,
                       void *stream);

/*
 * ps_backward -- gradients of L = sum_p g_p sigma_min(z_p I - A) from the singular pairs.
 * Passage: none in the paper (it has no gradients).  First-order perturbation of a simple
 * singular value: d sigma = Re(u^H dM v) with dM = dz I - dA.  Conjugate-Wirtinger
 * convention (d/dRe + i d/dIm), as torch uses for complex inputs:
 *     grad_z[p]    = g_p conj(u_p^H v_p)
 *     grad_A[i][j] = -sum_p g_p u_p[i] conj(v_p[j])      on the band only
 *   (with PS_REAL_A the band gradient's imaginary part is zeroed).
 *   grad_sigma_dev device double[npts];  u_dev, v_dev device ps_c128[npts][n] as returned by
 *   the eval calls.  grad_z_dev: device ps_c128[npts] or NULL.  grad_band_dev: device
 *   ps_c128 in the GB layout of ps_create_banded with ldab = kl + ku + 1 (n columns), or
 *   NULL; overwritten (not accumulated).  Both sums use a fixed order (deterministic).  With
 *   both outputs asked for, one pass reads u and v once for both gradients (partial sums per
 *   256 rows and per 64 shifts in the workspace, then reduced).
 *   ws_dev / ws_bytes >= ps_backward_workspace_size(m, npts) (needed when grad_band_dev is set).
 * Errors: PS_ERR_INVALID, PS_ERR_WORKSPACE, PS_ERR_HIP.
 */
ps_status ps_backward_workspace_size(ps_matrix m, int64_t npts, size_t *bytes);
ps_status ps_backward(ps_matrix m, int64_t npts, const double *grad_sigma_dev, const ps_c128 *u_dev,
                      const ps_c128 *v_dev, ps_c128 *grad_z_dev, ps_c128 *grad_band_dev, void *ws_dev,
                      size_t ws_bytes, void *stream);

/*
 * Batches of matrices.  A batch groups nmat registered matrices of possibly different n and
 * bandwidths, each with its own grid (Sec. 2.1), for one call that evaluates all of them
 * (the restricted evaluation of Sec. 4 applied to many matrices at once).  Outputs of all
 * matrices are concatenated: matrix m owns entries [off_m, off_m + nx_m * ny_m), with
 * off_m = sum of nx * ny of the matrices before m (ps_batch_info returns them).
 *
 * ps_create_batch -- mats: nmat handles (not owned; they must outlive the batch); grids:
 *   host array of nmat grids.  Copies the per-matrix descriptors to the device once.
 *   Errors: PS_ERR_INVALID (nmat < 1, NULL handle, bad grid), PS_ERR_NONFINITE, PS_ERR_HIP.
 * ps_destroy_batch -- frees the batch (not the matrices).  NULL is accepted.
 * ps_batch_info -- total number of grid points, and the offsets off_m (offsets may be NULL).
 * ps_batch_workspace_size -- device workspace for ps_eval_batch with options o.
 * ps_eval_batch -- sigma_min at the masked grid points of every matrix of the batch.
 *   masks_dev  device array of nmat device pointers to uint8 [ny_m][nx_m] masks; a NULL
 *              entry (or masks_dev == NULL) selects the full grid of that matrix.
 *   idx_dev    device int64[total]: in the section of matrix m, the ascending flat grid
 *              indices of its evaluated points (first counts_dev[m] entries).
 *   counts_dev device int64[nmat]: number of evaluated points per matrix.
 *   sigma_dev, info_dev, iters_dev: device arrays [total], indexed like idx_dev.
 *   Vectors are not produced in batch mode (o->want_vectors must be 0).
 *   Work: one compaction of all masks, then one persistent launch per (kl, ku) class whose
 *   shift queue lists larger matrices first.  Calls on one batch must not overlap.
 *   Errors: PS_ERR_INVALID, PS_ERR_WORKSPACE, PS_ERR_UNSUPPORTED (want_vectors), PS_ERR_HIP.
 */
typedef struct ps_batch_s *ps_batch;
ps_status ps_create_batch(int32_t nmat, const ps_matrix *mats, const ps_grid *grids, ps_batch *out);
ps_status ps_destroy_batch(ps_batch b);
ps_status ps_batch_info(ps_batch b, int64_t *total_points, int64_t *offsets);
ps_status ps_batch_workspace_size(ps_batch b, const ps_opts *o, size_t *bytes);
ps_status ps_eval_batch(ps_batch b, const uint8_t *const *masks_dev, const ps_opts *o, void *ws_dev, size_t ws_bytes,
                        int64_t *idx_dev, int64_t *counts_dev, double *sigma_dev, int32_t *info_dev,
                        int32_t *iters_dev, void *stream);

/*
 * ps_label_batch -- ps_label_grid for every matrix of a batch at once (the label generation
 * of Sec. 3.3 runs over many matrices): each level builds the masks of all matrices, evaluates
 * them as ps_eval_batch does (one bisection launch and one Golub-Kahan launch for all
 * matrices), then marks and excludes for all matrices together.  Matrix m's labels (and sigma) occupy
 * [offsets[m], offsets[m] + nx ny) of the concatenated outputs (offsets from ps_batch_info).
 *   label_dev  device uint8[total] (required; values as in ps_label_grid).
 *   sigma_dev  device double[total] or NULL.
 *   evals_dev  device int64[1] or NULL: shifts evaluated over all matrices.
 *   ws_dev / ws_bytes >= ps_label_batch_workspace_size(b, o).  Calls on one batch must not
 *   overlap.
 * Errors: PS_ERR_INVALID, PS_ERR_WORKSPACE, PS_ERR_UNSUPPORTED (vectors), PS_ERR_HIP.
 */
ps_status ps_label_batch_workspace_size(ps_batch b, const ps_opts *o, size_t *bytes);
ps_status ps_label_batch(ps_batch b, double eps, const ps_opts *o, void *ws_dev, size_t ws_bytes, uint8_t *label_dev,
                         double *sigma_dev, int64_t *evals_dev, void *stream);

/*
 * ps_newton_contour -- refine points toward the eps-level curve of sigma_min (the boundary of
 * the eps-pseudospectrum drawn as the level curve log10 eps in Sec. 2.1).  Each of `steps`
 * steps evaluates sigma_min with its singular vectors at every point, forms
 * g = conj(u^H v) (the gradient of sigma_min in the conjugate-Wirtinger convention) and
 * moves z <- z - sigma ln(sigma / eps) g / |g|^2 (Newton on ln(sigma / eps) along g).
 *   z_dev      device ps_c128[npts], updated in place.  sigma_dev: device double[npts],
 *              sigma_min at the final points.  info_dev: device int32[npts] or NULL.
 *   eps > 0, steps >= 0.  o: options of the evaluations (vectors are implied).
 *   ws_dev / ws_bytes >= ps_newton_workspace_size(m, npts, o).
 * Errors: PS_ERR_INVALID, PS_ERR_WORKSPACE, PS_ERR_HIP.
 */
ps_status ps_newton_workspace_size(ps_matrix m, int64_t npts, const ps_opts *o, size_t *bytes);
ps_status ps_newton_contour(ps_matrix m, ps_c128 *z_dev, int64_t npts, double eps, int32_t steps, const ps_opts *o,
                            void *ws_dev, size_t ws_bytes, double *sigma_dev, int32_t *info_dev, void *stream);

/* Stop flags of ps_trace_contour (flags_dev[p]). */
enum {
    PS_TRACE_CLOSED = 1,         /* point k >= 3 came within h of point 0: the curve closed    */
    PS_TRACE_LEFT_BOX = 2,       /* the last stored point lies outside the box                */
    PS_TRACE_NEWTON_FAILED = 4,  /* a corrected point missed the curve (|ln(sigma/eps)| >
                                    1e-6); it is not stored                                   */
    PS_TRACE_MAX_POINTS = 8      /* max_points points were stored                             */
};

/*
 * ps_trace_contour -- follow the eps-level curve sigma_min(zI - A) = eps (the boundary of the
 * eps-pseudospectrum, drawn as the level curve log10 eps in Sec. 2.1) from each seed, by
 * predictor-corrector steps: with g = conj(u^H v) the gradient of sigma_min at the current
 * point, the next point is the current one plus h i g / |g| (a step of length h along the
 * curve's tangent, counterclockwise around the region sigma < eps), corrected by
 * newton_steps Newton steps z <- z - sigma ln(sigma / eps) g / |g|^2 (as ps_newton_contour).
 * Point 0 is the seed after 2 newton_steps + 2 Newton steps.  Each Newton step and each
 * accepted point evaluates sigma_min with its singular vectors at every tracer.
 *   seeds_dev  device ps_c128[nseed] (e.g. from ps_contour_seeds).  nseed >= 0.
 *   eps > 0, h > 0 finite, max_points >= 1, newton_steps >= 1.
 *   box        host ps_grid whose a, b, c, d bound the tracing region (nx, ny unused), or NULL.
 *   points_dev device ps_c128[nseed][max_points]: the points of tracer p in order; entries
 *              past count_dev[p] are left as they were.
 *   count_dev  device int32[nseed]: points stored.  flags_dev: device int32[nseed], PS_TRACE_*.
 *   ws_dev / ws_bytes >= ps_trace_workspace_size(m, nseed, o) (vectors are implied in o).
 * Synchronous: every 8 points the call waits for the stream to learn whether any tracer is
 * still active, and returns when none is (so it cannot be captured in a graph).
 * Errors: PS_ERR_INVALID, PS_ERR_NONFINITE, PS_ERR_WORKSPACE, PS_ERR_HIP.
 */
ps_status ps_trace_workspace_size(ps_matrix m, int64_t nseed, const ps_opts *o, size_t *bytes);
ps_status ps_trace_contour(ps_matrix m, const ps_c128 *seeds_dev, int64_t nseed, double eps, double h,
                           int32_t max_points, int32_t newton_steps, const ps_grid *box, const ps_opts *o,
                           void *ws_dev, size_t ws_bytes, ps_c128 *points_dev, int32_t *count_dev,
                           int32_t *flags_dev, void *stream);

/*
 * ps_contour_seeds -- starting points for ps_newton_contour on the eps-level curve of sigma_min
 * (the boundary of the eps-pseudospectrum, drawn as the level curve log10 eps in Sec. 2.1):
 * one point on every grid edge whose two end points lie on different sides of the inclusive
 * test sigma <= eps (eq. sensitive_zone), at z1 + tau (z2 - z1) with
 * tau = (ln eps - ln s1) / (ln s2 - ln s1) (ln sigma linear along the edge; sigma is clamped to
 * 2^-1022 first).  Edge order: the horizontal edges (i, j)-(i, j+1) in row-major order of
 * (i, j), then the vertical edges (i, j)-(i+1, j) likewise.  No matrix is involved.
 *   g          the grid the values belong to (nx, ny >= 1).
 *   sigma_dev  device double[ny * nx], row-major (ps_eval_grid's output for mask NULL).
 *   eps > 0, finite.
 *   seeds_dev  device ps_c128[max_seeds] (may be NULL when max_seeds == 0): the first
 *              min(count, max_seeds) seeds in edge order.
 *   count_dev  device int64: the number of sign-change edges (may exceed max_seeds).
 *   ws_dev / ws_bytes >= ps_contour_seeds_workspace_size(g).
 * Errors: PS_ERR_INVALID, PS_ERR_NONFINITE, PS_ERR_WORKSPACE, PS_ERR_HIP.
 */
/*
 * ps_label_grid -- the sensitive zone S_eps of Sec. 2.1 (eq. sensitive_zone: z in S_eps iff
 * sigma_min(zI - A) <= eps) on the whole grid g, exactly, evaluating sigma_min only where the
 * answer is not already implied (the exclusion-region labelling the paper uses to generate
 * its training labels, Sec. 1 and Sec. 3.3).  sigma_min is 1-Lipschitz in z, so a computed
 * sigma(z0) > eps excludes every grid point closer to z0 than sigma(z0) - eps - margin
 * (margin = twice the evaluation tolerance tol_norm ||A||_F + tol_rel sigma(z0)).  The still
 * unknown points of the lattices of stride 8, 4, 2 and 1 (coarser strides are skipped on
 * small grids) are evaluated in turn, each level followed by the exclusion disks of its
 * points.  All steps run on the stream without host synchronisation.
 *   label_dev  device uint8[ny][nx] (required): 1 where sigma_min <= eps, 0 where it is
 *              above, 2 where neither is certified: the evaluation stopped at o->max_iter
 *              (PS_PT_MAXITER) with an estimate above eps.  A capped evaluation sizes no
 *              exclusion disk; it is labelled 1 when its estimate (an upper bound of sigma_min
 *              on the Golub-Kahan path) is <= eps.
 *   sigma_dev  device double[ny][nx] or NULL: sigma_min where it was evaluated, -1 where the
 *              point was excluded.
 *   evals_dev  device int64[1] or NULL: the number of shifts evaluated.
 *   eps > 0, finite.  o: options of the evaluations (vectors are not allowed).
 *   ws_dev / ws_bytes >= ps_label_workspace_size(m, g, o).
 * Errors: PS_ERR_INVALID, PS_ERR_NONFINITE, PS_ERR_WORKSPACE, PS_ERR_UNSUPPORTED (vectors),
 * PS_ERR_HIP.
 */
ps_status ps_label_workspace_size(ps_matrix m, const ps_grid *g, const ps_opts *o, size_t *bytes);
ps_status ps_label_grid(ps_matrix m, const ps_grid *g, double eps, const ps_opts *o, void *ws_dev, size_t ws_bytes,
                        uint8_t *label_dev, double *sigma_dev, int64_t *evals_dev, void *stream);

ps_status ps_contour_seeds_workspace_size(const ps_grid *g, size_t *bytes);
ps_status ps_contour_seeds(const ps_grid *g, const double *sigma_dev, double eps, ps_c128 *seeds_dev,
                           int64_t max_seeds, int64_t *count_dev, void *ws_dev, size_t ws_bytes, void *stream);

/*
 * ps_autotune -- choose the plan for ps_eval_points / ps_eval_grid on this matrix.  Passage:
 * none (an implementation choice; the paper computes each point by a dense SVD).
 *   Sigma-only calls that bisect (want_vectors = 0, bisect = 0, kl + ku >= 1): lanes per shift
 *   (1, 2, 4) times tests per lane (modes 2, 1, 3), nine plans.  Otherwise: the Golub-Kahan
 *   kernel's slot count (the default, a half and a quarter of it) times the Ritz-check
 *   interval (check_shift 5, 4, 3).  Each candidate runs once untimed and twice timed with HIP
 *   events on z_dev[0 .. npts) (a representative sample of the shifts to be evaluated, on the
 *   device; with vectors the timing runs sigma only); the fastest plan's fields (slots,
 *   check_shift, lanes, tests) are written into *o, everything else in *o is kept.  The first
 *   candidate is the default plan; another replaces it only when it takes under 98 % of its
 *   time (the faster of its timed runs).
 *   Plans are cached per process by (device architecture and compute-unit count, ceil(log2 n),
 *   kl, ku, ceil(log2 npts), want_vectors, bisect): a later call with the same key returns the
 *   cached plan without timing (ps_plan_cache_clear empties the cache).
 * Synchronous; allocates and frees its own workspace.  Results of the timed runs are
 * discarded.
 * Errors: PS_ERR_INVALID, PS_ERR_HIP.
 */
ps_status ps_autotune(ps_matrix m, const ps_c128 *z_dev, int64_t npts, ps_opts *o, void *stream);

/*
 * ps_autotune_batch -- the same for ps_eval_batch on this batch with these masks (masks_dev as
 * for ps_eval_batch): lanes per shift times tests per lane when the batch bisects (the plan
 * applies to all its matrices), else the Ritz-check interval.  One untimed call, then each
 * candidate timed twice over the whole batch call (the faster run counts; the default plan,
 * the first candidate, is kept unless another takes under 98 % of its time).  Cached by
 * (device, bisect, and per matrix
 * ceil(log2 n), kl, ku, ceil(log2 grid points)).  Synchronous; allocates and frees its own
 * workspace and outputs.
 * Errors: PS_ERR_INVALID, PS_ERR_UNSUPPORTED (vectors), PS_ERR_HIP.
 */
ps_status ps_autotune_batch(ps_batch b, const uint8_t *const *masks_dev, ps_opts *o, void *stream);

/* Empties the plan cache of ps_autotune and ps_autotune_batch. */
void ps_plan_cache_clear(void);

/* ------------------------------------------------------------------------------------------
 * Mask producer (Sec. 3.2, Sec. 3.5, Sec. 4): the classifier p(z, A) of the dual-path network
 * and its coarse-to-fine use over a grid, giving the restricted set R for ps_eval_grid.
 *
 * The network (Sec. 3.2, dual-path architecture).  Coordinates c = [Re z, Im z] are encoded
 * as phi(c) = [c, sin(2c), cos(2c), sin(4c), cos(4c), ..., sin(64c), cos(64c)] (26 values,
 * element-wise over c); the matrix features are f(z, A) = [f1 .. f30, g1, g2, g3] with the 30
 * global features supplied by the caller and the per-point distances of Sec. 3.1 eq. (dist)
 * computed here: g1 = min_i |z - lambda_i|, g2 = |z - lambda*|, g3 = mean_i |z - lambda_i|,
 * lambda* read as the eigenvalue centroid (the paper leaves it undefined).  Then
 *   h_c1 = SiLU(W_c1 phi + b_c1) (64), h_c2 = SiLU(W_c2 h_c1 + b_c2) (64),
 *   h_m1 = SiLU(W_m1 f + b_m1) (128), h_m2 = SiLU(W_m2 h_m1 + b_m2) (64),
 *   h4 = SiLU(W4 [h_c2, h_m2] + b4), h6 = h4 + SiLU(W5 h4 + b5) (128),
 *   h7 = SiLU(W7 h6 + b7) (64), p = 1 / (1 + exp(-(w . h7 + b))).
 * Parameter vector (PS_MLP_NPARAM floats): each layer's W (out x in, row-major) followed by
 * its b, in the order W_c1 (64x26), W_c2 (64x64), W_m1 (128x33), W_m2 (64x128), W4 (128x128),
 * W5 (128x128), W7 (64x128), w (1x64).
 * Arithmetic: float32 (the matrix cores' 16x16x4 float32 products, float32 accumulation);
 * the features are formed in float64 and rounded to float32; the global features enter
 * through a float64 fold into b_m1.  No trained weights ship with the library.
 * ---------------------------------------------------------------------------------------- */
#define PS_MLP_NPARAM 59841
#define PS_MLP_NGLOBAL 30

typedef struct ps_mlp_s *ps_mlp;

/* Options of ps_mask_predict (Sec. 3.5 hierarchical prediction, Sec. 3.6 threshold calibration). */
typedef struct {
    int32_t stride;   /* coarse stride s (default 4, 1 .. 32): coarse point (I, J) is fine
                         point (s I, s J) and owns the cell of fine rows s I .. s I + s - 1 and
                         columns likewise, cut at the grid's edge                             */
    int32_t dilate;   /* side of the square structuring element (default 5; odd, 1 .. 31)    */
    double coarse_q;  /* the coarse percentile as a fraction (default 0.8, in [0, 1])         */
    double tau;       /* the calibrated threshold tau (default 0.05, in (0, 1])               */
} ps_mask_opts;

void ps_mask_opts_default(ps_mask_opts *o);

/*
 * ps_mlp_create -- upload a parameter vector (layout above) and repack it for the kernels.
 *   params  PS_MLP_NPARAM floats; host pointer unless flags has PS_DEVICE_PTR.
 *   out     receives a handle owning device copies (freed by ps_mlp_destroy).
 * Synchronous on stream.  Errors: PS_ERR_INVALID, PS_ERR_NONFINITE (NaN/Inf), PS_ERR_HIP.
 */
ps_status ps_mlp_create(const float *params, uint32_t flags, ps_mlp *out, void *stream);
ps_status ps_mlp_destroy(ps_mlp net);

/*
 * ps_mask_workspace_size -- device workspace of ps_mask_predict on grid g with options o
 * (o NULL = defaults); g NULL gives the workspace of ps_mlp_prob.
 */
ps_status ps_mask_workspace_size(const ps_grid *g, const ps_mask_opts *o, size_t *bytes);

/*
 * ps_mlp_prob -- p(z, A) (Sec. 3.2) at npts arbitrary points.
 *   gfeat    host double[30]: f1 .. f30 of A (Tables matrix, matrixAdd, resolvent of Sec. 3.1).
 *   eig_dev  device ps_c128[neig], neig >= 1: the eigenvalues of A.
 *   z_dev    device ps_c128[npts] (npts >= 0).   prob_dev  device float[npts].
 *   ws_dev / ws_bytes >= ps_mask_workspace_size(NULL, NULL), 256-byte aligned.
 * Errors: PS_ERR_INVALID, PS_ERR_NONFINITE (gfeat), PS_ERR_WORKSPACE, PS_ERR_HIP.
 */
ps_status ps_mlp_prob(ps_mlp net, const double *gfeat, const ps_c128 *eig_dev, int64_t neig, const ps_c128 *z_dev,
                      int64_t npts, void *ws_dev, size_t ws_bytes, float *prob_dev, void *stream);

/*
 * ps_mask_predict -- the predicted region R of Sec. 4 on grid g by the hierarchical
 * prediction of Sec. 3.5:
 *   1. p at the coarse points -> P_coarse;
 *   2. tau_coarse = quantile_q(P_coarse), linear interpolation between the order statistics
 *      v_(k) <= v_(k+1) at h = q (m - 1), k = floor(h): v_(k) + (h - k)(v_(k+1) - v_(k));
 *   3. every cell whose coarse value is >= tau_coarse gets p at all its fine points; every
 *      other fine point gets probability 0;
 *   4. mask = {p >= tau} dilated by the dilate x dilate square (points outside the grid do
 *      not exist).
 * The comparisons are taken in double on the float32 probabilities.  All steps run on the
 * stream without host synchronisation.
 *   mask_dev        device uint8[ny][nx] (required), row-major (row <-> y): R, ready as
 *                   ps_eval_grid's mask.
 *   prob_dev        device float[ny][nx] or NULL: the fine probability map (0 outside the
 *                   refined cells).
 *   coarse_dev      device float[ceil(ny/s)][ceil(nx/s)] or NULL: P_coarse.
 *   tau_coarse_dev  device double or NULL.   evals_dev  device int64 or NULL: the number of
 *                   network evaluations (coarse points + fine points of the refined cells).
 *   gfeat, eig_dev, neig as in ps_mlp_prob.  o NULL = defaults.
 *   ws_dev / ws_bytes >= ps_mask_workspace_size(g, o), 256-byte aligned.
 * Errors: PS_ERR_INVALID, PS_ERR_NONFINITE, PS_ERR_WORKSPACE, PS_ERR_HIP.
 */
ps_status ps_mask_predict(ps_mlp net, const ps_grid *g, const double *gfeat, const ps_c128 *eig_dev, int64_t neig,
                          const ps_mask_opts *o, void *ws_dev, size_t ws_bytes, uint8_t *mask_dev, float *prob_dev,
                          float *coarse_dev, double *tau_coarse_dev, int64_t *evals_dev, void *stream);

/*
 * ps_mask_predict_batch -- ps_mask_predict for nmat matrices on one grid g, every step one launch
 * for all matrices (the setting of Sec. 3.3 and Sec. 5: many matrices, one grid).
 *   nmat            1 .. 65535.
 *   gfeat           host double[nmat][30]: the global features of each matrix.
 *   eig_dev         device ps_c128[eig_off[nmat]]: the eigenvalues of all matrices, matrix m's at
 *                   eig_off[m] .. eig_off[m+1] - 1.
 *   eig_off         host int64[nmat + 1]: eig_off[0] = 0, every matrix with at least one
 *                   eigenvalue.  gfeat and eig_off are copied to the workspace on the stream
 *                   before the call returns (host memory may be reused afterwards).
 *   mask_dev        device uint8[nmat][ny][nx] (required); prob_dev float[nmat][ny][nx],
 *                   coarse_dev float[nmat][ceil(ny/s)][ceil(nx/s)], tau_coarse_dev double[nmat],
 *                   evals_dev int64[nmat]: optional (NULL), as in ps_mask_predict, per matrix.
 *   ws_dev / ws_bytes >= ps_mask_batch_workspace_size(nmat, g, o), 256-byte aligned.
 * Errors: PS_ERR_INVALID, PS_ERR_NONFINITE, PS_ERR_WORKSPACE, PS_ERR_HIP.
 */
ps_status ps_mask_batch_workspace_size(int32_t nmat, const ps_grid *g, const ps_mask_opts *o, size_t *bytes);
ps_status ps_mask_predict_batch(ps_mlp net, int32_t nmat, const ps_grid *g, const double *gfeat,
                                const ps_c128 *eig_dev, const int64_t *eig_off, const ps_mask_opts *o, void *ws_dev,
                                size_t ws_bytes, uint8_t *mask_dev, float *prob_dev, float *coarse_dev,
                                double *tau_coarse_dev, int64_t *evals_dev, void *stream);

/*
 * ps_mask_calibrate -- the threshold calibration of Sec. 3.6 on a validation set of nval matrices
 * sharing grid g: for each candidate tau_k (ascending), the prediction {p >= tau_k} dilated by a
 * pred_dilate square is compared with the labels dilated by a label_dilate square; per matrix
 * recall = |both| / |dilated labels| (1 when a matrix has no labelled point).  Candidate k
 * qualifies when the median of the nval recalls is >= median_min and their 10th percentile is
 * >= p10_min (both by linear interpolation between order statistics, as for tau_coarse).  The
 * paper's tau* is the smallest qualifying candidate (recall cannot rise with tau, so it is the
 * first candidate whenever any qualifies); the largest qualifying candidate is the one that
 * predicts the fewest points within the same bounds.  Paper values: candidates 0.05, 0.06, ...,
 * 0.94, dilations 5 and 3, bounds 0.90 and 0.75, 30 validation matrices.
 *   prob_dev      device float[nval][ny][nx]: probability maps (e.g. ps_mask_predict_batch's).
 *   label_dev     device uint8[nval][ny][nx]: ground truth, nonzero = sensitive (e.g.
 *                 ps_label_batch's labels of the same matrices on the same grid).
 *   taus          host double[ntau], strictly ascending, 1 <= ntau <= PS_CAL_MAX_TAU.
 *   nval          1 .. PS_CAL_MAX_VAL.   pred_dilate, label_dilate: odd, 1 .. 31.
 *   index_dev     device int32[2] (required): the smallest and the largest qualifying candidate
 *                 index, -1 when none qualifies.
 *   recall_dev    device double[nval][ntau], median_dev / p10_dev double[ntau]: optional.
 *   ws_dev / ws_bytes >= ps_mask_calibrate_workspace_size(nval, ntau), 256-byte aligned.
 * Runs on the stream without host synchronisation; the candidates travel as kernel arguments.
 * Errors: PS_ERR_INVALID, PS_ERR_NONFINITE, PS_ERR_WORKSPACE, PS_ERR_HIP.
 */
#define PS_CAL_MAX_TAU 128
#define PS_CAL_MAX_VAL 256
ps_status ps_mask_calibrate_workspace_size(int32_t nval, int32_t ntau, size_t *bytes);
ps_status ps_mask_calibrate(int32_t nval, const ps_grid *g, const float *prob_dev, const uint8_t *label_dev,
                            const double *taus, int32_t ntau, int32_t pred_dilate, int32_t label_dilate,
                            double median_min, double p10_min, void *ws_dev, size_t ws_bytes, int32_t *index_dev,
                            double *recall_dev, double *median_dev, double *p10_dev, void *stream);

/*
 * ps_eval_points_noalloc -- ps_eval_points for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): sigma only, and the
 * workspace is a fixed device array of PS_NOALLOC_SCRATCH_BYTES inside the library instead
 * of a caller buffer.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine); it uses the matrix's own side stream as ps_eval_points does.
 *   z_dev, npts, o, sigma_dev, info_dev, iters_dev, stream   as in ps_eval_points
 *              (o->want_vectors must be 0).
 * Limit: the call needs the room ps_workspace_size would ask for npts shifts with at least one
 * wavefront (64) of Golub-Kahan slots: about 28 bytes per shift plus, per slot, about
 * (32 kl + 16 ku + 71) (n + 16) + 16 max_iter bytes (under 1 MiB per slot at n <= 4000 with
 * kl = ku = 4 and the default max_iter).  Requests that do not fit are refused with
 * PS_ERR_WORKSPACE and a message giving the bytes needed and the scratch size.
 * Each GPU holds one such array for the life of the process, shared by every call on that
 * GPU, and the array keeps the last call's contents: calls that overlap on one GPU (from
 * different streams or threads) race on it and must be serialised by the caller.  Everything
 * a call needs zeroed is cleared by its own kernels.
 * Errors: PS_ERR_INVALID, PS_ERR_UNSUPPORTED (vectors), PS_ERR_WORKSPACE (too large), PS_ERR_HIP.
 */
#define PS_NOALLOC_SCRATCH_BYTES (128u << 20)
ps_status ps_eval_points_noalloc(ps_matrix m, const ps_c128 *z_dev, int64_t npts, const ps_opts *o,
                                 double *sigma_dev, int32_t *info_dev, int32_t *iters_dev, void *stream);

/*
 * ps_set_timing_events -- measurement hook (no passage of the paper: it serves benchmarks).
 *   start, end   hipEvent_t (as void *) created by the caller, or both NULL to switch the hook off.
 * While set, every sigma-only evaluation on the calling thread that bisects (ps_eval_points,
 * ps_eval_grid, ps_eval_batch and the calls built on them) records start on the caller's
 * stream just before its bisection launches and end right after them, so that
 * hipEventElapsedTime(start, end) is the duration of the bisection kernel's launches (the
 * Golub-Kahan launches on the handle's side streams run beside them and are not included).
 * Meant for eager calls (under stream capture the records become capture-internal
 * dependencies, not timed nodes).  Thread-local; the caller keeps the events alive while the
 * hook is set.  Errors: PS_ERR_INVALID (one NULL).
 */
ps_status ps_set_timing_events(void *start, void *end);

/* Thread-local description of the last error on the calling thread ("" if none). */
const char *ps_last_error(void);

/* Library version string. */
const char *ps_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PS_H_ */
