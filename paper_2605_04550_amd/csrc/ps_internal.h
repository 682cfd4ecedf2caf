// Internal declarations shared by the host layer (ps_api.cpp) and the kernels
// (ps_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ps.h"

namespace ps {

// Maximum supported bandwidths of the compiled kernels.
constexpr int kMaxKL = 4;
constexpr int kMaxKU = 4;
// Wider bands (kl or ku above these) are taken as dense matrices, up to this order.
constexpr int kDenseMaxN = 64;
constexpr int kMaxIterCap = 4096;
// Rows per chunk of the triangular sweeps.  Per-row arrays are allocated with
// round_up(n, kChunk) + kChunk rows; rows past n hold zeros and make no contribution.
constexpr int kChunk = 8;
__host__ __device__ inline int64_t padded_rows(int64_t n) { return ((n + kChunk - 1) / kChunk) * kChunk + kChunk; }
// Zero rows stored before and after the row band of A (so that blocked reads near the ends
// of the matrix need no bounds checks): rows -kBandPadTop .. n + kBandPadBottom - 1 exist.
constexpr int kBandPadTop = 8;
constexpr int kBandPadBottom = 32;

// Size of the fixed device scratch of ps_eval_points_noalloc (see include/ps.h) and the
// lookup of its address on the current device.
constexpr size_t kNoallocScratchBytes = (size_t)PS_NOALLOC_SCRATCH_BYTES;
hipError_t noalloc_scratch(void **ptr);

// Where the shifts of one evaluation come from.
enum ShiftMode : int {
    kShiftList = 0,   // z[p] from a device array
    kShiftGrid = 1,   // grid point with flat index idx[p] (idx == nullptr: flat index p)
};

// Workspace carve-up of one evaluation: slots lanes, each with its own banded LU,
// three Lanczos vectors with block exponents and the Lanczos tridiagonal; with singular
// vectors also an accumulator vector and per-step bidiagonal entries and coefficients.
// Every per-slot array is tiled [wavefront][row][component][lane]: the 64 lanes of a
// wavefront touch 64 consecutive elements, and consecutive rows of one wavefront are
// contiguous (the shapes below list the logical indices).
struct Workspace {
    int64_t slots = 0;
    int64_t nrow = 0;              // allocated rows per slot of every per-row array
    double2 *L = nullptr;          // [n][kl][slots]   multipliers of column i
    double2 *U = nullptr;          // [n][w][slots]    U[i][i+d], d = 0 holds 1/U[i][i]
    uint8_t *piv = nullptr;        // [n][slots]       pivot row offset (0..kl)
    double2 *vu = nullptr;         // [n][slots]       Lanczos vector u (unnormalised)
    double2 *vv = nullptr;         // [n][slots]       Lanczos vector v (unnormalised)
    double2 *vy = nullptr;         // [n][slots]       intermediate of the two-factor solves
    int16_t *eu = nullptr;         // [n/8][slots]     binary exponent of each 8-row chunk of vu
    int16_t *ev = nullptr;
    int16_t *ey = nullptr;
    double *hist = nullptr;        // [kmax][2][slots] Lanczos tridiagonal: diag, offdiag^2
    double2 *vacc = nullptr;       // [n][slots]       singular-vector accumulator (vectors only)
    double *vmeta = nullptr;       // [kmax][4][slots] alpha', beta', Ritz work, coefficients (vectors only)
    // Calls with vectors: the normalised Lanczos vectors u_1 .. u_kstore of each slot, kept so
    // that the Ritz vector is one pass over them instead of a replay of the Lanczos steps
    // (see kstore_for); NULL and 0 otherwise.
    double2 *ustore = nullptr;     // [kstore][n][slots]
    int kstore = 0;
    unsigned long long *queue = nullptr;   // shift counter of the persistent launch
    int64_t *count = nullptr;      // number of shifts (device)
    int64_t *blocksums = nullptr;  // mask compaction scratch
    // Sigma-only calls: the queue positions the inertia bisection hands to the Golub-Kahan
    // kernel (allocated when npts_max > 0 and no vectors are wanted).
    int64_t *gk_list = nullptr;    // [npts_max]
    int64_t *gk_count = nullptr;   // [1]
    double *st_lo = nullptr;       // [npts_max] brackets saved between the two bisection launches
    double *st_hi = nullptr;
    int32_t *st_np = nullptr;
    int64_t npts_max = 0;
    int kmax = 0;
    int vec = 0;                   // 1: singular vectors wanted
};

// One matrix of a batch (device array, written once by ps_create_batch).  Matrices are
// stored grouped by (kl, ku); outputs of matrix m occupy [out_off, out_off + nx*ny) of the
// concatenated output arrays.
struct MatDesc {
    const double2 *arow;
    const double *gram;   // Gram band of the matrix (see the bisection kernel)
    int64_t n;
    double normA;
    double norm2A;    // upper bound on ||A||_2
    double ga, gb, gc, gd;
    int64_t nx, ny;
    int64_t out_off;
    int32_t kl, ku;
    int32_t cidx;     // position of the matrix in the caller's order
    int32_t cls;      // its (kl, ku) class
    int64_t cpos;     // its position in the class-sorted order
    int64_t cfirst;   // class-sorted position of the first matrix of its class
    int64_t gkbase;   // offset of its class's Golub-Kahan list
};

struct EvalArgs {
    int64_t n = 0;
    int kl = 0, ku = 0;
    const double2 *arow = nullptr; // [n][kl+ku+1] row band, zero outside the matrix
    double normA = 0.0;            // ||A||_F
    double norm2A = 0.0;           // upper bound on ||A||_2 (sqrt(||A||_1 ||A||_inf))
    int bisect = 1;                // 1: shifts that qualify take the inertia bisection
    const double *gram = nullptr;  // Gram band (sigma-only bisection)
    int lanes = 1;                 // lanes per shift of the bisection kernel (1, 2, 4, 64)
    int ktm = 1;                   // its test-count mode (tests_per_lane)
    const int64_t *perm = nullptr; // queue position -> shift position (the bisection's hand-off)
    int mode = kShiftList;
    const double2 *z = nullptr;
    const int64_t *idx = nullptr;
    double ga = 0, gb = 0, gc = 0, gd = 0;
    int64_t nx = 1, ny = 1;
    const int64_t *count_dev = nullptr;   // device count of shifts
    double tol_norm = 1e-10, tol_rel = 1e-8;
    int max_iter = 1000;
    int check_shift = 4;
    int want_vectors = 0;
    uint64_t seed = 0x2605045500000001ull;
    double *sigma = nullptr;
    double2 *u = nullptr;
    double2 *v = nullptr;
    int32_t *info = nullptr;
    int32_t *iters = nullptr;
    double eps = 0.0;
    uint8_t *sens = nullptr;
    // batch mode: the matrices of one (kl, ku) class
    const MatDesc *mats = nullptr;
    int nmat = 0;
    const int64_t *mfirst = nullptr;   // device: first queue position of each matrix
    int dense = 0;                     // 1: kl or ku above the banded kernels' limit, n <= kDenseMaxN
    // with vectors: brackets found beforehand by the bisection kernel (per shift position;
    // brk_np < 0: sigma below the bisection's limit, the Golub-Kahan path), or NULL
    const double *brk_lo = nullptr, *brk_hi = nullptr;
    const int32_t *brk_np = nullptr;
};

// sigma only for a matrix taken as dense (one wavefront per shift; at most npts_max shifts)
hipError_t launch_dense(const EvalArgs &a, int64_t npts_max, hipStream_t st);

// Arguments of the inertia-bisection kernel (sigma only): one matrix (batch == 0) or the
// chunks of a batch in longest-first order.
struct BisArgs {
    int batch = 0;
    const double *gram = nullptr;
    int64_t n = 0;
    int hb = 0;
    double normA = 0.0, norm2A = 0.0;
    int mode = kShiftList;
    const double2 *z = nullptr;
    const int64_t *idx = nullptr;
    double ga = 0, gb = 0, gc = 0, gd = 0;
    int64_t nx = 1, ny = 1;
    const int64_t *count_dev = nullptr;
    const MatDesc *mats = nullptr;          // batch: grouped by kl + ku, longest-first in a group
    int nmat = 0;
    int mlo = 0, mhi = 0;                   // batch: the launch's matrices mats[mlo .. mhi]
    const int64_t *chunkfirst = nullptr;    // [nmat] first chunk of each matrix
    const int64_t *total_chunks = nullptr;
    const int64_t *counts = nullptr;        // [nmat] shifts per matrix (caller order)
    const int64_t *mfirst = nullptr;        // [nmat] class-relative queue position (class order)
    double tol_norm = 1e-10, tol_rel = 1e-8;
    double *sigma = nullptr;
    int32_t *info = nullptr;
    int32_t *iters = nullptr;
    double eps = 0.0;
    uint8_t *sens = nullptr;
    int64_t *gk_list = nullptr;             // batch: base of all class lists
    int64_t *gk_count = nullptr;            // batch: one per class
    // 0: every pass in one launch; 1: first pass only, saving the bracket of every shift that
    // goes on (and handing over or finishing the others); 2: resume from the saved brackets;
    // 3: every pass, then save each final bracket (passes; -1 below the bisection's limit)
    // instead of writing sigma, for the singular vectors that follow
    int phase = 0;
    double *st_lo = nullptr, *st_hi = nullptr;   // saved brackets (queue position; output position
    int32_t *st_np = nullptr;                    // in phase 3 and in a batch); passes, -1 = settled
};

size_t gram_bytes(int64_t n, int kl, int ku);
hipError_t launch_gram_band(const double2 *arow, int64_t n, int kl, int ku, double *gram, hipStream_t st);
hipError_t launch_bis(const BisArgs &a, int hb, int ktm, int lanes, int64_t chunks, hipStream_t st);
hipError_t launch_bis_plan(const MatDesc *cls_order, const MatDesc *lpt_order, int nmat, int nclass,
                           const int64_t *counts, int spw, int64_t *pfx, int64_t *mfirst, int64_t *ctotal,
                           int64_t *chunkfirst, int64_t *total, int64_t *gk_count, hipStream_t st);
// The batch's Golub-Kahan launch: every (kl, ku) class at once, each on its own wavefronts
// and its own part of the workspace; a class takes count queue positions, from perm when it
// is not NULL.
struct GkClass {
    int32_t kl, ku;
    int32_t nmat;
    int32_t pad;
    int64_t first_block;   // first wavefront of the class in the launch
    int64_t nmax;          // largest n of the class
    int64_t slots;
    int64_t ws_off;        // its workspace, from the base
    const MatDesc *mats;   // its matrices (class-sorted order)
    const int64_t *mfirst;
    const int64_t *perm;
    const int64_t *count;
};
constexpr int kMaxClasses = (kMaxKL + 1) * (kMaxKU + 1);
struct GkBatchArgs {
    EvalArgs base;         // the fields every class shares (outputs, tolerances, shift source)
    char *ws;
    int32_t ncls;
    GkClass cls[kMaxClasses];
};
hipError_t launch_gk_batch(const GkBatchArgs &g, int64_t blocks, hipStream_t st);
// Sorting of the hand-off lists (list k starts at lists + base[k] and holds counts[k] entries).
struct ListBases {
    int64_t base[kMaxClasses];
};
hipError_t launch_sort_lists(int64_t *lists, const ListBases &bases, const int64_t *counts, int nlists,
                             hipStream_t st);

size_t workspace_bytes(int64_t n, int kl, int ku, int64_t slots, int kmax, int vec, int64_t npts_max,
                       int kstore = 0);
// The carve-up of one evaluation workspace (host and device: the batch's Golub-Kahan kernel
// carves each class's part itself).
// Lanczos vectors kept per slot in a call with vectors, by default: up to 64 (and up to kmax)
// while the store stays within 16 GiB (a short shift list keeps 64; a 65536-shift grid at
// n = 4000 keeps 3, all its Golub-Kahan shifts need there).  A call given less workspace keeps
// fewer (see prepare_eval).
constexpr int kStoreMaxK = 64;
constexpr double kStoreBudget = 16.0 * (1ull << 30);
__host__ __device__ inline int kstore_for(int64_t slots, int64_t nrow, int kmax, int vec) {
    if (!vec || slots < 1) return 0;
    const double per_k = 16.0 * (double)slots * (double)nrow;
    double k = kStoreBudget / per_k;
    if (k > kStoreMaxK) k = kStoreMaxK;
    if (k > kmax) k = kmax;
    return k >= 1.0 ? (int)k : 0;
}

__host__ __device__ inline void carve_workspace(void *base, int64_t n, int kl, int ku, int64_t slots, int kmax,
                                                int vec, int64_t npts_max, Workspace *w, int kstore = 0) {
    size_t off = 0;
    char *b = (char *)base;
    auto take = [&](size_t bytes) -> void * {
        void *p = (void *)(b + off);
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const int64_t nrow = padded_rows(n);
    const size_t ns = (size_t)nrow * (size_t)slots;
    const int wu = kl + ku + 1;
    w->slots = slots;
    w->nrow = nrow;
    w->kmax = kmax;
    w->vec = vec;
    w->queue = (unsigned long long *)take(sizeof(unsigned long long));
    w->count = (int64_t *)take(sizeof(int64_t));
    w->L = (double2 *)take(sizeof(double2) * ns * (size_t)(kl > 0 ? kl : 1));
    w->U = (double2 *)take(sizeof(double2) * ns * (size_t)wu);
    w->piv = (uint8_t *)take(ns);
    w->vu = (double2 *)take(sizeof(double2) * ns);
    w->vv = (double2 *)take(sizeof(double2) * ns);
    w->vy = (double2 *)take(sizeof(double2) * ns);
    w->eu = (int16_t *)take(sizeof(int16_t) * ns);
    w->ev = (int16_t *)take(sizeof(int16_t) * ns);
    w->ey = (int16_t *)take(sizeof(int16_t) * ns);
    w->hist = (double *)take(sizeof(double) * (size_t)kmax * 2 * (size_t)slots);
    if (vec) {
        w->vacc = (double2 *)take(sizeof(double2) * ns);
        w->vmeta = (double *)take(sizeof(double) * (size_t)kmax * 4 * (size_t)slots);
    } else {
        w->vacc = nullptr;
        w->vmeta = nullptr;
    }
    w->kstore = vec ? kstore : 0;
    w->ustore = w->kstore > 0 ? (double2 *)take(sizeof(double2) * ns * (size_t)w->kstore) : nullptr;
    if (npts_max > 0) {
        w->gk_list = (int64_t *)take(sizeof(int64_t) * (size_t)npts_max);
        w->gk_count = (int64_t *)take(sizeof(int64_t));
        w->st_lo = (double *)take(sizeof(double) * (size_t)npts_max);
        w->st_hi = (double *)take(sizeof(double) * (size_t)npts_max);
        w->st_np = (int32_t *)take(sizeof(int32_t) * (size_t)npts_max);
    } else {
        w->gk_list = nullptr;
        w->gk_count = nullptr;
        w->st_lo = w->st_hi = nullptr;
        w->st_np = nullptr;
    }
    w->npts_max = npts_max;
    w->blocksums = (int64_t *)take(8);   // extends to the end (sized by workspace_bytes)
}


// Kernel launchers (enqueue on stream; return hipError_t of the launch).
hipError_t launch_iota(int64_t *idx, int64_t npts, hipStream_t st);
hipError_t launch_set_count(int64_t *count, int64_t value, unsigned long long *queue, hipStream_t st);
hipError_t launch_compact_mask(const uint8_t *mask, int64_t npts, int64_t *idx, int64_t *count, int64_t *blocksums,
                               unsigned long long *queue, hipStream_t st);
// A second stream of a handle and the two events that fork work onto it and join it back.
struct SideStream {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
// The measurement hook of ps_set_timing_events (thread-local; NULL when off).
struct TimingEvents {
    hipEvent_t start = nullptr, end = nullptr;
};
TimingEvents &timing_events();
// side: if not NULL (and the call bisects), the Golub-Kahan launch runs on side->stream beside
// the bisection's second launch.
hipError_t launch_eval(const EvalArgs &a, const Workspace &ws, hipStream_t st, const SideStream *side);
// Batch: masks compaction for all matrices at once (masks: device array of nmat device
// pointers, NULL entries = full grid).
hipError_t launch_batch_compact(const MatDesc *mats, int nmat, int64_t max_npts, const uint8_t *const *masks,
                                int64_t *idx, int64_t *counts, int64_t *tilesums, hipStream_t st);
int64_t batch_tiles(int64_t max_npts);
hipError_t launch_backward(int64_t n, int kl, int ku, int64_t npts, const double *g, const double2 *u,
                           const double2 *v, double2 *grad_z, double2 *grad_band, double2 *partial, int real_a,
                           hipStream_t st);
int64_t backward_partial_rows(int64_t npts);
// Columns per shift of the z-gradient partials of the one-pass adjoint (after the band partials
// in its workspace: backward_partial_rows(npts) * n * (kl + ku + 1) + npts * cols complex values).
int64_t backward_zpart_cols(int64_t n);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);
int64_t contour_edge_tiles(int64_t nx, int64_t ny);
hipError_t launch_trace_init(int64_t m, const double2 *seeds, double2 *zt, int32_t *active, int32_t *count,
                             int32_t *flags, hipStream_t st);
hipError_t launch_trace_predict(int64_t m, const int32_t *active, const double2 *zc, const double2 *gc, double h,
                                double2 *zt, hipStream_t st);
hipError_t launch_trace_newton(int64_t m, const int32_t *active, double2 *zt, const double *sigma, const double2 *g,
                               double eps, hipStream_t st);
hipError_t launch_trace_accept(int64_t m, int32_t k, int32_t max_points, double eps, double h, const ps_grid *box,
                               const double2 *zt, const double *sigma, const double2 *g, int32_t *active, double2 *zc,
                               double2 *gc, double2 *z0, double2 *pts, int32_t *count, int32_t *flags,
                               hipStream_t st);
hipError_t launch_count_active(int64_t m, const int32_t *active, int32_t *n_active, hipStream_t st);
hipError_t launch_label_init(uint8_t *status, double *sig_out, int64_t npts, int64_t *evals, hipStream_t st);
hipError_t launch_label_mask(const uint8_t *status, int64_t nx, int64_t npts, int stride, uint8_t *mask,
                             hipStream_t st);
hipError_t launch_label_update(double a, double b, double c, double d, int64_t nx, int64_t ny, const int64_t *idx,
                               const int64_t *count, int64_t max_count, const double *sigma, const int32_t *info,
                               double eps, double tol_abs, double tol_rel, uint8_t *status, double *sig_out,
                               int64_t *evals, hipStream_t st);
hipError_t launch_label_finish(const uint8_t *status, uint8_t *label, int64_t npts, hipStream_t st);
hipError_t launch_blabel_init(const MatDesc *mats, int nmat, int64_t max_npts, uint8_t *status, double *sig_out,
                              uint8_t *mask_base, uint8_t **mask_ptrs, int64_t *evals, hipStream_t st);
hipError_t launch_blabel_mask(const MatDesc *mats, int nmat, int64_t max_npts, const uint8_t *status, int stride,
                              uint8_t *mask, hipStream_t st);
hipError_t launch_blabel_update(const MatDesc *mats, int nmat, int64_t max_count, const int64_t *idx,
                                const int64_t *counts, const double *sigma, const int32_t *info, double eps,
                                double tol_norm, double tol_rel, uint8_t *status, double *sig_out, int64_t *evals,
                                hipStream_t st);
hipError_t launch_contour_seeds(double a, double b, double c, double d, int64_t nx, int64_t ny, const double *sigma,
                                double eps, double2 *seeds, int64_t max_seeds, int64_t *count, int64_t *blocksums,
                                unsigned long long *scratch_queue, hipStream_t st);
hipError_t launch_newton_update(int64_t npts, double2 *z, const double *sigma, const double2 *grad_z, double eps,
                                hipStream_t st);

}  // namespace ps
