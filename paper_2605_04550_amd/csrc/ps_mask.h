// Internal interface of the mask-producer kernels (ps_mask.hip): the classifier of Sec. 3.2
// evaluated with the matrix cores, and its coarse-to-fine use over a grid (Sec. 3.5) that
// produces the restricted set R of Sec. 4.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ps {
namespace mlp {

// Parameter vector of the network (Sec. 3.2): per layer W (out x in, row-major) then b, in
// the order c1 (64x26), c2 (64x64), m1 (128x33), m2 (64x128), r4 (128x128), r5 (128x128),
// p7 (64x128), out (1x64).
constexpr int kNParam = 59841;
constexpr int kNGlobal = 30;

// Offsets (floats) of every W and b in the parameter vector.
constexpr int kWc1 = 0, kBc1 = kWc1 + 64 * 26;
constexpr int kWc2 = kBc1 + 64, kBc2 = kWc2 + 64 * 64;
constexpr int kWm1 = kBc2 + 64, kBm1 = kWm1 + 128 * 33;
constexpr int kWm2 = kBm1 + 128, kBm2 = kWm2 + 64 * 128;
constexpr int kW4 = kBm2 + 64, kB4 = kW4 + 128 * 128;
constexpr int kW5 = kB4 + 128, kB5 = kW5 + 128 * 128;
constexpr int kW7 = kB5 + 128, kB7 = kW7 + 64 * 128;
constexpr int kWout = kB7 + 64, kBout = kWout + 64;
static_assert(kBout + 1 == kNParam, "layer table");

// Packed weights (the A operands of the 16x16x4 MFMA): per layer, blocks [oc][kc] of 64 lanes
// x 4 floats, lane l element i = W[16 oc + l % 16][16 kc + 4 (l / 16) + i] (zero past K).
// m1 keeps only its three per-point columns (g1, g2, g3); its 30 global columns are folded
// into the bias per call.
constexpr int kPc1 = 0;                    // 64 x 32
constexpr int kPc2 = kPc1 + 64 * 32;       // 64 x 64
constexpr int kPm1 = kPc2 + 64 * 64;       // 128 x 16
constexpr int kPm2 = kPm1 + 128 * 16;      // 64 x 128
constexpr int kP4 = kPm2 + 64 * 128;       // 128 x 128
constexpr int kP5 = kP4 + 128 * 128;       // 128 x 128
constexpr int kP7 = kP5 + 128 * 128;       // 64 x 128
constexpr int kPackedFloats = kP7 + 64 * 128;

// Per-call state in the workspace (first kWsHeader bytes).
constexpr int kWsBfold = 0;                // float[128]: b_m1 + W_m1[:, :30] f
constexpr int kWsCent = 512;               // double2: eigenvalue centroid
constexpr int kWsTau = 528;                // double: tau_coarse
constexpr int kWsEvals = 536;              // int64: evaluations (when the caller passes none)
constexpr int kWsHeader = 1024;

struct Globals {
    double f[kNGlobal];
};

// Device tables of a batched call (nmat matrices on one grid); all NULL for a single matrix.
struct Batch {
    const double *gfeat;      // [nmat][30]
    const int64_t *eig_off;   // [nmat + 1]: matrix m's eigenvalues are eig[eig_off[m] .. eig_off[m+1])
};

struct GridArgs {
    double a, b, c, d;
    int64_t nx, ny;
};

hipError_t launch_pack(const float *raw, float *packed, hipStream_t s);

// Folded bias and centroid into each matrix's workspace header (matrix m's at ws + m * kWsHeader);
// the evaluation counters (evals[m], or the header's when evals is NULL) set to evals0.
hipError_t launch_prep(const float *raw, const Globals &gf, const Batch &bt, int nmat, const double2 *eig,
                       int64_t neig, char *ws, int64_t *evals, int64_t evals0, hipStream_t s);

// p at arbitrary points z[npts] (one matrix; launch_prep with nmat = 1 first).
hipError_t launch_points(const float *raw, const float *packed, const double2 *eig, int64_t neig, const char *ws,
                         const double2 *z, int64_t npts, float *prob, hipStream_t s);

// The hierarchical chain after launch_prep, for nmat matrices on one grid: coarse probabilities,
// tau_coarse, the refined cells, the thresholded and dilated mask.  Per-matrix outputs are
// consecutive: coarse [nmat][ncoarse], prob and mask [nmat][ny][nx], evals and tau [nmat].
hipError_t launch_mask(const float *raw, const float *packed, const Batch &bt, int nmat, const double2 *eig,
                       int64_t neig, char *ws, const GridArgs &g, int stride, int dilate, double coarse_q, double tau,
                       float *coarse, float *prob, uint8_t *mask, int64_t *evals, double *tau_coarse_out,
                       hipStream_t s);

// Threshold calibration (Sec. 3.6): candidates by value (ascending), counts in the workspace
// (nval * (ntau + 1) int64: labelled points per matrix, then the per-candidate bins).
constexpr int kCalMaxTau = 128;
constexpr int kCalMaxVal = 256;
struct Taus {
    double t[kCalMaxTau];
};
hipError_t launch_calibrate(const float *prob, const uint8_t *label, int nval, int64_t nx, int64_t ny, int rp, int rl,
                            const Taus &taus, int ntau, double median_min, double p10_min, int64_t *counts,
                            double *recall, double *median, double *p10, int32_t *index, hipStream_t s);

}  // namespace mlp
}  // namespace ps
