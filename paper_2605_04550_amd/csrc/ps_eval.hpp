// HIP device code for gfx950 (MI355X): sigma_min(zI - A) of a banded matrix at many shifts.
//
// One lane owns one shift at a time.  Per shift:
//   1. complex banded LU with partial pivoting of M = zI - A (gbtf2-style elimination
//      streamed row by row through a register window of (kl+1) x (kl+ku+1) entries),
//   2. Golub-Kahan bidiagonalisation of B = M^{-1} (inverse Lanczos):
//        p = B v_k - beta_{k-1} u_{k-1},  alpha_k = |p|,  u_k = p / alpha_k
//        q = B^H u_k - alpha_k v_k,       beta_k  = |q|,  v_{k+1} = q / beta_k
//      with B v = U^{-1} L^{-1} P^T v (forward sweep, backward sweep) and
//      B^H u = P L^{-H} U^{-H} u (forward sweep, backward sweep),
//   3. theta_k = largest eigenvalue of T_k = B_k^H B_k (B_k upper bidiagonal with
//      alpha on the diagonal, beta above it), found by a Sturm-safeguarded Newton iteration
//      on det(T_k - lambda I) from an upper bound; sigma_min(M) = 1/sqrt(theta) once theta
//      has converged.
// This reaches the quantity of the paper's Sec. 2.1 (sigma_min(z) = s_n of the SVD of
// zI - A) to a stated tolerance, without the O(n^3) dense SVD per shift.
//
// Memory layout: every per-shift array lives in a caller-provided workspace, tiled
// [wavefront][row][component][lane]: the 64 lanes of a wavefront sweep the same row at
// the same time, so each load or store of a wavefront is one contiguous 1 KiB (complex)
// segment, and consecutive rows of one wavefront are contiguous.  The band of A is read by
// all lanes at the same address (wave-uniform).
//
// Overflow safety: sigma_min can be far below the double range (it decays like
// 10^(-0.3 n) inside the pseudospectrum of a non-normal Toeplitz matrix), so every stored
// vector is kept in block floating point: one binary exponent per chunk of 8 rows.  A
// sweep carries a running exponent R; when a value would exceed 2^400 the chunk is redone
// row by row with rescaling, and readers bring each chunk to their own frame with ldexp.
//
// The persistent launch pulls shifts from a device counter; a lane whose shift has
// finished takes the next one at the start of the following cycle and factorises it
// during the forward sweep that the other lanes spend on their L solves.
//
// This header holds the persistent kernel (k_eval) and the complex helpers it shares with
// the small kernels.  ps_kernels.hip includes it for the helpers; each ps_eval_kl<K>.hip
// instantiates k_eval for one lower bandwidth, so the 75 instantiations compile in parallel.
#pragma once

#include "ps_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ps {

typedef double2 cd;

__device__ __forceinline__ cd C(double r, double i) { return make_double2(r, i); }
__device__ __forceinline__ cd czero() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ cd cmul(cd a, cd b) { return C(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)); }
__device__ __forceinline__ cd cconj(cd a) { return C(a.x, -a.y); }
// acc - a * b
__device__ __forceinline__ cd cfnma(cd a, cd b, cd acc) {
    return C(fma(a.y, b.y, fma(-a.x, b.x, acc.x)), fma(-a.y, b.x, fma(-a.x, b.y, acc.y)));
}
// acc - conj(a) * b
__device__ __forceinline__ cd cfnmac(cd a, cd b, cd acc) {
    return C(fma(-a.y, b.y, fma(-a.x, b.x, acc.x)), fma(a.y, b.x, fma(-a.x, b.y, acc.y)));
}
__device__ __forceinline__ double cabs1(cd a) { return fabs(a.x) + fabs(a.y); }
__device__ __forceinline__ double cabs2(cd a) { return fma(a.x, a.x, a.y * a.y); }
__device__ __forceinline__ cd cldexp(cd a, int e) { return C(ldexp(a.x, e), ldexp(a.y, e)); }
__device__ __forceinline__ cd cscale(cd a, double s) { return C(a.x * s, a.y * s); }
__device__ __forceinline__ cd csub(cd a, cd b) { return C(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cd crecip(cd a) {
    const double is = 1.0 / fmax(fabs(a.x), fabs(a.y));
    const double ar = a.x * is, ai = a.y * is;     // scaled so that ar^2 + ai^2 cannot under/overflow
    const double id = is / fma(ar, ar, ai * ai);
    return C(ar * id, -ai * id);
}
// Conditional swap written per component, so that it lowers to v_cndmask (a select of the
// whole struct would be lowered through private memory).
__device__ __forceinline__ void cswap_if(bool c, cd &a, cd &b) {
    const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
    a.x = c ? bx : ax;
    a.y = c ? by : ay;
    b.x = c ? ax : bx;
    b.y = c ? ay : by;
}

constexpr double kBig = 0x1p400;       // rescale when a sweep value reaches this
constexpr int kAfterRescale = 112;     // a rescaled value lands near 2^-112

// Shift needed to bring |t| (possibly Inf) well below kBig, given that t = r * s.
__device__ __forceinline__ int rescale_shift(double r_abs, double s_abs) {
    int e = ilogb(r_abs) + ilogb(s_abs) + 2;
    int sh = e + kAfterRescale;
    return sh < 64 ? 64 : sh;
}

// SplitMix64 (Steele, Lea, Flood 2014): counter-based start vector for inverse Lanczos.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__device__ __forceinline__ cd start_entry(uint64_t seed, int64_t i) {
    uint64_t h1 = splitmix64(seed ^ ((uint64_t)i * 0xD1B54A32D192ED03ull));
    uint64_t h2 = splitmix64(h1);
    return C((double)(h1 >> 11) * 0x1p-52 - 1.0, (double)(h2 >> 11) * 0x1p-52 - 1.0);
}

// Order in which a full-grid launch visits the grid: tiles of 8 x 8 points, tile rows top
// to bottom, tiles left to right, points row-major inside a tile (ragged tiles at the right
// and bottom edges).  Queue position id maps to the flat row-major index returned.  A
// wavefront takes 64 consecutive queue positions, i.e. one tile, whose shifts need similar
// Lanczos step counts because the count varies smoothly over the plane; a 64-point strip
// of one grid row spans a wider stretch and mixes short and long shifts.
__device__ __forceinline__ int64_t tile_flat(int64_t id, int64_t nx, int64_t ny) {
    const int64_t r0 = (id / (8 * nx)) * 8;          // first row of the tile row
    const int64_t h = ny - r0 < 8 ? ny - r0 : 8;       // its height
    const int64_t rem = id - r0 * nx;
    const int64_t ntx = (nx + 7) / 8;
    int64_t tx = rem / (8 * h);
    if (tx > ntx - 1) tx = ntx - 1;
    const int64_t tw = tx == ntx - 1 ? nx - 8 * (ntx - 1) : 8;
    const int64_t r2 = rem - tx * 8 * h;
    return (r0 + r2 / tw) * nx + 8 * tx + r2 % tw;
}

__device__ __forceinline__ cd grid_point(const EvalArgs &a, int64_t flat) {
    int64_t i = flat / a.nx, j = flat - i * a.nx;
    double x = a.nx > 1 ? __dadd_rn(a.ga, __ddiv_rn(__dmul_rn(a.gb - a.ga, (double)j), (double)(a.nx - 1))) : a.ga;
    double y = a.ny > 1 ? __dadd_rn(a.gc, __ddiv_rn(__dmul_rn(a.gd - a.gc, (double)i), (double)(a.ny - 1))) : a.gc;
    return C(x, y);
}

// Largest eigenvalue of the k x k symmetric tridiagonal T_k (diagonal hist[j][0], squared
// off-diagonal hist[j][1] between rows j and j+1) inside the bracket [lo, hi].
// One pass at lambda forms the LDL^T pivots d_j of T - lambda I: the number of positive
// pivots counts the eigenvalues above lambda (Sylvester inertia), and sum_j d_j'/d_j is
// d/dlambda log|det(T - lambda I)|, the Newton step for the largest root from above
// (monotone there).  Newton steps are taken while they at least halve; otherwise (a
// cluster of Ritz values) the bracket is bisected.  Returns the upper end of a bracket of
// relative width 2^-46.
// The same pass accumulates S = sum_j prod_{i>=j} l_i^2 (l_i = multipliers), so that
// x = (T - lambda I)^{-1} e_k has x_k^2 / |x|^2 = 1 / S: one step of inverse iteration
// from e_k, whose last component estimates y_k^2 for the top eigenvector y (it can only
// overestimate y_k^2 once y_k is below the shift's distance to theta).
struct TopEig {
    double theta;
    double yk2;
};

static __device__ TopEig top_eig(const double *hist, int64_t T, int64_t s, int k, double lo, double hi) {
    TopEig r;
    r.theta = hi;
    r.yk2 = 1.0;
    // Ritz values move little between checks: probe just above the previous value first
    // (lo > 0), widening the probe until it lies above every eigenvalue, then Newton.
    int probe = lo > 0.0 ? 0 : 3;          // probe p sits at lo (1 + 2^(10 p - 24))
    double lam = probe < 3 ? fmin(hi, lo * (1.0 + 0x1p-24)) : hi;
    double prev_step = INFINITY;
    double ssum_hi = 0.0;
    bool have_hi = false;
    for (int it = 0; it < 100; ++it) {
        double d = hist[s] - lam;
        double dd = -1.0;
        int cnt = d > 0.0;
        double rinv = 1.0 / d;
        double ssum = dd * rinv;
        double S = 1.0;
        for (int j = 1; j < k; ++j) {
            double b2 = hist[((int64_t)(j - 1) * 2 + 1) * T + s];
            double t = b2 * rinv;
            S = fma(S, t * rinv, 1.0);
            d = hist[((int64_t)j * 2 + 0) * T + s] - lam - t;
            dd = fma(t * dd, rinv, -1.0);
            cnt += d > 0.0;
            rinv = 1.0 / d;
            ssum = fma(dd, rinv, ssum);
        }
        if (cnt == 0) {
            hi = lam;
            r.theta = lam;
            r.yk2 = 1.0 / S;
            ssum_hi = ssum;
            have_hi = true;
        } else {
            lo = lam;
        }
        if (hi - lo <= 0x1p-46 * hi) break;
        if (!have_hi && probe < 2) {        // probe was below the top eigenvalue: widen it
            ++probe;
            lam = fmin(hi, lo * (1.0 + ldexp(1.0, 10 * probe - 24)));
            continue;
        }
        if (!have_hi && probe == 2) {       // fall back to the Gershgorin bound
            probe = 3;
            lam = hi;
            continue;
        }
        double next = 0.5 * (lo + hi);
        if (have_hi && ssum_hi > 0.0) {
            double step = 1.0 / ssum_hi;
            double cand = hi - step;
            if (cand > lo) {
                if (step <= 0x1p-47 * hi) next = hi * (1.0 - 0x1p-46);   // probe just below: closes the bracket
                else if (step <= 0.5 * prev_step) { next = cand; prev_step = step; }
            }
        }
        if (!(next > lo && next < hi)) break;
        lam = next;
    }
    return r;
}

struct Lane {
    int64_t pid;
    cd z;
    int k;            // number of alphas so far
    int next_check;   // Lanczos step at which theta is next evaluated
    int nchecks;
    int E0;           // reference exponent of the bidiagonal entries
    double theta;     // top Ritz value at the last check (units 2^(2 E0))
    double delta_prev, rho_prev;
    double ap_prev;   // alpha'_k in units of 2^E0
    double bp;        // beta'_k in units of 2^E0
    double gmax;      // Gershgorin bound over the closed rows of T_k
    double gopen;     // diagonal + left off-diagonal of the last row of T_k
    double a_m;       // alpha_k = a_m * 2^a_e, a_m in [1, 2)
    int a_e;
    double b_m;
    int b_e;
    int Eu, Ev, Ey;   // max row exponent of u, v, y
    double rdu, rdv;  // 1 / (norm mantissa) of u, v
    double nrm_h;     // squared norm of the start vector (fresh lanes)
    bool active, fresh, sing, exhausted;
    // Singular vectors (VEC): stage 0 runs the Lanczos process to convergence; stage 1
    // replays its first kfinal steps bit for bit from the same start vector, accumulating
    // v = sum_j p_j u_j (p = top left singular vector of B_kfinal) in vacc; stage 2 applies
    // one inverse-iteration step u = M^{-H} v / |M^{-H} v| and writes the pair.  With a
    // Lanczos-vector store (calls on few slots) stage 0 keeps every normalised u_j and v is
    // formed from them in one pass: no replay.  kfinal counts the kept vectors during stage 0.
    int stage;
    int kfinal;
    double vnorm2;    // |v|^2 of the accumulated vector (known after its last step)
    double vamax;     // largest |v_i|^2 so far (first index on ties)
    cd vph;           // the entry that attains it
    // Shifts bisected beforehand (calls with vectors): phase 2 while the lane computes the
    // singular pair from its bracket, 0 on the Golub-Kahan path.
    int phase;
    int nbis;         // bisection passes the bracket took
    double blo, bhi;  // bracket: blo < sigma_min (tested), sigma_min <= bhi
    // vectors after the bisection (phase 2): the step, sigma and flags to report, |x|^2
    int vit, vflags;
    double vsig, vx2;
    // batch mode: the matrix of the current shift
    int64_t n;
    const double2 *arow;
    double normA;
    double norm2A;
};

template <int KL, int KU, bool VEC, bool BATCH>
struct Kern {
    static constexpr int W = KL + KU + 1;

    // Order, band and Frobenius norm of the current shift's matrix (one matrix per launch,
    // or per shift in batch mode).
    static __device__ __forceinline__ int64_t nn(const EvalArgs &a, const Lane &ln) { return BATCH ? ln.n : a.n; }
    static __device__ __forceinline__ const double2 *band(const EvalArgs &a, const Lane &ln) {
        return BATCH ? ln.arow : a.arow;
    }
    static __device__ __forceinline__ double fro(const EvalArgs &a, const Lane &ln) { return BATCH ? ln.normA : a.normA; }
    static __device__ __forceinline__ double nrm2(const EvalArgs &a, const Lane &ln) {
        return BATCH ? ln.norm2A : a.norm2A;
    }

    // A lane is on the Golub-Kahan path unless it is computing a bisected shift's vectors.
    static __device__ __forceinline__ bool gk(const Lane &ln) { return ln.phase == 0; }

    // M[r][c] of M = zI - A from the row band (zero outside the matrix).
    static __device__ __forceinline__ cd mentry(const EvalArgs &a, const Lane &ln, int64_t r, int64_t c) {
        if (r >= nn(a, ln)) return czero();
        int64_t d = c - r + KL;
        if (d < 0 || d >= W) return czero();
        const cd z = ln.z;
        cd v = band(a, ln)[r * W + d];
        cd m = C(-v.x, -v.y);
        if (c == r) m = C(m.x + z.x, m.y + z.y);
        return m;
    }

    // Every sweep walks the rows in chunks of CH = 8: the loads of a whole chunk are issued
    // first (they do not depend on the recurrence), then the chunk's rows are computed.
    //
    // Block floating point: every stored vector carries one binary exponent per chunk of 8
    // rows (value of row r = mantissa * 2^e[r / 8]).  A chunk is first computed on the fast
    // path, where the sweep's running exponent R is fixed and every conversion is a
    // multiplication by a per-chunk factor, while one flag records whether any value left
    // the safe range (|x| >= 2^400, Inf or NaN).  Only if it did is the chunk recomputed on
    // the careful path from the state saved at its start, rescaling row by row; its outputs
    // are then brought to the chunk's final exponent before they are stored.
    static constexpr int CH = 8;

    static __device__ __forceinline__ double p2(int e) { return ldexp(1.0, e); }
    static __device__ __forceinline__ bool unsafe(cd v) { return !(cabs1(v) < kBig); }

    // ---------------------------------------------------------------- forward sweep 1
    // Fresh lanes: LU of M fused with the L solve of the start vector h (also stored as v).
    // Other lanes: y = L^{-1} P^T v_k with v_k read normalised.
    static __device__ void f1(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln) {
        const int64_t n = nn(a, ln), T = w.slots;
        cd b[KL + 1];
        cd Wm[KL + 1][W];
        int R = 0;
        double nrm_h = 0.0;
        const bool act = ln.active && gk(ln), fresh = ln.fresh;
        const bool lu = fresh && (!VEC || ln.stage == 0);   // a replay keeps the factors it has
        const double tiny = 0x1p-1000 * fmax(1.0, fro(a, ln) + cabs1(ln.z));
        bool sing = false;
        // input v: normalised stored v (mantissa * rdv * 2^(e - Ev)); fresh lanes read h
        const double rdv = fresh ? 1.0 : ln.rdv;
        const int Ev = fresh ? 0 : ln.Ev;
        const int64_t npad = ((n + CH - 1) / CH) * CH;
        auto gen = [&](int64_t i) -> cd {        // fresh lanes: start vector entry i, stored as v
            cd h = i < n ? start_entry(a.seed, i) : czero();   // padding rows stay zero
            w.vv[i * T + s] = h;
            nrm_h += cabs2(h);
            return h;
        };
        if (act) {
            if (fresh) {
                w.ev[s] = 0;
#pragma unroll
                for (int r = 0; r < KL; ++r) b[r] = gen(r);
                if (lu) {
#pragma unroll
                    for (int r = 0; r < KL; ++r)
#pragma unroll
                        for (int c = 0; c < W; ++c) Wm[r][c] = mentry(a, ln, r, c);
                }
            } else {
                const double f0 = rdv * p2((int)w.ev[s] - Ev);
#pragma unroll
                for (int r = 0; r < KL; ++r) b[r] = cscale(w.vv[r * T + s], f0);
            }
        }
        for (int64_t j0 = 0; j0 < npad; j0 += CH) {
            if (!act) continue;
            const int64_t q = j0 / CH;
            cd pin[CH];
            int pv[CH];
            cd Lr[CH][KL > 0 ? KL : 1];
            int ea = 0, eb = 0;
            if (!fresh) {
                ea = (int)w.ev[q * T + s];
                eb = KL > 0 ? (int)w.ev[(q + 1) * T + s] : ea;
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int64_t j = j0 + c;
                    pin[c] = w.vv[(j + KL) * T + s];
                    if (KL > 0) {
                        pv[c] = (int)w.piv[j * T + s];
#pragma unroll
                        for (int r = 0; r < KL; ++r) Lr[c][r] = w.L[(j * KL + r) * T + s];
                    } else {
                        pv[c] = 0;
                    }
                }
            } else {
                // LU rows of this chunk (stored once; multipliers and pivots kept for the solve)
                w.ev[(q + 1) * T + s] = 0;
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int64_t j = j0 + c;
                    pin[c] = gen(j + KL);
                    if (!lu) {       // replay: the multipliers and pivots stored by the LU
                        if (KL > 0) {
                            pv[c] = (int)w.piv[j * T + s];
#pragma unroll
                            for (int r = 0; r < KL; ++r) Lr[c][r] = w.L[(j * KL + r) * T + s];
                        } else {
                            pv[c] = 0;
                        }
                        continue;
                    }
#pragma unroll
                    for (int cc = 0; cc < W; ++cc) Wm[KL][cc] = mentry(a, ln, j + KL, j + cc);
                    double best = cabs1(Wm[0][0]);
                    int p = 0;
#pragma unroll
                    for (int r = 1; r <= KL; ++r) {
                        double v = cabs1(Wm[r][0]);
                        if (v > best) { best = v; p = r; }
                    }
#pragma unroll
                    for (int r = 1; r <= KL; ++r)
#pragma unroll
                        for (int cc = 0; cc < W; ++cc) cswap_if(p == r, Wm[0][cc], Wm[r][cc]);
                    // rows past n are zero rows: their pivot is 0 and they stay inert
                    const bool ok = best >= tiny;
                    sing = sing || (!ok && j < n);
                    const cd rc = crecip(Wm[0][0]);
                    const cd inv = C(ok ? rc.x : 0.0, ok ? rc.y : 0.0);
#pragma unroll
                    for (int r = 1; r <= KL; ++r) Lr[c][r - 1] = cmul(Wm[r][0], inv);
#pragma unroll
                    for (int r = 1; r <= KL; ++r)
#pragma unroll
                        for (int cc = 1; cc < W; ++cc) Wm[r][cc] = cfnma(Lr[c][r - 1], Wm[0][cc], Wm[r][cc]);
                    w.U[(j * W + 0) * T + s] = inv;
#pragma unroll
                    for (int cc = 1; cc < W; ++cc) w.U[(j * W + cc) * T + s] = Wm[0][cc];
#pragma unroll
                    for (int r = 0; r < KL; ++r) w.L[(j * KL + r) * T + s] = Lr[c][r];
                    w.piv[j * T + s] = (uint8_t)p;
                    pv[c] = p;
#pragma unroll
                    for (int r = 0; r < KL; ++r) {
#pragma unroll
                        for (int cc = 0; cc < W - 1; ++cc) Wm[r][cc] = Wm[r + 1][cc + 1];
                        Wm[r][W - 1] = czero();
                    }
                }
            }
            // L solve of the chunk
            cd bs[KL + 1];
#pragma unroll
            for (int r = 0; r <= KL; ++r) bs[r] = b[r];
            const int Rs = R;
            cd ob[CH];
            bool flag = false;
            {
                const double fa = rdv * p2(ea - Ev - R), fb = rdv * p2(eb - Ev - R);
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    b[KL] = cscale(pin[c], c + KL < CH ? fa : fb);
#pragma unroll
                    for (int r = 1; r <= KL; ++r) cswap_if(pv[c] == r, b[0], b[r]);
                    const cd y = b[0];
                    flag = flag || unsafe(y);
                    ob[c] = y;
#pragma unroll
                    for (int r = 1; r <= KL; ++r) b[r] = cfnma(Lr[c][r - 1], y, b[r]);
#pragma unroll
                    for (int r = 0; r < KL; ++r) b[r] = b[r + 1];
                }
            }
            if (flag) {   // careful path: rescale row by row
#pragma unroll
                for (int r = 0; r <= KL; ++r) b[r] = bs[r];
                R = Rs;
                int Rc[CH];
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    b[KL] = cscale(pin[c], rdv * p2((c + KL < CH ? ea : eb) - Ev - R));
#pragma unroll
                    for (int r = 1; r <= KL; ++r) cswap_if(pv[c] == r, b[0], b[r]);
                    cd y = b[0];
                    if (unsafe(y)) {
                        const int sh = rescale_shift(cabs1(y), 1.0);
#pragma unroll
                        for (int r = 0; r <= KL; ++r) b[r] = cldexp(b[r], -sh);
                        y = b[0];
                        R += sh;
                    }
                    ob[c] = y;
                    Rc[c] = R;
#pragma unroll
                    for (int r = 1; r <= KL; ++r) b[r] = cfnma(Lr[c][r - 1], y, b[r]);
#pragma unroll
                    for (int r = 0; r < KL; ++r) b[r] = b[r + 1];
                }
#pragma unroll
                for (int c = 0; c < CH; ++c) ob[c] = cldexp(ob[c], Rc[c] - R);
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) w.vy[(j0 + c) * T + s] = ob[c];
            w.ey[q * T + s] = (int16_t)R;
        }
        if (act) {
            ln.Ey = R;
            if (fresh) {
                ln.nrm_h = nrm_h;
                if (lu) ln.sing = sing;
                ln.Ev = 0;
                ln.rdv = 1.0 / sqrt(nrm_h);
            }
        }
    }

    // ---------------------------------------------------------------- backward sweep 1
    // x = U^{-1} y (= B v_k), out = x - beta u_{k-1}; out stored unnormalised; returns
    // |out|^2 = acc * 2^(2 Eacc).
    static __device__ void b1(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln, double &acc_out,
                              int &eacc_out) {
        const int64_t n = nn(a, ln), T = w.slots;
        const bool act = ln.active && gk(ln) && !ln.sing;
        const bool sub = !ln.fresh;
        int R = ln.Ey;
        cd xw[W];
#pragma unroll
        for (int d = 0; d < W; ++d) xw[d] = czero();
        double acc = 0.0;
        int Eacc = R;
        // u_{k-1} is read and u_k written in place (row i is read before it is written)
        double2 *uout = w.vu;
        int16_t *euout = w.eu;
        const double2 *uold = w.vu;
        const int16_t *euold = w.eu;
        const double rd_old = ln.rdu;
        const int E_old = ln.Eu;
        const double bm = ln.b_m;
        const int be = ln.b_e;
        const int64_t npad = ((n + CH - 1) / CH) * CH;
        for (int64_t q = npad / CH - 1; q >= 0; --q) {
            if (!act) continue;
            const int64_t i0 = q * CH + CH - 1;
            cd Ur[CH][W];
            cd yr[CH], ur[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int64_t i = i0 - c;
#pragma unroll
                for (int d = 0; d < W; ++d) Ur[c][d] = w.U[(i * W + d) * T + s];
                yr[c] = w.vy[i * T + s];
                ur[c] = uold[i * T + s];          // read even when unused (no branch); selected away below
            }
            const int ey = (int)w.ey[q * T + s];
            const int eu = (int)euold[q * T + s];
            cd xs[W];
#pragma unroll
            for (int d = 0; d < W; ++d) xs[d] = xw[d];
            const int Rs = R;
            cd ob[CH];
            bool flag = false;
            int eo;
            {
                const int es = R > be ? R : be;
                eo = sub ? es : R;
                const double fy = p2(ey - R), ft = p2(R - es);
                const double fu = bm * rd_old * p2(eu - E_old + be - es);
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    // the previous row's x (xw[1]) enters last: the row-to-row chain is one
                    // complex multiply-add and the scaling by 1/u_ii
                    cd rhs = cscale(yr[c], fy);
#pragma unroll
                    for (int d = W - 1; d >= 1; --d) rhs = cfnma(Ur[c][d], xw[d], rhs);
                    const cd t = cmul(rhs, Ur[c][0]);
                    flag = flag || unsafe(t);
                    const cd o = C(fma(-fu, ur[c].x, ft * t.x), fma(-fu, ur[c].y, ft * t.y));
                    ob[c] = sub ? o : t;
                    if constexpr (W > 1) {
#pragma unroll
                        for (int d = W - 1; d >= 2; --d) xw[d] = xw[d - 1];
                        xw[1] = t;
                    }
                }
            }
            if (flag) {   // careful path
#pragma unroll
                for (int d = 0; d < W; ++d) xw[d] = xs[d];
                R = Rs;
                int Ec[CH];
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    cd rhs = cldexp(yr[c], ey - R);
#pragma unroll
                    for (int d = W - 1; d >= 1; --d) rhs = cfnma(Ur[c][d], xw[d], rhs);
                    const cd inv = Ur[c][0];
                    cd t = cmul(rhs, inv);
                    if (unsafe(t)) {
                        const int sh = rescale_shift(cabs1(rhs), cabs1(inv));
                        rhs = cldexp(rhs, -sh);
#pragma unroll
                        for (int d = 1; d < W; ++d) xw[d] = cldexp(xw[d], -sh);
                        R += sh;
                        t = cmul(rhs, inv);
                    }
                    const int es = R > be ? R : be;
                    const cd tt = cldexp(t, R - es);
                    const cd bu = cscale(cldexp(ur[c], eu - E_old + be - es), bm * rd_old);
                    ob[c] = sub ? csub(tt, bu) : t;
                    Ec[c] = sub ? es : R;
                    if constexpr (W > 1) {
#pragma unroll
                        for (int d = W - 1; d >= 2; --d) xw[d] = xw[d - 1];
                        xw[1] = t;
                    }
                }
                eo = Ec[CH - 1];
#pragma unroll
                for (int c = 0; c < CH; ++c) ob[c] = cldexp(ob[c], Ec[c] - eo);
            }
            double cs = 0.0;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                uout[(i0 - c) * T + s] = ob[c];
                cs = fma(ob[c].x, ob[c].x, fma(ob[c].y, ob[c].y, cs));
            }
            euout[q * T + s] = (int16_t)eo;
            acc = ldexp(acc, 2 * (Eacc - eo)) + cs;     // exponents of a sweep's outputs never decrease
            Eacc = eo;
        }
        acc_out = acc;
        eacc_out = Eacc;
    }

    // ---------------------------------------------------------------- forward sweep 2
    // y = U^{-H} u_k (u_k read normalised), column-oriented forward substitution.
    // VEC stage 1 also adds p_k u_k to the accumulated singular vector (vacc); stage 2 solves
    // with the accumulated vector itself (plain doubles, exponent 0) instead of u_k.
    static __device__ void f2(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln) {
        const int64_t n = nn(a, ln), T = w.slots;
        const bool act = ln.active && gk(ln);
        const bool fin = VEC && ln.stage == 2;
        const bool rep = VEC && ln.stage == 1;
        // first pass with a Lanczos-vector store: keep the normalised u_k (the values a replay
        // would accumulate) in ustore[k - 1]
        const bool sto = VEC && ln.stage == 0 && act && w.ustore != nullptr && ln.k >= 1 && ln.k <= w.kstore;
        double2 *const ust = sto ? w.ustore + (int64_t)(ln.k - 1) * w.nrow * w.slots : nullptr;
        const double2 *uin = fin ? w.vacc : w.vu;
        const int16_t *euin = w.eu;
        const double rdu = fin ? 1.0 / sqrt(ln.vnorm2) : ln.rdu;
        const int Eu = fin ? 0 : ln.Eu;
        auto ex = [&](int64_t q) -> int { return fin ? 0 : (int)euin[q * T + s]; };
        // replay: vacc[r] (+)= p_k u_k[r]; the last replayed step also yields |v|^2 and the
        // first entry of largest modulus (for the phase convention)
        const bool first = rep && ln.k == 1, lastk = rep && ln.k == ln.kfinal;
        // (a lane held out of this sweep can be in the replay with k = 0: no read then)
        const double cf = act && rep && ln.k >= 1 ? w.vmeta[((int64_t)(ln.k - 1) * 4 + 3) * T + s] : 0.0;
        double vn = 0.0, vam = -1.0;
        cd vph = C(1.0, 0.0);
        auto accum = [&](int64_t r, cd un) {
            cd v = C(cf * un.x, cf * un.y);
            if (!first) {
                const cd o = w.vacc[r * T + s];
                v = C(o.x + v.x, o.y + v.y);
            }
            w.vacc[r * T + s] = v;
            if (lastk && r < n) {
                const double m = cabs2(v);
                vn += m;
                if (m > vam) {
                    vam = m;
                    vph = v;
                }
            }
        };
        int R = 0;
        cd acc[W];
        const int64_t npad = ((n + CH - 1) / CH) * CH;
        if (act) {
            const double f0 = rdu * p2(ex(0) - Eu);
#pragma unroll
            for (int d = 0; d < W - 1; ++d) {
                acc[d] = cscale(uin[d * T + s], f0);
                if (rep) accum(d, acc[d]);
                if (sto) ust[d * T + s] = acc[d];
            }
        }
        for (int64_t i0 = 0; i0 < npad; i0 += CH) {
            if (!act) continue;
            const int64_t q = i0 / CH;
            cd Ur[CH][W];
            cd pin[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int64_t i = i0 + c;
#pragma unroll
                for (int d = 0; d < W; ++d) Ur[c][d] = w.U[(i * W + d) * T + s];
                pin[c] = uin[(i + W - 1) * T + s];
            }
            const int ea = ex(q);
            const bool last = i0 + CH >= npad;                 // rows at or past npad were never written
            const int eb = (W > 1 && !last) ? ex(q + 1) : ea;
            if (rep || sto) {
                const double ga = rdu * p2(ea - Eu), gb = rdu * p2(eb - Eu);
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    if (c + W - 1 < CH || !last) {
                        const cd un = cscale(pin[c], c + W - 1 < CH ? ga : gb);
                        if (rep) accum(i0 + c + W - 1, un);
                        if (sto) ust[(i0 + c + W - 1) * T + s] = un;
                    }
            }
            cd as[W];
#pragma unroll
            for (int d = 0; d < W; ++d) as[d] = acc[d];
            const int Rs = R;
            cd ob[CH];
            bool flag = false;
            {
                const double fa = rdu * p2(ea - Eu - R), fb = last ? 0.0 : rdu * p2(eb - Eu - R);
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const cd x = cscale(pin[c], c + W - 1 < CH ? fa : fb);
                    acc[W - 1] = (c + W - 1 < CH || !last) ? x : czero();
                    const cd wv = cmul(acc[0], cconj(Ur[c][0]));
                    flag = flag || unsafe(wv);
                    ob[c] = wv;
#pragma unroll
                    for (int d = 1; d < W; ++d) acc[d] = cfnmac(Ur[c][d], wv, acc[d]);
#pragma unroll
                    for (int d = 0; d < W - 1; ++d) acc[d] = acc[d + 1];
                }
            }
            if (flag) {   // careful path
#pragma unroll
                for (int d = 0; d < W; ++d) acc[d] = as[d];
                R = Rs;
                int Rc[CH];
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const bool in = c + W - 1 < CH || !last;
                    const cd x = cscale(pin[c], rdu * p2((c + W - 1 < CH ? ea : eb) - Eu - R));
                    acc[W - 1] = in ? x : czero();
                    const cd inv = Ur[c][0];
                    cd wv = cmul(acc[0], cconj(inv));
                    if (unsafe(wv)) {
                        const int sh = rescale_shift(cabs1(acc[0]), cabs1(inv));
#pragma unroll
                        for (int d = 0; d < W; ++d) acc[d] = cldexp(acc[d], -sh);
                        R += sh;
                        wv = cmul(acc[0], cconj(inv));
                    }
                    ob[c] = wv;
                    Rc[c] = R;
#pragma unroll
                    for (int d = 1; d < W; ++d) acc[d] = cfnmac(Ur[c][d], wv, acc[d]);
#pragma unroll
                    for (int d = 0; d < W - 1; ++d) acc[d] = acc[d + 1];
                }
#pragma unroll
                for (int c = 0; c < CH; ++c) ob[c] = cldexp(ob[c], Rc[c] - R);
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) w.vy[(i0 + c) * T + s] = ob[c];
            w.ey[q * T + s] = (int16_t)R;
        }
        if (act) ln.Ey = R;
        if (sto) ln.kfinal = ln.k;      // Lanczos vectors kept so far (until the first pass ends)
        if (act && lastk) {
            ln.vnorm2 = vn;
            ln.vamax = vam;
            ln.vph = vph;
        }
    }

    // ---------------------------------------------------------------- backward sweep 2
    // q = P L^{-H} y - alpha_k v_k; v updated in place; returns |q|^2 = acc * 2^(2 Eacc).
    // Step j finalises entry j + kl, so the steps of output chunk p are j = 8p+7-kl .. 8p-kl;
    // the kl steps above the top chunk run first (their outputs lie past the padding), and
    // steps j < 0 carry zero data (they only flush the window).
    static __device__ void b2(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln, double &acc_out,
                              int &eacc_out) {
        const int64_t n = nn(a, ln), T = w.slots;
        const bool act = ln.active && gk(ln);
        // the final solve of the singular vectors (stage 2) has no -alpha v term: v is not read
        const bool fin = VEC && ln.stage == 2;
        int R = ln.Ey;
        cd b[KL + 1];
#pragma unroll
        for (int r = 0; r <= KL; ++r) b[r] = czero();
        double acc = 0.0;
        int Eacc = R;
        const double am = ln.a_m;
        const int ae = ln.a_e;
        const double rdv = ln.rdv;
        const int Ev = ln.Ev;
        const int64_t npad = ((n + CH - 1) / CH) * CH;
        // one step of the L^H P sweep at row j (careful form, used for the top kl steps)
        auto step_careful = [&](int64_t j, int ey) {
            cd b0 = cldexp(w.vy[j * T + s], ey - R);
#pragma unroll
            for (int r = 1; r <= KL; ++r) b0 = cfnmac(w.L[(j * KL + (r - 1)) * T + s], b[r], b0);
            if (unsafe(b0)) {
                const int sh = rescale_shift(cabs1(b0), 1.0);
                b0 = cldexp(b0, -sh);
#pragma unroll
                for (int r = 1; r <= KL; ++r) b[r] = cldexp(b[r], -sh);
                R += sh;
            }
            b[0] = b0;
            const int p = w.piv[j * T + s];
#pragma unroll
            for (int r = 1; r <= KL; ++r) cswap_if(p == r, b[0], b[r]);
#pragma unroll
            for (int r = KL; r >= 1; --r) b[r] = b[r - 1];
        };
        if (act && KL > 0) {
            const int eyt = (int)w.ey[(npad / CH - 1) * T + s];
            for (int64_t j = npad - 1; j >= npad - KL; --j) step_careful(j, eyt);
        }
        for (int64_t pq = npad / CH - 1; pq >= 0; --pq) {
            if (!act) continue;
            const int64_t jtop = pq * CH + CH - 1 - KL;
            cd yr[CH], vr[CH];
            int pv[CH];
            cd Lr[CH][KL > 0 ? KL : 1];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int64_t j = jtop - c;
                const int64_t jc = j >= 0 ? j : 0;              // steps j < 0 carry zero data
                const bool in = j >= 0;
                const cd y = w.vy[jc * T + s];
                yr[c] = C(in ? y.x : 0.0, in ? y.y : 0.0);
                if (KL > 0) {
                    pv[c] = in ? (int)w.piv[jc * T + s] : 0;
#pragma unroll
                    for (int r = 0; r < KL; ++r) {
                        const cd l = w.L[(jc * KL + r) * T + s];
                        Lr[c][r] = C(in ? l.x : 0.0, in ? l.y : 0.0);
                    }
                } else {
                    pv[c] = 0;
                }
                vr[c] = fin ? czero() : w.vv[(j + KL) * T + s];
            }
            const int eyh = (int)w.ey[pq * T + s];                  // rows >= 8 pq
            const int eyl = pq > 0 ? (int)w.ey[(pq - 1) * T + s] : eyh;   // rows < 8 pq
            const int evp = (int)w.ev[pq * T + s];
            cd bs[KL + 1];
#pragma unroll
            for (int r = 0; r <= KL; ++r) bs[r] = b[r];
            const int Rs = R;
            cd ob[CH];
            bool flag = false;
            int eo;
            {
                const int es = R > ae ? R : ae;
                eo = es;
                const double fh = p2(eyh - R), fl = p2(eyl - R), fbv = p2(R - es);
                const double fv = fin ? 0.0 : am * rdv * p2(evp - Ev + ae - es);
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    // row j = jtop - c lies in chunk pq iff c + kl < 8
                    cd b0 = cscale(yr[c], c + KL < CH ? fh : fl);
#pragma unroll
                    for (int r = 1; r <= KL; ++r) b0 = cfnmac(Lr[c][r - 1], b[r], b0);
                    flag = flag || unsafe(b0);
                    b[0] = b0;
#pragma unroll
                    for (int r = 1; r <= KL; ++r) cswap_if(pv[c] == r, b[0], b[r]);
                    const cd val = b[KL];
                    ob[c] = C(fma(-fv, vr[c].x, fbv * val.x), fma(-fv, vr[c].y, fbv * val.y));
#pragma unroll
                    for (int r = KL; r >= 1; --r) b[r] = b[r - 1];
                }
            }
            if (flag) {   // careful path
#pragma unroll
                for (int r = 0; r <= KL; ++r) b[r] = bs[r];
                R = Rs;
                int Ec[CH];
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    cd b0 = cldexp(yr[c], (c + KL < CH ? eyh : eyl) - R);
#pragma unroll
                    for (int r = 1; r <= KL; ++r) b0 = cfnmac(Lr[c][r - 1], b[r], b0);
                    if (unsafe(b0)) {
                        const int sh = rescale_shift(cabs1(b0), 1.0);
                        b0 = cldexp(b0, -sh);
#pragma unroll
                        for (int r = 1; r <= KL; ++r) b[r] = cldexp(b[r], -sh);
                        R += sh;
                    }
                    b[0] = b0;
#pragma unroll
                    for (int r = 1; r <= KL; ++r) cswap_if(pv[c] == r, b[0], b[r]);
                    const int es = R > ae ? R : ae;
                    const cd val = cldexp(b[KL], R - es);
                    const cd vo = fin ? czero() : cscale(cldexp(vr[c], evp - Ev + ae - es), am * rdv);
                    ob[c] = csub(val, vo);
                    Ec[c] = es;
#pragma unroll
                    for (int r = KL; r >= 1; --r) b[r] = b[r - 1];
                }
                eo = Ec[CH - 1];
#pragma unroll
                for (int c = 0; c < CH; ++c) ob[c] = cldexp(ob[c], Ec[c] - eo);
            }
            double cs = 0.0;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                w.vv[(pq * CH + CH - 1 - c) * T + s] = ob[c];
                cs = fma(ob[c].x, ob[c].x, fma(ob[c].y, ob[c].y, cs));
            }
            w.ev[pq * T + s] = (int16_t)eo;
            acc = ldexp(acc, 2 * (Eacc - eo)) + cs;
            Eacc = eo;
        }
        acc_out = acc;
        eacc_out = Eacc;
    }

    // ---------------------------------------------------------------- shifts bisected beforehand
    // Calls with singular vectors first run the bisection kernel over every shift (ps_bisect.hpp:
    // the inertia bisection on H = M^H M, sigma_min^2 its smallest eigenvalue), which saves each
    // final bracket lo < sigma_min <= hi, or -1 for a shift below the bisection's rounding limit.
    // This kernel starts from those brackets: the singular pair of a bisected shift comes from
    // inverse iteration on H - lo^2 I (below); the others take the Golub-Kahan path.
    static constexpr bool BIS = VEC && (KL + KU) >= 1;
    static constexpr int HB = KL + KU;          // half-bandwidth of H

    // 1 / d to full precision: the hardware reciprocal (about 24 correct bits) and two
    // Newton steps (each doubles the correct bits), without the library's special-case paths
    // (d is a positive normal number wherever the result is used).
    static __device__ __forceinline__ double recip(double d) {
        double r = __builtin_amdgcn_rcp(d);
        r = fma(r, fma(-d, r, 1.0), r);
        return fma(r, fma(-d, r, 1.0), r);
    }

    // A fresh shift: straight to its singular pair if the bisection kernel settled its bracket;
    // the Golub-Kahan path otherwise (below the bisection's limit, or no brackets given).
    static __device__ void bis_begin(const EvalArgs &a, Lane &ln) {
        ln.phase = 0;
        ln.nbis = 0;
        if (!BIS || !a.bisect || !a.brk_np) return;
        const int np = a.brk_np[ln.pid];
        if (np < 0) return;
        ln.phase = 1;
        ln.nbis = np;
        ln.blo = a.brk_lo[ln.pid];
        ln.bhi = a.brk_hi[ln.pid];
        const double target = a.tol_norm * fro(a, ln) + a.tol_rel * ln.blo;
        finish_bis(a, ln, 0.5 * (ln.blo + ln.bhi), ln.bhi - ln.blo <= target ? 0 : 2);
    }

    static __device__ void finish_bis(const EvalArgs &a, Lane &ln, double sigma, int flags) {
        flags |= PS_PT_BISECT | (ln.nbis << 8);
        if (VEC) {                    // the singular pair follows (vec_cycle)
            ln.phase = 2;
            ln.vit = 0;
            ln.vsig = sigma;
            ln.vflags = flags;
            return;
        }
        a.sigma[ln.pid] = sigma;
        if (a.info) a.info[ln.pid] = flags;
        if (a.iters) a.iters[ln.pid] = 0;
        if (a.sens) a.sens[ln.pid] = (uint8_t)(sigma <= a.eps);
        ln.active = false;
        ln.phase = 0;
    }

    // ---------------------------------------------------------------- vectors after the bisection
    // With vectors wanted, a bisection shift ends with lo < sigma_min <= hi, hi - lo <= target.
    // Its singular pair then comes from inverse iteration on H - lo^2 I = L D L^H (the test at
    // lo passed, so this factorisation exists): the top eigenvalue 1 / (sigma_min^2 - lo^2) of
    // (H - lo^2 I)^{-1} exceeds the next one by the factor (sigma_2^2 - lo^2) / (sigma_min^2 -
    // lo^2), the gap to sigma_2 over the bracket width (1e3 and more where sigma_2 / sigma_min
    // - 1 > 1e-5), so kInvIter steps from the start vector h give v; then u = M v / |M v|.  The
    // factor is stored in the U array (U[i][0].x = 1/d_i, U[i][e] = L[i][i-e]), x in vv, the
    // solves' middle vector in vy.  Phase convention as on the Golub-Kahan path.  One cycle of
    // the lane does one unit: the factorisation, one step, or the output.
    static constexpr int kInvIter = 4;

    // M[r][c] of M = zI - A (zero outside the matrix).
    static __device__ __forceinline__ cd mval(const EvalArgs &a, const Lane &ln, int64_t r, int64_t c) {
        const int64_t n = nn(a, ln);
        if (r < 0 || r >= n || c < 0 || c >= n) return czero();
        const int64_t d = c - r + KL;
        if (d < 0 || d >= W) return czero();
        const cd v = band(a, ln)[r * W + d];
        return r == c ? C(ln.z.x - v.x, ln.z.y - v.y) : C(-v.x, -v.y);
    }

    // Factorisation of H - sh I stored in U; x = h (the start vector) into vv; returns |h|^2.
    static __device__ double vec_factor(const EvalArgs &a, const Workspace &w, int64_t s, const Lane &ln, double sh) {
        const int64_t n = nn(a, ln), T = w.slots;
        constexpr int HA = HB > 0 ? HB : 1;
        cd P[HA][HA];
        double Q[HA];
#pragma unroll
        for (int e = 0; e < HA; ++e) {
            Q[e] = 0.0;
#pragma unroll
            for (int f = 0; f < HA; ++f) P[e][f] = czero();
        }
        double h2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            cd h[HB + 1];
#pragma unroll
            for (int e = 0; e <= HB; ++e) {
                double hx = 0.0, hy = 0.0;
#pragma unroll
                for (int t = 0; t <= HB - e; ++t) {
                    const int64_t r = i - KU + t;
                    const cd mi = mval(a, ln, r, i), mj = mval(a, ln, r, i - e);
                    hx = fma(mi.x, mj.x, fma(mi.y, mj.y, hx));
                    hy = fma(mi.x, mj.y, fma(-mi.y, mj.x, hy));
                }
                h[e] = C(hx, e > 0 ? hy : 0.0);
            }
            double d = h[0].x - sh;
            cd wv[HB + 1], lv[HB + 1];
#pragma unroll
            for (int e = HB; e >= 1; --e) {
                cd acc = h[e];
#pragma unroll
                for (int e2 = HB; e2 > e; --e2) acc = cfnmac(P[e - 1][e2 - e - 1], wv[e2], acc);
                wv[e] = acc;
                lv[e] = cscale(acc, Q[e - 1]);
                d = fma(-acc.x, lv[e].x, fma(-acc.y, lv[e].y, d));
            }
#pragma unroll
            for (int e = HB - 1; e >= 1; --e) {
                Q[e] = Q[e - 1];
#pragma unroll
                for (int f = 0; f + e + 1 < HB; ++f) P[e][f] = P[e - 1][f];
            }
            Q[0] = recip(d);
#pragma unroll
            for (int f = 1; f < HB; ++f) P[0][f - 1] = lv[f];
            w.U[(i * W + 0) * T + s] = C(Q[0], 0.0);
#pragma unroll
            for (int e = 1; e <= HB; ++e) w.U[(i * W + e) * T + s] = lv[e];
            const cd x = start_entry(a.seed, i);
            w.vv[i * T + s] = x;
            h2 += cabs2(x);
        }
        return h2;
    }

    // One step x <- (H - sh I)^{-1} (x / |x|) (forward L solve and the 1/d scaling into vy, then
    // the backward L^H solve into vv); returns the new |x|^2 and records in vamax / vph the first
    // entry of largest modulus.
    // The two solves run in chunks of VC rows: a chunk's workspace loads are all issued before
    // its rows are computed, so a lane waits for memory once per chunk rather than once per row
    // (the recurrence itself is short; one lane per shift has nothing else to hide the wait).
    // The workspace holds rows up to round_up(n, 8) + 8, so a chunk may read past row n - 1
    // (values unused); going backward, rows below 0 are clamped to row 0 (values unused).
    static constexpr int VC = HB <= 2 ? 8 : HB <= 4 ? 4 : 2;

    static __device__ double vec_step(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln, double scale) {
        const int64_t n = nn(a, ln), T = w.slots;
        constexpr int HA = HB > 0 ? HB : 1;
        cd y[HA];
#pragma unroll
        for (int e = 0; e < HA; ++e) y[e] = czero();   // y[e-1] = y_{i-e}
        for (int64_t i0 = 0; i0 < n; i0 += VC) {
            cd vin[VC], uu[VC][HB + 1];
#pragma unroll
            for (int r = 0; r < VC; ++r) {
                const int64_t i = i0 + r;
                vin[r] = w.vv[i * T + s];
#pragma unroll
                for (int e = 0; e <= HB; ++e) uu[r][e] = w.U[(i * W + e) * T + s];
            }
#pragma unroll
            for (int r = 0; r < VC; ++r) {
                const int64_t i = i0 + r;
                if (i < n) {
                    cd acc = cscale(vin[r], scale);
#pragma unroll
                    for (int e = HB; e >= 1; --e) acc = cfnma(uu[r][e], y[e - 1], acc);   // y[0] last
#pragma unroll
                    for (int e = HB - 1; e >= 1; --e) y[e] = y[e - 1];
                    y[0] = acc;
                    w.vy[i * T + s] = cscale(acc, uu[r][0].x);
                }
            }
        }
        cd x[HA];
#pragma unroll
        for (int e = 0; e < HA; ++e) x[e] = czero();   // x[e-1] = x_{i+e}
        double x2 = 0.0, am = -1.0;
        cd ph = C(1.0, 0.0);
        for (int64_t i0 = n - 1; i0 >= 0; i0 -= VC) {
            cd yin[VC], uu[VC][HB + 1];
#pragma unroll
            for (int r = 0; r < VC; ++r) {
                const int64_t i = i0 - r >= 0 ? i0 - r : 0;
                yin[r] = w.vy[i * T + s];
#pragma unroll
                for (int e = 1; e <= HB; ++e) uu[r][e] = w.U[((i + e) * W + e) * T + s];
            }
#pragma unroll
            for (int r = 0; r < VC; ++r) {
                const int64_t i = i0 - r;
                if (i >= 0) {
                    cd acc = yin[r];
#pragma unroll
                    for (int e = HB; e >= 1; --e)     // x[0] (the previous row's) last
                        if (i + e < n) acc = cfnmac(uu[r][e], x[e - 1], acc);
#pragma unroll
                    for (int e = HB - 1; e >= 1; --e) x[e] = x[e - 1];
                    x[0] = acc;
                    w.vv[i * T + s] = acc;
                    const double m = cabs2(acc);
                    x2 += m;
                    if (m >= am) {     // going backward, >= keeps the first index on ties
                        am = m;
                        ph = acc;
                    }
                }
            }
        }
        ln.vamax = am;
        ln.vph = ph;
        return x2;
    }

    // v = x / |x| with the phase convention, u = M v / |M v|, then sigma and flags.
    static __device__ void vec_output(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln) {
        const int64_t n = nn(a, ln), T = w.slots;
        const double am = sqrt(ln.vamax);
        const cd ph = am > 0.0 ? C(ln.vph.x / am, -ln.vph.y / am) : C(1.0, 0.0);
        const double rv = 1.0 / sqrt(ln.vx2);
        double2 *vout = a.v + ln.pid * n;
        double2 *uout = a.u + ln.pid * n;
        if constexpr (W <= 4) {
            // Pass 1: v = x / |x| with the phase (into v) and y = M v (into vy, with |y|^2), row by
            // row with the rows of v the product needs (v_{i-kl} .. v_{i+ku}) in a register window.
            // The raw rows are loaded PD rows ahead of their use, into a ring indexed at compile time
            // (the loop body is unrolled PD times), so a row's load is issued before the stores of the
            // rows in between and its wait overlaps them.  The workspace holds rows up to
            // round_up(n, 8) + 8 >= n + ku + 2 PD, so a prefetch may read past row n - 1 (unused).
            constexpr int PD = 2;
            cd win[W];
#pragma unroll
            for (int d = 0; d < W; ++d) win[d] = czero();
            auto vnorm = [&](int64_t r, cd raw) -> cd {      // normalised row r of v (zero past n - 1)
                const cd v = cscale(cmul(raw, ph), rv);
                return r < n ? v : czero();
            };
            // the window before row 0 (that of row -1): win[d] = v_{d-1-kl}, so v_0 .. v_{ku-1} in
            // win[kl+1] .. win[W-1] (rows below 0 are zero)
#pragma unroll
            for (int d = KL + 1; d < W; ++d) {
                const int64_t r = d - 1 - KL;
                win[d] = vnorm(r, w.vv[r * T + s]);
                if (r < n) vout[r] = win[d];
            }
            cd ring[PD];
#pragma unroll
            for (int c = 0; c < PD; ++c) ring[c] = w.vv[(KU + c) * T + s];
            double u2 = 0.0;
            for (int64_t i0 = 0; i0 < n; i0 += PD) {
#pragma unroll
                for (int c = 0; c < PD; ++c) {
                    const int64_t i = i0 + c;
                    const int64_t r = i + KU;              // the row the window gains
                    const cd raw = ring[c];
                    ring[c] = w.vv[(r + PD) * T + s];
                    const cd vr = vnorm(r, raw);
                    if (r < n) vout[r] = vr;
#pragma unroll
                    for (int d = 0; d < W - 1; ++d) win[d] = win[d + 1];
                    win[W - 1] = vr;
                    if (i < n) {
                        cd acc = czero();
#pragma unroll
                        for (int d = 0; d < W; ++d) {
                            const int64_t col = i - KL + d;
                            if (col >= 0 && col < n) {
                                const cd m = mval(a, ln, i, col), v = win[d];
                                acc = C(fma(m.x, v.x, fma(-m.y, v.y, acc.x)), fma(m.x, v.y, fma(m.y, v.x, acc.y)));
                            }
                        }
                        w.vy[i * T + s] = acc;
                        u2 += cabs2(acc);
                    }
                }
            }
            // Pass 2: u = y / |y|, with the same prefetch
            const double ru = 1.0 / sqrt(u2);
#pragma unroll
            for (int c = 0; c < PD; ++c) ring[c] = w.vy[c * T + s];
            for (int64_t i0 = 0; i0 < n; i0 += PD) {
#pragma unroll
                for (int c = 0; c < PD; ++c) {
                    const int64_t i = i0 + c;
                    const cd y = ring[c];
                    ring[c] = w.vy[(i + PD) * T + s];
                    if (i < n) uout[i] = cscale(y, ru);
                }
            }
        } else {
            // wider bands: three passes, one memory wait per row (the window and the ring
            // above make these kernels' register allocation spill)
            for (int64_t i = 0; i < n; ++i) {
                const cd v = cscale(cmul(w.vv[i * T + s], ph), rv);
                w.vv[i * T + s] = v;
                vout[i] = v;
            }
            double u2 = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                cd acc = czero();
#pragma unroll
                for (int d = 0; d < W; ++d) {
                    const int64_t c = i - KL + d;
                    if (c >= 0 && c < n) {
                        const cd m = mval(a, ln, i, c), v = w.vv[c * T + s];
                        acc = C(fma(m.x, v.x, fma(-m.y, v.y, acc.x)), fma(m.x, v.y, fma(m.y, v.x, acc.y)));
                    }
                }
                w.vy[i * T + s] = acc;
                u2 += cabs2(acc);
            }
            const double ru = 1.0 / sqrt(u2);
            for (int64_t i = 0; i < n; ++i) uout[i] = cscale(w.vy[i * T + s], ru);
        }
        a.sigma[ln.pid] = ln.vsig;
        if (a.info) a.info[ln.pid] = ln.vflags;
        if (a.iters) a.iters[ln.pid] = 0;
        if (a.sens) a.sens[ln.pid] = (uint8_t)(ln.vsig <= a.eps);
        ln.active = false;
        ln.phase = 0;
    }

    static __device__ void vec_cycle(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln) {
        if (ln.vit == 0) {
            ln.vx2 = vec_factor(a, w, s, ln, ln.blo * ln.blo);
        } else if (ln.vit <= kInvIter) {
            ln.vx2 = vec_step(a, w, s, ln, 1.0 / sqrt(ln.vx2));
        } else {
            vec_output(a, w, s, ln);
            return;
        }
        ln.vit += 1;
    }

    // ---------------------------------------------------------------- singular vectors
    // Coefficients of the Ritz vector for sigma_min (per lane, O(k)): with T_k = B_k^H B_k
    // (B_k upper bidiagonal, alpha'_j on the diagonal, beta'_j above it),
    //   q = top eigenvector of T_k (two steps of inverse iteration at theta (1 + 2^-40)),
    //   p = B_k q / |B_k q|  (top left singular vector of B_k).
    // The left Lanczos vectors u_j of B = M^{-1} then give v = sum_j p_j u_j, the Ritz
    // approximation of the top left singular vector of B, which is the right singular vector
    // of M = zI - A for sigma_min.  vmeta columns: 0 alpha'_j, 1 beta'_j, 2 q_j, 3 pivots of
    // the tridiagonal solve and finally p_j.
    static __device__ void ritz_coeffs(const Workspace &w, int64_t s, const Lane &ln) {
        const int64_t T = w.slots;
        const int k = ln.k;
        auto vm = [&](int j, int c) -> double & { return w.vmeta[((int64_t)j * 4 + c) * T + s]; };
        double mu = ln.theta * (1.0 + 0x1p-40);
        for (int j = 0; j < k; ++j) vm(j, 2) = 1.0;
        for (int it = 0; it < 2; ++it) {
            double dprev = 0.0;
            for (int j = 0; j < k; ++j) {
                double dj = w.hist[((int64_t)j * 2 + 0) * T + s] - mu;
                double rhs = vm(j, 2);
                if (j > 0) {
                    double e = sqrt(w.hist[((int64_t)(j - 1) * 2 + 1) * T + s]);
                    double lj = e / dprev;
                    dj -= lj * e;
                    rhs -= lj * vm(j - 1, 2);
                }
                vm(j, 2) = rhs;
                vm(j, 3) = dj;
                dprev = dj;
            }
            double xnext = 0.0, nrm = 0.0;
            for (int j = k - 1; j >= 0; --j) {
                double dj = vm(j, 3);
                double x = vm(j, 2) / dj;
                if (j < k - 1) x -= (sqrt(w.hist[((int64_t)j * 2 + 1) * T + s]) / dj) * xnext;
                vm(j, 2) = x;
                xnext = x;
                nrm += x * x;
            }
            double rn = 1.0 / sqrt(nrm);
            for (int j = 0; j < k; ++j) vm(j, 2) *= rn;
        }
        double pn = 0.0;
        for (int j = 0; j < k; ++j) {
            double pj = vm(j, 0) * vm(j, 2);
            if (j + 1 < k) pj += vm(j, 1) * vm(j + 1, 2);
            vm(j, 3) = pj;
            pn += pj * pj;
        }
        double rpn = 1.0 / sqrt(pn);
        for (int j = 0; j < k; ++j) vm(j, 3) *= rpn;
    }

    // Ritz vector v = sum_j p_j u_j (j = 1 .. kfinal) from the Lanczos vectors kept by the first
    // pass, into vacc, with |v|^2 and the first entry of largest modulus (as the replay's last
    // step gives them; same terms, same order).  A block of RB rows reads JB kept vectors per
    // memory wait.
    static __device__ __forceinline__ void ritz_from_store(const Workspace &w, int64_t s, Lane &ln, int64_t n) {
        const int64_t T = w.slots, nr = w.nrow;
        const int k = ln.kfinal;
        const int64_t npad = ((n + CH - 1) / CH) * CH;
        constexpr int RB = 4, JB = 8;
        double vn = 0.0, vam = -1.0;
        cd vph = C(1.0, 0.0);
        for (int64_t r0 = 0; r0 < npad; r0 += RB) {
            cd v[RB];
#pragma unroll
            for (int b = 0; b < RB; ++b) v[b] = czero();
            for (int j0 = 0; j0 < k; j0 += JB) {
                cd u[JB][RB];
                double c[JB];
#pragma unroll
                for (int jb = 0; jb < JB; ++jb) {
                    const int j = j0 + jb < k ? j0 + jb : k - 1;     // past k: a valid row, unused
                    c[jb] = w.vmeta[((int64_t)j * 4 + 3) * T + s];
#pragma unroll
                    for (int b = 0; b < RB; ++b) u[jb][b] = w.ustore[((int64_t)j * nr + r0 + b) * T + s];
                }
#pragma unroll
                for (int jb = 0; jb < JB; ++jb) {
                    if (j0 + jb < k) {
#pragma unroll
                        for (int b = 0; b < RB; ++b) {
                            const cd t = C(c[jb] * u[jb][b].x, c[jb] * u[jb][b].y);
                            v[b] = j0 + jb == 0 ? t : C(v[b].x + t.x, v[b].y + t.y);
                        }
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                const int64_t r = r0 + b;
                w.vacc[r * T + s] = v[b];
                if (r < n) {
                    const double m = cabs2(v[b]);
                    vn += m;
                    if (m > vam) {
                        vam = m;
                        vph = v[b];
                    }
                }
            }
        }
        ln.vnorm2 = vn;
        ln.vamax = vam;
        ln.vph = vph;
    }

    // Stage 2 output, after the inverse-iteration step left M^{-H} v in vv (|.|^2 = acc 2^(2 eacc)):
    // v = vacc / |vacc|, u = that direction normalised, both rotated by the unit scalar that
    // makes the first entry of v of largest modulus real and positive.
    static __device__ void write_vectors(const EvalArgs &a, const Workspace &w, int64_t s, const Lane &ln,
                                         double acc, int eacc) {
        const int64_t n = nn(a, ln), T = w.slots;
        const double am = sqrt(ln.vamax);
        const cd ph = am > 0.0 ? C(ln.vph.x / am, -ln.vph.y / am) : C(1.0, 0.0);
        const double rv = 1.0 / sqrt(ln.vnorm2);
        const double ru = 1.0 / sqrt(acc);
        double2 *vout = a.v + ln.pid * n;
        double2 *uout = a.u + ln.pid * n;
        for (int64_t i = 0; i < n; ++i) {
            vout[i] = cscale(cmul(w.vacc[i * T + s], ph), rv);
            const cd uu = cldexp(cscale(w.vv[i * T + s], ru), (int)w.ev[(i / CH) * T + s] - eacc);
            uout[i] = cmul(uu, ph);
        }
    }

    static __device__ void finish(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln, int flags) {
        double sigma;
        if (ln.sing) {
            sigma = 0.0;
            flags |= 1;
        } else {
            const double m = 1.0 / sqrt(ln.theta);      // sigma = m 2^-E0
            sigma = ldexp(m, -ln.E0);
            if (!(sigma >= 0x1p-1022) && m > 0.0 && m < INFINITY) {
                // below the normal range: reported as 0, with -floor(log2 sigma) in bits 8..31
                const int e2 = ilogb(m) - ln.E0;
                flags |= PS_PT_UNDERFLOW | ((-e2 < 0x7fffff ? -e2 : 0x7fffff) << 8);
                sigma = 0.0;
            } else if (!(sigma >= 0x1p-1022)) {
                flags |= PS_PT_UNDERFLOW;
                sigma = 0.0;
            }
        }
        a.sigma[ln.pid] = sigma;
        if (a.info) a.info[ln.pid] = flags;
        if (a.iters) a.iters[ln.pid] = ln.k;
        if (a.sens) a.sens[ln.pid] = (uint8_t)(sigma <= a.eps);
        if (VEC) {
            if (ln.sing) {
                // exactly singular (zero pivot): no Lanczos data; report zero vectors with the
                // SINGULAR bit set.
                for (int64_t i = 0; i < nn(a, ln); ++i) {
                    a.u[ln.pid * nn(a, ln) + i] = czero();
                    a.v[ln.pid * nn(a, ln) + i] = czero();
                }
            } else {
                ritz_coeffs(w, s, ln);
                const int kept = ln.kfinal;      // Lanczos vectors the first pass kept
                ln.kfinal = ln.k;
                if (w.ustore && ln.k >= 1 && kept == ln.k) {
                    // the Ritz vector from the kept vectors; the final solve follows (stage 2)
                    ritz_from_store(w, s, ln, nn(a, ln));
                    ln.stage = 2;
                    return;  // the lane stays active
                }
                // replay the same kfinal steps from the same start vector (the factors stay)
                ln.stage = 1;
                ln.fresh = true;
                ln.k = 0;
                ln.b_m = 0.0;
                ln.b_e = 0;
                return;      // the lane stays active
            }
        }
        ln.active = false;
    }

    // Convergence test at a check (theta_new = top Ritz value of T_k, r = residual norm
    // alpha_k beta_k |y_k| of its Ritz pair for (M M^H)^{-1}, both in units of 2^(2 E0)).
    // The target |sigma - sigma_min| <= tol_norm ||A|| + tol_rel sigma is a relative
    // tolerance tol_th = 2 (tol_norm ||A|| / sigma + tol_rel) on theta = 1 / sigma^2.
    //  * sigma_est <= tol_norm ||A|| / 2: done (the Ritz value only underestimates theta,
    //    so 0 <= sigma_est - sigma_min <= sigma_est).
    //  * r <= tol_th theta / 2: done (an eigenvalue lies within r of theta).
    //  * theta unchanged to 2^-44 (relative) over two consecutive checks: the Ritz value has settled
    //    at working precision (then y_k is below what the inverse-iteration estimate can
    //    resolve, and r is overestimated).
    static __device__ bool converged(const EvalArgs &a, Lane &ln, double theta_new, double r) {
        double r_abs = ldexp(a.tol_norm * fro(a, ln) * sqrt(theta_new), ln.E0);
        double tol_th = 2.0 * (r_abs + a.tol_rel);
        double delta = fmax(theta_new - ln.theta, 0.0);
        bool flat = ln.nchecks >= 1 && delta <= 0x1p-44 * theta_new;
        bool flat_prev = ln.rho_prev > 0.0;
        ln.delta_prev = delta;
        ln.rho_prev = flat ? 1.0 : 0.0;
        if (r_abs >= 2.0) return true;
        if (r <= 0.5 * tol_th * theta_new) return true;
        return flat && flat_prev;
    }

    static __device__ void check_theta(const Workspace &w, int64_t s, Lane &ln, TopEig &te) {
        if (ln.k == 1) {
            te.theta = w.hist[s];
            te.yk2 = 1.0;
        } else {
            te = top_eig(w.hist, w.slots, s, ln.k, ln.theta, fmax(ln.gmax, ln.gopen));
        }
    }

    static __device__ void after_b1(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln, double acc,
                                    int eacc) {
        const int64_t T = w.slots;
        double av = sqrt(ln.fresh ? acc / ln.nrm_h : acc);
        ln.Eu = eacc;
        ln.rdu = 1.0 / sqrt(acc);
        // a replay repeats the recurrence only; it ends before any step where the first pass stopped
        const bool first_pass = !VEC || ln.stage == 0;
        if (!(av > 0.0) && first_pass) {
            // B v_k = beta u_{k-1} exactly: the Krylov space is invariant and T_k is exact.
            if (ln.fresh) {
                ln.sing = true;
            } else {
                TopEig te;
                check_theta(w, s, ln, te);
                ln.theta = te.theta;
            }
            finish(a, w, s, ln, 0);
            return;
        }
        int ea = ilogb(av);
        ln.a_m = ldexp(av, -ea);
        ln.a_e = eacc + ea;
        auto vm = [&](int j, int c) -> double & { return w.vmeta[((int64_t)j * 4 + c) * T + s]; };
        if (ln.fresh) {
            ln.E0 = ln.a_e;
            double ap = ln.a_m;
            w.hist[s] = ap * ap;
            ln.theta = 0.0;
            ln.ap_prev = ap;
            ln.k = 1;
            ln.fresh = false;
            ln.next_check = 1;
            ln.nchecks = 0;
            ln.delta_prev = ln.rho_prev = 0.0;
            ln.gmax = 0.0;
            ln.gopen = ap * ap;
            if (VEC && first_pass) vm(0, 0) = ap;
            double r_abs = ldexp(a.tol_norm * fro(a, ln) * ap, ln.E0);
            if (r_abs >= 2.0 && first_pass) {
                ln.theta = ap * ap;
                finish(a, w, s, ln, 0);
            }
        } else {
            double ap = ldexp(ln.a_m, ln.a_e - ln.E0);
            double b2 = ln.ap_prev * ln.ap_prev * ln.bp * ln.bp;
            int k = ln.k;
            w.hist[((int64_t)(k - 1) * 2 + 1) * T + s] = b2;
            double dk = fma(ap, ap, ln.bp * ln.bp);
            w.hist[((int64_t)k * 2 + 0) * T + s] = dk;
            double off = sqrt(b2);
            ln.gmax = fmax(ln.gmax, ln.gopen + off);
            ln.gopen = dk + off;
            if (VEC && first_pass) {
                vm(k - 1, 1) = ln.bp;
                vm(k, 0) = ap;
            }
            ln.k = k + 1;
            ln.ap_prev = ap;
        }
    }

    static __device__ void after_b2(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln, double acc,
                                    int eacc, int kcap) {
        double bv = sqrt(acc);
        ln.Ev = eacc;
        ln.rdv = 1.0 / sqrt(acc);
        TopEig te;
        const bool first_pass = !VEC || ln.stage == 0;
        if (!(bv > 0.0) && first_pass) {
            // B^H u_k = alpha_k v_k exactly: invariant Krylov space, T_k exact.
            check_theta(w, s, ln, te);
            ln.theta = te.theta;
            finish(a, w, s, ln, 0);
            return;
        }
        int eb = ilogb(bv);
        ln.b_m = ldexp(bv, -eb);
        ln.b_e = eacc + eb;
        ln.bp = ldexp(ln.b_m, ln.b_e - ln.E0);
        if (!first_pass) return;     // replay: no checks (it stops at the first pass's step count)
        bool checked = false;
        if (ln.k >= ln.next_check) {
            check_theta(w, s, ln, te);
            double r = ln.ap_prev * ln.bp * sqrt(te.yk2);
            bool conv = converged(a, ln, te.theta, r);
            ln.theta = te.theta;
            ln.nchecks += 1;
            int step = ln.k >> a.check_shift;
            ln.next_check = ln.k + (step > 1 ? step : 1);
            checked = true;
            if (conv) {
                finish(a, w, s, ln, 0);
                return;
            }
        }
        if (ln.k >= kcap) {
            if (!checked) {
                check_theta(w, s, ln, te);
                ln.theta = te.theta;
            }
            finish(a, w, s, ln, 2);
        }
    }

    // In the kernels with kl = 4 and singular vectors the four sweeps are compiled as
    // functions of their own: inlined there, the kl = 4, ku = 2 kernel returns wrong sigma on
    // the Golub-Kahan path (about 1e-4 where sigma is below 1e-8), although the same lane code
    // is correct on the CPU, with the sweeps compiled separately, and inlined in the sigma-only
    // kernels at every kl.  It does so with or without the bisection that these kernels once
    // held beside the sweeps.  Separate functions cost their calls' register saves to scratch,
    // but inlined, these kernels spill as well (944 against 1204 bytes a lane at ku = 2).
    // Every mode of all 25 band shapes is checked against the oracle by the all-band-shapes
    // test.
    static constexpr bool kSplitSweeps = KL >= 4 && VEC;
    static __device__ __noinline__ void f1_sep(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln) {
        f1(a, w, s, ln);
    }
    static __device__ __noinline__ void b1_sep(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln,
                                               double &acc, int &eacc) {
        b1(a, w, s, ln, acc, eacc);
    }
    static __device__ __noinline__ void f2_sep(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln) {
        f2(a, w, s, ln);
    }
    static __device__ __noinline__ void b2_sep(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln,
                                               double &acc, int &eacc) {
        b2(a, w, s, ln, acc, eacc);
    }
    static __device__ __forceinline__ void sweep_f1(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln) {
        if constexpr (kSplitSweeps) f1_sep(a, w, s, ln);
        else f1(a, w, s, ln);
    }
    static __device__ __forceinline__ void sweep_b1(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln,
                                                    double &acc, int &eacc) {
        if constexpr (kSplitSweeps) b1_sep(a, w, s, ln, acc, eacc);
        else b1(a, w, s, ln, acc, eacc);
    }
    static __device__ __forceinline__ void sweep_f2(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln) {
        if constexpr (kSplitSweeps) f2_sep(a, w, s, ln);
        else f2(a, w, s, ln);
    }
    static __device__ __forceinline__ void sweep_b2(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln,
                                                    double &acc, int &eacc) {
        if constexpr (kSplitSweeps) b2_sep(a, w, s, ln, acc, eacc);
        else b2(a, w, s, ln, acc, eacc);
    }

    // Shift position id -> output index (pid), shift z and, in batch mode, its matrix.
    static __device__ void locate(const EvalArgs &a, int64_t id, Lane &ln) {
        ln.pid = id;
        if (BATCH) {
            // matrix of position id: the last m with mfirst[m] <= id
            int lo = 0, hi = a.nmat - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (a.mfirst[mid] <= id) lo = mid;
                else hi = mid - 1;
            }
            const MatDesc d = a.mats[lo];
            const int64_t q = id - a.mfirst[lo];
            ln.n = d.n;
            ln.arow = d.arow;
            ln.normA = d.normA;
            ln.norm2A = d.norm2A;
            ln.pid = d.out_off + q;
            const int64_t flat = a.idx[ln.pid];
            const int64_t gi = flat / d.nx, gj = flat - gi * d.nx;
            const double x = d.nx > 1 ? __dadd_rn(d.ga, __ddiv_rn(__dmul_rn(d.gb - d.ga, (double)gj),
                                                                   (double)(d.nx - 1))) : d.ga;
            const double y = d.ny > 1 ? __dadd_rn(d.gc, __ddiv_rn(__dmul_rn(d.gd - d.gc, (double)gi),
                                                                   (double)(d.ny - 1))) : d.gc;
            ln.z = C(x, y);
        } else if (a.mode == kShiftList) {
            ln.z = a.z[ln.pid];
        } else if (a.idx) {
            ln.z = grid_point(a, a.idx[ln.pid]);
        } else {
            ln.pid = tile_flat(id, a.nx, a.ny);   // full grid: output at the flat index
            ln.z = grid_point(a, ln.pid);
        }
    }

    // The workspace is laid out [wavefront][row][component][lane]: the 64 lanes of a
    // wavefront touch one contiguous 1 KiB (complex) segment per access, and a chunk of
    // consecutive rows of one wavefront is contiguous as well.  Each lane works on a view
    // whose pointers are offset to its own column (slots = 64, lane index 0).
    static __device__ Workspace lane_view(const Workspace &g, int64_t sg) {
        Workspace w = g;
        const int64_t wv = sg >> 6, l = sg & 63;
        const int64_t wl = KL > 0 ? KL : 1;
        const int64_t nr = g.nrow;
        w.slots = 64;
        w.L = g.L + wv * nr * wl * 64 + l;
        w.U = g.U + wv * nr * W * 64 + l;
        w.piv = g.piv + wv * nr * 64 + l;
        w.vu = g.vu + wv * nr * 64 + l;
        w.vv = g.vv + wv * nr * 64 + l;
        w.vy = g.vy + wv * nr * 64 + l;
        w.eu = g.eu + wv * nr * 64 + l;
        w.ev = g.ev + wv * nr * 64 + l;
        w.ey = g.ey + wv * nr * 64 + l;
        w.hist = g.hist + wv * (int64_t)g.kmax * 2 * 64 + l;
        if (VEC) {
            w.vacc = g.vacc + wv * nr * 64 + l;
            w.vmeta = g.vmeta + wv * (int64_t)g.kmax * 4 * 64 + l;
            if (g.ustore) w.ustore = g.ustore + wv * (int64_t)g.kstore * nr * 64 + l;
        }
        return w;
    }

    // sg: the lane's slot in the workspace (its global thread index in a one-class launch)
    static __device__ void run(const EvalArgs a, const Workspace wg, int64_t sg) {
        const Workspace w = lane_view(wg, sg);
        const int64_t s = 0;
        const int64_t npts = *a.count_dev;
        const int kcap = a.max_iter;
        Lane ln;
        ln.active = false;
        ln.exhausted = false;
        ln.fresh = false;
        ln.sing = false;
        ln.k = 0;
        ln.next_check = 1;
        ln.nchecks = 0;
        ln.pid = -1;
        ln.z = czero();
        ln.theta = 0.0;
        ln.b_m = 0.0;
        ln.b_e = 0;
        ln.a_m = 0.0;
        ln.a_e = 0;
        ln.Eu = ln.Ev = ln.Ey = 0;
        ln.rdu = ln.rdv = 1.0;
        ln.E0 = 0;
        ln.nrm_h = 1.0;
        ln.ap_prev = ln.bp = 0.0;
        ln.gmax = ln.gopen = 0.0;
        ln.delta_prev = ln.rho_prev = 0.0;
        ln.stage = 0;
        ln.kfinal = 0;
        ln.vnorm2 = 1.0;
        ln.vamax = -1.0;
        ln.vph = C(1.0, 0.0);
        ln.n = a.n;
        ln.arow = a.arow;
        ln.normA = a.normA;
        ln.norm2A = a.norm2A;
        ln.phase = 0;
        ln.nbis = 0;
        ln.blo = ln.bhi = 0.0;
        ln.vit = ln.vflags = 0;
        ln.vsig = ln.vx2 = 0.0;
        while (true) {
            bool may_refill = !ln.active && !ln.exhausted;
            if (may_refill) {
                const unsigned long long id = atomicAdd(w.queue, 1ull);
                if ((int64_t)id >= npts) {
                    ln.exhausted = true;
                } else {
                    // queue position (the shifts the bisection kernel handed over, or all)
                    const int64_t qid = a.perm ? a.perm[id] : (int64_t)id;
                    ln.active = qid >= 0;
                    ln.exhausted = qid < 0;
                    ln.fresh = true;
                    ln.stage = 0;
                    ln.kfinal = 0;
                    ln.phase = 0;
                    ln.sing = false;
                    ln.k = 0;
                    ln.b_m = 0.0;
                    ln.b_e = 0;
                    locate(a, qid >= 0 ? qid : 0, ln);
                    if (ln.active) bis_begin(a, ln);   // a settled bracket: on to the singular pair
                }
            }
            if (__all(!ln.active && ln.exhausted)) break;
            if (__all(!ln.active)) continue;

            double acc;
            int eacc;
            if (!VEC) {
                // Sigma only: every lane is on the Golub-Kahan path (four sweeps per cycle).
                if (__any(ln.active)) {
                    sweep_f1(a, w, s, ln);
                    if (ln.active && gk(ln) && ln.sing) finish(a, w, s, ln, 0);
                    sweep_b1(a, w, s, ln, acc, eacc);
                    if (ln.active && gk(ln)) after_b1(a, w, s, ln, acc, eacc);
                    sweep_f2(a, w, s, ln);
                    sweep_b2(a, w, s, ln, acc, eacc);
                    if (ln.active && gk(ln)) after_b2(a, w, s, ln, acc, eacc, kcap);
                }
                continue;
            }
            // Lanes computing their vectors after the bisection take one unit of that work per
            // cycle.
            if (BIS && __any(ln.active && !gk(ln))) {
                if (ln.active && ln.phase == 2) vec_cycle(a, w, s, ln);
            }
            if (!__any(ln.active && gk(ln))) continue;
            // With vectors a cycle serves lanes in all three stages; lanes sit out the sweeps
            // their stage does not need (ln.active is cleared around those calls).
            const bool act0 = ln.active;
            const bool fin = act0 && ln.stage == 2;        // only f2 and b2, from vacc
            if (fin) ln.active = false;
            sweep_f1(a, w, s, ln);
            if (ln.active && ln.sing) finish(a, w, s, ln, 0);
            sweep_b1(a, w, s, ln, acc, eacc);
            const int st0 = ln.stage;
            if (ln.active && gk(ln)) after_b1(a, w, s, ln, acc, eacc);
            const bool hold = ln.active && ln.stage != st0;   // entered the replay: starts next cycle
            if (fin) {
                ln.active = true;
                ln.a_m = 0.0;                               // no -alpha v term
                ln.a_e = 0;
            }
            if (hold) ln.active = false;
            sweep_f2(a, w, s, ln);
            const bool endrep = ln.active && ln.stage == 1 && ln.k == ln.kfinal;   // vacc is complete
            if (endrep) ln.active = false;
            sweep_b2(a, w, s, ln, acc, eacc);
            if (hold || endrep) ln.active = true;
            if (endrep) {
                ln.stage = 2;
            } else if (fin) {
                write_vectors(a, w, s, ln, acc, eacc);
                ln.active = false;
            } else if (ln.active && !hold && gk(ln)) {
                after_b2(a, w, s, ln, acc, eacc, kcap);
            }
        }
    }
};

// One wavefront per workgroup: a launch of S slots is S / 64 workgroups, which the dispatcher
// spreads over all compute units (and their four SIMDs) even when S / 64 is below the SIMD
// count, instead of packing four wavefronts onto each of S / 256 compute units.
constexpr int kEvalBlock = 64;

template <int KL, int KU, bool VEC, bool BATCH>
__global__ void __launch_bounds__(kEvalBlock) k_eval(EvalArgs a, Workspace w) {
    Kern<KL, KU, VEC, BATCH>::run(a, w, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

typedef void (*EvalKernel)(EvalArgs, Workspace);

// mode 0: one matrix, sigma only; 1: one matrix with vectors (batches: ps_eval_batch.hip)
template <int KL, int KU>
EvalKernel pick_mode(int mode) {
    switch (mode) {
    case 0: return k_eval<KL, KU, false, false>;
    case 1: return k_eval<KL, KU, true, false>;
    }
    return nullptr;
}

template <int KL>
EvalKernel pick_ku(int ku, int mode) {
    switch (ku) {
    case 0: return pick_mode<KL, 0>(mode);
    case 1: return pick_mode<KL, 1>(mode);
    case 2: return pick_mode<KL, 2>(mode);
    case 3: return pick_mode<KL, 3>(mode);
    case 4: return pick_mode<KL, 4>(mode);
    }
    return nullptr;
}

// Defined in ps_eval_kl<K>.hip.
EvalKernel pick_eval_kl0(int ku, int mode);
EvalKernel pick_eval_kl1(int ku, int mode);
EvalKernel pick_eval_kl2(int ku, int mode);
EvalKernel pick_eval_kl3(int ku, int mode);
EvalKernel pick_eval_kl4(int ku, int mode);

}  // namespace ps
