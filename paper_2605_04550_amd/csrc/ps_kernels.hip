// HIP kernels for gfx950 (MI355X): sigma_min(zI - A) of a banded matrix at many shifts.
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
//      alpha on the diagonal, beta above it), found by Newton on det(T_k - lambda I)
//      from an upper bound; sigma_min(M) = 1/sqrt(theta) once theta has settled.
// This reaches the quantity of the paper's Sec. 2.1 (sigma_min(z) = s_n of the SVD of
// zI - A) to a stated tolerance, without the O(n^3) dense SVD per shift.
//
// Memory layout: every per-shift array lives in a caller-provided workspace, laid out
// [row][component][slot]; the lanes of a wavefront sweep the same row at the same time,
// so each load or store of a wavefront is one contiguous 1 KiB (complex) segment.  The
// band of A is read by all lanes at the same address (wave-uniform).
//
// Overflow safety: sigma_min can be far below the double range (it decays like
// 10^(-0.3 n) inside the pseudospectrum of a non-normal Toeplitz matrix), so every
// triangular sweep keeps a running binary exponent R and stores each row together with
// the exponent that was current when it was written (value = mantissa * 2^e).  When a
// value would exceed 2^400, the sweep's window is scaled down and R grows.  Readers
// rescale each row to their own frame with ldexp, which only ever shifts downward.
//
// The persistent launch pulls shifts from a device counter; a lane whose shift has
// finished takes the next one at the start of the following cycle and factorises it
// during the forward sweep that the other lanes spend on their L solves.

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

__device__ TopEig top_eig(const double *hist, int64_t T, int64_t s, int k, double lo, double hi) {
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
    bool active, fresh, sing, exhausted, pending;
    // batch mode: the matrix of the current shift
    int64_t n;
    const double2 *arow;
    double normA;
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
        const bool act = ln.active, fresh = ln.fresh;
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
#pragma unroll
                for (int r = 0; r < KL; ++r)
#pragma unroll
                    for (int c = 0; c < W; ++c) Wm[r][c] = mentry(a, ln, r, c);
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
                ln.sing = sing;
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
        const bool act = ln.active && !ln.sing;
        const bool sub = !ln.fresh;
        int R = ln.Ey;
        cd xw[W];
#pragma unroll
        for (int d = 0; d < W; ++d) xw[d] = czero();
        double acc = 0.0;
        int Eacc = R;
        // VEC: write u_k into basis slot k (k = ln.k), read u_{k-1} from slot k-1.
        double2 *uout = w.vu;
        int16_t *euout = w.eu;
        const double2 *uold = w.vu;
        const int16_t *euold = w.eu;
        const double rd_old = ln.rdu;
        const int E_old = ln.Eu;
        if (VEC) {
            int64_t stride = w.nrow * T;
            uout = w.basis + (int64_t)ln.k * stride;
            euout = w.ebasis + (int64_t)ln.k * stride;
            if (ln.k > 0) {
                uold = w.basis + (int64_t)(ln.k - 1) * stride;
                euold = w.ebasis + (int64_t)(ln.k - 1) * stride;
            }
        }
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
                    cd rhs = cscale(yr[c], fy);
#pragma unroll
                    for (int d = 1; d < W; ++d) rhs = cfnma(Ur[c][d], xw[d], rhs);
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
                    for (int d = 1; d < W; ++d) rhs = cfnma(Ur[c][d], xw[d], rhs);
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
    static __device__ void f2(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln, bool from_vu = false) {
        const int64_t n = nn(a, ln), T = w.slots;
        const bool act = ln.active;
        const double2 *uin = w.vu;
        const int16_t *euin = w.eu;
        if (VEC && !from_vu) {
            int64_t stride = w.nrow * T;
            uin = w.basis + (int64_t)(ln.k - 1) * stride;
            euin = w.ebasis + (int64_t)(ln.k - 1) * stride;
        }
        const double rdu = ln.rdu;
        const int Eu = ln.Eu;
        int R = 0;
        cd acc[W];
        const int64_t npad = ((n + CH - 1) / CH) * CH;
        if (act) {
            const double f0 = rdu * p2((int)euin[s] - Eu);
#pragma unroll
            for (int d = 0; d < W - 1; ++d) acc[d] = cscale(uin[d * T + s], f0);
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
            const int ea = (int)euin[q * T + s];
            const bool last = i0 + CH >= npad;                 // rows at or past npad were never written
            const int eb = (W > 1 && !last) ? (int)euin[(q + 1) * T + s] : ea;
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
    }

    // ---------------------------------------------------------------- backward sweep 2
    // q = P L^{-H} y - alpha_k v_k; v updated in place; returns |q|^2 = acc * 2^(2 Eacc).
    // Step j finalises entry j + kl, so the steps of output chunk p are j = 8p+7-kl .. 8p-kl;
    // the kl steps above the top chunk run first (their outputs lie past the padding), and
    // steps j < 0 carry zero data (they only flush the window).
    static __device__ void b2(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln, double &acc_out,
                              int &eacc_out) {
        const int64_t n = nn(a, ln), T = w.slots;
        const bool act = ln.active;
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
                vr[c] = w.vv[(j + KL) * T + s];
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
                const double fv = am * rdv * p2(evp - Ev + ae - es);
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
                    const cd vo = cscale(cldexp(vr[c], evp - Ev + ae - es), am * rdv);
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

    // ---------------------------------------------------------------- singular vectors
    // For every lane whose shift converged (ln.pending), all lanes of the wavefront together:
    //   q = top eigenvector of T_k (two steps of inverse iteration at theta (1 + 2^-40)),
    //   p = B_k q / |B_k q| (top left singular vector of the bidiagonal),
    //   v = U_k p  (Ritz vector: right singular vector of M = zI - A), assembled in vu,
    //   u = M^{-H} v / |M^{-H} v| through the lane's LU factors (one inverse-iteration
    //       step: M^{-H} v_min = u_min / sigma_min, so the error in u shrinks by the gap
    //       instead of growing by |M| / sigma as it would for u = M v / sigma),
    // then both are written to the caller's [npts][n] arrays with the joint phase that makes
    // the first entry of v of largest modulus real and positive.
    static __device__ void ritz_coeffs(const Workspace &w, int64_t s, const Lane &ln) {
        const int64_t T = w.slots;
        const int k = ln.k;
        // bmeta rows: [0, 2kvec) basis meta (1/norm, exponent); [2kvec, 3kvec) q;
        // [3kvec, 4kvec) pivots, then p; [4kvec, 6kvec) alpha'_j, beta'_j.
        double *q = w.bmeta + (int64_t)(2 * w.kvec) * T;
        double *aux = q + (int64_t)w.kvec * T;
        const double *ab = q + (int64_t)(2 * w.kvec) * T;
        double mu = ln.theta * (1.0 + 0x1p-40);
        for (int j = 0; j < k; ++j) q[(int64_t)j * T + s] = 1.0;
        for (int it = 0; it < 2; ++it) {
            double dprev = 0.0;
            for (int j = 0; j < k; ++j) {
                double dj = w.hist[((int64_t)j * 2 + 0) * T + s] - mu;
                double rhs = q[(int64_t)j * T + s];
                if (j > 0) {
                    double e = sqrt(w.hist[((int64_t)(j - 1) * 2 + 1) * T + s]);
                    double lj = e / dprev;
                    dj -= lj * e;
                    rhs -= lj * q[(int64_t)(j - 1) * T + s];
                }
                q[(int64_t)j * T + s] = rhs;
                aux[(int64_t)j * T + s] = dj;
                dprev = dj;
            }
            double xnext = 0.0, nrm = 0.0;
            for (int j = k - 1; j >= 0; --j) {
                double dj = aux[(int64_t)j * T + s];
                double x = q[(int64_t)j * T + s] / dj;
                if (j < k - 1) x -= (sqrt(w.hist[((int64_t)j * 2 + 1) * T + s]) / dj) * xnext;
                q[(int64_t)j * T + s] = x;
                xnext = x;
                nrm += x * x;
            }
            double rn = 1.0 / sqrt(nrm);
            for (int j = 0; j < k; ++j) q[(int64_t)j * T + s] *= rn;
        }
        double pn = 0.0;
        for (int j = 0; j < k; ++j) {
            double pj = ab[((int64_t)j * 2 + 0) * T + s] * q[(int64_t)j * T + s];
            if (j + 1 < k) pj += ab[((int64_t)j * 2 + 1) * T + s] * q[(int64_t)(j + 1) * T + s];
            aux[(int64_t)j * T + s] = pj;
            pn += pj * pj;
        }
        double rpn = 1.0 / sqrt(pn);
        for (int j = 0; j < k; ++j) aux[(int64_t)j * T + s] *= rpn;
    }

    static __device__ void vec_finalize(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln) {
        const int64_t n = nn(a, ln), T = w.slots;
        const bool pend = ln.pending;
        if (pend) ritz_coeffs(w, s, ln);
        const double *coef = w.bmeta + (int64_t)(3 * w.kvec) * T;
        const int64_t stride = w.nrow * T;
        const int k = ln.k;
        double vn = 0.0, amax = -1.0;
        cd vph = C(1.0, 0.0);
        for (int64_t i = 0; i < n; ++i) {
            if (!pend) continue;
            cd acc = czero();
            for (int j = 0; j < k; ++j) {
                double rd = w.bmeta[((int64_t)j * 2 + 0) * T + s];
                int Ej = (int)w.bmeta[((int64_t)j * 2 + 1) * T + s];
                cd uj = cldexp(cscale(w.basis[j * stride + i * T + s], rd),
                               (int)w.ebasis[j * stride + (i / CH) * T + s] - Ej);
                double c = coef[(int64_t)j * T + s];
                acc = C(fma(c, uj.x, acc.x), fma(c, uj.y, acc.y));
            }
            w.vu[i * T + s] = acc;
            vn += cabs2(acc);
            double m = cabs2(acc);
            if (m > amax) { amax = m; vph = acc; }
        }
        for (int64_t i = n; i < w.nrow; ++i) {
            if (!pend) continue;
            w.vu[i * T + s] = czero();
        }
        for (int64_t q = 0; q < w.nrow / CH; ++q) {
            if (!pend) continue;
            w.eu[q * T + s] = 0;
        }
        // u direction: M^{-H} v through the factors (alpha = 0: no three-term correction)
        const bool saved = ln.active;
        ln.active = pend;
        if (pend) {
            ln.Eu = 0;
            ln.rdu = 1.0 / sqrt(vn);
            ln.a_m = 0.0;
            ln.a_e = 0;
        }
        f2(a, w, s, ln, true);
        double accu;
        int eaccu;
        b2(a, w, s, ln, accu, eaccu);
        ln.active = saved;
        if (!pend) return;
        double am = sqrt(amax);
        cd ph = am > 0.0 ? C(vph.x / am, -vph.y / am) : C(1.0, 0.0);
        double rv = 1.0 / sqrt(vn);
        double ru = 1.0 / sqrt(accu);
        double2 *vout = a.v + ln.pid * n;
        double2 *uout = a.u + ln.pid * n;
        for (int64_t i = 0; i < n; ++i) {
            vout[i] = cscale(cmul(w.vu[i * T + s], ph), rv);
            cd uu = cldexp(cscale(w.vv[i * T + s], ru), (int)w.ev[(i / CH) * T + s] - eaccu);
            uout[i] = cmul(uu, ph);
        }
        ln.pending = false;
    }

    static __device__ void finish(const EvalArgs &a, const Workspace &w, int64_t s, Lane &ln, int flags) {
        double sigma;
        if (ln.sing) {
            sigma = 0.0;
            flags |= 1;
        } else {
            sigma = ldexp(1.0 / sqrt(ln.theta), -ln.E0);
            if (!(sigma >= 0x1p-1022)) flags |= 4;
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
                ln.pending = true;   // assembled by vec_finalize with the whole wavefront
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
        if (VEC) {
            w.bmeta[((int64_t)ln.k * 2 + 0) * T + s] = ln.rdu;
            w.bmeta[((int64_t)ln.k * 2 + 1) * T + s] = (double)ln.Eu;
        }
        if (!(av > 0.0)) {
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
        double *abq = VEC ? w.bmeta + (int64_t)(4 * w.kvec) * T : nullptr;
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
            if (VEC) abq[s] = ap;
            double r_abs = ldexp(a.tol_norm * fro(a, ln) * ap, ln.E0);
            if (r_abs >= 2.0) {
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
            if (VEC) {
                abq[((int64_t)(k - 1) * 2 + 1) * T + s] = ln.bp;
                abq[((int64_t)k * 2 + 0) * T + s] = ap;
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
        if (!(bv > 0.0)) {
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
            w.basis = g.basis + wv * (int64_t)g.kvec * nr * 64 + l;
            w.ebasis = g.ebasis + wv * (int64_t)g.kvec * nr * 64 + l;
            w.bmeta = g.bmeta + wv * (int64_t)g.kvec * 6 * 64 + l;
        }
        return w;
    }

    static __device__ void run(const EvalArgs a, const Workspace wg) {
        const int64_t sg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const Workspace w = lane_view(wg, sg);
        const int64_t s = 0;
        const int64_t npts = *a.count_dev;
        const int kcap = VEC ? (a.max_iter < w.kvec ? a.max_iter : w.kvec) : a.max_iter;
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
        ln.pending = false;
        ln.n = a.n;
        ln.arow = a.arow;
        ln.normA = a.normA;
        while (true) {
            if (VEC && __all(!ln.active) && __any(ln.pending)) vec_finalize(a, w, s, ln);
            bool may_refill = !ln.active && !ln.exhausted;
            if (VEC) may_refill = may_refill && __all(!ln.active);
            if (may_refill) {
                unsigned long long id = atomicAdd(w.queue, 1ull);
                if ((int64_t)id >= npts) {
                    ln.exhausted = true;
                } else {
                    ln.pid = (int64_t)id;
                    ln.active = true;
                    ln.fresh = true;
                    ln.sing = false;
                    ln.k = 0;
                    ln.b_m = 0.0;
                    ln.b_e = 0;
                    if (BATCH) {
                        // matrix of queue position id: the last m with mfirst[m] <= id
                        int lo = 0, hi = a.nmat - 1;
                        while (lo < hi) {
                            int mid = (lo + hi + 1) >> 1;
                            if (a.mfirst[mid] <= (int64_t)id) lo = mid;
                            else hi = mid - 1;
                        }
                        const MatDesc d = a.mats[lo];
                        const int64_t q = (int64_t)id - a.mfirst[lo];
                        ln.n = d.n;
                        ln.arow = d.arow;
                        ln.normA = d.normA;
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
                    } else {
                        ln.z = grid_point(a, a.idx ? a.idx[ln.pid] : ln.pid);
                    }
                }
            }
            if (__all(!ln.active && ln.exhausted)) break;
            if (__all(!ln.active)) continue;

            double acc;
            int eacc;
            f1(a, w, s, ln);
            if (ln.active && ln.sing) finish(a, w, s, ln, 0);
            b1(a, w, s, ln, acc, eacc);
            if (ln.active) after_b1(a, w, s, ln, acc, eacc);
            f2(a, w, s, ln);
            b2(a, w, s, ln, acc, eacc);
            if (ln.active) after_b2(a, w, s, ln, acc, eacc, kcap);
        }
    }
};

// One wavefront per workgroup: a launch of S slots is S / 64 workgroups, which the dispatcher
// spreads over all compute units (and their four SIMDs) even when S / 64 is below the SIMD
// count, instead of packing four wavefronts onto each of S / 256 compute units.
constexpr int kEvalBlock = 64;

template <int KL, int KU, bool VEC, bool BATCH>
__global__ void __launch_bounds__(kEvalBlock) k_eval(EvalArgs a, Workspace w) {
    Kern<KL, KU, VEC, BATCH>::run(a, w);
}

// ------------------------------------------------------------------------ small kernels

__global__ void k_set_count(int64_t *count, int64_t value, unsigned long long *queue) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (count) *count = value;
        *queue = 0ull;
    }
}

__global__ void k_iota(int64_t *idx, int64_t npts) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < npts) idx[t] = t;
}

constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

// Block-local exclusive scan of flags in LDS.
__device__ int64_t block_scan(int64_t v, int64_t *sh, int64_t &total) {
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int64_t x = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    total = sh[kScanBlock - 1];
    int64_t excl = sh[t] - v;
    __syncthreads();
    return excl;
}

__global__ void __launch_bounds__(kScanBlock) k_mask_count(const uint8_t *mask, int64_t npts, int64_t *blocksums) {
    __shared__ int64_t sh[kScanBlock];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t c = 0;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < npts && mask[base + q]) ++c;
    int64_t total;
    block_scan(c, sh, total);
    if (threadIdx.x == 0) blocksums[blockIdx.x] = total;
}

// Single-block exclusive scan over the block sums (any number of blocks), total -> count.
__global__ void __launch_bounds__(kScanBlock) k_scan_sums(int64_t *blocksums, int64_t nblocks, int64_t *count,
                                                          unsigned long long *queue) {
    __shared__ int64_t sh[kScanBlock];
    int64_t carry = 0;
    for (int64_t base = 0; base < nblocks; base += kScanBlock) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < nblocks ? blocksums[i] : 0;
        int64_t total;
        int64_t ex = block_scan(v, sh, total);
        if (i < nblocks) blocksums[i] = carry + ex;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *count = carry;
        *queue = 0ull;
    }
}

__global__ void __launch_bounds__(kScanBlock) k_mask_scatter(const uint8_t *mask, int64_t npts,
                                                             const int64_t *blocksums, int64_t *idx) {
    __shared__ int64_t sh[kScanBlock];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t c = 0;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < npts && mask[base + q]) ++c;
    int64_t total;
    int64_t ex = block_scan(c, sh, total);
    int64_t pos = blocksums[blockIdx.x] + ex;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < npts && mask[base + q]) idx[pos++] = base + q;
}

// ------------------------------------------------------------------------ adjoint

// grad_z[p] = g_p conj(u_p^H v_p): one wavefront per shift, lanes stride over rows.
__global__ void __launch_bounds__(256) k_grad_z(int64_t n, int64_t npts, const double *g, const double2 *u,
                                                const double2 *v, double2 *grad_z) {
    int lane = threadIdx.x & 63;
    int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= npts) return;
    const double2 *up = u + p * n;
    const double2 *vp = v + p * n;
    double re = 0.0, im = 0.0;
    for (int64_t i = lane; i < n; i += 64) {
        double2 a = up[i], b = vp[i];
        re = fma(a.x, b.x, fma(a.y, b.y, re));   // conj(a) b
        im = fma(a.x, b.y, fma(-a.y, b.x, im));
    }
    for (int off = 32; off >= 1; off >>= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
    }
    const double gp = g ? g[p] : 1.0;     // NULL weights: the plain gradient of sigma_min
    if (lane == 0) grad_z[p] = make_double2(gp * re, -gp * im);
}

constexpr int kBwdRows = 64;   // shifts summed per partial row (fixed order)

// Partial band gradient: partial[r][t] = -sum_{p in block r} g_p u_p[i] conj(v_p[j]) for
// band entry t = (j, d) of the GB layout, i = j + d - ku.  Threads stride over entries.
__global__ void __launch_bounds__(256) k_grad_band_partial(int64_t n, int kl, int ku, int64_t npts, const double *g,
                                                           const double2 *u, const double2 *v, double2 *partial) {
    int w = kl + ku + 1;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t r = blockIdx.y;
    if (t >= n * w) return;
    int64_t j = t / w;
    int d = (int)(t - j * w);
    int64_t i = j + d - ku;
    double re = 0.0, im = 0.0;
    if (i >= 0 && i < n) {
        int64_t p0 = r * kBwdRows, p1 = p0 + kBwdRows < npts ? p0 + kBwdRows : npts;
        for (int64_t p = p0; p < p1; ++p) {
            double2 a = u[p * n + i], b = v[p * n + j];
            double gp = g[p];
            // a conj(b)
            re = fma(gp, fma(a.x, b.x, a.y * b.y), re);
            im = fma(gp, fma(a.y, b.x, -a.x * b.y), im);
        }
    }
    partial[r * n * w + t] = make_double2(-re, -im);
}

__global__ void __launch_bounds__(256) k_grad_band_sum(int64_t n, int w, int64_t rows, const double2 *partial,
                                                       double2 *grad_band, int real_a) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * w) return;
    double re = 0.0, im = 0.0;
    for (int64_t r = 0; r < rows; ++r) {
        double2 x = partial[r * n * w + t];
        re += x.x;
        im += x.y;
    }
    grad_band[t] = make_double2(re, real_a ? 0.0 : im);
}

// ------------------------------------------------------------------------ host launchers

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t workspace_bytes(int64_t n, int kl, int ku, int64_t slots, int kmax, int kvec, int64_t npts_max) {
    Workspace w;
    carve_workspace(nullptr, n, kl, ku, slots, kmax, kvec, npts_max, &w);
    return (size_t)(uintptr_t)w.blocksums + align256(sizeof(int64_t) * (size_t)((npts_max + kScanTile - 1) / kScanTile + 1));
}

void carve_workspace(void *base, int64_t n, int kl, int ku, int64_t slots, int kmax, int kvec, int64_t npts_max,
                     Workspace *w) {
    size_t off = 0;
    char *b = (char *)base;
    auto take = [&](size_t bytes) -> void * {
        void *p = (void *)(b + off);
        off += align256(bytes);
        return p;
    };
    const int64_t nrow = padded_rows(n);
    const size_t ns = (size_t)nrow * (size_t)slots;
    const int wu = kl + ku + 1;
    w->slots = slots;
    w->nrow = nrow;
    w->kmax = kmax;
    w->kvec = kvec;
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
    if (kvec > 0) {
        w->basis = (double2 *)take(sizeof(double2) * ns * (size_t)kvec);
        w->ebasis = (int16_t *)take(sizeof(int16_t) * ns * (size_t)kvec);
        // meta pairs [kvec][2], q [kvec], pivots/p [kvec], alpha'/beta' [kvec][2]
        w->bmeta = (double *)take(sizeof(double) * (size_t)kvec * 6 * (size_t)slots);
    } else {
        w->basis = nullptr;
        w->ebasis = nullptr;
        w->bmeta = nullptr;
    }
    w->blocksums = (int64_t *)take(8);
    // blocksums extends to the end (sized by workspace_bytes)
    (void)npts_max;
}

hipError_t launch_set_count(int64_t *count, int64_t value, unsigned long long *queue, hipStream_t st) {
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(64), 0, st, count, value, queue);
    return hipGetLastError();
}

hipError_t launch_iota(int64_t *idx, int64_t npts, hipStream_t st) {
    if (npts > 0) hipLaunchKernelGGL(k_iota, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, idx, npts);
    return hipGetLastError();
}

hipError_t launch_compact_mask(const uint8_t *mask, int64_t npts, int64_t *idx, int64_t *count, int64_t *blocksums,
                               unsigned long long *queue, hipStream_t st) {
    int64_t nb = (npts + kScanTile - 1) / kScanTile;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_mask_count, dim3((unsigned)nb), dim3(kScanBlock), 0, st, mask, npts, blocksums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, blocksums, nb, count, queue);
    hipLaunchKernelGGL(k_mask_scatter, dim3((unsigned)nb), dim3(kScanBlock), 0, st, mask, npts,
                       (const int64_t *)blocksums, idx);
    return hipGetLastError();
}

typedef void (*EvalKernel)(EvalArgs, Workspace);

// mode 0: one matrix, sigma only; 1: one matrix with vectors; 2: batch, sigma only
template <int KL, int KU>
static EvalKernel pick_mode(int mode) {
    switch (mode) {
    case 0: return k_eval<KL, KU, false, false>;
    case 1: return k_eval<KL, KU, true, false>;
    case 2: return k_eval<KL, KU, false, true>;
    }
    return nullptr;
}

template <int KL>
static EvalKernel pick_ku(int ku, int mode) {
    switch (ku) {
    case 0: return pick_mode<KL, 0>(mode);
    case 1: return pick_mode<KL, 1>(mode);
    case 2: return pick_mode<KL, 2>(mode);
    case 3: return pick_mode<KL, 3>(mode);
    case 4: return pick_mode<KL, 4>(mode);
    }
    return nullptr;
}

static EvalKernel pick(int kl, int ku, int mode) {
    switch (kl) {
    case 0: return pick_ku<0>(ku, mode);
    case 1: return pick_ku<1>(ku, mode);
    case 2: return pick_ku<2>(ku, mode);
    case 3: return pick_ku<3>(ku, mode);
    case 4: return pick_ku<4>(ku, mode);
    }
    return nullptr;
}

hipError_t launch_eval(const EvalArgs &a, const Workspace &ws, hipStream_t st) {
    EvalKernel k = pick(a.kl, a.ku, a.want_vectors != 0 ? 1 : 0);
    if (!k) return hipErrorInvalidValue;
    int64_t blocks = ws.slots / kEvalBlock;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kEvalBlock), 0, st, a, ws);
    return hipGetLastError();
}

hipError_t launch_eval_batch(const EvalArgs &a, const Workspace &ws, int kl, int ku, hipStream_t st) {
    EvalKernel k = pick(kl, ku, 2);
    if (!k) return hipErrorInvalidValue;
    int64_t blocks = ws.slots / kEvalBlock;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kEvalBlock), 0, st, a, ws);
    return hipGetLastError();
}

int64_t batch_tiles(int64_t max_npts) { return (max_npts + kScanTile - 1) / kScanTile; }

// Batched compaction: blockIdx.y = matrix, blockIdx.x = tile of kScanTile grid points.
// A NULL mask selects every grid point of that matrix.
__global__ void __launch_bounds__(kScanBlock) k_bmask_count(const MatDesc *mats, const uint8_t *const *masks,
                                                            int64_t ntiles, int64_t *tilesums) {
    __shared__ int64_t sh[kScanBlock];
    const int m = blockIdx.y;
    const int64_t npts = mats[m].nx * mats[m].ny;
    const uint8_t *mask = masks ? masks[m] : nullptr;
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t c = 0;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < npts && (!mask || mask[base + q])) ++c;
    int64_t total;
    block_scan(c, sh, total);
    if (threadIdx.x == 0) tilesums[(int64_t)m * ntiles + blockIdx.x] = total;
}

// One block per matrix: exclusive scan of its tile sums, count -> counts[m].
__global__ void __launch_bounds__(kScanBlock) k_bscan(int64_t ntiles, int64_t *tilesums, int64_t *counts) {
    __shared__ int64_t sh[kScanBlock];
    const int m = blockIdx.x;
    int64_t *ts = tilesums + (int64_t)m * ntiles;
    int64_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += kScanBlock) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < ntiles ? ts[i] : 0;
        int64_t total;
        int64_t ex = block_scan(v, sh, total);
        if (i < ntiles) ts[i] = carry + ex;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[m] = carry;
}

__global__ void __launch_bounds__(kScanBlock) k_bmask_scatter(const MatDesc *mats, const uint8_t *const *masks,
                                                              int64_t ntiles, const int64_t *tilesums, int64_t *idx) {
    __shared__ int64_t sh[kScanBlock];
    const int m = blockIdx.y;
    const int64_t npts = mats[m].nx * mats[m].ny;
    const uint8_t *mask = masks ? masks[m] : nullptr;
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t c = 0;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < npts && (!mask || mask[base + q])) ++c;
    int64_t total;
    int64_t ex = block_scan(c, sh, total);
    int64_t pos = tilesums[(int64_t)m * ntiles + blockIdx.x] + ex;
    int64_t *out = idx + mats[m].out_off;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < npts && (!mask || mask[base + q])) out[pos++] = base + q;
}

// Queue positions of one class: mfirst[m] = sum of counts before m; total -> *total.
__global__ void k_batch_prefix(const MatDesc *mats, const int64_t *counts, int nmat, int64_t *mfirst,
                               int64_t *total, unsigned long long *queue) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t acc = 0;
        for (int m = 0; m < nmat; ++m) {
            mfirst[m] = acc;
            acc += counts[mats[m].cidx];
        }
        *total = acc;
        *queue = 0ull;
    }
}

hipError_t launch_batch_compact(const MatDesc *mats, int nmat, int64_t max_npts, const uint8_t *const *masks,
                                int64_t *idx, int64_t *counts, int64_t *tilesums, hipStream_t st) {
    int64_t nt = batch_tiles(max_npts);
    if (nt < 1) nt = 1;
    hipLaunchKernelGGL(k_bmask_count, dim3((unsigned)nt, (unsigned)nmat), dim3(kScanBlock), 0, st, mats, masks, nt,
                       tilesums);
    hipLaunchKernelGGL(k_bscan, dim3((unsigned)nmat), dim3(kScanBlock), 0, st, nt, tilesums, counts);
    hipLaunchKernelGGL(k_bmask_scatter, dim3((unsigned)nt, (unsigned)nmat), dim3(kScanBlock), 0, st, mats, masks, nt,
                       (const int64_t *)tilesums, idx);
    return hipGetLastError();
}

hipError_t launch_batch_prefix(const MatDesc *mats_cls, const int64_t *counts, int nmat, int64_t *mfirst,
                               int64_t *total, unsigned long long *queue, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_prefix, dim3(1), dim3(64), 0, st, mats_cls, counts, nmat, mfirst, total, queue);
    return hipGetLastError();
}

int64_t backward_partial_rows(int64_t npts) { return (npts + kBwdRows - 1) / kBwdRows; }

// Zero fill (used where a memset node must not appear in captured graphs).
__global__ void k_zero(uint64_t *p, int64_t words) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < words) p[t] = 0ull;
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
    int64_t words = (int64_t)(bytes / 8);
    if (words > 0)
        hipLaunchKernelGGL(k_zero, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st, (uint64_t *)p, words);
    return hipGetLastError();
}

// Newton step toward the level curve sigma = eps: z <- z - sigma ln(sigma/eps) g / |g|^2,
// with g = grad_z (conjugate-Wirtinger gradient of sigma_min).  Points with sigma = 0 or a
// vanishing gradient stay where they are.
__global__ void k_newton_update(int64_t npts, double2 *z, const double *sigma, const double2 *g, double eps) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    const double s = sigma[p];
    const double2 gp = g[p];
    const double g2 = fma(gp.x, gp.x, gp.y * gp.y);
    if (!(s > 0.0) || !(g2 > 0.0)) return;
    const double f = s * log(s / eps) / g2;
    z[p] = make_double2(z[p].x - f * gp.x, z[p].y - f * gp.y);
}

hipError_t launch_newton_update(int64_t npts, double2 *z, const double *sigma, const double2 *grad_z, double eps,
                                hipStream_t st) {
    if (npts > 0)
        hipLaunchKernelGGL(k_newton_update, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, npts, z, sigma,
                           grad_z, eps);
    return hipGetLastError();
}

hipError_t launch_backward(int64_t n, int kl, int ku, int64_t npts, const double *g, const double2 *u,
                           const double2 *v, double2 *grad_z, double2 *grad_band, double2 *partial, int real_a,
                           hipStream_t st) {
    if (grad_z) {
        int64_t threads = npts * 64;
        hipLaunchKernelGGL(k_grad_z, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, n, npts, g, u, v,
                           grad_z);
    }
    if (grad_band) {
        int w = kl + ku + 1;
        int64_t tot = n * w;
        int64_t rows = backward_partial_rows(npts);
        hipLaunchKernelGGL(k_grad_band_partial, dim3((unsigned)((tot + 255) / 256), (unsigned)rows), dim3(256), 0, st,
                           n, kl, ku, npts, g, u, v, partial);
        hipLaunchKernelGGL(k_grad_band_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, w, rows,
                           (const double2 *)partial, grad_band, real_a);
    }
    return hipGetLastError();
}

}  // namespace ps
