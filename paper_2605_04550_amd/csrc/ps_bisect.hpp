// HIP device code for gfx950 (MI355X): sigma_min(zI - A) by inertia bisection, one kernel
// for a whole call (one matrix, or every matrix of a batch).
//
// sigma_min^2 is the smallest eigenvalue of H = M^H M, M = zI - A (sigma_min = s_n of the SVD
// of zI - A, Sec. 2.1).  For t >= 0, t < sigma_min exactly when H - t^2 I is positive
// definite, i.e. when its root-free factorisation H - t^2 I = L D L^H (L unit lower
// triangular) meets no non-positive pivot (Sylvester's law of inertia).  A test is one pass
// over the n rows; a bracket lo < sigma_min <= hi shrinks with every pass.
//
// H is banded with half-bandwidth hb = kl + ku and depends on z through
//     H = G - conj(z) A - z A^H + |z|^2 I,     G = A^H A,
// so row i of H is  H[i][i-e] = G[i][i-e] - x s_e + i y d_e  (z = x + i y) with
// s_e = A[i][i-e] + conj(A[i-e][i]) and d_e = A[i][i-e] - conj(A[i-e][i]).  G, s and d do not
// depend on z: the handle stores them once per matrix (the "Gram band", written by
// k_gram_band at ps_create_banded), and a pass forms a row of H with 4 fused multiply-adds
// per entry from data that every lane of a wavefront reads at the same address.  The
// factor's state (the hb previous rows of L and their 1/d) stays in registers, so a pass
// moves no per-shift data through memory.
//
// Parallel layout: L lanes own one shift (L = 1, 2, 4, or 64 = a whole wavefront), each lane
// runs KT tests per pass, so one pass splits the bracket into L*KT + 1 parts.  A wavefront
// works on 64 / L consecutive shifts of one matrix (a "chunk"); a batch launch orders the
// chunks longest-first by the predicted cost of their matrix.  A shift whose sigma_min lies
// below the bisection's rounding limit (its first test fails) is handed to the Golub-Kahan
// kernel through a list.
#pragma once

#include "ps_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <utility>

namespace ps {

namespace bis {

typedef double2 cd;

// Doubles per row of the Gram band for half-bandwidth hb: e = 0 uses 3 (G_ii, 2 Re A_ii,
// 2 Im A_ii) padded to 4, then 6 per e = 1..hb (G, s, d as complex numbers).
__host__ __device__ constexpr int gram_stride(int hb) { return 4 + 6 * hb; }

// Tests per lane and pass for half-bandwidth HB under test-count mode KTM:
// 0: one test; 1: three for hb <= 2, two for hb <= 6, one above; 2: two for hb <= 6, else one.
// (Measured: at hb <= 2 three tests share the row formation best; at hb = 5, 6 two tests beat
// one by 13-15 %; at hb = 7, 8 a second test's registers cost more than it saves.)
__host__ __device__ constexpr int tests_per_lane(int hb, int ktm) {
    return ktm == 0 ? 1 : ktm == 1 ? (hb <= 2 ? 3 : hb <= 6 ? 2 : 1) : (hb <= 6 ? 2 : 1);
}

constexpr int kMaxPasses = 128;   // far above the ~30 passes a shift needs with one test per pass

// 1 / d to full precision: the hardware reciprocal (about 24 correct bits) and two Newton
// steps, each doubling the correct bits (d is a positive normal number wherever it matters).
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return fma(r, fma(-d, r, 1.0), r);
}

// Load of two doubles of the Gram band.  The band is the same for every lane of the
// wavefront and does not change during the launch: read through the constant address space,
// it comes in by scalar loads into scalar registers (one copy per wavefront, used directly as
// operands) instead of vector loads that would copy every value into all 64 lanes.
// The address of a row as a wavefront-uniform value (the compiler cannot always prove it).
__device__ __forceinline__ const double *uniform_ptr(const double *p) {
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (const double *)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double2 kload2(const double *p) {
#if defined(__HIP_DEVICE_COMPILE__)
    const __attribute__((address_space(4))) double *q = (const __attribute__((address_space(4))) double *)p;
    return make_double2(q[0], q[1]);
#else
    return *(const double2 *)p;
#endif
}

// One pass of KT tests at shifts sh[j] = t_j^2: bit j of the result is set when every pivot of
// H - sh[j] I = L D L^H is positive.  Every pass runs over all n rows (a failed test computes
// on with meaningless values): every pass then costs the same known work, and the lanes of a
// wavefront run in step anyway.  hmin = min_i H[i][i] = min_i |M e_i|^2 >= sigma_min^2.
//
// Row i, m = i - e (e = hb .. 1):  w_e = H[i][m] - sum_{e2 > e} w_e2 conj(L[m][i - e2]),
// L[i][m] = w_e / d_m,  d_i = H[i][i] - t^2 - sum_e Re(w_e conj(L[i][m])).
// Registers: the hb previous rows of the factor sit in hb slots, row r in slot r mod hb:
// Ls[k][f] = L[r][r-1-f] (f = 0 .. hb-2) and Qs[k] = 1 / d_r; rows before the first are zero.
// The row loop is unrolled by hb, so that every slot index is a compile-time constant and a
// new row simply takes the registers of the row hb back (whose last use is this row's e = hb
// term): nothing is shifted from register to register.
template <int HB, int KT>
__device__ __forceinline__ unsigned pass(const double *gb, int64_t n, double x, double y, const double (&sh)[KT],
                                         double &hmin) {
    constexpr int RS = gram_stride(HB);
    constexpr int HA = HB > 1 ? HB - 1 : 1;
    cd Ls[KT][HB][HA];
    double Qs[KT][HB];
    bool ok[KT];
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        ok[j] = true;
#pragma unroll
        for (int k = 0; k < HB; ++k) {
            Qs[j][k] = 0.0;
#pragma unroll
            for (int f = 0; f < HA; ++f) Ls[j][k][f] = make_double2(0.0, 0.0);
        }
    }
    // The Gram band is the same for every lane of the wavefront and does not change during
    // the launch: read through the constant address space, its rows come in by scalar loads
    // into scalar registers (one copy per wavefront, used directly as operands), instead of
    // vector loads that would copy every value into all 64 lanes.
    const double zz = fma(x, x, y * y);
    double hm = 0x1p1000;
    // Row data of the Gram band (RS doubles).  The part a row needs first (the diagonal entry
    // and the PFB outermost e blocks, all of it at narrow bands) is loaded one row ahead, so
    // that those scalar loads are in flight while the previous row is computed; the rest of
    // the row is loaded when the row starts and arrives while its first blocks are computed.
    // (Loading every row completely ahead would not fit the scalar register file at wider
    // bands.)  The band has zero rows past n, so the load ahead of the last row stays inside.
    constexpr int PFB = HB <= 2 ? HB : HB <= 4 ? 2 : 1;
    struct Row {
        double v[RS];
    };
    auto load_part = [&](Row &rw, int64_t i, bool ahead) {
        const double *r = uniform_ptr(gb + i * RS);
        if (ahead) {
            const double2 a = kload2(r), b = kload2(r + 2);
            rw.v[0] = a.x;
            rw.v[1] = a.y;
            rw.v[2] = b.x;
            rw.v[3] = b.y;
        }
#pragma unroll
        for (int e = 1; e <= HB; ++e) {
            if ((e > HB - PFB) != ahead) continue;
#pragma unroll
            for (int q = 4 + 6 * (e - 1); q < 10 + 6 * (e - 1); q += 2) {
                const double2 t = kload2(r + q);
                rw.v[q] = t.x;
                rw.v[q + 1] = t.y;
            }
        }
    };
    // row i of the factorisations, held in slot K = i mod hb.  H[i][i-e] is formed just before
    // its e step (for all tests), with one scalar operand per instruction (the limit of the
    // instruction set): t = y d_y, t = g_x - t, H_x = t - x s_x (and likewise for H_y); with
    // contraction off the compiler does not fuse them into a form with two.
    auto step = [&](int64_t i, Row &rw, auto kc) {
        constexpr int K = decltype(kc)::value;
        load_part(rw, i, false);
        double h0;
        {
#pragma clang fp contract(off)
            h0 = fma(-x, rw.v[1], rw.v[0] + fma(-y, rw.v[2], zz));
        }
        hm = fmin(hm, h0);
        double dd[KT];
        cd wv[KT][HB + 1], lv[KT][HB + 1];
#pragma unroll
        for (int j = 0; j < KT; ++j) dd[j] = h0 - sh[j];
#pragma unroll
        for (int e = HB; e >= 1; --e) {
            const double *q = rw.v + 4 + 6 * (e - 1);   // G, s, d of entry e
            cd he;
            {
#pragma clang fp contract(off)
                he = make_double2(fma(-x, q[2], q[0] - y * q[5]), fma(-x, q[3], q[1] + y * q[4]));
            }
            const int se = (K - e + HB) % HB;   // slot of row i - e (a constant)
#pragma unroll
            for (int j = 0; j < KT; ++j) {
                cd acc = he;
#pragma unroll
                for (int e2 = HB; e2 > e; --e2) {
                    // acc -= wv[e2] * conj(L[i-e][i-e2]),  L[i-e][i-e2] = Ls[se][e2-e-1]
                    const cd p = Ls[j][se][e2 - e - 1];
                    acc.x = fma(-wv[j][e2].x, p.x, fma(-wv[j][e2].y, p.y, acc.x));
                    acc.y = fma(-wv[j][e2].y, p.x, fma(wv[j][e2].x, p.y, acc.y));
                }
                wv[j][e] = acc;
                lv[j][e] = make_double2(acc.x * Qs[j][se], acc.y * Qs[j][se]);
                dd[j] = fma(-acc.x, lv[j][e].x, fma(-acc.y, lv[j][e].y, dd[j]));
            }
        }
#pragma unroll
        for (int j = 0; j < KT; ++j) {
            ok[j] = ok[j] && dd[j] > 0.0;
            Qs[j][K] = recip(dd[j]);
#pragma unroll
            for (int f = 0; f + 1 < HB; ++f) Ls[j][K][f] = lv[j][f + 1];
        }
    };
    // one row: the loads of the next row are issued first, then the row is computed; rows are
    // scheduled one by one (interleaving them would only lengthen register lifetimes)
    Row cur;
    load_part(cur, 0, true);
    auto advance = [&](int64_t i, auto kc) {
        Row nxt;
        load_part(nxt, i + 1, true);
        step(i, cur, kc);
        cur = nxt;
        __builtin_amdgcn_sched_barrier(0);
    };
    int64_t i0 = 0;
    for (; i0 + HB <= n; i0 += HB) {
        [&]<int... U>(std::integer_sequence<int, U...>) {
            (advance(i0 + U, std::integral_constant<int, U>{}), ...);
        }(std::make_integer_sequence<int, HB>{});
    }
    [&]<int... U>(std::integer_sequence<int, U...>) {
        ((i0 + U < n ? advance(i0 + U, std::integral_constant<int, U>{}) : void()), ...);
    }(std::make_integer_sequence<int, HB>{});
    hmin = hm;
    unsigned bits = 0;
#pragma unroll
    for (int j = 0; j < KT; ++j) bits |= ok[j] ? (1u << j) : 0u;
    return bits;
}

// Minimum / maximum over the L lanes of a group (L a power of two, groups aligned in the
// wavefront).
template <int L>
__device__ __forceinline__ double group_min(double v) {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
template <int L>
__device__ __forceinline__ double group_max(double v) {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// The shift a lane group works on.
struct Shift {
    double x, y;          // z
    int64_t pid;          // output position
    int64_t qpos;         // queue position handed to the Golub-Kahan kernel
    int64_t sid;          // index of its saved bracket between a first-pass and a resuming launch
    bool valid;
};

// Matrix-level data of the current chunk.
struct MatView {
    const double *gb;     // Gram band rows
    int64_t n;
    double normA, norm2A;
    int64_t *gk_list;     // this matrix's Golub-Kahan list (its class's, in a batch)
    int64_t *gk_count;
};

// Bisection of the group's shift: T = L * KT test points per pass.  The first pass tests
// sigma_adm (the smallest t the rounding allows) and T - 1 points spread geometrically up to
// mn = |z| + ||A||_2 >= sigma_min; later passes split the bracket into T + 1 parts,
// geometrically while hi > 2 lo, then evenly, until hi - lo <= tol_norm ||A||_F + tol_rel lo.
// sigma = the midpoint of the final bracket.
template <int HB, int KT, int L>
__device__ void bisect(const BisArgs &a, const MatView &mv, const Shift &sf) {
    constexpr int T = L * KT;
    const int gl = (int)(threadIdx.x & (L - 1));
    // admission: the rounding of forming and factorising H, about 32 eps mn^2 in sigma^2,
    // must stay below an eighth of sigma * target(sigma): sigma >= sigma_adm, the positive
    // root of tol_rel s^2 + tol_norm ||A||_F s = 256 eps mn^2
    const double mn = hypot(sf.x, sf.y) + mv.norm2A;
    const double b = a.tol_norm * mv.normA, c = 256.0 * 0x1p-52 * mn * mn;
    const double adm = 2.0 * c / (b + sqrt(b * b + 4.0 * a.tol_rel * c));
    bool gk = !(mn < 1e100 && mn > 1e-100) || !(adm < mn);
    double lo = adm, hi = mn;
    int passes = 0;
    bool done = !sf.valid || gk;
    if (a.phase == 2 && sf.valid) {
        // resume after a first-pass launch (passes < 0: the shift was finished or handed over)
        passes = a.st_np[sf.sid];
        lo = a.st_lo[sf.sid];
        hi = a.st_hi[sf.sid];
        gk = false;
        done = passes < 0;
    }
    const bool resumable = !done;
    bool capped = false, pending = false;
    while (__any(!done)) {
        if (!done) {
            const bool first = passes == 0;
            const bool geo = first || hi > 2.0 * lo;
            const double lr = geo ? log2(hi / lo) : 0.0;
            double t[KT], sh[KT];
#pragma unroll
            for (int j = 0; j < KT; ++j) {
                const int k = gl * KT + j;
                const double f = first ? (double)k / T : (double)(k + 1) / (T + 1);
                t[j] = geo ? (k == 0 && first ? lo : lo * exp2(f * lr)) : fma(hi - lo, f, lo);
                sh[j] = t[j] * t[j];
            }
            double hmin = 0.0;
            const unsigned bits = pass<HB, KT>(mv.gb, mv.n, sf.x, sf.y, sh, hmin);
            ++passes;
            // leading passed tests of this lane: t_c-1 < sigma_min <= t_c
            int cnt = 0;
#pragma unroll
            for (int j = 0; j < KT; ++j) cnt += (cnt == j && ((bits >> j) & 1u)) ? 1 : 0;
            double pl = -1.0, fl = INFINITY;
#pragma unroll
            for (int j = 0; j < KT; ++j) {
                if (j == cnt - 1) pl = t[j];
                if (j == cnt) fl = t[j];
            }
            // the group's lowest failed point, then its highest passed point below that
            const double nh = group_min<L>(fl);
            const double np = group_max<L>(pl < nh ? pl : -1.0);
            if (first && !(nh > lo)) {          // sigma_min <= sigma_adm: the Golub-Kahan path
                gk = true;
                done = true;
            } else {
                if (np > lo) lo = np;
                if (nh < hi) hi = nh;
                if (first) hi = fmin(hi, sqrt(hmin));
                const double target = a.tol_norm * mv.normA + a.tol_rel * lo;
                const double mid = 0.5 * (lo + hi);
                done = hi - lo <= target || !(mid > lo && mid < hi);
                if (!done && passes >= kMaxPasses) {
                    done = true;
                    capped = true;
                }
                if (!done && a.phase == 1) {     // first-pass launch: the rest comes later
                    done = true;
                    pending = true;
                }
            }
        }
    }
    if (!sf.valid || gl != 0) return;
    if (a.phase == 1) {
        a.st_np[sf.sid] = pending ? passes : -1;
        a.st_lo[sf.sid] = lo;
        a.st_hi[sf.sid] = hi;
        if (pending) return;
    }
    if (gk) {
        const int64_t at = (int64_t)atomicAdd((unsigned long long *)mv.gk_count, 1ull);
        mv.gk_list[at] = sf.qpos;
        return;
    }
    if (!resumable) return;
    const double sigma = 0.5 * (lo + hi);
    a.sigma[sf.pid] = sigma;
    if (a.info) a.info[sf.pid] = PS_PT_BISECT | (capped ? PS_PT_MAXITER : 0) | (passes << 8);
    if (a.iters) a.iters[sf.pid] = 0;
    if (a.sens) a.sens[sf.pid] = (uint8_t)(sigma <= a.eps);
}

__device__ __forceinline__ double grid_coord(double lo, double hi, int64_t k, int64_t n) {
    return n > 1 ? __dadd_rn(lo, __ddiv_rn(__dmul_rn(hi - lo, (double)k), (double)(n - 1))) : lo;
}

// Queue position -> flat grid index of a full-grid call: tiles of 8 x 8 points (see the
// Golub-Kahan kernel's tile_flat; the same order, so that both kernels agree on positions).
__device__ __forceinline__ int64_t tile_order(int64_t id, int64_t nx, int64_t ny) {
    const int64_t r0 = (id / (8 * nx)) * 8;
    const int64_t h = ny - r0 < 8 ? ny - r0 : 8;
    const int64_t rem = id - r0 * nx;
    const int64_t ntx = (nx + 7) / 8;
    int64_t tx = rem / (8 * h);
    if (tx > ntx - 1) tx = ntx - 1;
    const int64_t tw = tx == ntx - 1 ? nx - 8 * (ntx - 1) : 8;
    const int64_t r2 = rem - tx * 8 * h;
    return (r0 + r2 / tw) * nx + 8 * tx + r2 % tw;
}

template <int HB, int KTM, int L>
__device__ __forceinline__ void run_hb(const BisArgs &a, const MatView &mv, const Shift &sf) {
    bisect<HB, tests_per_lane(HB, KTM), L>(a, mv, sf);
}

// One wavefront per workgroup, one chunk of 64 / L shifts per wavefront.  Half-bandwidths
// HBLO .. HBHI are compiled in; the chunk's matrix picks one (the same for the whole
// wavefront).
template <int HBLO, int HBHI, int KTM, int L>
__global__ void __launch_bounds__(64) k_bis(BisArgs a) {
    constexpr int SPW = 64 / L;
    const int64_t b = blockIdx.x;
    const int lane = (int)threadIdx.x;
    MatView mv;
    Shift sf;
    int hb;
    if (a.batch) {
        if (b >= *a.total_chunks) return;
        // matrix of chunk b: the last k with chunkfirst[k] <= b (longest-first order)
        int lo = 0, hi = a.nmat - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.chunkfirst[mid] <= b) lo = mid;
            else hi = mid - 1;
        }
        const MatDesc &d = a.mats[lo];
        const int64_t q = (b - a.chunkfirst[lo]) * SPW + lane / L;
        const int64_t cnt = a.counts[d.cidx];
        mv.gb = d.gram;
        mv.n = d.n;
        mv.normA = d.normA;
        mv.norm2A = d.norm2A;
        mv.gk_list = a.gk_list + d.gkbase;
        mv.gk_count = a.gk_count + d.cls;
        hb = d.kl + d.ku;
        sf.valid = q < cnt;
        const int64_t qq = sf.valid ? q : 0;
        sf.pid = d.out_off + qq;
        sf.qpos = a.mfirst[d.cpos] + qq;
        sf.sid = sf.pid;
        const int64_t flat = a.idx[sf.pid];
        const int64_t gi = flat / d.nx, gj = flat - gi * d.nx;
        sf.x = grid_coord(d.ga, d.gb, gj, d.nx);
        sf.y = grid_coord(d.gc, d.gd, gi, d.ny);
    } else {
        const int64_t cnt = *a.count_dev;
        const int64_t q = b * SPW + lane / L;
        mv.gb = a.gram;
        mv.n = a.n;
        mv.normA = a.normA;
        mv.norm2A = a.norm2A;
        mv.gk_list = a.gk_list;
        mv.gk_count = a.gk_count;
        hb = a.hb;
        sf.valid = q < cnt;
        const int64_t qq = sf.valid ? q : 0;
        sf.qpos = qq;
        sf.sid = qq;
        if (a.mode == kShiftList) {
            sf.pid = qq;
            sf.x = a.z[qq].x;
            sf.y = a.z[qq].y;
        } else {
            const int64_t flat = a.idx ? a.idx[qq] : tile_order(qq, a.nx, a.ny);
            sf.pid = a.idx ? qq : flat;
            const int64_t gi = flat / a.nx, gj = flat - gi * a.nx;
            sf.x = grid_coord(a.ga, a.gb, gj, a.nx);
            sf.y = grid_coord(a.gc, a.gd, gi, a.ny);
        }
    }
    if (!__any(sf.valid)) return;
    switch (hb) {
#define PS_BIS_CASE(H)                                                   \
    case H:                                                              \
        if constexpr (H >= HBLO && H <= HBHI) run_hb<H, KTM, L>(a, mv, sf); \
        break;
        PS_BIS_CASE(1)
        PS_BIS_CASE(2)
        PS_BIS_CASE(3)
        PS_BIS_CASE(4)
        PS_BIS_CASE(5)
        PS_BIS_CASE(6)
        PS_BIS_CASE(7)
        PS_BIS_CASE(8)
#undef PS_BIS_CASE
    default: break;
    }
}

}  // namespace bis

typedef void (*BisKernel)(BisArgs);

}  // namespace ps
