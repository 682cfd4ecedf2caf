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
// 0: one test; 1: three for hb <= 2, two for hb <= 5, one above; 2: two for hb <= 6, else one.
// (Measured: at hb <= 2 three tests share the row formation best; at hb = 5 two tests beat one
// by about 10 %; at hb = 6 two tests take the registers of a second wavefront per SIMD and
// gain nothing; at hb = 7, 8 a second test does not fit.)
__host__ __device__ constexpr int tests_per_lane(int hb, int ktm) {
    return ktm == 0 ? 1 : ktm == 1 ? (hb <= 2 ? 3 : hb <= 5 ? 2 : 1) : (hb <= 6 ? 2 : 1);
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
// Right-looking elimination over a sliding window.  Before step i the registers hold the
// trailing matrix S (H with the updates of pivots 0 .. i-1 applied) on rows i .. i+hb-1,
// columns from i on; step i
//   brings in row i+hb of H (no earlier pivot reaches it),
//   takes the pivot d_i = S[i][i] (the test fails if it is not positive), and
//   updates S[i+k][i+k'] -= S[i+k][i] conj(S[i+k'][i]) / d_i for 1 <= k' <= k <= hb.
// The hb^2 / 2 updates of a step are independent of each other; only the next pivot
// (row i+1's diagonal, updated first) and its reciprocal lie on the path from step to step.
// Row r sits in slot r mod (hb+1), its entry (r, r-e) at position e of the slot: a row keeps
// its registers while the window slides, and the row loop is unrolled by hb+1 so that every
// slot index is a compile-time constant.
template <int HB, int KT>
__device__ __forceinline__ unsigned pass(const double *gb, int64_t n, double x, double y, const double (&sh)[KT],
                                         double &hmin) {
    constexpr int RS = gram_stride(HB);
    constexpr int NS = HB + 1;
    cd S[KT][NS][NS];
    double dcur[KT], rcur[KT];
    bool ok[KT];
    const double zz = fma(x, x, y * y);
    double hm = 0x1p1000;
    // Row r of H - sh[j] I (the diagonal shifted per test) into slot F.  The Gram band is the
    // same for every lane of the wavefront and does not change during the launch: read through
    // the constant address space, it comes in by scalar loads into scalar registers (one copy
    // per wavefront, used directly as operands).  Each formula has one scalar operand per
    // instruction (the limit of the instruction set); with contraction off the compiler does
    // not fuse them into a form with two.  The band has zero rows past n (read by the last hb
    // steps, never pivoted).
    struct Row {
        double v[RS];
    };
    auto load_row = [&](int64_t r) {
        Row rw;
        const double *p = uniform_ptr(gb + r * RS);
#pragma unroll
        for (int q = 0; q < RS; q += 2) {
            const double2 t = kload2(p + q);
            rw.v[q] = t.x;
            rw.v[q + 1] = t.y;
        }
        return rw;
    };
    auto form = [&](const Row &rw, int64_t r, cd (&h)[HB + 1]) {
#pragma clang fp contract(off)
        const double hd = fma(-x, rw.v[1], rw.v[0] + fma(-y, rw.v[2], zz));
        hm = r < n ? fmin(hm, hd) : hm;
        h[0] = make_double2(hd, 0.0);
#pragma unroll
        for (int e = 1; e <= HB; ++e) {
            const double *q = rw.v + 4 + 6 * (e - 1);   // G, s, d of entry (r, r - e)
            h[e] = make_double2(fma(-x, q[2], q[0] - y * q[5]), fma(-x, q[3], q[1] + y * q[4]));
        }
    };
    // s -= c conj(p), and its real part alone on the diagonal
    auto upd = [](cd &s, const cd c, const cd p) {
        s.x = fma(-c.x, p.x, fma(-c.y, p.y, s.x));
        s.y = fma(-c.y, p.x, fma(c.x, p.y, s.y));
    };
    auto upd_diag = [](cd &s, const cd c, const cd p) { s.x = fma(-c.x, p.x, fma(-c.y, p.y, s.x)); };
    // rows 0 .. hb-1 (entries left of column 0 are never read)
    [&]<int... U>(std::integer_sequence<int, U...>) {
        auto one = [&](auto uc) {
            constexpr int R = decltype(uc)::value;
            cd h[HB + 1];
            form(load_row(R), R, h);
#pragma unroll
            for (int j = 0; j < KT; ++j) {
                S[j][R][0] = make_double2(h[0].x - sh[j], 0.0);
#pragma unroll
                for (int e = 1; e <= HB; ++e) S[j][R][e] = h[e];
            }
        };
        (one(std::integral_constant<int, U>{}), ...);
    }(std::make_integer_sequence<int, HB>{});
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        ok[j] = true;
        dcur[j] = S[j][0][0].x;
        rcur[j] = recip(dcur[j]);
    }
    auto step = [&](int64_t i, auto kc) {
        constexpr int K = decltype(kc)::value;   // slot of row i
        constexpr int F = (K + HB) % NS;         // slot of the incoming row i + hb
        const Row rw = load_row(i + HB);         // arrives while the window rows are updated
        cd cp[KT][HB + 1];                       // S[i+k][i] / d_i
        double ri[KT];
#pragma unroll
        for (int j = 0; j < KT; ++j) {
            ok[j] = ok[j] && dcur[j] > 0.0;
            ri[j] = rcur[j];
#pragma unroll
            for (int k = 1; k < HB; ++k) {
                const cd c = S[j][(K + k) % NS][k];
                cp[j][k] = make_double2(c.x * ri[j], c.y * ri[j]);
            }
        }
        // window rows i+1 .. i+hb-1, row i+1 first: its diagonal is the next pivot
#pragma unroll
        for (int k = 1; k < HB; ++k) {
#pragma unroll
            for (int j = 0; j < KT; ++j) {
                cd *row = S[j][(K + k) % NS];
                const cd c = row[k];
#pragma unroll
                for (int k2 = 1; k2 < k; ++k2) upd(row[k - k2], c, cp[j][k2]);
                upd_diag(row[0], c, cp[j][k]);
                if (k == 1) {
                    dcur[j] = row[0].x;
                    rcur[j] = recip(dcur[j]);
                }
            }
        }
        // the incoming row
        cd h[HB + 1];
        form(rw, i + HB, h);
#pragma unroll
        for (int j = 0; j < KT; ++j) {
            cd *row = S[j][F];
            const cd c = h[HB];
            cp[j][HB] = make_double2(c.x * ri[j], c.y * ri[j]);
            row[0] = make_double2(h[0].x - sh[j], 0.0);
#pragma unroll
            for (int e = 1; e < HB; ++e) row[e] = h[e];
#pragma unroll
            for (int k2 = 1; k2 < HB; ++k2) upd(row[HB - k2], c, cp[j][k2]);
            upd_diag(row[0], c, cp[j][HB]);
            if (HB == 1) {
                dcur[j] = row[0].x;
                rcur[j] = recip(dcur[j]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    int64_t i0 = 0;
    for (; i0 + NS <= n; i0 += NS) {
        [&]<int... U>(std::integer_sequence<int, U...>) {
            (step(i0 + U, std::integral_constant<int, U>{}), ...);
        }(std::make_integer_sequence<int, NS>{});
    }
    [&]<int... U>(std::integer_sequence<int, U...>) {
        ((i0 + U < n ? step(i0 + U, std::integral_constant<int, U>{}) : void()), ...);
    }(std::make_integer_sequence<int, NS>{});
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
    if (a.phase == 3) {                  // brackets for a call with vectors, at output positions
        a.st_np[sf.pid] = gk ? -1 : passes;
        a.st_lo[sf.pid] = lo;
        a.st_hi[sf.pid] = hi;
        return;
    }
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

// Wavefronts per SIMD the register allocation aims at: two where a single test per lane
// leaves the window of the widest bands just over half the register file (the allocator then
// keeps it within half), no demand otherwise.
__host__ __device__ constexpr int bis_waves(int hb, int kt) { return hb >= 7 && kt == 1 ? 2 : 1; }

// One wavefront per workgroup, one chunk of 64 / L shifts per wavefront.  Half-bandwidths
// HBLO .. HBHI are compiled in; the chunk's matrix picks one (the same for the whole
// wavefront).
template <int HBLO, int HBHI, int KTM, int L>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(bis_waves(HBHI, tests_per_lane(HBHI, KTM)))))
k_bis(BisArgs a) {
    constexpr int SPW = 64 / L;
    int64_t b = blockIdx.x;
    const int lane = (int)threadIdx.x;
    MatView mv;
    Shift sf;
    int hb;
    if (a.batch) {
        // the launch covers the chunks of mats[mlo .. mhi], numbered on from chunkfirst[mlo]
        const int64_t c0 = a.chunkfirst[a.mlo];
        const int64_t c1 = a.mhi + 1 < a.nmat ? a.chunkfirst[a.mhi + 1] : *a.total_chunks;
        b += c0;
        if (b >= c1) return;
        // matrix of chunk b: the last k with chunkfirst[k] <= b
        int lo = a.mlo, hi = a.mhi;
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
