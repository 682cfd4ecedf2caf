// Mask producer: the dual-path classifier of Sec. 3.2 on the matrix cores, its coarse-to-fine
// evaluation over a grid (Sec. 3.5) and the threshold + dilation that give the restricted set R
// of Sec. 4.
//
// Arithmetic: float32 network (v_mfma_f32_16x16x4f32, float32 accumulation), features in
// float64 rounded to float32, the 30 global features folded into the m1 bias in float64.
//
// Layout of a tile.  A wavefront evaluates 16 points at once: lane l works on point l % 16
// and on the input rows 4 (l / 16) .. 4 (l / 16) + 3 of each group of 16.  A layer
// y = W h + b is a chain of 16x16x4 MFMAs with A = a 16 x 4 block of W (packed once per
// network so that each lane loads one float4 per 16 inputs) and B = 4 rows of h.  The output
// accumulator of a 16-row block leaves row 16 oc + 4 (l / 16) + i of point l % 16 in lane l,
// register i -- exactly the rows the next layer's B operand wants from that lane when its
// input index k is enumerated as 16 kc + 4 (l / 16) + i.  So activations never move between
// lanes: every layer reads the previous one's accumulators in place, and only the packed
// weight order encodes the permutation.
#include "ps_mask.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ps {
namespace mlp {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;   // four wavefronts, one 16-point tile each

__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// SiLU(y) = y / (1 + e^-y) and the logistic function, in float32 (exp through the hardware
// exp2 with the argument scaled, hardware reciprocal).
__device__ __forceinline__ float silu(float y) { return y * __builtin_amdgcn_rcpf(1.0f + __expf(-y)); }
__device__ __forceinline__ float logistic(float y) { return __builtin_amdgcn_rcpf(1.0f + __expf(-y)); }

__device__ __forceinline__ v4f silu4(v4f y) {
    v4f r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = silu(y[i]);
    return r;
}

// y[oc] = W h + b for O outputs over KC groups of 16 inputs (see the layout note above).  The
// A operands stream through a two-deep register queue: the load for step s + 2 is issued before
// the four MFMAs of step s (a scheduling barrier keeps it there), so each operand has two
// steps of matrix-core work to arrive from L2.
template <int O, int KC>
__device__ __forceinline__ void dense(const float4 *__restrict__ P, const float *__restrict__ bias, const v4f *h,
                                      v4f *y, int lane) {
    constexpr int N = (O / 16) * KC;
    const int q = lane >> 4;
    float4 q0 = P[lane];
    float4 q1 = N > 1 ? P[64 + lane] : q0;
    v4f acc;
#pragma unroll
    for (int s = 0; s < N; ++s) {
        const int oc = s / KC, kc = s % KC;
        float4 nxt = q1;
        if (s + 2 < N) nxt = P[(s + 2) * 64 + lane];
        __builtin_amdgcn_sched_barrier(0);
        if (kc == 0) {
            const float4 bb = *(const float4 *)(bias + 16 * oc + 4 * q);
            acc = v4f{bb.x, bb.y, bb.z, bb.w};
        }
        acc = mfma(q0.x, h[kc][0], acc);
        acc = mfma(q0.y, h[kc][1], acc);
        acc = mfma(q0.z, h[kc][2], acc);
        acc = mfma(q0.w, h[kc][3], acc);
        if (kc == KC - 1) y[oc] = acc;
        q0 = q1;
        q1 = nxt;
    }
}

// phi_j of Sec. 3.2 (Fourier feature encoding): j = 0, 1 -> x, y; j = 2 + 4 b + t (b = 0..5)
// -> sin(2^(b+1) x), sin(2^(b+1) y), cos(2^(b+1) x), cos(2^(b+1) y) for t = 0..3; 0 past 25.
__device__ __forceinline__ float fourier(int j, double x, double y) {
    if (j < 2) return (float)(j == 0 ? x : y);
    if (j >= 26) return 0.0f;
    const int t = j - 2, band = t >> 2, kind = t & 3;
    const double arg = (double)(2 << band) * ((kind & 1) ? y : x);
    double s, c;
    sincos(arg, &s, &c);
    return (float)((kind & 2) ? c : s);
}

struct Net {
    const float *raw;
    const float4 *packed;
    const float *bfold;
    const double2 *eig;
    int64_t neig;
    double2 cent;
};

__device__ __forceinline__ Net make_net(const float *raw, const float *packed, const double2 *eig, int64_t neig,
                                        const char *ws) {
    Net n;
    n.raw = raw;
    n.packed = (const float4 *)packed;
    n.bfold = (const float *)(ws + kWsBfold);
    n.eig = eig;
    n.neig = neig;
    n.cent = *(const double2 *)(ws + kWsCent);
    return n;
}

// p(z) for the 16 points of a tile; lane l passes the coordinates of point l % 16 and gets its
// probability back (all four lanes of a point hold it).
__device__ float eval_tile(const Net &net, double x, double y, int lane) {
    const int q = lane >> 4;
    // per-point features g1, g2, g3 (Sec. 3.1, eq. dist): the four lanes of a point split the
    // spectrum, then combine
    double dmin2 = INFINITY, dsum = 0.0;
    for (int64_t e = q; e < net.neig; e += 4) {
        const double2 l = net.eig[e];
        const double dx = x - l.x, dy = y - l.y;
        const double d2 = dx * dx + dy * dy;
        dmin2 = fmin(dmin2, d2);
        dsum += sqrt(d2);
    }
    dmin2 = fmin(dmin2, __shfl_xor(dmin2, 16));
    dsum += __shfl_xor(dsum, 16);
    dmin2 = fmin(dmin2, __shfl_xor(dmin2, 32));
    dsum += __shfl_xor(dsum, 32);
    const double cx = x - net.cent.x, cy = y - net.cent.y;
    const float g1 = (float)sqrt(dmin2), g2 = (float)sqrt(cx * cx + cy * cy), g3 = (float)(dsum / (double)net.neig);

    // coordinate path: phi (26 inputs, two groups of 16) -> 64 -> 64
    v4f hin[2];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc)
#pragma unroll
        for (int i = 0; i < 4; ++i) hin[kc][i] = fourier(16 * kc + 4 * q + i, x, y);
    v4f t1[8], h3[8];
    dense<64, 2>(net.packed + kPc1 / 4, net.raw + kBc1, hin, t1, lane);
#pragma unroll
    for (int oc = 0; oc < 4; ++oc) t1[oc] = silu4(t1[oc]);
    dense<64, 4>(net.packed + kPc2 / 4, net.raw + kBc2, t1, h3, lane);
#pragma unroll
    for (int oc = 0; oc < 4; ++oc) h3[oc] = silu4(h3[oc]);

    // matrix path: [g1, g2, g3] (the global features are in the folded bias) -> 128 -> 64
    v4f gin[1];
    gin[0][0] = q == 0 ? g1 : 0.0f;
    gin[0][1] = q == 0 ? g2 : 0.0f;
    gin[0][2] = q == 0 ? g3 : 0.0f;
    gin[0][3] = 0.0f;
    dense<128, 1>(net.packed + kPm1 / 4, net.bfold, gin, t1, lane);
#pragma unroll
    for (int oc = 0; oc < 8; ++oc) t1[oc] = silu4(t1[oc]);
    dense<64, 8>(net.packed + kPm2 / 4, net.raw + kBm2, t1, h3 + 4, lane);
#pragma unroll
    for (int oc = 4; oc < 8; ++oc) h3[oc] = silu4(h3[oc]);

    // h4 = SiLU(W4 [h_c2, h_m2] + b4); h6 = h4 + SiLU(W5 h4 + b5)
    v4f h4[8];
    dense<128, 8>(net.packed + kP4 / 4, net.raw + kB4, h3, h4, lane);
#pragma unroll
    for (int oc = 0; oc < 8; ++oc) h4[oc] = silu4(h4[oc]);
    dense<128, 8>(net.packed + kP5 / 4, net.raw + kB5, h4, t1, lane);
#pragma unroll
    for (int oc = 0; oc < 8; ++oc) t1[oc] = h4[oc] + silu4(t1[oc]);

    // h7 = SiLU(W7 h6 + b7); p = logistic(w . h7 + b)
    v4f h7[4];
    dense<64, 8>(net.packed + kP7 / 4, net.raw + kB7, t1, h7, lane);
    float part = 0.0f;
#pragma unroll
    for (int oc = 0; oc < 4; ++oc) {
        const float4 w = *(const float4 *)(net.raw + kWout + 16 * oc + 4 * q);
        const v4f a = silu4(h7[oc]);
        part = fmaf(w.x, a[0], part);
        part = fmaf(w.y, a[1], part);
        part = fmaf(w.z, a[2], part);
        part = fmaf(w.w, a[3], part);
    }
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    return logistic(part + net.raw[kBout]);
}

// Grid coordinate of Sec. 2.1 (inclusive ends; a single point sits at the start).
__device__ __forceinline__ double grid_x(const GridArgs &g, int64_t j) {
    return g.nx > 1 ? g.a + ((g.b - g.a) * (double)j) / (double)(g.nx - 1) : g.a;
}
__device__ __forceinline__ double grid_y(const GridArgs &g, int64_t i) {
    return g.ny > 1 ? g.c + ((g.d - g.c) * (double)i) / (double)(g.ny - 1) : g.c;
}

__global__ void __launch_bounds__(kBlock) k_pack(const float *__restrict__ raw, float *__restrict__ packed) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kPackedFloats) return;
    // which packed matrix
    int base, O, K, KC, woff, col0;
    if (t < kPc2) { base = kPc1; O = 64; K = 26; KC = 2; woff = kWc1; col0 = 0; }
    else if (t < kPm1) { base = kPc2; O = 64; K = 64; KC = 4; woff = kWc2; col0 = 0; }
    else if (t < kPm2) { base = kPm1; O = 128; K = 3; KC = 1; woff = kWm1; col0 = 30; }
    else if (t < kP4) { base = kPm2; O = 64; K = 128; KC = 8; woff = kWm2; col0 = 0; }
    else if (t < kP5) { base = kP4; O = 128; K = 128; KC = 8; woff = kW4; col0 = 0; }
    else if (t < kP7) { base = kP5; O = 128; K = 128; KC = 8; woff = kW5; col0 = 0; }
    else { base = kP7; O = 64; K = 128; KC = 8; woff = kW7; col0 = 0; }
    const int r = (int)(t - base);
    const int i = r & 3, lane = (r >> 2) & 63, blk = r >> 8;
    const int oc = blk / KC, kc = blk % KC;
    const int o = 16 * oc + (lane & 15), k = 16 * kc + 4 * (lane >> 4) + i;
    // the row width of W in the parameter vector: 33 for m1 (its per-point columns start at 30)
    const int ld = woff == kWm1 ? 33 : K;
    packed[t] = (o < O && k < K) ? raw[woff + o * ld + col0 + k] : 0.0f;
}

// Per-matrix view of a (possibly batched) call: matrix m = blockIdx.y.  A single-matrix call
// has no device tables (gfeat / eig_off NULL) and one matrix.
struct Mat {
    const double2 *eig;
    int64_t neig;
    char *ws;          // this matrix's header (kWsHeader bytes)
};

__device__ __forceinline__ Mat mat_of(const Batch &b, const double2 *eig, int64_t neig, char *ws) {
    const int m = blockIdx.y;
    Mat r;
    if (b.eig_off) {
        const int64_t o0 = b.eig_off[m], o1 = b.eig_off[m + 1];
        r.eig = eig + o0;
        r.neig = o1 - o0;
    } else {
        r.eig = eig;
        r.neig = neig;
    }
    r.ws = ws + (int64_t)m * kWsHeader;
    return r;
}

__global__ void __launch_bounds__(kBlock) k_prep(const float *__restrict__ raw, Globals gf, Batch bt,
                                                 const double2 *__restrict__ eig, int64_t neig, char *ws,
                                                 int64_t *evals, int64_t evals0) {
    __shared__ double sx[kBlock], sy[kBlock];
    const Mat mt = mat_of(bt, eig, neig, ws);
    double ax = 0.0, ay = 0.0;
    for (int64_t e = threadIdx.x; e < mt.neig; e += kBlock) {
        ax += mt.eig[e].x;
        ay += mt.eig[e].y;
    }
    sx[threadIdx.x] = ax;
    sy[threadIdx.x] = ay;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sx[threadIdx.x] += sx[threadIdx.x + w];
            sy[threadIdx.x] += sy[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *(double2 *)(mt.ws + kWsCent) = make_double2(sx[0] / (double)mt.neig, sy[0] / (double)mt.neig);
        int64_t *ev = evals ? evals + blockIdx.y : (int64_t *)(mt.ws + kWsEvals);
        *ev = evals0;
    }
    if (threadIdx.x < 128) {
        const int o = threadIdx.x;
        const double *f = bt.gfeat ? bt.gfeat + (int64_t)blockIdx.y * kNGlobal : gf.f;
        double acc = raw[kBm1 + o];
        for (int k = 0; k < kNGlobal; ++k) acc += (double)raw[kWm1 + o * 33 + k] * f[k];
        ((float *)(mt.ws + kWsBfold))[o] = (float)acc;
    }
}

__global__ void __launch_bounds__(kBlock) k_points(const float *__restrict__ raw, const float *__restrict__ packed,
                                                   const double2 *__restrict__ eig, int64_t neig, const char *ws,
                                                   const double2 *__restrict__ z, int64_t npts, float *prob) {
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (tile * 16 >= npts) return;                      // uniform per wavefront
    const Net net = make_net(raw, packed, eig, neig, ws);
    const int64_t pt = tile * 16 + (lane & 15);
    const int64_t src = pt < npts ? pt : npts - 1;
    const double2 zz = z[src];
    const float p = eval_tile(net, zz.x, zz.y, lane);
    if (lane < 16 && pt < npts) prob[pt] = p;
}

__global__ void __launch_bounds__(kBlock) k_coarse(const float *__restrict__ raw, const float *__restrict__ packed,
                                                   Batch bt, const double2 *__restrict__ eig, int64_t neig, char *ws,
                                                   GridArgs g, int stride, int64_t ncx, int64_t ncoarse,
                                                   float *coarse) {
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (tile * 16 >= ncoarse) return;
    const Mat mt = mat_of(bt, eig, neig, ws);
    const Net net = make_net(raw, packed, mt.eig, mt.neig, mt.ws);
    const int64_t c = tile * 16 + (lane & 15);
    const int64_t cc = c < ncoarse ? c : ncoarse - 1;
    const int64_t I = cc / ncx, J = cc - I * ncx;
    const float p = eval_tile(net, grid_x(g, (int64_t)stride * J), grid_y(g, (int64_t)stride * I), lane);
    if (lane < 16 && c < ncoarse) coarse[(int64_t)blockIdx.y * ncoarse + c] = p;
}

// Order statistic of rank k of m floats by radix selection on order-preserving keys (one
// workgroup; 8 bits per pass).
__device__ __forceinline__ unsigned key_of(float v) {
    const unsigned b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float value_of(unsigned k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__device__ float select_rank(const float *__restrict__ v, int64_t m, int64_t k, unsigned *hist, int64_t *sk,
                             unsigned *sprefix) {
    unsigned prefix = 0, pmask = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int t = threadIdx.x; t < 256; t += blockDim.x) hist[t] = 0;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
            const unsigned key = key_of(v[i]);
            if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t kk = k;
            unsigned d = 0;
            for (; d < 255u; ++d) {
                if (kk < (int64_t)hist[d]) break;
                kk -= hist[d];
            }
            *sk = kk;
            *sprefix = prefix | (d << shift);
        }
        __syncthreads();
        k = *sk;
        prefix = *sprefix;
        pmask |= 255u << shift;
        __syncthreads();
    }
    return value_of(prefix);
}

// Bitonic sort of the m <= kSortMax order-preserving keys of one matrix in LDS (padded with the
// largest key), for the quantile.
constexpr int kSortMax = 8192;

__device__ void bitonic_sort(unsigned *key, int n) {
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < n / 2; t += blockDim.x) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const unsigned a = key[lo], b = key[hi];
                if ((a > b) == up) {
                    key[lo] = b;
                    key[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

// tau_coarse = v_(k) + (h - k)(v_(k+1) - v_(k)), h = q (m - 1), k = floor(h): the quantile of
// Sec. 3.5 by linear interpolation between order statistics, with contraction into fused
// multiply-adds switched off for the operators written here, so the value is the one the plain
// formula gives.  One workgroup per matrix.
__global__ void __launch_bounds__(kBlock) k_quantile(const float *__restrict__ coarse, int64_t m, double q, char *ws,
                                                     double *tau_out) {
#pragma clang fp contract(off)
    __shared__ unsigned keys[kSortMax];
    __shared__ unsigned hist[256];
    __shared__ int64_t sk;
    __shared__ unsigned sprefix;
    const float *v = coarse + (int64_t)blockIdx.x * m;
    const double h = q * (double)(m - 1);
    const int64_t k0 = (int64_t)floor(h);
    const double g = h - (double)k0;
    float v0, v1;
    if (m <= kSortMax) {
        int n = 2;
        while (n < m) n <<= 1;
        for (int i = threadIdx.x; i < n; i += blockDim.x) keys[i] = i < m ? key_of(v[i]) : 0xffffffffu;
        __syncthreads();
        bitonic_sort(keys, n);
        v0 = value_of(keys[k0]);
        v1 = k0 + 1 < m ? value_of(keys[k0 + 1]) : v0;
    } else {
        v0 = select_rank(v, m, k0, hist, &sk, &sprefix);
        v1 = k0 + 1 < m ? select_rank(v, m, k0 + 1, hist, &sk, &sprefix) : v0;
    }
    if (threadIdx.x == 0) {
        const double tau = (double)v0 + g * ((double)v1 - (double)v0);
        *(double *)(ws + (int64_t)blockIdx.x * kWsHeader + kWsTau) = tau;
        if (tau_out) tau_out[blockIdx.x] = tau;
    }
}

// One wavefront per 16-point tile of a coarse cell (ceil(s^2 / 16) tiles per cell, s = stride):
// if the cell's coarse value reaches tau_coarse, p at the tile's fine points, else probability
// 0 there.  (No loop over tiles inside a wavefront: the weight loads are the same for every
// tile, and a loop would invite the compiler to hoist all of them into registers.)
__global__ void __launch_bounds__(kBlock) k_fine(const float *__restrict__ raw, const float *__restrict__ packed,
                                                 Batch bt, const double2 *__restrict__ eig, int64_t neig, char *ws,
                                                 GridArgs g, int stride, int64_t ncx, int64_t ncells, int tpc,
                                                 const float *__restrict__ coarse, float *prob, int64_t *evals) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (wid >= ncells * tpc) return;
    const int64_t cell = wid / tpc;
    const int t0 = (int)(wid - cell * tpc) * 16;
    const int64_t I = cell / ncx, J = cell - I * ncx;
    const int64_t r0 = (int64_t)stride * I, c0 = (int64_t)stride * J;
    const int h = (int)(r0 + stride <= g.ny ? stride : g.ny - r0);
    const int w = (int)(c0 + stride <= g.nx ? stride : g.nx - c0);
    const int cnt = h * w;
    if (t0 >= cnt) return;                               // a tile past a cut cell's points
    const Mat mt = mat_of(bt, eig, neig, ws);
    float *pm = prob + (int64_t)blockIdx.y * g.nx * g.ny;
    const bool sel = (double)coarse[(int64_t)blockIdx.y * ncells + cell] >= *(const double *)(mt.ws + kWsTau);
    const int li = t0 + (lane & 15);
    const int lc = li < cnt ? li : cnt - 1;
    const int64_t i = r0 + lc / w, j = c0 + lc % w;
    if (!sel) {
        if (lane < 16 && li < cnt) pm[i * g.nx + j] = 0.0f;
        return;
    }
    if (lane == 0) {
        int64_t *ev = evals ? evals + blockIdx.y : (int64_t *)(mt.ws + kWsEvals);
        atomicAdd((unsigned long long *)ev, (unsigned long long)(cnt - t0 < 16 ? cnt - t0 : 16));
    }
    const Net net = make_net(raw, packed, mt.eig, mt.neig, mt.ws);
    const float p = eval_tile(net, grid_x(g, j), grid_y(g, i), lane);
    if (lane < 16 && li < cnt) pm[i * g.nx + j] = p;
}

// mask = the points within the (2r+1) x (2r+1) square of a point with p >= tau.
__global__ void __launch_bounds__(kBlock) k_dilate(const float *__restrict__ prob, int64_t nx, int64_t ny, double tau,
                                                   int r, uint8_t *mask) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nx * ny) return;
    const float *pm = prob + (int64_t)blockIdx.y * nx * ny;
    const int64_t i = t / nx, j = t - i * nx;
    const int64_t i0 = i - r > 0 ? i - r : 0, i1 = i + r < ny - 1 ? i + r : ny - 1;
    const int64_t j0 = j - r > 0 ? j - r : 0, j1 = j + r < nx - 1 ? j + r : nx - 1;
    uint8_t hit = 0;
    for (int64_t a = i0; a <= i1 && !hit; ++a)
        for (int64_t b = j0; b <= j1; ++b)
            if ((double)pm[a * nx + b] >= tau) {
                hit = 1;
                break;
            }
    mask[(int64_t)blockIdx.y * nx * ny + t] = hit;
}

// ------------------------------------------------------------------ threshold calibration
// Sec. 3.6: per validation matrix and candidate tau, recall of the prediction {p >= tau} dilated
// by a square of radius rp against the labels dilated by a square of radius rl.  A point lies
// in the dilated prediction at tau exactly when the maximum of p over its (2 rp + 1)^2 window
// is >= tau, so one pass per point bins the labelled points by how many candidates they pass.

__global__ void __launch_bounds__(kBlock) k_cal_zero(int64_t *cnt, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) cnt[t] = 0;
}

__global__ void __launch_bounds__(kBlock) k_cal_count(const float *__restrict__ prob,
                                                      const uint8_t *__restrict__ label, int64_t nx, int64_t ny,
                                                      int rp, int rl, Taus taus, int ntau, int64_t *nlab,
                                                      int64_t *hist) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nx * ny) return;
    const int m = blockIdx.y;
    const uint8_t *L = label + (int64_t)m * nx * ny;
    const float *P = prob + (int64_t)m * nx * ny;
    const int64_t i = t / nx, j = t - i * nx;
    bool lab = false;
    for (int64_t a = (i - rl > 0 ? i - rl : 0); a <= (i + rl < ny - 1 ? i + rl : ny - 1) && !lab; ++a)
        for (int64_t b = (j - rl > 0 ? j - rl : 0); b <= (j + rl < nx - 1 ? j + rl : nx - 1); ++b)
            if (L[a * nx + b]) {
                lab = true;
                break;
            }
    if (!lab) return;
    atomicAdd((unsigned long long *)(nlab + m), 1ull);
    float pmax = -INFINITY;
    for (int64_t a = (i - rp > 0 ? i - rp : 0); a <= (i + rp < ny - 1 ? i + rp : ny - 1); ++a)
        for (int64_t b = (j - rp > 0 ? j - rp : 0); b <= (j + rp < nx - 1 ? j + rp : nx - 1); ++b)
            pmax = fmaxf(pmax, P[a * nx + b]);
    const double pm = (double)pmax;
    int k = 0;
    while (k < ntau && taus.t[k] <= pm) ++k;
    if (k > 0) atomicAdd((unsigned long long *)(hist + (int64_t)m * ntau + (k - 1)), 1ull);
}

// v_(k) + (h - k)(v_(k+1) - v_(k)) at h = q (n - 1) on sorted v (no fused multiply-add).
__device__ double quantile_sorted(const double *v, int n, double q) {
#pragma clang fp contract(off)
    const double h = q * (double)(n - 1);
    const int k = (int)floor(h);
    const double g = h - (double)k;
    const double v0 = v[k], v1 = k + 1 < n ? v[k + 1] : v0;
    return v0 + g * (v1 - v0);
}

__global__ void __launch_bounds__(kBlock) k_cal_select(const int64_t *__restrict__ nlab,
                                                       const int64_t *__restrict__ hist, int nval, int ntau,
                                                       double median_min, double p10_min, double *recall_out,
                                                       double *median_out, double *p10_out, int32_t *index_out) {
    __shared__ double rec[kCalMaxVal];
    __shared__ double srt[kCalMaxVal];
    __shared__ int first, last;
    if (threadIdx.x == 0) first = last = -1;
    for (int k = 0; k < ntau; ++k) {
        for (int m = threadIdx.x; m < nval; m += blockDim.x) {
            int64_t hit = 0;
            for (int i = k; i < ntau; ++i) hit += hist[(int64_t)m * ntau + i];
            const int64_t nl = nlab[m];
            const double r = nl > 0 ? (double)hit / (double)nl : 1.0;
            rec[m] = r;
            if (recall_out) recall_out[(int64_t)m * ntau + k] = r;
        }
        __syncthreads();
        for (int m = threadIdx.x; m < nval; m += blockDim.x) {
            int r = 0;
            for (int j = 0; j < nval; ++j) r += (rec[j] < rec[m]) || (rec[j] == rec[m] && j < m);
            srt[r] = rec[m];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const double med = quantile_sorted(srt, nval, 0.5), p10 = quantile_sorted(srt, nval, 0.1);
            if (median_out) median_out[k] = med;
            if (p10_out) p10_out[k] = p10;
            if (med >= median_min && p10 >= p10_min) {
                if (first < 0) first = k;
                last = k;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        index_out[0] = first;
        index_out[1] = last;
    }
}

int64_t blocks_for(int64_t n, int64_t per) { return (n + per - 1) / per; }

}  // namespace

hipError_t launch_pack(const float *raw, float *packed, hipStream_t s) {
    hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks_for(kPackedFloats, kBlock)), dim3(kBlock), 0, s, raw, packed);
    return hipGetLastError();
}

hipError_t launch_prep(const float *raw, const Globals &gf, const Batch &bt, int nmat, const double2 *eig,
                       int64_t neig, char *ws, int64_t *evals, int64_t evals0, hipStream_t s) {
    hipLaunchKernelGGL(k_prep, dim3(1, nmat), dim3(kBlock), 0, s, raw, gf, bt, eig, neig, ws, evals, evals0);
    return hipGetLastError();
}

hipError_t launch_points(const float *raw, const float *packed, const double2 *eig, int64_t neig, const char *ws,
                         const double2 *z, int64_t npts, float *prob, hipStream_t s) {
    if (npts == 0) return hipSuccess;
    const int64_t tiles = blocks_for(npts, 16);
    hipLaunchKernelGGL(k_points, dim3((unsigned)blocks_for(tiles, kBlock / 64)), dim3(kBlock), 0, s, raw, packed,
                       eig, neig, ws, z, npts, prob);
    return hipGetLastError();
}

hipError_t launch_mask(const float *raw, const float *packed, const Batch &bt, int nmat, const double2 *eig,
                       int64_t neig, char *ws, const GridArgs &g, int stride, int dilate, double coarse_q, double tau,
                       float *coarse, float *prob, uint8_t *mask, int64_t *evals, double *tau_coarse_out,
                       hipStream_t s) {
    const int64_t ncy = (g.ny + stride - 1) / stride, ncx = (g.nx + stride - 1) / stride;
    const int64_t ncoarse = ncy * ncx;
    hipLaunchKernelGGL(k_coarse, dim3((unsigned)blocks_for(blocks_for(ncoarse, 16), kBlock / 64), nmat), dim3(kBlock),
                       0, s, raw, packed, bt, eig, neig, ws, g, stride, ncx, ncoarse, coarse);
    hipLaunchKernelGGL(k_quantile, dim3(nmat), dim3(kBlock), 0, s, coarse, ncoarse, coarse_q, ws, tau_coarse_out);
    const int tpc = (stride * stride + 15) / 16;
    hipLaunchKernelGGL(k_fine, dim3((unsigned)blocks_for(ncoarse * tpc, kBlock / 64), nmat), dim3(kBlock), 0, s, raw,
                       packed, bt, eig, neig, ws, g, stride, ncx, ncoarse, tpc, coarse, prob, evals);
    hipLaunchKernelGGL(k_dilate, dim3((unsigned)blocks_for(g.nx * g.ny, kBlock), nmat), dim3(kBlock), 0, s, prob, g.nx,
                       g.ny, tau, (dilate - 1) / 2, mask);
    return hipGetLastError();
}

hipError_t launch_calibrate(const float *prob, const uint8_t *label, int nval, int64_t nx, int64_t ny, int rp, int rl,
                            const Taus &taus, int ntau, double median_min, double p10_min, int64_t *counts,
                            double *recall, double *median, double *p10, int32_t *index, hipStream_t s) {
    const int64_t ncnt = (int64_t)nval * (ntau + 1);
    int64_t *nlab = counts, *hist = counts + nval;
    hipLaunchKernelGGL(k_cal_zero, dim3((unsigned)blocks_for(ncnt, kBlock)), dim3(kBlock), 0, s, counts, ncnt);
    hipLaunchKernelGGL(k_cal_count, dim3((unsigned)blocks_for(nx * ny, kBlock), nval), dim3(kBlock), 0, s, prob, label,
                       nx, ny, rp, rl, taus, ntau, nlab, hist);
    hipLaunchKernelGGL(k_cal_select, dim3(1), dim3(kBlock), 0, s, nlab, hist, nval, ntau, median_min, p10_min, recall,
                       median, p10, index);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace ps
