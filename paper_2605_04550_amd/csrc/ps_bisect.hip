// Host launchers of the inertia-bisection kernel, the Gram band it reads, and the batch plan
// (queue positions per (kl, ku) class and the longest-first chunk order).
#include "ps_bisect.hpp"

namespace ps {

BisKernel pick_bis_h1(bool batch, int ktm, int lanes);
BisKernel pick_bis_h2(bool batch, int ktm, int lanes);
BisKernel pick_bis_h3(bool batch, int ktm, int lanes);
BisKernel pick_bis_h4(bool batch, int ktm, int lanes);
BisKernel pick_bis_h5(bool batch, int ktm, int lanes);
BisKernel pick_bis_h6(bool batch, int ktm, int lanes);
BisKernel pick_bis_h7(bool batch, int ktm, int lanes);
BisKernel pick_bis_h8(bool batch, int ktm, int lanes);

namespace {

// Row i of the Gram band (doubles, stride gram_stride(hb)):
//   [0] G[i][i] (real), [1] 2 Re A[i][i], [2] 2 Im A[i][i], [3] 0,
//   then for e = 1 .. hb at 4 + 6 (e - 1): G[i][i-e], s_e, d_e (complex), with
//   G = A^H A, s_e = A[i][i-e] + conj(A[i-e][i]), d_e = A[i][i-e] - conj(A[i-e][i]);
// entries with i - e < 0 are zero, and so are the rows past n.
// G[i][i-e] = sum_r conj(A[r][i]) A[r][i-e] over the rows r in [i - ku, i - e + kl].
__global__ void k_gram_band(const double2 *arow, int64_t n, int kl, int ku, int64_t rows, double *gram) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    const int w = kl + ku + 1, hb = kl + ku, rs = bis::gram_stride(hb);
    double *out = gram + i * rs;
    for (int k = 0; k < rs; ++k) out[k] = 0.0;
    if (i >= n) return;
    // A[r][c] from the row band (zero outside the band and the matrix)
    auto at = [&](int64_t r, int64_t c) -> double2 {
        const int64_t d = c - r + kl;
        if (r < 0 || r >= n || c < 0 || c >= n || d < 0 || d >= w) return make_double2(0.0, 0.0);
        return arow[r * w + d];
    };
    for (int e = 0; e <= hb && e <= i; ++e) {
        double gx = 0.0, gy = 0.0;
        for (int64_t r = i - ku; r <= i - e + kl; ++r) {
            const double2 p = at(r, i), q = at(r, i - e);
            // conj(p) * q
            gx += p.x * q.x + p.y * q.y;
            gy += p.x * q.y - p.y * q.x;
        }
        const double2 al = e <= kl ? at(i, i - e) : make_double2(0.0, 0.0);
        const double2 up = e <= ku ? at(i - e, i) : make_double2(0.0, 0.0);
        const double2 au = make_double2(up.x, -up.y);
        if (e == 0) {
            out[0] = gx;
            out[1] = 2.0 * al.x;
            out[2] = 2.0 * al.y;
        } else {
            double *o = out + 4 + 6 * (e - 1);
            o[0] = gx;
            o[1] = gy;
            o[2] = al.x + au.x;
            o[3] = al.y + au.y;
            o[4] = al.x - au.x;
            o[5] = al.y - au.y;
        }
    }
}

constexpr int kPlanBlock = 256;

// Block-wide inclusive scan of one int64 per thread.
__device__ int64_t block_incl_scan(int64_t v, int64_t *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kPlanBlock; o <<= 1) {
        const int64_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    const int64_t r = sh[threadIdx.x];
    __syncthreads();
    return r;
}

// The batch plan, one workgroup:
//   pfx[p]        exclusive prefix of the counts over the class-sorted matrices,
//   mfirst[p]     queue position of matrix p inside its class (pfx[p] - pfx[first of class]),
//   ctotal[c]     shifts of class c,
//   chunkfirst[k] first chunk of the k-th matrix in longest-first order (chunks of spw shifts),
//   *total        number of chunks; gk_count[c] = 0.
__global__ void __launch_bounds__(kPlanBlock) k_bis_plan(const MatDesc *cls_order, const MatDesc *lpt_order, int nmat,
                                                         int nclass, const int64_t *counts, int spw, int64_t *pfx,
                                                         int64_t *mfirst, int64_t *ctotal, int64_t *chunkfirst,
                                                         int64_t *total, int64_t *gk_count) {
    __shared__ int64_t sh[kPlanBlock];
    int64_t carry = 0;
    for (int base = 0; base < nmat; base += kPlanBlock) {
        const int p = base + (int)threadIdx.x;
        const int64_t v = p < nmat ? counts[cls_order[p].cidx] : 0;
        const int64_t inc = block_incl_scan(v, sh);
        if (p < nmat) pfx[p] = carry + inc - v;
        if (threadIdx.x == kPlanBlock - 1) sh[0] = inc;
        __syncthreads();
        carry += sh[0];
        __syncthreads();
    }
    const int64_t all = carry;
    __syncthreads();
    for (int p = (int)threadIdx.x; p < nmat; p += kPlanBlock) {
        mfirst[p] = pfx[p] - pfx[cls_order[p].cfirst];
    }
    for (int c = (int)threadIdx.x; c < nclass; c += kPlanBlock) gk_count[c] = 0;
    __syncthreads();
    // class totals: the last matrix of a class ends it
    for (int p = (int)threadIdx.x; p < nmat; p += kPlanBlock) {
        const bool last = p == nmat - 1 || cls_order[p + 1].cls != cls_order[p].cls;
        if (last) ctotal[cls_order[p].cls] = (p == nmat - 1 ? all : pfx[p + 1]) - pfx[cls_order[p].cfirst];
    }
    carry = 0;
    for (int base = 0; base < nmat; base += kPlanBlock) {
        const int k = base + (int)threadIdx.x;
        const int64_t v = k < nmat ? (counts[lpt_order[k].cidx] + spw - 1) / spw : 0;
        const int64_t inc = block_incl_scan(v, sh);
        if (k < nmat) chunkfirst[k] = carry + inc - v;
        if (threadIdx.x == kPlanBlock - 1) sh[0] = inc;
        __syncthreads();
        carry += sh[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// Sorts each list of shifts handed to the Golub-Kahan kernel (one workgroup per list; the
// first pass appends to them in no particular order) into increasing queue position, so that
// the lanes of a Golub-Kahan wavefront take neighbouring shifts of one matrix: their band
// reads coincide and their step counts are alike.  Lists longer than kSortMax stay as they are.
constexpr int kSortMax = 8192;

__global__ void __launch_bounds__(kPlanBlock) k_sort_lists(int64_t *lists, ListBases bases, const int64_t *counts) {
    __shared__ int64_t v[kSortMax];
    int64_t *list = lists + bases.base[blockIdx.x];
    const int64_t cnt = counts[blockIdx.x];
    if (cnt < 2 || cnt > kSortMax) return;
    int m = 1;
    while (m < cnt) m <<= 1;
    for (int i = (int)threadIdx.x; i < m; i += kPlanBlock) v[i] = i < cnt ? list[i] : INT64_MAX;
    __syncthreads();
    for (int k = 2; k <= m; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = (int)threadIdx.x; i < m; i += kPlanBlock) {
                const int p = i ^ j;
                if (p > i) {
                    const bool up = (i & k) == 0;
                    const int64_t a = v[i], b = v[p];
                    if ((a > b) == up) {
                        v[i] = b;
                        v[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = (int)threadIdx.x; i < cnt; i += kPlanBlock) list[i] = v[i];
}

}  // namespace

hipError_t launch_sort_lists(int64_t *lists, const ListBases &bases, const int64_t *counts, int nlists,
                             hipStream_t st) {
    if (nlists < 1) return hipSuccess;
    hipLaunchKernelGGL(k_sort_lists, dim3((unsigned)nlists), dim3(kPlanBlock), 0, st, lists, bases, counts);
    return hipGetLastError();
}

// Batch kernels exist for even largest half-bandwidths (they compile in every smaller one).
BisKernel pick_bis(bool batch, int hb, int ktm, int lanes) {
    if (batch) hb = (hb + 1) & ~1;
    switch (hb) {
    case 1: return pick_bis_h1(batch, ktm, lanes);
    case 2: return pick_bis_h2(batch, ktm, lanes);
    case 3: return pick_bis_h3(batch, ktm, lanes);
    case 4: return pick_bis_h4(batch, ktm, lanes);
    case 5: return pick_bis_h5(batch, ktm, lanes);
    case 6: return pick_bis_h6(batch, ktm, lanes);
    case 7: return pick_bis_h7(batch, ktm, lanes);
    case 8: return pick_bis_h8(batch, ktm, lanes);
    }
    return nullptr;
}

int64_t gram_rows(int64_t n) { return n + 8; }
size_t gram_bytes(int64_t n, int kl, int ku) {
    return sizeof(double) * (size_t)gram_rows(n) * (size_t)bis::gram_stride(kl + ku);
}

hipError_t launch_gram_band(const double2 *arow, int64_t n, int kl, int ku, double *gram, hipStream_t st) {
    const int64_t rows = gram_rows(n);
    hipLaunchKernelGGL(k_gram_band, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, arow, n, kl, ku, rows,
                       gram);
    return hipGetLastError();
}

hipError_t launch_bis(const BisArgs &a, int hb, int ktm, int lanes, int64_t chunks, hipStream_t st) {
    // a wavefront per shift already tests 64 points per pass: one test per lane
    BisKernel k = pick_bis(a.batch != 0, hb, lanes == 64 ? 0 : ktm, lanes);
    if (!k) return hipErrorInvalidValue;
    if (chunks < 1) return hipSuccess;
    hipLaunchKernelGGL(k, dim3((unsigned)chunks), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_bis_plan(const MatDesc *cls_order, const MatDesc *lpt_order, int nmat, int nclass,
                           const int64_t *counts, int spw, int64_t *pfx, int64_t *mfirst, int64_t *ctotal,
                           int64_t *chunkfirst, int64_t *total, int64_t *gk_count, hipStream_t st) {
    hipLaunchKernelGGL(k_bis_plan, dim3(1), dim3(kPlanBlock), 0, st, cls_order, lpt_order, nmat, nclass, counts, spw,
                       pfx, mfirst, ctotal, chunkfirst, total, gk_count);
    return hipGetLastError();
}

}  // namespace ps
