// Launchers of the persistent sigma_min kernel (instantiated in ps_eval_kl<K>.hip) and the
// small kernels around it: queue and count set-up, mask compaction (a block scan over the
// mask, then a scatter of the selected flat indices in grid order), the batch variants of
// both, workspace carving, the adjoint (gradients of sigma_min with respect to z and to the
// band of A), seeds on the eps-level curve from grid-edge sign changes, the Newton update of
// contour points, and the exclusion-region labelling of the sensitive zone.

#include "ps_eval.hpp"

namespace ps {

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

// Queue order of a call with vectors: the shifts the bisection settled (saved passes >= 0)
// first, then those on the Golub-Kahan path, each in queue order.  A wavefront then holds
// shifts of one kind: a lane computing its vectors by inverse iteration and a lane on the
// Golub-Kahan path would otherwise pay for each other's work every cycle.  np is indexed by
// output position: the flat index of the tile order for a full grid, the queue position
// otherwise (as the bisection kernel saved it).
__device__ __forceinline__ int64_t part_out_pos(int mode, const int64_t *idx, int64_t q, int64_t nx, int64_t ny) {
    return (mode != kShiftList && !idx) ? tile_flat(q, nx, ny) : q;
}

__global__ void __launch_bounds__(kScanBlock) k_part_count(const int32_t *np, const int64_t *count, int mode,
                                                           const int64_t *idx, int64_t nx, int64_t ny,
                                                           int64_t *blocksums) {
    __shared__ int64_t sh[kScanBlock];
    const int64_t cnt = *count;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t c = 0;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < cnt && np[part_out_pos(mode, idx, base + q, nx, ny)] >= 0) ++c;
    int64_t total;
    block_scan(c, sh, total);
    if (threadIdx.x == 0) blocksums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) k_part_scatter(const int32_t *np, const int64_t *count, int mode,
                                                             const int64_t *idx, int64_t nx, int64_t ny,
                                                             const int64_t *blocksums, const int64_t *nbis,
                                                             int64_t *perm) {
    __shared__ int64_t sh[kScanBlock];
    const int64_t cnt = *count, nb = *nbis;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    bool bis[kScanItems];
    int64_t c = 0;
    for (int q = 0; q < kScanItems; ++q) {
        bis[q] = base + q < cnt && np[part_out_pos(mode, idx, base + q, nx, ny)] >= 0;
        c += bis[q] ? 1 : 0;
    }
    int64_t total;
    int64_t pos = blocksums[blockIdx.x] + block_scan(c, sh, total);   // settled shifts before base
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t i = base + q;
        if (i >= cnt) break;
        if (bis[q]) perm[pos++] = i;
        else perm[nb + (i - pos)] = i;      // i - pos: Golub-Kahan shifts before i
    }
}

// ------------------------------------------------------------------------ contour seeds
// Edge e of an nx x ny grid: the first ny (nx - 1) edges are horizontal, (i, j)-(i, j+1) in
// row-major order; the next (ny - 1) nx are vertical, (i, j)-(i+1, j).  An edge seeds the
// eps-level curve when its ends lie on different sides of sigma <= eps.

struct EdgeGrid {
    double a, b, c, d;
    int64_t nx, ny, nh, ne;   // nh horizontal edges, ne edges in all
};

__device__ __forceinline__ void edge_ends(const EdgeGrid &g, int64_t e, int64_t &p1, int64_t &p2) {
    if (e < g.nh) {
        const int64_t i = e / (g.nx - 1), j = e - i * (g.nx - 1);
        p1 = i * g.nx + j;
        p2 = p1 + 1;
    } else {
        p1 = e - g.nh;
        p2 = p1 + g.nx;
    }
}

__device__ __forceinline__ bool edge_flag(const EdgeGrid &g, const double *sigma, double eps, int64_t e) {
    if (e >= g.ne) return false;
    int64_t p1, p2;
    edge_ends(g, e, p1, p2);
    return (sigma[p1] <= eps) != (sigma[p2] <= eps);
}

__device__ __forceinline__ cd edge_grid_point(const EdgeGrid &g, int64_t flat) {
    const int64_t i = flat / g.nx, j = flat - i * g.nx;
    const double x = g.nx > 1 ? __dadd_rn(g.a, __ddiv_rn(__dmul_rn(g.b - g.a, (double)j), (double)(g.nx - 1))) : g.a;
    const double y = g.ny > 1 ? __dadd_rn(g.c, __ddiv_rn(__dmul_rn(g.d - g.c, (double)i), (double)(g.ny - 1))) : g.c;
    return C(x, y);
}

__global__ void __launch_bounds__(kScanBlock) k_edge_count(EdgeGrid g, const double *sigma, double eps,
                                                           int64_t *blocksums) {
    __shared__ int64_t sh[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t c = 0;
    for (int q = 0; q < kScanItems; ++q) c += edge_flag(g, sigma, eps, base + q) ? 1 : 0;
    int64_t total;
    block_scan(c, sh, total);
    if (threadIdx.x == 0) blocksums[blockIdx.x] = total;
}

// Seed on a flagged edge z1 -> z2: z1 + tau (z2 - z1), tau = (ln eps - ln s1)/(ln s2 - ln s1),
// sigma clamped to the smallest normal double before the logarithm.
__global__ void __launch_bounds__(kScanBlock) k_edge_scatter(EdgeGrid g, const double *sigma, double eps,
                                                             const int64_t *blocksums, double2 *seeds,
                                                             int64_t max_seeds) {
    __shared__ int64_t sh[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t c = 0;
    for (int q = 0; q < kScanItems; ++q) c += edge_flag(g, sigma, eps, base + q) ? 1 : 0;
    int64_t total;
    int64_t pos = blocksums[blockIdx.x] + block_scan(c, sh, total);
    const double le = log(eps);
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t e = base + q;
        if (!edge_flag(g, sigma, eps, e)) continue;
        if (pos < max_seeds) {
            int64_t p1, p2;
            edge_ends(g, e, p1, p2);
            const double l1 = log(fmax(sigma[p1], 0x1p-1022)), l2 = log(fmax(sigma[p2], 0x1p-1022));
            const double tau = (le - l1) / (l2 - l1);
            const cd z1 = edge_grid_point(g, p1), z2 = edge_grid_point(g, p2);
            seeds[pos] = C(fma(tau, z2.x - z1.x, z1.x), fma(tau, z2.y - z1.y, z1.y));
        }
        ++pos;
    }
}

int64_t contour_edge_tiles(int64_t nx, int64_t ny) {
    const int64_t ne = ny * (nx - 1) + (ny - 1) * nx;
    const int64_t nt = (ne + kScanTile - 1) / kScanTile;
    return nt > 0 ? nt : 1;
}

hipError_t launch_contour_seeds(double a, double b, double c, double d, int64_t nx, int64_t ny, const double *sigma,
                                double eps, double2 *seeds, int64_t max_seeds, int64_t *count, int64_t *blocksums,
                                unsigned long long *scratch_queue, hipStream_t st) {
    EdgeGrid g;
    g.a = a;
    g.b = b;
    g.c = c;
    g.d = d;
    g.nx = nx;
    g.ny = ny;
    g.nh = ny * (nx - 1);
    g.ne = g.nh + (ny - 1) * nx;
    const int64_t nt = contour_edge_tiles(nx, ny);
    hipLaunchKernelGGL(k_edge_count, dim3((unsigned)nt), dim3(kScanBlock), 0, st, g, sigma, eps, blocksums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, blocksums, nt, count, scratch_queue);
    hipLaunchKernelGGL(k_edge_scatter, dim3((unsigned)nt), dim3(kScanBlock), 0, st, g, sigma, eps,
                       (const int64_t *)blocksums, seeds, max_seeds);
    return hipGetLastError();
}

// ------------------------------------------------------------------------ exclusion-region labels
// Status of a grid point: 0 unknown, 1 sigma <= eps (evaluated), 2 sigma > eps (evaluated, or
// inside the exclusion disk of an evaluated point), 3 undecided: the evaluation stopped at its
// iteration cap (PS_PT_MAXITER) with an estimate above eps.  A capped estimate is not the
// certified value: such a point gets no exclusion disk, and it is labelled 1 only when the
// estimate, an upper bound of sigma_min on the Golub-Kahan path, is <= eps.

// The outcome of an evaluated point from its sigma and info word.
__device__ __forceinline__ uint8_t label_status(double sg, int32_t info, double eps) {
    const bool capped = (info & PS_PT_MAXITER) != 0;
    if (sg <= eps && !(capped && (info & PS_PT_BISECT))) return 1;
    return capped ? 3 : 2;
}

__global__ void k_label_init(uint8_t *status, double *sig_out, int64_t npts, int64_t *evals) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < npts) {
        status[t] = 0;
        if (sig_out) sig_out[t] = -1.0;
    }
    if (t == 0 && evals) *evals = 0;
}

// Points of the lattice of the given stride that are still unknown (stride 1: all unknown).
__global__ void k_label_mask(const uint8_t *status, int64_t nx, int64_t npts, int stride, uint8_t *mask) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npts) return;
    const int64_t i = t / nx, j = t - i * nx;
    mask[t] = (uint8_t)(status[t] == 0 && i % stride == 0 && j % stride == 0);
}

__global__ void k_label_mark(const int64_t *idx, const int64_t *count, const double *sigma, const int32_t *info,
                             double eps, uint8_t *status, double *sig_out, int64_t *evals) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = *count;
    if (p == 0 && evals) *evals += c;
    if (p >= c) return;
    const int64_t f = idx[p];
    status[f] = label_status(sigma[p], info[p], eps);
    if (sig_out) sig_out[f] = sigma[p];
}

// One workgroup per evaluated point z0 with sigma(z0) > eps: sigma_min is 1-Lipschitz in z
// (|sigma(z) - sigma(z0)| <= |z - z0|), so every grid point with
// |z - z0| < sigma(z0) - eps - margin has sigma(z) > eps, where margin (twice the evaluation
// tolerance) covers the error of the computed sigma(z0).
__global__ void __launch_bounds__(256) k_label_exclude(EdgeGrid g, const int64_t *idx, const int64_t *count,
                                                       const double *sigma, const int32_t *info, double eps,
                                                       double tol_abs, double tol_rel, uint8_t *status) {
    const int64_t p = blockIdx.x;
    if (p >= *count) return;
    if (info[p] & PS_PT_MAXITER) return;       // not certified: no exclusion disk
    const double sg = sigma[p];
    const double rho = sg - eps - 2.0 * (tol_abs + tol_rel * sg);
    if (!(rho > 0.0)) return;
    const int64_t f = idx[p];
    const int64_t i0 = f / g.nx, j0 = f - i0 * g.nx;
    const cd z0 = edge_grid_point(g, f);
    const double hx = g.nx > 1 ? (g.b - g.a) / (double)(g.nx - 1) : 0.0;
    const double hy = g.ny > 1 ? (g.d - g.c) / (double)(g.ny - 1) : 0.0;
    const int64_t rj = hx > 0.0 ? (int64_t)fmin(rho / hx + 1.0, (double)g.nx) : 0;
    const int64_t ri = hy > 0.0 ? (int64_t)fmin(rho / hy + 1.0, (double)g.ny) : 0;
    const int64_t ilo = i0 - ri > 0 ? i0 - ri : 0, ihi = i0 + ri < g.ny - 1 ? i0 + ri : g.ny - 1;
    const int64_t jlo = j0 - rj > 0 ? j0 - rj : 0, jhi = j0 + rj < g.nx - 1 ? j0 + rj : g.nx - 1;
    const int64_t bw = jhi - jlo + 1, cells = (ihi - ilo + 1) * bw;
    for (int64_t q = threadIdx.x; q < cells; q += blockDim.x) {
        const int64_t i = ilo + q / bw, j = jlo + q % bw;
        const int64_t t = i * g.nx + j;
        if (status[t] != 0) continue;
        const cd zq = edge_grid_point(g, t);
        if (hypot(zq.x - z0.x, zq.y - z0.y) < rho) status[t] = 2;
    }
}

__global__ void k_label_finish(const uint8_t *status, uint8_t *label, int64_t npts) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < npts) label[t] = status[t] == 1 ? 1 : status[t] == 3 ? 2 : 0;
}

static EdgeGrid make_edge_grid(double a, double b, double c, double d, int64_t nx, int64_t ny) {
    EdgeGrid g;
    g.a = a;
    g.b = b;
    g.c = c;
    g.d = d;
    g.nx = nx;
    g.ny = ny;
    g.nh = ny * (nx - 1);
    g.ne = g.nh + (ny - 1) * nx;
    return g;
}

hipError_t launch_label_init(uint8_t *status, double *sig_out, int64_t npts, int64_t *evals, hipStream_t st) {
    hipLaunchKernelGGL(k_label_init, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, status, sig_out, npts,
                       evals);
    return hipGetLastError();
}

hipError_t launch_label_mask(const uint8_t *status, int64_t nx, int64_t npts, int stride, uint8_t *mask,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_label_mask, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, status, nx, npts, stride,
                       mask);
    return hipGetLastError();
}

hipError_t launch_label_update(double a, double b, double c, double d, int64_t nx, int64_t ny, const int64_t *idx,
                               const int64_t *count, int64_t max_count, const double *sigma, const int32_t *info,
                               double eps, double tol_abs, double tol_rel, uint8_t *status, double *sig_out,
                               int64_t *evals, hipStream_t st) {
    if (max_count < 1) return hipSuccess;
    hipLaunchKernelGGL(k_label_mark, dim3((unsigned)((max_count + 255) / 256)), dim3(256), 0, st, idx, count, sigma,
                       info, eps, status, sig_out, evals);
    const EdgeGrid g = make_edge_grid(a, b, c, d, nx, ny);
    hipLaunchKernelGGL(k_label_exclude, dim3((unsigned)max_count), dim3(256), 0, st, g, idx, count, sigma, info, eps,
                       tol_abs, tol_rel, status);
    return hipGetLastError();
}

hipError_t launch_label_finish(const uint8_t *status, uint8_t *label, int64_t npts, hipStream_t st) {
    hipLaunchKernelGGL(k_label_finish, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, status, label, npts);
    return hipGetLastError();
}

// Batched labelling: the same steps for every matrix of a batch at once.  Matrix m's points
// occupy [out_off, out_off + nx ny) of the concatenated status, mask, label and sigma arrays
// (its grid from its MatDesc); blockIdx.y is the matrix.

__global__ void k_blabel_init(const MatDesc *mats, uint8_t *status, double *sig_out, uint8_t *mask_base,
                              uint8_t **mask_ptrs, int64_t *evals) {
    const int m = blockIdx.y;
    const MatDesc d = mats[m];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < d.nx * d.ny) {
        status[d.out_off + t] = 0;
        if (sig_out) sig_out[d.out_off + t] = -1.0;
    }
    if (t == 0) mask_ptrs[m] = mask_base + d.out_off;
    if (t == 0 && m == 0 && evals) *evals = 0;
}

__global__ void k_blabel_mask(const MatDesc *mats, const uint8_t *status, int stride, uint8_t *mask) {
    const MatDesc d = mats[blockIdx.y];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d.nx * d.ny) return;
    const int64_t i = t / d.nx, j = t - i * d.nx;
    mask[d.out_off + t] = (uint8_t)(status[d.out_off + t] == 0 && i % stride == 0 && j % stride == 0);
}

__global__ void k_blabel_mark(const MatDesc *mats, const int64_t *idx, const int64_t *counts, const double *sigma,
                              const int32_t *info, double eps, uint8_t *status, double *sig_out, int64_t *evals) {
    const int m = blockIdx.y;
    const MatDesc d = mats[m];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = counts[m];
    if (p == 0 && evals) atomicAdd((unsigned long long *)evals, (unsigned long long)c);
    if (p >= c) return;
    const int64_t f = idx[d.out_off + p];
    const double sg = sigma[d.out_off + p];
    status[d.out_off + f] = label_status(sg, info[d.out_off + p], eps);
    if (sig_out) sig_out[d.out_off + f] = sg;
}

__global__ void __launch_bounds__(256) k_blabel_exclude(const MatDesc *mats, const int64_t *idx,
                                                        const int64_t *counts, const double *sigma,
                                                        const int32_t *info, double eps, double tol_norm,
                                                        double tol_rel, uint8_t *status) {
    const int m = blockIdx.y;
    const MatDesc d = mats[m];
    const int64_t p = blockIdx.x;
    if (p >= counts[m]) return;
    if (info[d.out_off + p] & PS_PT_MAXITER) return;   // not certified: no exclusion disk
    const double sg = sigma[d.out_off + p];
    const double rho = sg - eps - 2.0 * (tol_norm * d.normA + tol_rel * sg);
    if (!(rho > 0.0)) return;
    EdgeGrid g;
    g.a = d.ga;
    g.b = d.gb;
    g.c = d.gc;
    g.d = d.gd;
    g.nx = d.nx;
    g.ny = d.ny;
    g.nh = g.ne = 0;
    const int64_t f = idx[d.out_off + p];
    const int64_t i0 = f / g.nx, j0 = f - i0 * g.nx;
    const cd z0 = edge_grid_point(g, f);
    const double hx = g.nx > 1 ? (g.b - g.a) / (double)(g.nx - 1) : 0.0;
    const double hy = g.ny > 1 ? (g.d - g.c) / (double)(g.ny - 1) : 0.0;
    const int64_t rj = hx > 0.0 ? (int64_t)fmin(rho / hx + 1.0, (double)g.nx) : 0;
    const int64_t ri = hy > 0.0 ? (int64_t)fmin(rho / hy + 1.0, (double)g.ny) : 0;
    const int64_t ilo = i0 - ri > 0 ? i0 - ri : 0, ihi = i0 + ri < g.ny - 1 ? i0 + ri : g.ny - 1;
    const int64_t jlo = j0 - rj > 0 ? j0 - rj : 0, jhi = j0 + rj < g.nx - 1 ? j0 + rj : g.nx - 1;
    const int64_t bw = jhi - jlo + 1, cells = (ihi - ilo + 1) * bw;
    uint8_t *st = status + d.out_off;
    for (int64_t q = threadIdx.x; q < cells; q += blockDim.x) {
        const int64_t i = ilo + q / bw, j = jlo + q % bw;
        const int64_t t = i * g.nx + j;
        if (st[t] != 0) continue;
        const cd zq = edge_grid_point(g, t);
        if (hypot(zq.x - z0.x, zq.y - z0.y) < rho) st[t] = 2;
    }
}

hipError_t launch_blabel_init(const MatDesc *mats, int nmat, int64_t max_npts, uint8_t *status, double *sig_out,
                              uint8_t *mask_base, uint8_t **mask_ptrs, int64_t *evals, hipStream_t st) {
    hipLaunchKernelGGL(k_blabel_init, dim3((unsigned)((max_npts + 255) / 256), (unsigned)nmat), dim3(256), 0, st,
                       mats, status, sig_out, mask_base, mask_ptrs, evals);
    return hipGetLastError();
}

hipError_t launch_blabel_mask(const MatDesc *mats, int nmat, int64_t max_npts, const uint8_t *status, int stride,
                              uint8_t *mask, hipStream_t st) {
    hipLaunchKernelGGL(k_blabel_mask, dim3((unsigned)((max_npts + 255) / 256), (unsigned)nmat), dim3(256), 0, st,
                       mats, status, stride, mask);
    return hipGetLastError();
}

hipError_t launch_blabel_update(const MatDesc *mats, int nmat, int64_t max_count, const int64_t *idx,
                                const int64_t *counts, const double *sigma, const int32_t *info, double eps,
                                double tol_norm, double tol_rel, uint8_t *status, double *sig_out, int64_t *evals,
                                hipStream_t st) {
    if (max_count < 1) return hipSuccess;
    hipLaunchKernelGGL(k_blabel_mark, dim3((unsigned)((max_count + 255) / 256), (unsigned)nmat), dim3(256), 0, st,
                       mats, idx, counts, sigma, info, eps, status, sig_out, evals);
    hipLaunchKernelGGL(k_blabel_exclude, dim3((unsigned)max_count, (unsigned)nmat), dim3(256), 0, st, mats, idx,
                       counts, sigma, info, eps, tol_norm, tol_rel, status);
    return hipGetLastError();
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

constexpr int kBwdRows = 256;  // shifts summed per partial row (fixed order)

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

// Both gradients in one pass over u and v (each element read once from memory): workgroup
// (x, y) takes rows 256 x .. 256 x + 255 of the kBwdRows shifts of block y, one row per thread.
// A thread adds g_p u_p[i] conj(v_p[j]) of its row j to its band entries (i = j + d - ku, the
// neighbouring rows of u coming from the cache) and each wavefront sums conj(u_p) v_p over its
// 64 rows into LDS; the next shift's rows are loaded while a shift is summed.  After the block
// the wavefront sums go to zpart[p][4 x + wave] and the band sums to partial[y][j][d] (the
// layout of k_grad_band_partial).
constexpr int kBwdRowBlock = 256;
int64_t backward_zpart_cols(int64_t n) { return ((n + kBwdRowBlock - 1) / kBwdRowBlock) * (kBwdRowBlock / 64); }

template <int W>
__global__ void __launch_bounds__(kBwdRowBlock) k_grad_fused(int64_t n, int ku, int64_t npts, const double *g,
                                                             const double2 *u, const double2 *v, double2 *partial,
                                                             double2 *zpart) {
    __shared__ double2 zsh[kBwdRowBlock / 64][kBwdRows];   // 16 KiB
    const int64_t j = (int64_t)blockIdx.x * kBwdRowBlock + threadIdx.x;
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const int64_t p0 = (int64_t)blockIdx.y * kBwdRows;
    const int np = (int)(npts - p0 < kBwdRows ? npts - p0 : kBwdRows);
    const bool in = j < n;
    bool ok[W];                       // row i = j + d - ku inside the matrix
#pragma unroll
    for (int d = 0; d < W; ++d) ok[d] = in && j + d - ku >= 0 && j + d - ku < n;
    double re[W], im[W];
#pragma unroll
    for (int d = 0; d < W; ++d) re[d] = im[d] = 0.0;
    // rows of shift p0 + q: v_p[j] and u_p[j + d - ku]
    double2 bn = make_double2(0.0, 0.0), an[W];
    auto fetch = [&](int q) {
        const int64_t off = (p0 + q) * n;
        bn = in ? v[off + j] : make_double2(0.0, 0.0);
#pragma unroll
        for (int d = 0; d < W; ++d) an[d] = ok[d] ? u[off + j + d - ku] : make_double2(0.0, 0.0);
    };
    if (np > 0) fetch(0);
    for (int q = 0; q < np; ++q) {
        const double2 b = bn;
        double2 a[W];
#pragma unroll
        for (int d = 0; d < W; ++d) a[d] = an[d];
        if (q + 1 < np) fetch(q + 1);
        const double gp = g ? g[p0 + q] : 1.0;
        double zr = 0.0, zi = 0.0;
#pragma unroll
        for (int d = 0; d < W; ++d) {          // a conj(b), weighted (zero outside the matrix)
            re[d] = fma(gp, fma(a[d].x, b.x, a[d].y * b.y), re[d]);
            im[d] = fma(gp, fma(a[d].y, b.x, -a[d].x * b.y), im[d]);
            if (d == ku) {                     // row i = j: conj(u_p[j]) v_p[j]
                zr = fma(a[d].x, b.x, a[d].y * b.y);
                zi = fma(a[d].x, b.y, -a[d].y * b.x);
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            zr += __shfl_xor(zr, off);
            zi += __shfl_xor(zi, off);
        }
        if (lane == 0) zsh[wave][q] = make_double2(zr, zi);
    }
    __syncthreads();
    const int64_t zcols = (int64_t)gridDim.x * (kBwdRowBlock / 64);
    for (int t = (int)threadIdx.x; t < np * (kBwdRowBlock / 64); t += kBwdRowBlock) {
        const int q = t / (kBwdRowBlock / 64), wv = t % (kBwdRowBlock / 64);
        zpart[(p0 + q) * zcols + (int64_t)blockIdx.x * (kBwdRowBlock / 64) + wv] = zsh[wv][q];
    }
    if (in) {
        double2 *pr = partial + (int64_t)blockIdx.y * n * W + j * W;
#pragma unroll
        for (int d = 0; d < W; ++d) pr[d] = make_double2(-re[d], -im[d]);
    }
}

// grad_z[p] = g_p conj(sum of the row-block partials of p): one wavefront per shift, lane l
// summing columns l, l + 64, ... (coalesced), then a fixed butterfly over the lanes.
__global__ void __launch_bounds__(256) k_grad_zsum(int64_t npts, int64_t zcols, const double *g,
                                                   const double2 *zpart, double2 *grad_z) {
    const int lane = (int)(threadIdx.x & 63);
    const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= npts) return;                       // whole wavefronts
    double re = 0.0, im = 0.0;
    for (int64_t c = lane; c < zcols; c += 64) {
        const double2 x = zpart[p * zcols + c];
        re += x.x;
        im += x.y;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
    }
    const double gp = g ? g[p] : 1.0;
    if (lane == 0) grad_z[p] = make_double2(gp * re, -gp * im);
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

size_t workspace_bytes(int64_t n, int kl, int ku, int64_t slots, int kmax, int vec, int64_t npts_max, int kstore) {
    Workspace w;
    carve_workspace(nullptr, n, kl, ku, slots, kmax, vec, npts_max, &w, kstore);
    return (size_t)(uintptr_t)w.blocksums + align256(sizeof(int64_t) * (size_t)((npts_max + kScanTile - 1) / kScanTile + 1));
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

static EvalKernel pick(int kl, int ku, int mode) {
    switch (kl) {
    case 0: return pick_eval_kl0(ku, mode);
    case 1: return pick_eval_kl1(ku, mode);
    case 2: return pick_eval_kl2(ku, mode);
    case 3: return pick_eval_kl3(ku, mode);
    case 4: return pick_eval_kl4(ku, mode);
    }
    return nullptr;
}

// Sigma-only calls with the bisection on (kl + ku >= 1): the bisection kernel evaluates
// every shift it can and lists the others (sigma_min below its rounding limit) for the
// Golub-Kahan kernel, which then takes only those.
static bool bisects(const EvalArgs &a, const Workspace &ws) {
    return !a.want_vectors && a.bisect && a.kl + a.ku >= 1 && a.gram && ws.gk_list && ws.npts_max > 0;
}

// Calls with vectors and the bisection on: the Golub-Kahan kernel's own bisection runs at one
// wavefront per SIMD (its registers hold the Lanczos state as well), so the bisection kernel
// first finds every shift's final bracket (phase 3: saved at the shift's output position)
// and the vector kernel starts from those brackets: inverse iteration for the shifts that
// qualified, the Golub-Kahan process for the others.  Short shift sets (contour refinement
// and tracing evaluate one shift per contour point) take a whole wavefront per shift, 64
// tests per pass; larger ones the call's lanes per shift.
constexpr int64_t kWaveBracketMax = 2048;

static bool brackets_first(const EvalArgs &a, const Workspace &ws) {
    return a.want_vectors && a.bisect && a.kl + a.ku >= 1 && a.gram && ws.st_np && ws.npts_max > 0;
}

hipError_t launch_eval(const EvalArgs &a0, const Workspace &ws, hipStream_t st, const SideStream *side) {
    if (a0.dense) return launch_dense(a0, ws.npts_max, st);
    EvalArgs a = a0;
    EvalKernel k = pick(a.kl, a.ku, a.want_vectors != 0 ? 1 : 0);
    if (!k) return hipErrorInvalidValue;
    const int64_t blocks = ws.slots / kEvalBlock;
    if (brackets_first(a, ws)) {
        BisArgs b;
        b.gram = a.gram;
        b.n = a.n;
        b.hb = a.kl + a.ku;
        b.normA = a.normA;
        b.norm2A = a.norm2A;
        b.mode = a.mode;
        b.z = a.z;
        b.idx = a.idx;
        b.ga = a.ga;
        b.gb = a.gb;
        b.gc = a.gc;
        b.gd = a.gd;
        b.nx = a.nx;
        b.ny = a.ny;
        b.count_dev = a.count_dev;
        b.tol_norm = a.tol_norm;
        b.tol_rel = a.tol_rel;
        b.st_lo = ws.st_lo;
        b.st_hi = ws.st_hi;
        b.st_np = ws.st_np;
        b.phase = 3;
        const int lanes = ws.npts_max <= kWaveBracketMax ? 64 : a.lanes;
        const int64_t spw = 64 / lanes;
        hipError_t e = launch_bis(b, b.hb, a.ktm, lanes, (ws.npts_max + spw - 1) / spw, st);
        if (e != hipSuccess) return e;
        if (ws.gk_list && ws.gk_count && ws.blocksums) {   // settled shifts first (k_part_*)
            const int64_t nb = ws.npts_max > kScanTile ? (ws.npts_max + kScanTile - 1) / kScanTile : 1;
            hipLaunchKernelGGL(k_part_count, dim3((unsigned)nb), dim3(kScanBlock), 0, st, (const int32_t *)ws.st_np,
                               a.count_dev, a.mode, a.idx, a.nx, a.ny, ws.blocksums);
            hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, ws.blocksums, nb, ws.gk_count,
                               ws.queue);
            hipLaunchKernelGGL(k_part_scatter, dim3((unsigned)nb), dim3(kScanBlock), 0, st,
                               (const int32_t *)ws.st_np, a.count_dev, a.mode, a.idx, a.nx, a.ny,
                               (const int64_t *)ws.blocksums, (const int64_t *)ws.gk_count, ws.gk_list);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            a.perm = ws.gk_list;
        }
        a.brk_lo = ws.st_lo;
        a.brk_hi = ws.st_hi;
        a.brk_np = ws.st_np;
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kEvalBlock), 0, st, a, ws);
        return hipGetLastError();
    }
    if (bisects(a, ws)) {
        BisArgs b;
        b.gram = a.gram;
        b.n = a.n;
        b.hb = a.kl + a.ku;
        b.normA = a.normA;
        b.norm2A = a.norm2A;
        b.mode = a.mode;
        b.z = a.z;
        b.idx = a.idx;
        b.ga = a.ga;
        b.gb = a.gb;
        b.gc = a.gc;
        b.gd = a.gd;
        b.nx = a.nx;
        b.ny = a.ny;
        b.count_dev = a.count_dev;
        b.tol_norm = a.tol_norm;
        b.tol_rel = a.tol_rel;
        b.sigma = a.sigma;
        b.info = a.info;
        b.iters = a.iters;
        b.eps = a.eps;
        b.sens = a.sens;
        b.gk_list = ws.gk_list;
        b.gk_count = ws.gk_count;
        b.st_lo = ws.st_lo;
        b.st_hi = ws.st_hi;
        b.st_np = ws.st_np;
        hipError_t e = launch_zero(ws.gk_count, sizeof(int64_t), st);
        if (e != hipSuccess) return e;
        const int64_t spw = 64 / a.lanes;
        const int64_t chunks = (ws.npts_max + spw - 1) / spw;
        a.perm = ws.gk_list;
        a.count_dev = ws.gk_count;
        if (!side || !side->stream) {
            const TimingEvents &tv = timing_events();
            if (tv.start && (e = hipEventRecord(tv.start, st)) != hipSuccess)
                return e;
            b.phase = 0;
            e = launch_bis(b, b.hb, a.ktm, a.lanes, chunks, st);
            if (e != hipSuccess) return e;
            if (tv.end && (e = hipEventRecord(tv.end, st)) != hipSuccess)
                return e;
            ListBases lb = {};
            if ((e = launch_sort_lists(ws.gk_list, lb, ws.gk_count, 1, st)) != hipSuccess) return e;
            hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kEvalBlock), 0, st, a, ws);
            return hipGetLastError();
        }
        // first pass of every shift; then the Golub-Kahan launch over the shifts it handed
        // over runs on the side stream while the bisection resumes on this one
        const TimingEvents &tev = timing_events();
        if (tev.start && (e = hipEventRecord(tev.start, st)) != hipSuccess)
            return e;
        b.phase = 1;
        if ((e = launch_bis(b, b.hb, a.ktm, a.lanes, chunks, st)) != hipSuccess) return e;
        ListBases lb = {};
        if ((e = launch_sort_lists(ws.gk_list, lb, ws.gk_count, 1, st)) != hipSuccess) return e;
        if ((e = hipEventRecord(side->fork, st)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(side->stream, side->fork, 0)) != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kEvalBlock), 0, side->stream, a, ws);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipEventRecord(side->join, side->stream)) != hipSuccess) return e;
        b.phase = 2;
        if ((e = launch_bis(b, b.hb, a.ktm, a.lanes, chunks, st)) != hipSuccess) return e;
        if (tev.end && (e = hipEventRecord(tev.end, st)) != hipSuccess) return e;
        return hipStreamWaitEvent(st, side->join, 0);
    }
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kEvalBlock), 0, st, a, ws);
    return hipGetLastError();
}

TimingEvents &timing_events() {
    static thread_local TimingEvents t;
    return t;
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

// ------------------------------------------------------------------------ contour tracing
// One thread per tracer.  zc: current point on the curve, gc: the gradient there, zt: the
// point being corrected, z0: point 0 (closure test).

__global__ void k_trace_init(int64_t m, const double2 *seeds, double2 *zt, int32_t *active, int32_t *count,
                             int32_t *flags) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    zt[p] = seeds[p];
    active[p] = 1;
    count[p] = 0;
    flags[p] = 0;
}

// Predictor: a step of length h along the tangent i g / |g| (active tracers only).
__global__ void k_trace_predict(int64_t m, const int32_t *active, const double2 *zc, const double2 *gc, double h,
                                double2 *zt) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m || !active[p]) return;
    const double2 g = gc[p];
    const double f = h / sqrt(fma(g.x, g.x, g.y * g.y));
    zt[p] = make_double2(zc[p].x - f * g.y, zc[p].y + f * g.x);
}

// Corrector: one Newton step on ln(sigma / eps) along g (active tracers only).
__global__ void k_trace_newton(int64_t m, const int32_t *active, double2 *zt, const double *sigma, const double2 *g,
                               double eps) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m || !active[p]) return;
    const double s = sigma[p];
    const double2 gp = g[p];
    const double g2 = fma(gp.x, gp.x, gp.y * gp.y);
    if (!(s > 0.0) || !(g2 > 0.0)) return;
    const double f = s * log(s / eps) / g2;
    zt[p] = make_double2(zt[p].x - f * gp.x, zt[p].y - f * gp.y);
}

// Acceptance of point k: store it and set the stop flags (bits as PS_TRACE_*).
__global__ void k_trace_accept(int64_t m, int32_t k, int32_t max_points, double eps, double h, int use_box,
                               double ba, double bb, double bc, double bd, const double2 *zt, const double *sigma,
                               const double2 *g, int32_t *active, double2 *zc, double2 *gc, double2 *z0,
                               double2 *pts, int32_t *count, int32_t *flags) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m || !active[p]) return;
    const double s = sigma[p];
    if (!(s > 0.0) || !(fabs(log(s / eps)) <= 1e-6)) {
        flags[p] |= PS_TRACE_NEWTON_FAILED;
        active[p] = 0;
        return;
    }
    const double2 z = zt[p];
    pts[p * max_points + k] = z;
    count[p] = k + 1;
    zc[p] = z;
    gc[p] = g[p];
    if (k == 0) z0[p] = z;
    int stop = 0;
    if (use_box && !(z.x >= ba && z.x <= bb && z.y >= bc && z.y <= bd)) stop |= PS_TRACE_LEFT_BOX;
    const double2 o = k == 0 ? z : z0[p];
    if (k >= 3 && hypot(z.x - o.x, z.y - o.y) < h) stop |= PS_TRACE_CLOSED;
    if (!stop && k == max_points - 1) stop |= PS_TRACE_MAX_POINTS;
    if (stop) {
        flags[p] |= stop;
        active[p] = 0;
    }
}

__global__ void k_count_active(int64_t m, const int32_t *active, int32_t *n_active) {
    __shared__ int32_t sh[256];
    int32_t c = 0;
    for (int64_t p = threadIdx.x; p < m; p += 256) c += active[p] != 0;
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_active = sh[0];
}

static dim3 grid_for(int64_t m) { return dim3((unsigned)((m + 255) / 256)); }

hipError_t launch_trace_init(int64_t m, const double2 *seeds, double2 *zt, int32_t *active, int32_t *count,
                             int32_t *flags, hipStream_t st) {
    hipLaunchKernelGGL(k_trace_init, grid_for(m), dim3(256), 0, st, m, seeds, zt, active, count, flags);
    return hipGetLastError();
}

hipError_t launch_trace_predict(int64_t m, const int32_t *active, const double2 *zc, const double2 *gc, double h,
                                double2 *zt, hipStream_t st) {
    hipLaunchKernelGGL(k_trace_predict, grid_for(m), dim3(256), 0, st, m, active, zc, gc, h, zt);
    return hipGetLastError();
}

hipError_t launch_trace_newton(int64_t m, const int32_t *active, double2 *zt, const double *sigma, const double2 *g,
                               double eps, hipStream_t st) {
    hipLaunchKernelGGL(k_trace_newton, grid_for(m), dim3(256), 0, st, m, active, zt, sigma, g, eps);
    return hipGetLastError();
}

hipError_t launch_trace_accept(int64_t m, int32_t k, int32_t max_points, double eps, double h, const ps_grid *box,
                               const double2 *zt, const double *sigma, const double2 *g, int32_t *active, double2 *zc,
                               double2 *gc, double2 *z0, double2 *pts, int32_t *count, int32_t *flags,
                               hipStream_t st) {
    const int use_box = box != nullptr;
    const double ba = box ? box->a : 0.0, bb = box ? box->b : 0.0, bc = box ? box->c : 0.0, bd = box ? box->d : 0.0;
    hipLaunchKernelGGL(k_trace_accept, grid_for(m), dim3(256), 0, st, m, k, max_points, eps, h, use_box, ba, bb, bc,
                       bd, zt, sigma, g, active, zc, gc, z0, pts, count, flags);
    return hipGetLastError();
}

hipError_t launch_count_active(int64_t m, const int32_t *active, int32_t *n_active, hipStream_t st) {
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, st, m, active, n_active);
    return hipGetLastError();
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
    if (grad_z && grad_band && partial) {
        // both gradients: one pass over u and v, then the two fixed-order reductions
        const int w = kl + ku + 1;
        const int64_t rows = backward_partial_rows(npts);
        const int64_t rb = (n + kBwdRowBlock - 1) / kBwdRowBlock;
        double2 *zpart = partial + rows * n * w;
        const dim3 grid((unsigned)rb, (unsigned)rows);
        switch (w) {
#define PS_FUSED_CASE(WW) \
    case WW: hipLaunchKernelGGL(k_grad_fused<WW>, grid, dim3(kBwdRowBlock), 0, st, n, ku, npts, g, u, v, partial, zpart); \
        break;
            PS_FUSED_CASE(1) PS_FUSED_CASE(2) PS_FUSED_CASE(3) PS_FUSED_CASE(4) PS_FUSED_CASE(5)
            PS_FUSED_CASE(6) PS_FUSED_CASE(7) PS_FUSED_CASE(8) PS_FUSED_CASE(9)
#undef PS_FUSED_CASE
        default: return hipErrorInvalidValue;
        }
        hipLaunchKernelGGL(k_grad_zsum, dim3((unsigned)((npts * 64 + 255) / 256)), dim3(256), 0, st, npts,
                           backward_zpart_cols(n), g, (const double2 *)zpart, grad_z);
        hipLaunchKernelGGL(k_grad_band_sum, dim3((unsigned)((n * w + 255) / 256)), dim3(256), 0, st, n, w, rows,
                           (const double2 *)partial, grad_band, real_a);
        return hipGetLastError();
    }
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
