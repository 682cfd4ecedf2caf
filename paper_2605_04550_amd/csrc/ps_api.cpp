// Host side of the C ABI declared in include/ps.h: argument validation, the matrix
// handle, workspace planning and kernel launches on the caller's stream.

#include "ps.h"
#include "ps_internal.h"
#include "ps_mask.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

struct ps_mlp_s {
    float *raw;      // device, the parameter vector
    float *packed;   // device, the MFMA operand order of the hidden layers
    int device;
};

struct ps_matrix_s {
    int64_t n;
    int32_t kl, ku;
    uint32_t flags;
    double fro;
    double norm2;    // sqrt(||A||_1 ||A||_inf) >= ||A||_2
    double2 *arow;   // device, [n][kl+ku+1] rows 0 .. n-1 of the band
    double2 *abase;  // the allocation: kBandPadTop zero rows, the band, kBandPadBottom zero rows
    double *gram;    // device, the Gram band read by the bisection kernel (kl + ku >= 1)
    // Second streams for the Golub-Kahan launch beside the bisection, one per caller stream
    // seen (so that concurrent calls on different streams do not queue their Golub-Kahan
    // launches behind one another): side[0] is created with the handle, the others on the
    // handle's device on first use by another stream (never while that stream is capturing a
    // graph: such a call shares side[0]); beyond kMatSides callers, side[0] is shared.  A call
    // holds its side stream's mutex while it enqueues the fork, the launch and the join, so
    // that calls sharing a side stream from several threads do not interleave its events.
    static constexpr int kMatSides = 4;
    ps::SideStream side[kMatSides];
    hipStream_t side_key[kMatSides];
    bool side_bound[kMatSides];
    int nside;
    std::mutex side_mu;                   // the table above
    std::mutex side_call_mu[kMatSides];   // one enqueue sequence at a time per side stream
    int device;
    bool dense;      // kl or ku above the banded kernels' limit: sigma only, n <= kDenseMaxN
};

namespace {

thread_local char g_err[512] = "";

ps_status fail(ps_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

ps_status ok() {
    g_err[0] = 0;
    return PS_OK;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return fail(PS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int64_t kSlotQuantum = 256;
constexpr int64_t kMaxSlots = 131072;
// Bytes the default plan may use: enough slots to give every SIMD a wavefront at n = 10^4
// (1.9 MB per slot there), under half of the 288 GB of HBM.
constexpr double kDefaultWsBudget = 128.0 * (1ull << 30);

ps_opts resolve(const ps_opts *o) {
    ps_opts r;
    ps_opts_default(&r);
    if (o) r = *o;
    return r;
}

ps_status check_opts(const ps_opts &o) {
    if (!(o.tol_norm >= 0.0) || !(o.tol_rel >= 0.0) || !isfinite(o.tol_norm) || !isfinite(o.tol_rel))
        return fail(PS_ERR_INVALID, "tolerances must be finite and >= 0");
    if (o.tol_norm == 0.0 && o.tol_rel == 0.0) return fail(PS_ERR_INVALID, "tol_norm and tol_rel are both 0");
    if (o.max_iter < 1 || o.max_iter > ps::kMaxIterCap)
        return fail(PS_ERR_INVALID, "max_iter must be in [1, %d]", ps::kMaxIterCap);
    if (o.slots < 0) return fail(PS_ERR_INVALID, "slots must be >= 0");
    if (o.check_shift < 0 || o.check_shift > 12) return fail(PS_ERR_INVALID, "check_shift must be in [0, 12]");
    if (o.bisect != 0 && o.bisect != -1) return fail(PS_ERR_INVALID, "bisect must be 0 or -1");
    if (o.lanes != 0 && o.lanes != 1 && o.lanes != 2 && o.lanes != 4 && o.lanes != 64)
        return fail(PS_ERR_INVALID, "lanes must be 0, 1, 2, 4 or 64");
    if (o.tests < 0 || o.tests > 3) return fail(PS_ERR_INVALID, "tests must be in [0, 3]");
    return PS_OK;
}

int check_shift_of(const ps_opts &o) { return o.check_shift > 0 ? o.check_shift : 5; }

// Lanes per shift of the bisection kernel (default 1) and its test-count mode: tests 1 -> one
// test per lane and pass; 0 and 2 -> three for kl + ku <= 2, two for <= 5, one above; 3 -> two
// for kl + ku <= 6, one above.
int lanes_of(const ps_opts &o) { return o.lanes > 0 ? o.lanes : 1; }
int ktm_of(const ps_opts &o) { return o.tests == 1 ? 0 : o.tests == 3 ? 2 : 1; }

// 1: shifts that qualify take the inertia bisection; 0: every shift takes Golub-Kahan.
int bisect_of(const ps_opts &o) { return o.bisect < 0 ? 0 : 1; }

int vec_of(const ps_opts &o) { return o.want_vectors ? 1 : 0; }

int64_t round_slots(int64_t s) {
    s = (s / kSlotQuantum) * kSlotQuantum;
    return s;
}

// Slots of the default plan for npts shifts.
int64_t default_slots(const ps_matrix_s *m, int64_t npts, const ps_opts &o) {
    int64_t want = ((npts + kSlotQuantum - 1) / kSlotQuantum) * kSlotQuantum;
    if (o.slots > 0) want = round_slots(o.slots);
    if (want < kSlotQuantum) want = kSlotQuantum;
    if (want > kMaxSlots) want = kMaxSlots;
    const int vec = vec_of(o);
    // shrink until the workspace fits the default budget
    while (want > kSlotQuantum &&
           (double)ps::workspace_bytes(m->n, m->kl, m->ku, want, o.max_iter, vec, npts) > kDefaultWsBudget)
        want -= kSlotQuantum;
    return want;
}

// Largest slot count <= the default whose workspace fits ws_bytes (0 if none).
int64_t slots_for(const ps_matrix_s *m, int64_t npts, const ps_opts &o, size_t ws_bytes) {
    int64_t s = default_slots(m, npts, o);
    const int vec = vec_of(o);
    while (s >= kSlotQuantum && ps::workspace_bytes(m->n, m->kl, m->ku, s, o.max_iter, vec, npts) > ws_bytes)
        s -= kSlotQuantum;
    return s >= kSlotQuantum ? s : 0;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// A non-blocking stream at the default priority and its fork and join events (no timing).
hipError_t create_side(ps::SideStream *s) {
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->join, hipEventDisableTiming);
    return e;
}

void destroy_side(ps::SideStream *s) {
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->fork) (void)hipEventDestroy(s->fork);
    if (s->join) (void)hipEventDestroy(s->join);
    s->stream = nullptr;
    s->fork = s->join = nullptr;
}

// Index of the side stream of a call on `caller` (see ps_matrix_s::side).
int side_index(ps_matrix m, hipStream_t caller) {
    std::lock_guard<std::mutex> g(m->side_mu);
    for (int i = 0; i < m->nside; ++i)
        if (m->side_bound[i] && m->side_key[i] == caller) return i;
    if (!m->side_bound[0]) {
        m->side_bound[0] = true;
        m->side_key[0] = caller;
        return 0;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (m->nside < ps_matrix_s::kMatSides && hipStreamIsCapturing(caller, &cs) == hipSuccess &&
        cs == hipStreamCaptureStatusNone) {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (cur != m->device) (void)hipSetDevice(m->device);
        ps::SideStream sd;
        const hipError_t e = create_side(&sd);
        if (cur != m->device) (void)hipSetDevice(cur);
        if (e == hipSuccess) {
            const int i = m->nside++;
            m->side[i] = sd;
            m->side_key[i] = caller;
            m->side_bound[i] = true;
            return i;
        }
        destroy_side(&sd);
    }
    return 0;
}

// The side stream of a call on `caller`, held for the call's enqueue sequence.
struct SideLock {
    const ps::SideStream *side;
    std::unique_lock<std::mutex> lk;
    SideLock(ps_matrix m, hipStream_t caller) {
        const int i = side_index(m, caller);
        side = &m->side[i];
        lk = std::unique_lock<std::mutex>(m->side_call_mu[i]);
    }
};

ps_status check_grid(const ps_grid *g) {
    if (!g) return fail(PS_ERR_INVALID, "grid is NULL");
    if (g->nx < 1 || g->ny < 1) return fail(PS_ERR_INVALID, "grid needs nx, ny >= 1");
    if (!isfinite(g->a) || !isfinite(g->b) || !isfinite(g->c) || !isfinite(g->d))
        return fail(PS_ERR_NONFINITE, "non-finite grid bounds");
    if (g->nx > (int64_t)1 << 31 || g->ny > (int64_t)1 << 31 || g->nx * g->ny > ((int64_t)1 << 40))
        return fail(PS_ERR_INVALID, "grid too large");
    return PS_OK;
}

ps_status check_handle(ps_matrix m) {
    if (!m) return fail(PS_ERR_INVALID, "matrix handle is NULL");
    return PS_OK;
}

// Entry points that need the banded kernels (vectors, labels, batches, ...); called after
// their argument checks, where the handle is first used.
ps_status check_banded(ps_matrix m, const char *what) {
    if (m->dense)
        return fail(PS_ERR_UNSUPPORTED, "%s needs kl, ku <= %d (this matrix has kl=%d ku=%d and takes the dense "
                    "sigma-only path)", what, ps::kMaxKL, m->kl, m->ku);
    return PS_OK;
}

// Workspace of a dense-path evaluation: the shift counter and the mask compaction only.
size_t dense_ws_bytes(const ps_matrix_s *m, int64_t npts) {
    return ps::workspace_bytes(m->n, 0, 0, kSlotQuantum, 1, 0, npts);
}

ps_status prepare_eval(ps_matrix m, int64_t npts_max, const ps_opts &o, void *ws, size_t ws_bytes, double *sigma,
                       ps_c128 *u, ps_c128 *v, ps::Workspace *w, ps::EvalArgs *a) {
    if (!sigma) return fail(PS_ERR_INVALID, "sigma output is NULL");
    if (o.want_vectors && (!u || !v)) return fail(PS_ERR_INVALID, "want_vectors needs u and v outputs");
    if (!ws) return fail(PS_ERR_WORKSPACE, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(PS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (m->dense) {
        if (o.want_vectors)
            return fail(PS_ERR_UNSUPPORTED, "singular vectors need kl, ku <= %d (kl=%d ku=%d)", ps::kMaxKL, m->kl,
                        m->ku);
        const size_t need = dense_ws_bytes(m, npts_max);
        if (ws_bytes < need) return fail(PS_ERR_WORKSPACE, "workspace needs %zu bytes (got %zu)", need, ws_bytes);
        ps::carve_workspace(ws, m->n, 0, 0, kSlotQuantum, 1, 0, npts_max, w);
        a->n = m->n;
        a->kl = m->kl;
        a->ku = m->ku;
        a->arow = m->arow;
        a->normA = m->fro;
        a->norm2A = m->norm2;
        a->tol_norm = o.tol_norm;
        a->tol_rel = o.tol_rel;
        a->sigma = sigma;
        a->count_dev = w->count;
        a->dense = 1;
        return PS_OK;
    }
    int64_t slots = slots_for(m, npts_max, o, ws_bytes);
    if (slots == 0)
        return fail(PS_ERR_WORKSPACE, "workspace of %zu bytes is below the minimum %zu", ws_bytes,
                    ps::workspace_bytes(m->n, m->kl, m->ku, kSlotQuantum, o.max_iter, vec_of(o), npts_max));
    // kept Lanczos vectors (calls with vectors): the default number where the workspace holds
    // them beyond the slots' own needs, else as many as it does hold (0: the replay)
    int kst = ps::kstore_for(slots, ps::padded_rows(m->n), o.max_iter, vec_of(o));
    while (kst > 0 &&
           ps::workspace_bytes(m->n, m->kl, m->ku, slots, o.max_iter, vec_of(o), npts_max, kst) > ws_bytes)
        --kst;
    ps::carve_workspace(ws, m->n, m->kl, m->ku, slots, o.max_iter, vec_of(o), npts_max, w, kst);
    a->n = m->n;
    a->kl = m->kl;
    a->ku = m->ku;
    a->arow = m->arow;
    a->normA = m->fro;
    a->norm2A = m->norm2;
    a->bisect = bisect_of(o);
    a->gram = m->gram;
    a->lanes = lanes_of(o);
    a->ktm = ktm_of(o);
    a->tol_norm = o.tol_norm;
    a->tol_rel = o.tol_rel;
    a->max_iter = o.max_iter;
    a->check_shift = check_shift_of(o);
    a->want_vectors = o.want_vectors;
    a->sigma = sigma;
    a->u = (double2 *)u;
    a->v = (double2 *)v;
    a->count_dev = w->count;
    return PS_OK;
}

}  // namespace

extern "C" {

void ps_opts_default(ps_opts *o) {
    if (!o) return;
    o->tol_norm = 1e-10;
    o->tol_rel = 1e-8;
    o->max_iter = 3000;
    o->want_vectors = 0;
    o->slots = 0;
    o->check_shift = 0;
    o->bisect = 0;
    o->lanes = 0;
    o->tests = 0;
}

// ------------------------------------------------------------------------------------------
// Mask producer (classifier of Sec. 3.2, hierarchical prediction of Sec. 3.5).

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

ps_mask_opts resolve_mask(const ps_mask_opts *o) {
    ps_mask_opts r;
    ps_mask_opts_default(&r);
    if (o) r = *o;
    return r;
}

ps_status check_mask_opts(const ps_mask_opts &o) {
    if (o.stride < 1 || o.stride > 32) return fail(PS_ERR_INVALID, "stride must be in [1, 32]");
    if (o.dilate < 1 || o.dilate > 31 || o.dilate % 2 == 0) return fail(PS_ERR_INVALID, "dilate must be odd, 1 .. 31");
    if (!(o.coarse_q >= 0.0 && o.coarse_q <= 1.0)) return fail(PS_ERR_INVALID, "coarse_q must be in [0, 1]");
    if (!(o.tau > 0.0 && o.tau <= 1.0)) return fail(PS_ERR_INVALID, "tau must be in (0, 1]");
    return PS_OK;
}

ps_status check_net_inputs(ps_mlp net, const double *gfeat, const ps_c128 *eig, int64_t neig,
                           ps::mlp::Globals *gf) {
    if (!net) return fail(PS_ERR_INVALID, "network handle is NULL");
    if (!gfeat) return fail(PS_ERR_INVALID, "global features are NULL");
    if (!eig || neig < 1) return fail(PS_ERR_INVALID, "the spectrum needs neig >= 1 eigenvalues");
    for (int k = 0; k < ps::mlp::kNGlobal; ++k) {
        if (!isfinite(gfeat[k])) return fail(PS_ERR_NONFINITE, "global feature %d is not finite", k);
        gf->f[k] = gfeat[k];
    }
    return PS_OK;
}

}  // namespace

void ps_mask_opts_default(ps_mask_opts *o) {
    if (!o) return;
    o->stride = 4;
    o->dilate = 5;
    o->coarse_q = 0.8;
    o->tau = 0.05;
}

ps_status ps_mlp_create(const float *params, uint32_t flags, ps_mlp *out, void *stream) {
    if (!params || !out) return fail(PS_ERR_INVALID, "params and out are required");
    if (flags & ~(uint32_t)PS_DEVICE_PTR) return fail(PS_ERR_INVALID, "unknown flags");
    *out = nullptr;
    const size_t bytes = sizeof(float) * ps::mlp::kNParam;
    std::vector<float> h(ps::mlp::kNParam);
    if (flags & PS_DEVICE_PTR)
        HIP_TRY(hipMemcpy(h.data(), params, bytes, hipMemcpyDeviceToHost));
    else
        memcpy(h.data(), params, bytes);
    for (int i = 0; i < ps::mlp::kNParam; ++i)
        if (!isfinite(h[i])) return fail(PS_ERR_NONFINITE, "parameter %d is not finite", i);
    ps_mlp_s *n = new ps_mlp_s();
    HIP_TRY(hipGetDevice(&n->device));
    hipError_t e = hipMalloc((void **)&n->raw, bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&n->packed, sizeof(float) * ps::mlp::kPackedFloats);
    hipStream_t s = (hipStream_t)stream;
    if (e == hipSuccess) e = hipMemcpyAsync(n->raw, h.data(), bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = ps::mlp::launch_pack(n->raw, n->packed, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        if (n->raw) (void)hipFree(n->raw);
        if (n->packed) (void)hipFree(n->packed);
        delete n;
        return fail(PS_ERR_HIP, "ps_mlp_create: %s", hipGetErrorString(e));
    }
    *out = n;
    return ok();
}

ps_status ps_mlp_destroy(ps_mlp net) {
    if (!net) return ok();
    hipError_t e1 = hipFree(net->raw), e2 = hipFree(net->packed);
    delete net;
    if (e1 != hipSuccess || e2 != hipSuccess) return fail(PS_ERR_HIP, "ps_mlp_destroy: hipFree failed");
    return ok();
}

ps_status ps_mask_workspace_size(const ps_grid *g, const ps_mask_opts *o, size_t *bytes) {
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    if (!g) {
        *bytes = ps::mlp::kWsHeader;
        return ok();
    }
    ps_status st = check_grid(g);
    if (st) return st;
    const ps_mask_opts r = resolve_mask(o);
    if ((st = check_mask_opts(r))) return st;
    const int64_t ncoarse = ((g->ny + r.stride - 1) / r.stride) * ((g->nx + r.stride - 1) / r.stride);
    *bytes = ps::mlp::kWsHeader + align256(sizeof(float) * (size_t)ncoarse) +
             align256(sizeof(float) * (size_t)(g->nx * g->ny));
    return ok();
}

ps_status ps_mlp_prob(ps_mlp net, const double *gfeat, const ps_c128 *eig_dev, int64_t neig, const ps_c128 *z_dev,
                      int64_t npts, void *ws_dev, size_t ws_bytes, float *prob_dev, void *stream) {
    ps::mlp::Globals gf;
    ps_status st = check_net_inputs(net, gfeat, eig_dev, neig, &gf);
    if (st) return st;
    if (npts < 0) return fail(PS_ERR_INVALID, "npts must be >= 0");
    if (npts > 0 && (!z_dev || !prob_dev)) return fail(PS_ERR_INVALID, "z and prob are required");
    if (!ws_dev || ws_bytes < (size_t)ps::mlp::kWsHeader)
        return fail(PS_ERR_WORKSPACE, "network workspace needs %d bytes", ps::mlp::kWsHeader);
    if (!aligned(ws_dev, 256)) return fail(PS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)ws_dev;
    const ps::mlp::Batch none{nullptr, nullptr};
    HIP_TRY(ps::mlp::launch_prep(net->raw, gf, none, 1, (const double2 *)eig_dev, neig, ws,
                                 (int64_t *)(ws + ps::mlp::kWsEvals), 0, s));
    HIP_TRY(ps::mlp::launch_points(net->raw, net->packed, (const double2 *)eig_dev, neig, ws, (const double2 *)z_dev,
                                   npts, prob_dev, s));
    return ok();
}

ps_status ps_mask_predict(ps_mlp net, const ps_grid *g, const double *gfeat, const ps_c128 *eig_dev, int64_t neig,
                          const ps_mask_opts *o, void *ws_dev, size_t ws_bytes, uint8_t *mask_dev, float *prob_dev,
                          float *coarse_dev, double *tau_coarse_dev, int64_t *evals_dev, void *stream) {
    ps::mlp::Globals gf;
    ps_status st = check_net_inputs(net, gfeat, eig_dev, neig, &gf);
    if (st) return st;
    if ((st = check_grid(g))) return st;
    const ps_mask_opts r = resolve_mask(o);
    if ((st = check_mask_opts(r))) return st;
    if (!mask_dev) return fail(PS_ERR_INVALID, "mask output is NULL");
    const int64_t ncy = (g->ny + r.stride - 1) / r.stride, ncx = (g->nx + r.stride - 1) / r.stride;
    if (ncy * ncx >= ((int64_t)1 << 31)) return fail(PS_ERR_INVALID, "too many coarse points");
    size_t need = 0;
    ps_mask_workspace_size(g, &r, &need);
    if (!ws_dev || ws_bytes < need) return fail(PS_ERR_WORKSPACE, "mask workspace needs %zu bytes", need);
    if (!aligned(ws_dev, 256)) return fail(PS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    char *ws = (char *)ws_dev;
    float *coarse = coarse_dev ? coarse_dev : (float *)(ws + ps::mlp::kWsHeader);
    float *prob = prob_dev ? prob_dev
                           : (float *)(ws + ps::mlp::kWsHeader + align256(sizeof(float) * (size_t)(ncy * ncx)));
    int64_t *evals = evals_dev ? evals_dev : (int64_t *)(ws + ps::mlp::kWsEvals);
    ps::mlp::GridArgs ga{g->a, g->b, g->c, g->d, g->nx, g->ny};
    hipStream_t s = (hipStream_t)stream;
    const ps::mlp::Batch none{nullptr, nullptr};
    HIP_TRY(ps::mlp::launch_prep(net->raw, gf, none, 1, (const double2 *)eig_dev, neig, ws, evals, ncy * ncx, s));
    HIP_TRY(ps::mlp::launch_mask(net->raw, net->packed, none, 1, (const double2 *)eig_dev, neig, ws, ga, r.stride,
                                 r.dilate, r.coarse_q, r.tau, coarse, prob, mask_dev, evals, tau_coarse_dev, s));
    return ok();
}

namespace {

// Workspace of a batched call: the per-matrix headers, the uploaded tables (global features,
// eigenvalue offsets), the coarse and the probability maps.
struct MaskBatchLayout {
    size_t headers, gfeat, eig_off, coarse, prob, total;
};

MaskBatchLayout mask_batch_layout(int32_t nmat, const ps_grid *g, const ps_mask_opts &r) {
    const int64_t ncoarse = ((g->ny + r.stride - 1) / r.stride) * ((g->nx + r.stride - 1) / r.stride);
    MaskBatchLayout L;
    L.headers = 0;
    L.gfeat = L.headers + (size_t)nmat * ps::mlp::kWsHeader;
    L.eig_off = L.gfeat + align256(sizeof(double) * ps::mlp::kNGlobal * (size_t)nmat);
    L.coarse = L.eig_off + align256(sizeof(int64_t) * ((size_t)nmat + 1));
    L.prob = L.coarse + align256(sizeof(float) * (size_t)ncoarse * (size_t)nmat);
    L.total = L.prob + align256(sizeof(float) * (size_t)(g->nx * g->ny) * (size_t)nmat);
    return L;
}

}  // namespace

ps_status ps_mask_batch_workspace_size(int32_t nmat, const ps_grid *g, const ps_mask_opts *o, size_t *bytes) {
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    if (nmat < 1 || nmat > 65535) return fail(PS_ERR_INVALID, "nmat must be in [1, 65535]");
    ps_status st = check_grid(g);
    if (st) return st;
    const ps_mask_opts r = resolve_mask(o);
    if ((st = check_mask_opts(r))) return st;
    *bytes = mask_batch_layout(nmat, g, r).total;
    return ok();
}

ps_status ps_mask_predict_batch(ps_mlp net, int32_t nmat, const ps_grid *g, const double *gfeat,
                                const ps_c128 *eig_dev, const int64_t *eig_off, const ps_mask_opts *o, void *ws_dev,
                                size_t ws_bytes, uint8_t *mask_dev, float *prob_dev, float *coarse_dev,
                                double *tau_coarse_dev, int64_t *evals_dev, void *stream) {
    if (!net) return fail(PS_ERR_INVALID, "network handle is NULL");
    if (nmat < 1 || nmat > 65535) return fail(PS_ERR_INVALID, "nmat must be in [1, 65535]");
    if (!gfeat || !eig_off || !eig_dev) return fail(PS_ERR_INVALID, "gfeat, eig and eig_off are required");
    ps_status st = check_grid(g);
    if (st) return st;
    const ps_mask_opts r = resolve_mask(o);
    if ((st = check_mask_opts(r))) return st;
    if (!mask_dev) return fail(PS_ERR_INVALID, "mask output is NULL");
    if (eig_off[0] != 0) return fail(PS_ERR_INVALID, "eig_off[0] must be 0");
    for (int32_t m = 0; m < nmat; ++m)
        if (eig_off[m + 1] - eig_off[m] < 1) return fail(PS_ERR_INVALID, "matrix %d has no eigenvalues", m);
    for (size_t k = 0; k < (size_t)nmat * ps::mlp::kNGlobal; ++k)
        if (!isfinite(gfeat[k])) return fail(PS_ERR_NONFINITE, "global feature %zu is not finite", k);
    const int64_t ncy = (g->ny + r.stride - 1) / r.stride, ncx = (g->nx + r.stride - 1) / r.stride;
    if (ncy * ncx >= ((int64_t)1 << 31)) return fail(PS_ERR_INVALID, "too many coarse points");
    const MaskBatchLayout L = mask_batch_layout(nmat, g, r);
    if (!ws_dev || ws_bytes < L.total) return fail(PS_ERR_WORKSPACE, "mask batch workspace needs %zu bytes", L.total);
    if (!aligned(ws_dev, 256)) return fail(PS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    char *ws = (char *)ws_dev;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(ws + L.gfeat, gfeat, sizeof(double) * ps::mlp::kNGlobal * (size_t)nmat,
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ws + L.eig_off, eig_off, sizeof(int64_t) * ((size_t)nmat + 1), hipMemcpyHostToDevice, s));
    const ps::mlp::Batch bt{(const double *)(ws + L.gfeat), (const int64_t *)(ws + L.eig_off)};
    float *coarse = coarse_dev ? coarse_dev : (float *)(ws + L.coarse);
    float *prob = prob_dev ? prob_dev : (float *)(ws + L.prob);
    ps::mlp::GridArgs ga{g->a, g->b, g->c, g->d, g->nx, g->ny};
    ps::mlp::Globals unused{};
    HIP_TRY(ps::mlp::launch_prep(net->raw, unused, bt, nmat, (const double2 *)eig_dev, 0, ws, evals_dev, ncy * ncx,
                                 s));
    HIP_TRY(ps::mlp::launch_mask(net->raw, net->packed, bt, nmat, (const double2 *)eig_dev, 0, ws, ga, r.stride,
                                 r.dilate, r.coarse_q, r.tau, coarse, prob, mask_dev, evals_dev, tau_coarse_dev, s));
    return ok();
}

ps_status ps_mask_calibrate_workspace_size(int32_t nval, int32_t ntau, size_t *bytes) {
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    if (nval < 1 || nval > ps::mlp::kCalMaxVal) return fail(PS_ERR_INVALID, "nval must be in [1, %d]", ps::mlp::kCalMaxVal);
    if (ntau < 1 || ntau > ps::mlp::kCalMaxTau) return fail(PS_ERR_INVALID, "ntau must be in [1, %d]", ps::mlp::kCalMaxTau);
    *bytes = align256(sizeof(int64_t) * (size_t)nval * ((size_t)ntau + 1));
    return ok();
}

ps_status ps_mask_calibrate(int32_t nval, const ps_grid *g, const float *prob_dev, const uint8_t *label_dev,
                            const double *taus, int32_t ntau, int32_t pred_dilate, int32_t label_dilate,
                            double median_min, double p10_min, void *ws_dev, size_t ws_bytes, int32_t *index_dev,
                            double *recall_dev, double *median_dev, double *p10_dev, void *stream) {
    size_t need = 0;
    ps_status st = ps_mask_calibrate_workspace_size(nval, ntau, &need);
    if (st) return st;
    if ((st = check_grid(g))) return st;
    if (!prob_dev || !label_dev || !index_dev || !taus) return fail(PS_ERR_INVALID, "prob, label, taus and index are required");
    for (int32_t k = 0; k < ntau; ++k) {
        if (!isfinite(taus[k])) return fail(PS_ERR_NONFINITE, "tau %d is not finite", k);
        if (k > 0 && !(taus[k] > taus[k - 1])) return fail(PS_ERR_INVALID, "taus must be strictly ascending");
    }
    for (int32_t d : {pred_dilate, label_dilate})
        if (d < 1 || d > 31 || d % 2 == 0) return fail(PS_ERR_INVALID, "dilation sides must be odd, 1 .. 31");
    if (!isfinite(median_min) || !isfinite(p10_min)) return fail(PS_ERR_NONFINITE, "recall bounds must be finite");
    if (!ws_dev || ws_bytes < need) return fail(PS_ERR_WORKSPACE, "calibration workspace needs %zu bytes", need);
    if (!aligned(ws_dev, 256)) return fail(PS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    ps::mlp::Taus tv{};
    for (int32_t k = 0; k < ntau; ++k) tv.t[k] = taus[k];
    HIP_TRY(ps::mlp::launch_calibrate(prob_dev, label_dev, nval, g->nx, g->ny, (pred_dilate - 1) / 2,
                                      (label_dilate - 1) / 2, tv, ntau, median_min, p10_min, (int64_t *)ws_dev,
                                      recall_dev, median_dev, p10_dev, index_dev, (hipStream_t)stream));
    return ok();
}

const char *ps_last_error(void) { return g_err; }

ps_status ps_set_timing_events(void *start, void *end) {
    if ((start == nullptr) != (end == nullptr)) return fail(PS_ERR_INVALID, "start and end must both be set or NULL");
    ps::timing_events().start = (hipEvent_t)start;
    ps::timing_events().end = (hipEvent_t)end;
    return ok();
}

const char *ps_version(void) { return "ps-mi355x 0.1 (gfx950, fp64)"; }

ps_status ps_create_banded(const ps_c128 *ab, int64_t ldab, int64_t n, int32_t kl, int32_t ku, uint32_t flags,
                           void *stream, ps_matrix *out) {
    if (!out) return fail(PS_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!ab) return fail(PS_ERR_INVALID, "ab is NULL");
    if (n < 1) return fail(PS_ERR_INVALID, "n must be >= 1 (got %lld)", (long long)n);
    if (kl < 0 || ku < 0 || kl > n - 1 || ku > n - 1)
        return fail(PS_ERR_INVALID, "need 0 <= kl, ku <= n - 1 (kl=%d ku=%d n=%lld)", kl, ku, (long long)n);
    if (ldab < (int64_t)kl + ku + 1) return fail(PS_ERR_INVALID, "ldab must be >= kl + ku + 1");
    if (flags & ~(uint32_t)(PS_DEVICE_PTR | PS_REAL_A)) return fail(PS_ERR_INVALID, "unknown flags");
    const bool dense = kl > ps::kMaxKL || ku > ps::kMaxKU;
    if (dense && n > ps::kDenseMaxN)
        return fail(PS_ERR_UNSUPPORTED, "kl and ku must be <= %d, or n <= %d for wider bands (got n=%lld kl=%d ku=%d)",
                    ps::kMaxKL, ps::kDenseMaxN, (long long)n, kl, ku);
    hipStream_t st = (hipStream_t)stream;
    const int64_t w = (int64_t)kl + ku + 1;
    std::vector<ps_c128> gb((size_t)(ldab * n));
    if (flags & PS_DEVICE_PTR) {
        HIP_TRY(hipMemcpyAsync(gb.data(), ab, sizeof(ps_c128) * gb.size(), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    } else {
        memcpy(gb.data(), ab, sizeof(ps_c128) * gb.size());
    }
    std::vector<double2> rows((size_t)(n * w));
    std::vector<double> colsum((size_t)n, 0.0);
    double fro2 = 0.0, rowmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t d = 0; d < w; ++d) {
            int64_t j = i - kl + d;
            double2 v = make_double2(0.0, 0.0);
            if (j >= 0 && j < n) {
                ps_c128 e = gb[(size_t)((ku + i - j) + j * ldab)];
                if (!isfinite(e.re) || !isfinite(e.im))
                    return fail(PS_ERR_NONFINITE, "non-finite band entry A[%lld][%lld]", (long long)i, (long long)j);
                v = make_double2(e.re, e.im);
                fro2 += e.re * e.re + e.im * e.im;
            }
            rows[(size_t)(i * w + d)] = v;
        }
        double rs = 0.0;
        for (int64_t d = 0; d < w; ++d) {
            const double a = hypot(rows[(size_t)(i * w + d)].x, rows[(size_t)(i * w + d)].y);
            rs += a;
            if (i - kl + d >= 0 && i - kl + d < n) colsum[(size_t)(i - kl + d)] += a;
        }
        rowmax = rs > rowmax ? rs : rowmax;
    }
    double colmax = 0.0;
    for (double c : colsum) colmax = c > colmax ? c : colmax;
    ps_matrix m = new ps_matrix_s();
    m->n = n;
    m->kl = kl;
    m->ku = ku;
    m->flags = flags;
    m->fro = sqrt(fro2);
    m->norm2 = sqrt(rowmax * colmax);
    m->arow = nullptr;
    m->abase = nullptr;
    m->gram = nullptr;
    for (int i = 0; i < ps_matrix_s::kMatSides; ++i) {
        m->side[i] = ps::SideStream();
        m->side_key[i] = nullptr;
        m->side_bound[i] = false;
    }
    m->nside = 1;
    m->dense = dense;
    (void)hipGetDevice(&m->device);
    // zero rows around the band: kernels may read rows -kBandPadTop .. n + kBandPadBottom - 1
    const size_t padded = (size_t)(ps::kBandPadTop + n + ps::kBandPadBottom) * (size_t)w;
    std::vector<double2> store(padded, make_double2(0.0, 0.0));
    std::copy(rows.begin(), rows.end(), store.begin() + (size_t)ps::kBandPadTop * (size_t)w);
    hipError_t e = hipMalloc((void **)&m->abase, sizeof(double2) * padded);
    if (e != hipSuccess) {
        delete m;
        return fail(PS_ERR_HIP, "hipMalloc of the band: %s", hipGetErrorString(e));
    }
    m->arow = m->abase + (size_t)ps::kBandPadTop * (size_t)w;
    e = hipMemcpyAsync(m->abase, store.data(), sizeof(double2) * padded, hipMemcpyHostToDevice, st);
    // the Gram band of the bisection kernel (computed on the device from the uploaded band)
    if (e == hipSuccess && kl + ku >= 1 && !dense) {
        e = hipMalloc((void **)&m->gram, ps::gram_bytes(n, kl, ku));
        if (e == hipSuccess) e = ps::launch_gram_band(m->arow, n, kl, ku, m->gram, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = create_side(&m->side[0]);
    if (e != hipSuccess) {
        (void)hipFree(m->abase);
        if (m->gram) (void)hipFree(m->gram);
        destroy_side(&m->side[0]);
        delete m;
        return fail(PS_ERR_HIP, "band upload: %s", hipGetErrorString(e));
    }
    *out = m;
    return ok();
}

ps_status ps_destroy(ps_matrix m) {
    if (!m) return ok();
    if (m->abase) (void)hipFree(m->abase);
    if (m->gram) (void)hipFree(m->gram);
    for (int i = 0; i < m->nside; ++i) destroy_side(&m->side[i]);
    delete m;
    return ok();
}

ps_status ps_matrix_info(ps_matrix m, int64_t *n, int32_t *kl, int32_t *ku, double *fro) {
    ps_status st = check_handle(m);
    if (st) return st;
    if (n) *n = m->n;
    if (kl) *kl = m->kl;
    if (ku) *ku = m->ku;
    if (fro) *fro = m->fro;
    return ok();
}

ps_status ps_workspace_size(ps_matrix m, int64_t npts, const ps_opts *o, size_t *bytes) {
    ps_status st = check_handle(m);
    if (st) return st;
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    if (npts < 0) return fail(PS_ERR_INVALID, "npts must be >= 0");
    ps_opts r = resolve(o);
    if ((st = check_opts(r))) return st;
    if (m->dense) {
        if (r.want_vectors) return fail(PS_ERR_UNSUPPORTED, "singular vectors need kl, ku <= %d", ps::kMaxKL);
        *bytes = dense_ws_bytes(m, npts);
        return ok();
    }
    int64_t slots = default_slots(m, npts, r);
    const int vec = vec_of(r);
    *bytes = ps::workspace_bytes(m->n, m->kl, m->ku, slots, r.max_iter, vec, npts,
                                 ps::kstore_for(slots, ps::padded_rows(m->n), r.max_iter, vec));
    return ok();
}

ps_status ps_eval_points(ps_matrix m, const ps_c128 *z_dev, int64_t npts, const ps_opts *o, void *ws_dev,
                         size_t ws_bytes, double *sigma_dev, ps_c128 *u_dev, ps_c128 *v_dev, int32_t *info_dev,
                         int32_t *iters_dev, void *stream) {
    ps_status st = check_handle(m);
    if (st) return st;
    if (npts < 0) return fail(PS_ERR_INVALID, "npts must be >= 0");
    ps_opts r = resolve(o);
    if ((st = check_opts(r))) return st;
    if (npts == 0) return ok();
    if (!z_dev) return fail(PS_ERR_INVALID, "z is NULL");
    ps::Workspace w;
    ps::EvalArgs a;
    if ((st = prepare_eval(m, npts, r, ws_dev, ws_bytes, sigma_dev, u_dev, v_dev, &w, &a))) return st;
    a.mode = ps::kShiftList;
    a.z = (const double2 *)z_dev;
    a.info = info_dev;
    a.iters = iters_dev;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ps::launch_set_count(w.count, npts, w.queue, s));
    {
        SideLock sl(m, s);
        HIP_TRY(ps::launch_eval(a, w, s, sl.side));
    }
    return ok();
}

ps_status ps_eval_points_noalloc(ps_matrix m, const ps_c128 *z_dev, int64_t npts, const ps_opts *o,
                                 double *sigma_dev, int32_t *info_dev, int32_t *iters_dev, void *stream) {
    ps_status st = check_handle(m);
    if (st) return st;
    if (npts < 0) return fail(PS_ERR_INVALID, "npts must be >= 0");
    ps_opts r = resolve(o);
    if ((st = check_opts(r))) return st;
    if (r.want_vectors) return fail(PS_ERR_UNSUPPORTED, "the allocation-free call computes sigma only");
    if (npts == 0) return ok();
    if (!z_dev) return fail(PS_ERR_INVALID, "z is NULL");
    if ((st = check_banded(m, "the allocation-free call"))) return st;
    void *scratch = nullptr;
    HIP_TRY(ps::noalloc_scratch(&scratch));
    // the largest slot count (a multiple of one wavefront, at most the default plan's) whose
    // workspace fits the fixed scratch
    const int64_t quantum = 64;
    int64_t slots = default_slots(m, npts, r);
    slots -= slots % quantum;
    while (slots >= quantum && ps::workspace_bytes(m->n, m->kl, m->ku, slots, r.max_iter, 0, npts) >
                                   ps::kNoallocScratchBytes)
        slots -= quantum;
    if (slots < quantum)
        return fail(PS_ERR_WORKSPACE,
                    "%lld shifts at n=%lld need %zu bytes with one wavefront of slots; the fixed scratch holds %zu",
                    (long long)npts, (long long)m->n,
                    ps::workspace_bytes(m->n, m->kl, m->ku, quantum, r.max_iter, 0, npts),
                    ps::kNoallocScratchBytes);
    r.slots = (int32_t)slots;
    ps::Workspace w;
    ps::EvalArgs a;
    ps::carve_workspace(scratch, m->n, m->kl, m->ku, slots, r.max_iter, 0, npts, &w);
    if (!sigma_dev) return fail(PS_ERR_INVALID, "sigma output is NULL");
    a.n = m->n;
    a.kl = m->kl;
    a.ku = m->ku;
    a.arow = m->arow;
    a.normA = m->fro;
    a.norm2A = m->norm2;
    a.bisect = bisect_of(r);
    a.gram = m->gram;
    a.lanes = lanes_of(r);
    a.ktm = ktm_of(r);
    a.tol_norm = r.tol_norm;
    a.tol_rel = r.tol_rel;
    a.max_iter = r.max_iter;
    a.check_shift = check_shift_of(r);
    a.want_vectors = 0;
    a.sigma = sigma_dev;
    a.count_dev = w.count;
    a.mode = ps::kShiftList;
    a.z = (const double2 *)z_dev;
    a.info = info_dev;
    a.iters = iters_dev;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ps::launch_set_count(w.count, npts, w.queue, s));
    {
        SideLock sl(m, s);
        HIP_TRY(ps::launch_eval(a, w, s, sl.side));
    }
    return ok();
}

ps_status ps_eval_grid(ps_matrix m, const ps_grid *g, const uint8_t *mask_dev, const ps_opts *o, void *ws_dev,
                       size_t ws_bytes, int64_t *idx_dev, int64_t *count_dev, double *sigma_dev, ps_c128 *u_dev,
                       ps_c128 *v_dev, int32_t *info_dev, int32_t *iters_dev, double eps, uint8_t *sens_dev,
                       void *stream) {
    ps_status st = check_handle(m);
    if (st) return st;
    if ((st = check_grid(g))) return st;
    if (!idx_dev || !count_dev) return fail(PS_ERR_INVALID, "idx and count outputs are required");
    if (sens_dev && !isfinite(eps)) return fail(PS_ERR_INVALID, "eps must be finite");
    ps_opts r = resolve(o);
    if ((st = check_opts(r))) return st;
    const int64_t npts = g->nx * g->ny;
    ps::Workspace w;
    ps::EvalArgs a;
    if ((st = prepare_eval(m, npts, r, ws_dev, ws_bytes, sigma_dev, u_dev, v_dev, &w, &a))) return st;
    a.mode = ps::kShiftGrid;
    a.ga = g->a;
    a.gb = g->b;
    a.gc = g->c;
    a.gd = g->d;
    a.nx = g->nx;
    a.ny = g->ny;
    a.info = info_dev;
    a.iters = iters_dev;
    a.eps = eps;
    a.sens = sens_dev;
    hipStream_t s = (hipStream_t)stream;
    if (mask_dev) {
        HIP_TRY(ps::launch_compact_mask(mask_dev, npts, idx_dev, w.count, w.blocksums, w.queue, s));
        a.idx = idx_dev;
    } else {
        HIP_TRY(ps::launch_iota(idx_dev, npts, s));
        HIP_TRY(ps::launch_set_count(w.count, npts, w.queue, s));
        a.idx = nullptr;
    }
    a.count_dev = w.count;
    HIP_TRY(hipMemcpyAsync(count_dev, w.count, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    {
        SideLock sl(m, s);
        HIP_TRY(ps::launch_eval(a, w, s, sl.side));
    }
    return ok();
}

ps_status ps_backward_workspace_size(ps_matrix m, int64_t npts, size_t *bytes) {
    ps_status st = check_handle(m);
    if (st) return st;
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    if (npts < 0) return fail(PS_ERR_INVALID, "npts must be >= 0");
    if ((st = check_banded(m, "the adjoint"))) return st;
    int64_t rows = ps::backward_partial_rows(npts);
    *bytes = sizeof(double2) * ((size_t)(rows > 0 ? rows : 1) * (size_t)m->n * (size_t)(m->kl + m->ku + 1) +
                                (size_t)npts * (size_t)ps::backward_zpart_cols(m->n));
    return ok();
}

ps_status ps_backward(ps_matrix m, int64_t npts, const double *grad_sigma_dev, const ps_c128 *u_dev,
                      const ps_c128 *v_dev, ps_c128 *grad_z_dev, ps_c128 *grad_band_dev, void *ws_dev,
                      size_t ws_bytes, void *stream) {
    ps_status st = check_handle(m);
    if (st) return st;
    if (npts < 0) return fail(PS_ERR_INVALID, "npts must be >= 0");
    if (!grad_z_dev && !grad_band_dev) return ok();
    if (npts > 0 && (!grad_sigma_dev || !u_dev || !v_dev))
        return fail(PS_ERR_INVALID, "grad_sigma, u and v are required");
    if ((st = check_banded(m, "the adjoint"))) return st;
    hipStream_t s = (hipStream_t)stream;
    if (npts == 0) {
        if (grad_band_dev)
            HIP_TRY(ps::launch_zero(grad_band_dev, sizeof(ps_c128) * (size_t)m->n * (m->kl + m->ku + 1), s));
        return ok();
    }
    size_t need = 0;
    ps_backward_workspace_size(m, npts, &need);
    if (grad_band_dev && (!ws_dev || ws_bytes < need))
        return fail(PS_ERR_WORKSPACE, "backward workspace needs %zu bytes (got %zu)", need, ws_bytes);
    HIP_TRY(ps::launch_backward(m->n, m->kl, m->ku, npts, grad_sigma_dev, (const double2 *)u_dev,
                                (const double2 *)v_dev, (double2 *)grad_z_dev, (double2 *)grad_band_dev,
                                (double2 *)ws_dev, (m->flags & PS_REAL_A) ? 1 : 0, s));
    return ok();
}

}  // extern "C"

struct ps_batch_s {
    int32_t nmat = 0;
    std::vector<ps_grid> grids;
    std::vector<int64_t> off;
    std::vector<int64_t> npts;
    std::vector<int64_t> mat_n;           // per matrix, caller order (plan-cache key)
    std::vector<int32_t> mat_kl, mat_ku;
    int64_t total = 0;
    int64_t max_npts = 0;
    ps::MatDesc *desc_caller = nullptr;   // device, caller order
    ps::MatDesc *desc_class = nullptr;    // device, grouped by (kl, ku), larger n first
    ps::MatDesc *desc_lpt = nullptr;      // device, longest-first by predicted bisection cost
    static constexpr int kSides = 1;      // the stream of the Golub-Kahan launch
    ps::SideStream side[kSides];
    std::mutex side_mu;                   // held while a call enqueues its fork, launch and join
    int max_hb = 0;                       // largest kl + ku
    int64_t lpt_chunks[3] = {0, 0, 0};    // chunks of 64, 32, 16 shifts over the full grids
    struct Cls {
        int kl, ku, begin, count;
        int64_t nmax, npts;
        int64_t gkbase;   // offset of the class's Golub-Kahan list in the batch scratch
    };
    std::vector<Cls> classes;
};

namespace {

// Slots of one class's Golub-Kahan launch.  The classes run concurrently, so each has its own
// workspace within an equal share of the default budget.  A class that bisects hands only the
// shifts below the bisection's rounding limit to this launch (a few per cent on the measured
// workloads): an eighth of its shifts, at least 256, get a slot of their own; lanes take
// further shifts as they finish.
int64_t class_slots(const ps_batch_s::Cls &c, const ps_opts &o, bool bis, size_t nclass) {
    int64_t need = bis && c.kl + c.ku >= 1 ? (c.npts + 7) / 8 : c.npts;
    int64_t want = ((need + kSlotQuantum - 1) / kSlotQuantum) * kSlotQuantum;
    if (o.slots > 0) want = round_slots(o.slots);
    if (want < kSlotQuantum) want = kSlotQuantum;
    if (want > kMaxSlots) want = kMaxSlots;
    const double budget = kDefaultWsBudget / (double)(nclass > 0 ? nclass : 1);
    while (want > kSlotQuantum &&
           (double)ps::workspace_bytes(c.nmax, c.kl, c.ku, want, o.max_iter, 0, 0) > budget)
        want -= kSlotQuantum;
    return want;
}

size_t class_ws_bytes(const ps_batch_s::Cls &c, const ps_opts &o, bool bis, size_t nclass) {
    const size_t b = ps::workspace_bytes(c.nmax, c.kl, c.ku, class_slots(c, o, bis, nclass), o.max_iter, 0, 0);
    return (b + 255) & ~(size_t)255;
}

// Batch scratch, 256-byte aligned pieces: compaction tile sums [tiles * nmat], then
// mfirst, pfx, chunkfirst [nmat], ctotal, gk_count [classes], the chunk total, and the
// Golub-Kahan lists [total points].
struct BatchScratch {
    int64_t *tilesums, *mfirst, *pfx, *chunkfirst, *ctotal, *gk_count, *total_chunks, *gk_list;
    double *st_lo, *st_hi;
    int32_t *st_np;
    size_t bytes;
};

BatchScratch batch_scratch(const ps_batch_s *b, char *base) {
    int64_t nt = ps::batch_tiles(b->max_npts);
    if (nt < 1) nt = 1;
    size_t off = 0;
    auto take = [&](size_t bytes) -> int64_t * {
        int64_t *p = (int64_t *)(base + off);
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const size_t nm = sizeof(int64_t) * (size_t)b->nmat, nc = sizeof(int64_t) * b->classes.size();
    BatchScratch r;
    r.tilesums = take(sizeof(int64_t) * (size_t)(nt * b->nmat));
    r.mfirst = take(nm);
    r.pfx = take(nm);
    r.chunkfirst = take(nm);
    r.ctotal = take(nc);
    r.gk_count = take(nc);
    r.total_chunks = take(sizeof(int64_t));
    r.gk_list = take(sizeof(int64_t) * (size_t)b->total);
    r.st_lo = (double *)take(sizeof(double) * (size_t)b->total);
    r.st_hi = (double *)take(sizeof(double) * (size_t)b->total);
    r.st_np = (int32_t *)take(sizeof(int32_t) * (size_t)b->total);
    r.bytes = off;
    return r;
}

size_t batch_scratch_bytes(const ps_batch_s *b) { return batch_scratch(b, nullptr).bytes; }

// A candidate plan replaces the default only when it runs in under this fraction of its time
// (differences below that are within the run-to-run spread of a call).
constexpr float kTuneMargin = 0.98f;

// Plans chosen by ps_autotune / ps_autotune_batch, by device and problem shape.
std::mutex &plan_mutex() {
    static std::mutex mu;
    return mu;
}
std::map<std::string, ps_opts> &plan_cache() {
    static std::map<std::string, ps_opts> c;
    return c;
}
std::string device_tag() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    return std::string(p.gcnArchName) + "/" + std::to_string(p.multiProcessorCount);
}
int log2_bucket(int64_t v) {
    int b = 0;
    while (b < 62 && ((int64_t)1 << b) < v) ++b;
    return b;
}
// the fields a plan sets
void copy_plan(const ps_opts &from, ps_opts *to) {
    to->slots = from.slots;
    to->check_shift = from.check_shift;
    to->lanes = from.lanes;
    to->tests = from.tests;
}
bool plan_lookup(const std::string &key, ps_opts *o) {
    std::lock_guard<std::mutex> g(plan_mutex());
    auto it = plan_cache().find(key);
    if (it == plan_cache().end()) return false;
    copy_plan(it->second, o);
    return true;
}
void plan_store(const std::string &key, const ps_opts &o) {
    std::lock_guard<std::mutex> g(plan_mutex());
    plan_cache()[key] = o;
}


}  // namespace

extern "C" {

// Label workspace: the evaluation workspace for every grid point, then status and mask bytes,
// compacted indices, compacted sigma and the evaluation counter.
static size_t label_aux_bytes(int64_t npts) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return 2 * al((size_t)npts) + 2 * al(sizeof(int64_t) * (size_t)npts) + al(sizeof(int32_t) * (size_t)npts) + 256;
}

ps_status ps_label_workspace_size(ps_matrix m, const ps_grid *g, const ps_opts *o, size_t *bytes) {
    ps_status st = check_handle(m);
    if (st) return st;
    if ((st = check_grid(g))) return st;
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    ps_opts r = resolve(o);
    if ((st = check_opts(r))) return st;
    if (r.want_vectors) return fail(PS_ERR_UNSUPPORTED, "labelling does not produce vectors");
    if ((st = check_banded(m, "labelling"))) return st;
    const int64_t npts = g->nx * g->ny;
    size_t ev = 0;
    if ((st = ps_workspace_size(m, npts, &r, &ev))) return st;
    *bytes = ((ev + 255) & ~(size_t)255) + label_aux_bytes(npts);
    return ok();
}

ps_status ps_label_grid(ps_matrix m, const ps_grid *g, double eps, const ps_opts *o, void *ws_dev, size_t ws_bytes,
                        uint8_t *label_dev, double *sigma_dev, int64_t *evals_dev, void *stream) {
    ps_status st = check_handle(m);
    if (st) return st;
    if ((st = check_grid(g))) return st;
    if (!(eps > 0.0) || !isfinite(eps)) return fail(PS_ERR_INVALID, "eps must be finite and > 0");
    if (!label_dev) return fail(PS_ERR_INVALID, "label output is NULL");
    ps_opts r = resolve(o);
    if ((st = check_opts(r))) return st;
    if (r.want_vectors) return fail(PS_ERR_UNSUPPORTED, "labelling does not produce vectors");
    size_t need = 0;
    if ((st = ps_label_workspace_size(m, g, &r, &need))) return st;
    if (!ws_dev || ws_bytes < need) return fail(PS_ERR_WORKSPACE, "label workspace needs %zu bytes", need);
    if (!aligned(ws_dev, 256)) return fail(PS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    const int64_t npts = g->nx * g->ny;
    const size_t evb = ((need - label_aux_bytes(npts)) + 255) & ~(size_t)255;
    char *aux = (char *)ws_dev + evb;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    uint8_t *status = (uint8_t *)aux;
    uint8_t *mask = status + al((size_t)npts);
    int64_t *idx = (int64_t *)(mask + al((size_t)npts));
    double *sig_c = (double *)((char *)idx + al(sizeof(int64_t) * (size_t)npts));
    int32_t *info_c = (int32_t *)((char *)sig_c + al(sizeof(double) * (size_t)npts));
    int64_t *evals = (int64_t *)((char *)info_c + al(sizeof(int32_t) * (size_t)npts));
    if (evals_dev) evals = evals_dev;
    ps::Workspace w;
    ps::EvalArgs a;
    if ((st = prepare_eval(m, npts, r, ws_dev, evb, sig_c, nullptr, nullptr, &w, &a))) return st;
    a.info = info_c;
    a.mode = ps::kShiftGrid;
    a.ga = g->a;
    a.gb = g->b;
    a.gc = g->c;
    a.gd = g->d;
    a.nx = g->nx;
    a.ny = g->ny;
    a.idx = idx;
    a.count_dev = w.count;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ps::launch_label_init(status, sigma_dev, npts, evals, s));
    int stride = 1;
    while (stride < 8 && (g->nx >= 24 * stride || g->ny >= 24 * stride)) stride *= 2;
    for (; stride >= 1; stride /= 2) {
        const int64_t lattice = ((g->ny + stride - 1) / stride) * ((g->nx + stride - 1) / stride);
        HIP_TRY(ps::launch_label_mask(status, g->nx, npts, stride, mask, s));
        HIP_TRY(ps::launch_compact_mask(mask, npts, idx, w.count, w.blocksums, w.queue, s));
        {
            SideLock sl(m, s);
            HIP_TRY(ps::launch_eval(a, w, s, sl.side));
        }
        HIP_TRY(ps::launch_label_update(g->a, g->b, g->c, g->d, g->nx, g->ny, idx, w.count, lattice, sig_c, info_c, eps,
                                        r.tol_norm * m->fro, r.tol_rel, status, sigma_dev, evals, s));
    }
    HIP_TRY(ps::launch_label_finish(status, label_dev, npts, s));
    return ok();
}

ps_status ps_contour_seeds_workspace_size(const ps_grid *g, size_t *bytes) {
    ps_status st = check_grid(g);
    if (st) return st;
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    // scan queue word (unused by the seeds) + one block sum per tile of edges
    *bytes = 256 + sizeof(int64_t) * (size_t)ps::contour_edge_tiles(g->nx, g->ny);
    return ok();
}

ps_status ps_contour_seeds(const ps_grid *g, const double *sigma_dev, double eps, ps_c128 *seeds_dev,
                           int64_t max_seeds, int64_t *count_dev, void *ws_dev, size_t ws_bytes, void *stream) {
    ps_status st = check_grid(g);
    if (st) return st;
    if (!(eps > 0.0) || !isfinite(eps)) return fail(PS_ERR_INVALID, "eps must be finite and > 0");
    if (max_seeds < 0) return fail(PS_ERR_INVALID, "max_seeds must be >= 0");
    if (!sigma_dev || !count_dev) return fail(PS_ERR_INVALID, "sigma and count are required");
    if (max_seeds > 0 && !seeds_dev) return fail(PS_ERR_INVALID, "seeds is NULL with max_seeds > 0");
    size_t need = 0;
    ps_contour_seeds_workspace_size(g, &need);
    if (!ws_dev || ws_bytes < need) return fail(PS_ERR_WORKSPACE, "contour-seed workspace needs %zu bytes", need);
    if (!aligned(ws_dev, 256)) return fail(PS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    char *base = (char *)ws_dev;
    HIP_TRY(ps::launch_contour_seeds(g->a, g->b, g->c, g->d, g->nx, g->ny, sigma_dev, eps, (double2 *)seeds_dev,
                                     max_seeds, count_dev, (int64_t *)(base + 256), (unsigned long long *)base,
                                     (hipStream_t)stream));
    return ok();
}

ps_status ps_newton_workspace_size(ps_matrix m, int64_t npts, const ps_opts *o, size_t *bytes) {
    ps_status st = check_handle(m);
    if (st) return st;
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    if (npts < 0) return fail(PS_ERR_INVALID, "npts must be >= 0");
    ps_opts r = resolve(o);
    r.want_vectors = 1;
    if ((st = check_opts(r))) return st;
    size_t ev = 0;
    if ((st = ps_workspace_size(m, npts, &r, &ev))) return st;
    ev = (ev + 255) & ~(size_t)255;
    size_t vec = ((sizeof(ps_c128) * (size_t)npts * (size_t)m->n) + 255) & ~(size_t)255;
    size_t gz = ((sizeof(ps_c128) * (size_t)npts) + 255) & ~(size_t)255;
    *bytes = ev + 2 * vec + gz;
    return ok();
}

ps_status ps_newton_contour(ps_matrix m, ps_c128 *z_dev, int64_t npts, double eps, int32_t steps, const ps_opts *o,
                            void *ws_dev, size_t ws_bytes, double *sigma_dev, int32_t *info_dev, void *stream) {
    ps_status st = check_handle(m);
    if (st) return st;
    if (npts < 0 || steps < 0) return fail(PS_ERR_INVALID, "npts and steps must be >= 0");
    if (!(eps > 0.0) || !isfinite(eps)) return fail(PS_ERR_INVALID, "eps must be finite and > 0");
    if (npts == 0) return ok();
    if (!z_dev || !sigma_dev) return fail(PS_ERR_INVALID, "z and sigma are required");
    ps_opts rv = resolve(o);
    rv.want_vectors = 1;
    if ((st = check_opts(rv))) return st;
    size_t need = 0;
    ps_newton_workspace_size(m, npts, &rv, &need);
    if (!ws_dev || ws_bytes < need) return fail(PS_ERR_WORKSPACE, "Newton workspace needs %zu bytes", need);
    size_t ev = 0;
    ps_workspace_size(m, npts, &rv, &ev);
    ev = (ev + 255) & ~(size_t)255;
    size_t vec = ((sizeof(ps_c128) * (size_t)npts * (size_t)m->n) + 255) & ~(size_t)255;
    char *base = (char *)ws_dev;
    ps_c128 *u = (ps_c128 *)(base + ev);
    ps_c128 *v = (ps_c128 *)(base + ev + vec);
    double2 *gz = (double2 *)(base + ev + 2 * vec);
    hipStream_t s = (hipStream_t)stream;
    for (int32_t it = 0; it < steps; ++it) {
        if ((st = ps_eval_points(m, z_dev, npts, &rv, ws_dev, ev, sigma_dev, u, v, info_dev, nullptr, stream)))
            return st;
        HIP_TRY(ps::launch_backward(m->n, m->kl, m->ku, npts, nullptr, (const double2 *)u, (const double2 *)v, gz,
                                    nullptr, nullptr, 0, s));
        HIP_TRY(ps::launch_newton_update(npts, (double2 *)z_dev, sigma_dev, gz, eps, s));
    }
    ps_opts rs = rv;
    rs.want_vectors = 0;
    if ((st = ps_eval_points(m, z_dev, npts, &rs, ws_dev, ev, sigma_dev, nullptr, nullptr, info_dev, nullptr,
                             stream)))
        return st;
    return ok();
}

// Workspace of ps_trace_contour: the evaluation workspace (with vectors) for nseed shifts,
// u and v, then per tracer the gradient, trial point, current point, its gradient, point 0,
// sigma, the active flag, and the active count.
ps_status ps_trace_workspace_size(ps_matrix m, int64_t nseed, const ps_opts *o, size_t *bytes) {
    ps_status st = check_handle(m);
    if (st) return st;
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    if (nseed < 0) return fail(PS_ERR_INVALID, "nseed must be >= 0");
    ps_opts r = resolve(o);
    r.want_vectors = 1;
    if ((st = check_opts(r))) return st;
    size_t ev = 0;
    if ((st = ps_workspace_size(m, nseed, &r, &ev))) return st;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t k = (size_t)nseed;
    *bytes = al(ev) + 2 * al(sizeof(ps_c128) * k * (size_t)m->n) + 5 * al(sizeof(ps_c128) * k) +
             al(sizeof(double) * k) + al(sizeof(int32_t) * k) + 256;
    return ok();
}

ps_status ps_trace_contour(ps_matrix m, const ps_c128 *seeds_dev, int64_t nseed, double eps, double h,
                           int32_t max_points, int32_t newton_steps, const ps_grid *box, const ps_opts *o,
                           void *ws_dev, size_t ws_bytes, ps_c128 *points_dev, int32_t *count_dev,
                           int32_t *flags_dev, void *stream) {
    ps_status st = check_handle(m);
    if (st) return st;
    if (nseed < 0) return fail(PS_ERR_INVALID, "nseed must be >= 0");
    if (!(eps > 0.0) || !isfinite(eps)) return fail(PS_ERR_INVALID, "eps must be finite and > 0");
    if (!(h > 0.0) || !isfinite(h)) return fail(PS_ERR_INVALID, "h must be finite and > 0");
    if (max_points < 1 || newton_steps < 1) return fail(PS_ERR_INVALID, "need max_points >= 1 and newton_steps >= 1");
    if (box && (!isfinite(box->a) || !isfinite(box->b) || !isfinite(box->c) || !isfinite(box->d)))
        return fail(PS_ERR_NONFINITE, "non-finite box");
    if (nseed == 0) return ok();
    if (!seeds_dev || !points_dev || !count_dev || !flags_dev)
        return fail(PS_ERR_INVALID, "seeds, points, count and flags are required");
    ps_opts rv = resolve(o);
    rv.want_vectors = 1;
    if ((st = check_opts(rv))) return st;
    size_t need = 0;
    if ((st = ps_trace_workspace_size(m, nseed, &rv, &need))) return st;
    if (!ws_dev || ws_bytes < need) return fail(PS_ERR_WORKSPACE, "trace workspace needs %zu bytes", need);
    if (!aligned(ws_dev, 256)) return fail(PS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t ev = 0;
    ps_workspace_size(m, nseed, &rv, &ev);
    ev = al(ev);
    const size_t k = (size_t)nseed;
    char *p = (char *)ws_dev + ev;
    auto take = [&](size_t bytes) -> char * {
        char *q = p;
        p += al(bytes);
        return q;
    };
    ps_c128 *u = (ps_c128 *)take(sizeof(ps_c128) * k * (size_t)m->n);
    ps_c128 *v = (ps_c128 *)take(sizeof(ps_c128) * k * (size_t)m->n);
    double2 *gz = (double2 *)take(sizeof(ps_c128) * k);
    double2 *zt = (double2 *)take(sizeof(ps_c128) * k);
    double2 *zc = (double2 *)take(sizeof(ps_c128) * k);
    double2 *gc = (double2 *)take(sizeof(ps_c128) * k);
    double2 *z0 = (double2 *)take(sizeof(ps_c128) * k);
    double *sig = (double *)take(sizeof(double) * k);
    int32_t *active = (int32_t *)take(sizeof(int32_t) * k);
    int32_t *n_active = (int32_t *)take(sizeof(int32_t));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ps::launch_trace_init(nseed, (const double2 *)seeds_dev, zt, active, count_dev, flags_dev, s));
    auto evaluate = [&]() -> ps_status {
        ps_status e = ps_eval_points(m, (const ps_c128 *)zt, nseed, &rv, ws_dev, ev, sig, u, v, nullptr, nullptr,
                                     stream);
        if (e) return e;
        HIP_TRY(ps::launch_backward(m->n, m->kl, m->ku, nseed, nullptr, (const double2 *)u, (const double2 *)v, gz,
                                    nullptr, nullptr, 0, s));
        return PS_OK;
    };
    for (int32_t kp = 0; kp < max_points; ++kp) {
        if (kp > 0) HIP_TRY(ps::launch_trace_predict(nseed, active, zc, gc, h, zt, s));
        const int32_t steps = kp == 0 ? 2 * newton_steps + 2 : newton_steps;
        for (int32_t it = 0; it < steps; ++it) {
            if ((st = evaluate())) return st;
            HIP_TRY(ps::launch_trace_newton(nseed, active, zt, sig, gz, eps, s));
        }
        if ((st = evaluate())) return st;
        HIP_TRY(ps::launch_trace_accept(nseed, kp, max_points, eps, h, box, zt, sig, gz, active, zc, gc, z0,
                                        (double2 *)points_dev, count_dev, flags_dev, s));
        if ((kp & 7) == 7 && kp + 1 < max_points) {
            int32_t h_active = 0;
            HIP_TRY(ps::launch_count_active(nseed, active, n_active, s));
            HIP_TRY(hipMemcpyAsync(&h_active, n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (h_active == 0) break;
        }
    }
    HIP_TRY(hipStreamSynchronize(s));
    return ok();
}

ps_status ps_autotune(ps_matrix m, const ps_c128 *z_dev, int64_t npts, ps_opts *o, void *stream) {
    ps_status st = check_handle(m);
    if (st) return st;
    if (!o || !z_dev || npts < 1) return fail(PS_ERR_INVALID, "need options, shifts and npts >= 1");
    if ((st = check_opts(*o))) return st;
    if (m->dense) return ok();   // the dense path has no plan to choose
    const bool bis = !o->want_vectors && bisect_of(*o) && m->kl + m->ku >= 1;
    char key[160];
    snprintf(key, sizeof key, "m|%s|n%d|kl%d|ku%d|p%d|v%d|b%d", device_tag().c_str(), log2_bucket(m->n), m->kl,
             m->ku, log2_bucket(npts), o->want_vectors ? 1 : 0, bisect_of(*o));
    if (plan_lookup(key, o)) return ok();
    hipStream_t s = (hipStream_t)stream;
    ps_opts base = *o;
    base.slots = 0;
    // candidates: the bisection's lanes per shift and tests per lane (sigma-only calls that
    // bisect), otherwise the Golub-Kahan kernel's slot count and Ritz-check interval
    std::vector<ps_opts> cands;
    if (bis) {
        for (int lanes : {1, 2, 4})
            for (int tests : {2, 1, 3}) {
                ps_opts t = base;
                t.lanes = lanes;
                t.tests = tests;
                cands.push_back(t);
            }
    } else {
        const int64_t s0 = default_slots(m, npts, base);
        for (int64_t sl = s0; sl >= kSlotQuantum && cands.size() < 9; sl = round_slots(sl / 2))
            for (int c : {5, 4, 3}) {
                ps_opts t = base;
                t.slots = (int32_t)sl;
                t.check_shift = c;
                cands.push_back(t);
            }
    }
    size_t wsb = 0;
    for (const auto &t : cands) {
        size_t b = 0;
        if ((st = ps_workspace_size(m, npts, &t, &b))) return st;
        wsb = std::max(wsb, b);
    }
    void *ws = nullptr;
    double *sig = nullptr;
    HIP_TRY(hipMalloc(&ws, wsb));
    hipError_t e = hipMalloc((void **)&sig, sizeof(double) * (size_t)npts);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = INFINITY;
    ps_opts pick = cands[0];
    // sigma only while timing: the plan fields do not change what vectors cost per step
    for (size_t i = 0; e == hipSuccess && !st && i < cands.size(); ++i) {
        ps_opts t = cands[i];
        const int32_t vec = t.want_vectors;
        if (!bis) t.want_vectors = 0;
        float ms = INFINITY;
        for (int rep = 0; rep < 3 && e == hipSuccess && !st; ++rep) {   // the first call is untimed
            float one = INFINITY;
            if (rep > 0) e = hipEventRecord(e0, s);
            if (e == hipSuccess)
                st = ps_eval_points(m, z_dev, npts, &t, ws, wsb, sig, nullptr, nullptr, nullptr, nullptr, stream);
            if (rep > 0 && e == hipSuccess && !st) e = hipEventRecord(e1, s);
            if (rep > 0 && e == hipSuccess && !st) e = hipEventSynchronize(e1);
            if (rep > 0 && e == hipSuccess && !st) e = hipEventElapsedTime(&one, e0, e1);
            ms = std::min(ms, one);
        }
        t.want_vectors = vec;
        // the first candidate is the default plan: another replaces it only when clearly faster
        if (e == hipSuccess && !st && (i == 0 || ms < kTuneMargin * best)) {
            best = ms;
            pick = t;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sig);
    (void)hipFree(ws);
    if (st) return st;
    if (e != hipSuccess) return fail(PS_ERR_HIP, "autotune: %s", hipGetErrorString(e));
    copy_plan(pick, o);
    plan_store(key, *o);
    return ok();
}

void ps_plan_cache_clear(void) {
    std::lock_guard<std::mutex> g(plan_mutex());
    plan_cache().clear();
}

ps_status ps_create_batch(int32_t nmat, const ps_matrix *mats, const ps_grid *grids, ps_batch *out) {
    if (!out) return fail(PS_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (nmat < 1 || !mats || !grids) return fail(PS_ERR_INVALID, "need nmat >= 1, mats and grids");
    ps_batch b = new ps_batch_s();
    b->nmat = nmat;
    std::vector<ps::MatDesc> dc((size_t)nmat);
    for (int32_t m = 0; m < nmat; ++m) {
        const ps_matrix a = mats[m];
        const ps_grid &g = grids[m];
        if (!a) { delete b; return fail(PS_ERR_INVALID, "matrix %d is NULL", m); }
        if (a->dense) {
            delete b;
            return fail(PS_ERR_UNSUPPORTED, "matrix %d has kl=%d ku=%d: batches need kl, ku <= %d", m, a->kl, a->ku,
                        ps::kMaxKL);
        }
        if (g.nx < 1 || g.ny < 1 || g.nx * g.ny > ((int64_t)1 << 40)) {
            delete b;
            return fail(PS_ERR_INVALID, "bad grid size for matrix %d", m);
        }
        if (!isfinite(g.a) || !isfinite(g.b) || !isfinite(g.c) || !isfinite(g.d)) {
            delete b;
            return fail(PS_ERR_NONFINITE, "non-finite grid bounds for matrix %d", m);
        }
        ps::MatDesc d;
        d.arow = a->arow;
        d.gram = a->gram;
        d.n = a->n;
        d.normA = a->fro;
        d.norm2A = a->norm2;
        d.ga = g.a;
        d.gb = g.b;
        d.gc = g.c;
        d.gd = g.d;
        d.nx = g.nx;
        d.ny = g.ny;
        d.out_off = b->total;
        d.kl = a->kl;
        d.ku = a->ku;
        d.cidx = m;
        d.cls = 0;
        d.cpos = 0;
        d.cfirst = 0;
        d.gkbase = 0;
        dc[(size_t)m] = d;
        b->max_hb = std::max(b->max_hb, a->kl + a->ku);
        b->grids.push_back(g);
        b->off.push_back(b->total);
        b->npts.push_back(g.nx * g.ny);
        b->mat_n.push_back(a->n);
        b->mat_kl.push_back(a->kl);
        b->mat_ku.push_back(a->ku);
        b->total += g.nx * g.ny;
        b->max_npts = std::max(b->max_npts, g.nx * g.ny);
    }
    std::vector<ps::MatDesc> dk = dc;
    std::stable_sort(dk.begin(), dk.end(), [](const ps::MatDesc &x, const ps::MatDesc &y) {
        if (x.kl != y.kl) return x.kl < y.kl;
        if (x.ku != y.ku) return x.ku < y.ku;
        return x.n > y.n;
    });
    for (int32_t i = 0; i < nmat;) {
        ps_batch_s::Cls c;
        c.kl = dk[(size_t)i].kl;
        c.ku = dk[(size_t)i].ku;
        c.begin = i;
        c.count = 0;
        c.nmax = 0;
        c.npts = 0;
        while (i < nmat && dk[(size_t)i].kl == c.kl && dk[(size_t)i].ku == c.ku) {
            c.nmax = std::max(c.nmax, dk[(size_t)i].n);
            c.npts += dk[(size_t)i].nx * dk[(size_t)i].ny;
            ++c.count;
            ++i;
        }
        b->classes.push_back(c);
    }
    // class of every matrix, its class-sorted position, the first matrix of its class, and the
    // offset of its class's Golub-Kahan list (classes in order, each sized by its grid points)
    int64_t gkbase = 0;
    for (size_t ci = 0; ci < b->classes.size(); ++ci) {
        auto &c = b->classes[ci];
        c.gkbase = gkbase;
        for (int p = c.begin; p < c.begin + c.count; ++p) {
            dk[(size_t)p].cls = (int32_t)ci;
            dk[(size_t)p].cpos = p;
            dk[(size_t)p].cfirst = c.begin;
            dk[(size_t)p].gkbase = gkbase;
            dc[(size_t)dk[(size_t)p].cidx] = dk[(size_t)p];
        }
        gkbase += c.npts;
    }
    // longest-first order of the bisection chunks: predicted cost per shift ~ n times the work
    // of one row of a pass (forming the row of H and one test)
    std::vector<ps::MatDesc> dl = dk;
    auto cost = [](const ps::MatDesc &x) {
        const double hb = (double)(x.kl + x.ku);
        return (double)x.n * (2.0 * hb * hb + 8.0 * hb + 8.0);
    };
    std::stable_sort(dl.begin(), dl.end(),
                     [&](const ps::MatDesc &x, const ps::MatDesc &y) { return cost(x) > cost(y); });
    for (int k = 0; k < 3; ++k) {
        const int64_t spw = 64 >> k;
        for (const auto &d : dl) b->lpt_chunks[k] += (d.nx * d.ny + spw - 1) / spw;
    }
    hipError_t e = hipMalloc((void **)&b->desc_caller, sizeof(ps::MatDesc) * (size_t)nmat);
    if (e == hipSuccess) e = hipMalloc((void **)&b->desc_class, sizeof(ps::MatDesc) * (size_t)nmat);
    if (e == hipSuccess) e = hipMalloc((void **)&b->desc_lpt, sizeof(ps::MatDesc) * (size_t)nmat);
    if (e == hipSuccess)
        e = hipMemcpy(b->desc_caller, dc.data(), sizeof(ps::MatDesc) * (size_t)nmat, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->desc_class, dk.data(), sizeof(ps::MatDesc) * (size_t)nmat, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->desc_lpt, dl.data(), sizeof(ps::MatDesc) * (size_t)nmat, hipMemcpyHostToDevice);
    for (auto &sd : b->side)
        if (e == hipSuccess) e = create_side(&sd);
    if (e != hipSuccess) {
        ps_destroy_batch(b);
        return fail(PS_ERR_HIP, "batch descriptors: %s", hipGetErrorString(e));
    }
    *out = b;
    return ok();
}

ps_status ps_destroy_batch(ps_batch b) {
    if (!b) return ok();
    if (b->desc_caller) (void)hipFree(b->desc_caller);
    if (b->desc_class) (void)hipFree(b->desc_class);
    if (b->desc_lpt) (void)hipFree(b->desc_lpt);
    for (auto &sd : b->side) destroy_side(&sd);
    delete b;
    return ok();
}

ps_status ps_batch_info(ps_batch b, int64_t *total_points, int64_t *offsets) {
    if (!b) return fail(PS_ERR_INVALID, "batch is NULL");
    if (total_points) *total_points = b->total;
    if (offsets)
        for (int32_t m = 0; m < b->nmat; ++m) offsets[m] = b->off[(size_t)m];
    return ok();
}

ps_status ps_batch_workspace_size(ps_batch b, const ps_opts *o, size_t *bytes) {
    if (!b) return fail(PS_ERR_INVALID, "batch is NULL");
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    ps_opts r = resolve(o);
    ps_status st;
    if ((st = check_opts(r))) return st;
    const bool bis = bisect_of(r) && b->max_hb >= 1;
    size_t sum = 0;
    for (const auto &c : b->classes) sum += class_ws_bytes(c, r, bis, b->classes.size());
    *bytes = batch_scratch_bytes(b) + sum;
    return ok();
}

// Compaction of the masks, the plan (queue positions per (kl, ku) class, longest-first chunk
// order), the bisection's first pass over every shift of every matrix, then at once: the
// bisection resumed on the caller's stream, and one Golub-Kahan launch per class over the
// shifts the first pass handed over (all shifts of a class that does not bisect) on the side
// streams, longest classes first, each class with its own workspace past the batch scratch.
static ps_status batch_eval_core(ps_batch b, const uint8_t *const *masks_dev, const ps_opts &r, char *base,
                                 int64_t *idx_dev, int64_t *counts_dev, double *sigma_dev, int32_t *info_dev,
                                 int32_t *iters_dev, hipStream_t s) {
    const BatchScratch bs = batch_scratch(b, base);
    const int lanes = lanes_of(r);
    if (lanes == 64) return fail(PS_ERR_INVALID, "lanes = 64 (a wavefront per shift) is not a batch plan: use 1, 2 or 4");
    const bool bis = bisect_of(r) && b->max_hb >= 1;
    const size_t ncls = b->classes.size();
    HIP_TRY(ps::launch_batch_compact(b->desc_caller, b->nmat, b->max_npts, masks_dev, idx_dev, counts_dev,
                                     bs.tilesums, s));
    HIP_TRY(ps::launch_bis_plan(b->desc_class, b->desc_lpt, b->nmat, (int)ncls, counts_dev, 64 / lanes, bs.pfx,
                                bs.mfirst, bs.ctotal, bs.chunkfirst, bs.total_chunks, bs.gk_count, s));
    ps::BisArgs ba;
    const int64_t chunks = b->lpt_chunks[lanes == 1 ? 0 : lanes == 2 ? 1 : 2];
    if (bis) {
        ba.batch = 1;
        ba.mats = b->desc_lpt;
        ba.nmat = b->nmat;
        ba.mlo = 0;
        ba.mhi = b->nmat - 1;
        ba.chunkfirst = bs.chunkfirst;
        ba.total_chunks = bs.total_chunks;
        ba.counts = counts_dev;
        ba.mfirst = bs.mfirst;
        ba.idx = idx_dev;
        ba.tol_norm = r.tol_norm;
        ba.tol_rel = r.tol_rel;
        ba.sigma = sigma_dev;
        ba.info = info_dev;
        ba.iters = iters_dev;
        ba.gk_list = bs.gk_list;
        ba.gk_count = bs.gk_count;
        ba.st_lo = bs.st_lo;
        ba.st_hi = bs.st_hi;
        ba.st_np = bs.st_np;
        ba.phase = 1;
        if (ps::timing_events().start)
            HIP_TRY(hipEventRecord(ps::timing_events().start, s));
        HIP_TRY(ps::launch_bis(ba, b->max_hb, ktm_of(r), lanes, chunks, s));
    }
    // one Golub-Kahan launch for all classes on a side stream, beside the resumed bisection
    ps::GkBatchArgs g;
    g.base.mode = ps::kShiftGrid;
    g.base.idx = idx_dev;
    g.base.tol_norm = r.tol_norm;
    g.base.tol_rel = r.tol_rel;
    g.base.max_iter = r.max_iter;
    g.base.check_shift = check_shift_of(r);
    g.base.bisect = 0;
    g.base.want_vectors = 0;
    g.base.sigma = sigma_dev;
    g.base.info = info_dev;
    g.base.iters = iters_dev;
    g.ws = base;
    g.ncls = (int32_t)ncls;
    size_t off = bs.bytes;
    int64_t blocks = 0;
    for (size_t ci = 0; ci < ncls; ++ci) {
        const auto &c = b->classes[ci];
        const bool handed = bis && c.kl + c.ku >= 1;
        ps::GkClass &q = g.cls[ci];
        q.kl = c.kl;
        q.ku = c.ku;
        q.nmat = c.count;
        q.pad = 0;
        q.first_block = blocks;
        q.nmax = c.nmax;
        q.slots = class_slots(c, r, bis, ncls);
        q.ws_off = (int64_t)off;
        q.mats = b->desc_class + c.begin;
        q.mfirst = bs.mfirst + c.begin;
        q.perm = handed ? bs.gk_list + c.gkbase : nullptr;
        q.count = handed ? bs.gk_count + ci : bs.ctotal + ci;
        HIP_TRY(ps::launch_zero(base + off, sizeof(unsigned long long), s));   // the class's queue counter
        blocks += q.slots / 64;
        off += class_ws_bytes(c, r, bis, ncls);
    }
    if (bis) {
        ps::ListBases lb = {};
        for (size_t ci = 0; ci < ncls; ++ci) lb.base[ci] = b->classes[ci].gkbase;
        HIP_TRY(ps::launch_sort_lists(bs.gk_list, lb, bs.gk_count, (int)ncls, s));
    }
    ps::SideStream &sd = b->side[0];
    std::lock_guard<std::mutex> side_lock(b->side_mu);
    HIP_TRY(hipEventRecord(sd.fork, s));
    HIP_TRY(hipStreamWaitEvent(sd.stream, sd.fork, 0));
    HIP_TRY(ps::launch_gk_batch(g, blocks, sd.stream));
    HIP_TRY(hipEventRecord(sd.join, sd.stream));
    if (bis) {
        ba.phase = 2;
        HIP_TRY(ps::launch_bis(ba, b->max_hb, ktm_of(r), lanes, chunks, s));
        if (ps::timing_events().end)
            HIP_TRY(hipEventRecord(ps::timing_events().end, s));
    }
    HIP_TRY(hipStreamWaitEvent(s, sd.join, 0));
    return ok();
}

ps_status ps_eval_batch(ps_batch b, const uint8_t *const *masks_dev, const ps_opts *o, void *ws_dev, size_t ws_bytes,
                        int64_t *idx_dev, int64_t *counts_dev, double *sigma_dev, int32_t *info_dev,
                        int32_t *iters_dev, void *stream) {
    if (!b) return fail(PS_ERR_INVALID, "batch is NULL");
    ps_opts r = resolve(o);
    ps_status st;
    if ((st = check_opts(r))) return st;
    if (r.want_vectors) return fail(PS_ERR_UNSUPPORTED, "vectors are not produced in batch mode");
    if (!idx_dev || !counts_dev || !sigma_dev) return fail(PS_ERR_INVALID, "idx, counts and sigma are required");
    if (!ws_dev) return fail(PS_ERR_WORKSPACE, "workspace is NULL");
    if (!aligned(ws_dev, 256)) return fail(PS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    size_t need = 0;
    ps_batch_workspace_size(b, &r, &need);
    if (ws_bytes < need) return fail(PS_ERR_WORKSPACE, "batch workspace needs %zu bytes (got %zu)", need, ws_bytes);
    return batch_eval_core(b, masks_dev, r, (char *)ws_dev, idx_dev, counts_dev, sigma_dev, info_dev, iters_dev,
                           (hipStream_t)stream);
}

ps_status ps_autotune_batch(ps_batch b, const uint8_t *const *masks_dev, ps_opts *o, void *stream) {
    if (!b) return fail(PS_ERR_INVALID, "batch is NULL");
    if (!o) return fail(PS_ERR_INVALID, "options are NULL");
    ps_status st;
    if ((st = check_opts(*o))) return st;
    if (o->want_vectors) return fail(PS_ERR_UNSUPPORTED, "vectors are not produced in batch mode");
    if (o->lanes == 64) return fail(PS_ERR_INVALID, "lanes = 64 is not a batch plan");
    const bool bis = bisect_of(*o) && b->max_hb >= 1;
    std::string key = "b|" + device_tag() + "|b" + std::to_string(bisect_of(*o)) + "|m" + std::to_string(b->nmat);
    for (int32_t m = 0; m < b->nmat; ++m) {
        key += "|" + std::to_string(log2_bucket(b->mat_n[(size_t)m])) + "," + std::to_string(b->mat_kl[(size_t)m]) +
               "," + std::to_string(b->mat_ku[(size_t)m]) + "," + std::to_string(log2_bucket(b->npts[(size_t)m]));
    }
    if (plan_lookup(key, o)) return ok();
    hipStream_t s = (hipStream_t)stream;
    std::vector<ps_opts> cands;
    if (bis) {
        for (int lanes : {1, 2, 4})
            for (int tests : {2, 1, 3}) {
                ps_opts t = *o;
                t.lanes = lanes;
                t.tests = tests;
                cands.push_back(t);
            }
    } else {
        for (int c : {5, 4, 3}) {
            ps_opts t = *o;
            t.check_shift = c;
            cands.push_back(t);
        }
    }
    size_t wsb = 0;
    for (const auto &t : cands) {
        size_t x = 0;
        if ((st = ps_batch_workspace_size(b, &t, &x))) return st;
        wsb = std::max(wsb, x);
    }
    void *ws = nullptr;
    int64_t *idx = nullptr, *counts = nullptr;
    double *sig = nullptr;
    HIP_TRY(hipMalloc(&ws, wsb));
    hipError_t e = hipMalloc((void **)&idx, sizeof(int64_t) * (size_t)b->total);
    if (e == hipSuccess) e = hipMalloc((void **)&counts, sizeof(int64_t) * (size_t)b->nmat);
    if (e == hipSuccess) e = hipMalloc((void **)&sig, sizeof(double) * (size_t)b->total);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = INFINITY;
    ps_opts pick = cands[0];
    // one untimed call first (set-up), then each candidate twice (the faster run counts); the
    // first candidate is the default plan, which another replaces only when clearly faster
    if (e == hipSuccess)
        st = ps_eval_batch(b, masks_dev, &cands[0], ws, wsb, idx, counts, sig, nullptr, nullptr, stream);
    for (size_t i = 0; e == hipSuccess && !st && i < cands.size(); ++i) {
        float ms = INFINITY;
        for (int rep = 0; rep < 2 && e == hipSuccess && !st; ++rep) {
            float one = INFINITY;
            e = hipEventRecord(e0, s);
            if (e == hipSuccess)
                st = ps_eval_batch(b, masks_dev, &cands[i], ws, wsb, idx, counts, sig, nullptr, nullptr, stream);
            if (e == hipSuccess && !st) e = hipEventRecord(e1, s);
            if (e == hipSuccess && !st) e = hipEventSynchronize(e1);
            if (e == hipSuccess && !st) e = hipEventElapsedTime(&one, e0, e1);
            ms = std::min(ms, one);
        }
        if (e == hipSuccess && !st && (i == 0 || ms < kTuneMargin * best)) {
            best = ms;
            pick = cands[i];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sig);
    (void)hipFree(counts);
    (void)hipFree(idx);
    (void)hipFree(ws);
    if (st) return st;
    if (e != hipSuccess) return fail(PS_ERR_HIP, "batch autotune: %s", hipGetErrorString(e));
    copy_plan(pick, o);
    plan_store(key, *o);
    return ok();
}

// Batched labelling workspace past the batch evaluation workspace: status and mask bytes for
// every point, the mask pointer array, compacted indices and sigma, counts, the counter.
static size_t blabel_aux_bytes(ps_batch b) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t tot = (size_t)b->total;
    return 2 * al(tot) + al(sizeof(void *) * (size_t)b->nmat) + 2 * al(8 * tot) + al(4 * tot) + al(8 * (size_t)b->nmat) + 256;
}

ps_status ps_label_batch_workspace_size(ps_batch b, const ps_opts *o, size_t *bytes) {
    if (!b) return fail(PS_ERR_INVALID, "batch is NULL");
    if (!bytes) return fail(PS_ERR_INVALID, "bytes is NULL");
    size_t ev = 0;
    ps_status st = ps_batch_workspace_size(b, o, &ev);
    if (st) return st;
    *bytes = ((ev + 255) & ~(size_t)255) + blabel_aux_bytes(b);
    return ok();
}

ps_status ps_label_batch(ps_batch b, double eps, const ps_opts *o, void *ws_dev, size_t ws_bytes, uint8_t *label_dev,
                         double *sigma_dev, int64_t *evals_dev, void *stream) {
    if (!b) return fail(PS_ERR_INVALID, "batch is NULL");
    if (!(eps > 0.0) || !isfinite(eps)) return fail(PS_ERR_INVALID, "eps must be finite and > 0");
    if (!label_dev) return fail(PS_ERR_INVALID, "label output is NULL");
    ps_opts r = resolve(o);
    ps_status st;
    if ((st = check_opts(r))) return st;
    if (r.want_vectors) return fail(PS_ERR_UNSUPPORTED, "labelling does not produce vectors");
    size_t need = 0;
    if ((st = ps_label_batch_workspace_size(b, &r, &need))) return st;
    if (!ws_dev || ws_bytes < need) return fail(PS_ERR_WORKSPACE, "batch label workspace needs %zu bytes", need);
    if (!aligned(ws_dev, 256)) return fail(PS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t tot = (size_t)b->total;
    char *aux = (char *)ws_dev + (need - blabel_aux_bytes(b));
    uint8_t *status = (uint8_t *)aux;
    uint8_t *mask = status + al(tot);
    uint8_t **mptr = (uint8_t **)(mask + al(tot));
    int64_t *idx = (int64_t *)((char *)mptr + al(sizeof(void *) * (size_t)b->nmat));
    double *sig_c = (double *)((char *)idx + al(8 * tot));
    int32_t *info_c = (int32_t *)((char *)sig_c + al(8 * tot));
    int64_t *counts = (int64_t *)((char *)info_c + al(4 * tot));
    int64_t *evals = (int64_t *)((char *)counts + al(8 * (size_t)b->nmat));
    if (evals_dev) evals = evals_dev;
    hipStream_t s = (hipStream_t)stream;
    int64_t nxmax = 0, nymax = 0;
    for (size_t m = 0; m < b->grids.size(); ++m) {
        nxmax = std::max(nxmax, b->grids[m].nx);
        nymax = std::max(nymax, b->grids[m].ny);
    }
    HIP_TRY(ps::launch_blabel_init(b->desc_caller, b->nmat, b->max_npts, status, sigma_dev, mask, mptr, evals, s));
    int stride = 1;
    while (stride < 8 && (nxmax >= 24 * stride || nymax >= 24 * stride)) stride *= 2;
    for (; stride >= 1; stride /= 2) {
        const int64_t lattice = ((nymax + stride - 1) / stride) * ((nxmax + stride - 1) / stride);
        HIP_TRY(ps::launch_blabel_mask(b->desc_caller, b->nmat, b->max_npts, status, stride, mask, s));
        if ((st = batch_eval_core(b, (const uint8_t *const *)mptr, r, (char *)ws_dev, idx, counts, sig_c, info_c,
                                  nullptr, s)))
            return st;
        HIP_TRY(ps::launch_blabel_update(b->desc_caller, b->nmat, lattice, idx, counts, sig_c, info_c, eps,
                                         r.tol_norm, r.tol_rel, status, sigma_dev, evals, s));
    }
    HIP_TRY(ps::launch_label_finish(status, label_dev, b->total, s));
    return ok();
}

}  // extern "C"
