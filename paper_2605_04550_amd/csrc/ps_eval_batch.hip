// The Golub-Kahan kernel of a batch: one launch for every (kl, ku) class of the batch, so that
// the classes' shifts run at the same time instead of one class after another.  Each
// wavefront belongs to one class (a table in the kernel arguments), carves that class's part
// of the workspace and runs the class's compiled kernel body on its slot.
#include "ps_eval.hpp"

namespace ps {

namespace {

template <int KL, int KU>
__device__ void run_class(const EvalArgs &a, const Workspace &w, int64_t sg) {
    Kern<KL, KU, false, true>::run(a, w, sg);
}

__global__ void __launch_bounds__(kEvalBlock) k_eval_batch(GkBatchArgs g) {
    int c = 0;
    for (int k = 1; k < g.ncls; ++k)
        if (g.cls[k].first_block <= (int64_t)blockIdx.x) c = k;
    const GkClass &q = g.cls[c];
    EvalArgs a = g.base;
    a.n = q.nmax;
    a.kl = q.kl;
    a.ku = q.ku;
    a.mats = q.mats;
    a.nmat = q.nmat;
    a.mfirst = q.mfirst;
    a.perm = q.perm;
    a.count_dev = q.count;
    Workspace w;
    carve_workspace(g.ws + q.ws_off, q.nmax, q.kl, q.ku, q.slots, a.max_iter, 0, 0, &w);
    const int64_t sg = ((int64_t)blockIdx.x - q.first_block) * kEvalBlock + threadIdx.x;
    switch (q.kl * (kMaxKU + 1) + q.ku) {
#define PS_GK_CASE(KL, KU) \
    case KL * (kMaxKU + 1) + KU: run_class<KL, KU>(a, w, sg); break;
        PS_GK_CASE(0, 0) PS_GK_CASE(0, 1) PS_GK_CASE(0, 2) PS_GK_CASE(0, 3) PS_GK_CASE(0, 4)
        PS_GK_CASE(1, 0) PS_GK_CASE(1, 1) PS_GK_CASE(1, 2) PS_GK_CASE(1, 3) PS_GK_CASE(1, 4)
        PS_GK_CASE(2, 0) PS_GK_CASE(2, 1) PS_GK_CASE(2, 2) PS_GK_CASE(2, 3) PS_GK_CASE(2, 4)
        PS_GK_CASE(3, 0) PS_GK_CASE(3, 1) PS_GK_CASE(3, 2) PS_GK_CASE(3, 3) PS_GK_CASE(3, 4)
        PS_GK_CASE(4, 0) PS_GK_CASE(4, 1) PS_GK_CASE(4, 2) PS_GK_CASE(4, 3) PS_GK_CASE(4, 4)
#undef PS_GK_CASE
    default: break;
    }
}

}  // namespace

hipError_t launch_gk_batch(const GkBatchArgs &g, int64_t blocks, hipStream_t st) {
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(k_eval_batch, dim3((unsigned)blocks), dim3(kEvalBlock), 0, st, g);
    return hipGetLastError();
}

}  // namespace ps
