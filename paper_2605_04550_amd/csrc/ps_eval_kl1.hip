// k_eval instantiations for lower bandwidth 1 (every upper bandwidth 0..4, three modes).
#include "ps_eval.hpp"

namespace ps {

EvalKernel pick_eval_kl1(int ku, int mode) { return pick_ku<1>(ku, mode); }

}  // namespace ps
