// k_eval instantiations for lower bandwidth 3 (every upper bandwidth 0..4, three modes).
#include "ps_eval.hpp"

namespace ps {

EvalKernel pick_eval_kl3(int ku, int mode) { return pick_ku<3>(ku, mode); }

}  // namespace ps
