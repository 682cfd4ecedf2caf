// Inertia-bisection kernel instantiations for half-bandwidth 1 (one matrix), and for batches
// whose largest half-bandwidth is 1 (even bounds only); one file per bound so that they
// compile in parallel.
#include "ps_bisect.hpp"

namespace ps {

namespace {

template <int LO, int HI, bool SINGLE>
BisKernel pick_range(int ktm, int lanes) {
    switch (ktm * 100 + lanes) {
    case 1: return bis::k_bis<LO, HI, 0, 1>;
    case 2: return bis::k_bis<LO, HI, 0, 2>;
    case 4: return bis::k_bis<LO, HI, 0, 4>;
    case 101: return bis::k_bis<LO, HI, 1, 1>;
    case 102: return bis::k_bis<LO, HI, 1, 2>;
    case 104: return bis::k_bis<LO, HI, 1, 4>;
    case 201: return bis::k_bis<LO, HI, 2, 1>;
    case 202: return bis::k_bis<LO, HI, 2, 2>;
    case 204: return bis::k_bis<LO, HI, 2, 4>;
    case 64:
        if constexpr (SINGLE) return bis::k_bis<LO, HI, 0, 64>;
        return nullptr;
    }
    return nullptr;
}

}  // namespace

BisKernel pick_bis_h1(bool batch, int ktm, int lanes) {
    if (batch) return nullptr;   // batch launches use the even upper bounds
    return pick_range<1, 1, true>(ktm, lanes);
}

}  // namespace ps
