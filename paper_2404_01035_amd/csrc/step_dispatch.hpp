// Dispatch of one step to the kernel instance for (N, K-1, anisotropy, potential).
#pragma once

#include "step2d.hpp"
#include "step3d.hpp"

namespace mp {

template <typename R, int NP, int NM, bool D3, bool ANISO, bool OBST>
int call_variant(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    if constexpr (D3)
        return call_3d<R, NP, NM, ANISO, OBST>(L, c, k);
    else
        return call_2d<R, NP, NM, ANISO, OBST>(L, c, k);
}

template <typename R, int NP, int NM, bool D3>
int call_flags(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    const bool obst = L.potential == MP_OBSTACLE;
    if (L.aniso)
        return obst ? call_variant<R, NP, NM, D3, true, true>(L, c, k)
                    : call_variant<R, NP, NM, D3, true, false>(L, c, k);
    return obst ? call_variant<R, NP, NM, D3, false, true>(L, c, k)
                : call_variant<R, NP, NM, D3, false, false>(L, c, k);
}

template <typename R, bool D3>
int call_step_dim(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    if (L.nphases == 2 && L.nmu == 1) return call_flags<R, 2, 1, D3>(L, c, k);
    if (L.nphases == 2 && L.nmu == 2) return call_flags<R, 2, 2, D3>(L, c, k);
    if (L.nphases == 3 && L.nmu == 1) return call_flags<R, 3, 1, D3>(L, c, k);
    if (L.nphases == 3 && L.nmu == 2) return call_flags<R, 3, 2, D3>(L, c, k);
    return MP_E_PARAM;
}

}  // namespace mp
