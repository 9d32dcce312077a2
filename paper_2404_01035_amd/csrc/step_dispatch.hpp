// Dispatch of one step to the kernel instance for (N, K-1, anisotropy, potential).
#pragma once

#include "step2d.hpp"
#include "step3d.hpp"

namespace mp {

template <typename R, int NP, int NM, bool D3, bool ANISO, bool OBST>
int launch_variant(const StepLaunch& L, const Coef<R>& c, hipStream_t s) {
    if constexpr (D3)
        return launch_3d<R, NP, NM, ANISO, OBST>(L, c, s);
    else
        return launch_2d<R, NP, NM, ANISO, OBST>(L, c, s);
}

template <typename R, int NP, int NM, bool D3>
int launch_flags(const StepLaunch& L, const Coef<R>& c, hipStream_t s) {
    const bool obst = L.potential == MP_OBSTACLE;
    if (L.aniso)
        return obst ? launch_variant<R, NP, NM, D3, true, true>(L, c, s)
                    : launch_variant<R, NP, NM, D3, true, false>(L, c, s);
    return obst ? launch_variant<R, NP, NM, D3, false, true>(L, c, s)
                : launch_variant<R, NP, NM, D3, false, false>(L, c, s);
}

template <typename R, bool D3>
int launch_step_dim(const StepLaunch& L, const Coef<R>& c, hipStream_t s) {
    if (L.nphases == 2 && L.nmu == 1) return launch_flags<R, 2, 1, D3>(L, c, s);
    if (L.nphases == 2 && L.nmu == 2) return launch_flags<R, 2, 2, D3>(L, c, s);
    if (L.nphases == 3 && L.nmu == 1) return launch_flags<R, 3, 1, D3>(L, c, s);
    if (L.nphases == 3 && L.nmu == 2) return launch_flags<R, 3, 2, D3>(L, c, s);
    return MP_E_PARAM;
}

}  // namespace mp
