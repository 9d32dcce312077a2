// Dispatch of one step to the kernel instance for (N, K-1, anisotropy, potential).
// DIAG selects the instances that also write the partial diagnostics records
// of the stored state.
#pragma once

#include "step2d.hpp"
#include "step3d.hpp"

namespace mp {

template <typename R, int NP, int NM, bool D3, bool ANISO, bool OBST, bool DIAG>
int call_variant(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    if constexpr (D3)
        return call_3d<R, NP, NM, ANISO, OBST, DIAG>(L, c, k);
    else
        return call_2d<R, NP, NM, ANISO, OBST, DIAG>(L, c, k);
}

template <typename R, int NP, int NM, bool D3, bool DIAG>
int call_flags(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    const bool obst = L.potential == MP_OBSTACLE;
    if (L.aniso)
        return obst ? call_variant<R, NP, NM, D3, true, true, DIAG>(L, c, k)
                    : call_variant<R, NP, NM, D3, true, false, DIAG>(L, c, k);
    return obst ? call_variant<R, NP, NM, D3, false, true, DIAG>(L, c, k)
                : call_variant<R, NP, NM, D3, false, false, DIAG>(L, c, k);
}

// The general kernels (both obstacle projections share one instance: the
// choice is CoefX::proj).
template <typename R, int NP, int NM, bool D3, bool DIAG>
int call_gen_flags(const StepLaunch& L, const Coef<R>& c, const CoefX<R>& x, KernelCall& k) {
    const bool obst = L.potential != MP_WELL;
    if constexpr (D3) {
        if (L.aniso)
            return obst ? call_3d_gen<R, NP, NM, true, true, DIAG>(L, c, x, k)
                        : call_3d_gen<R, NP, NM, true, false, DIAG>(L, c, x, k);
        return obst ? call_3d_gen<R, NP, NM, false, true, DIAG>(L, c, x, k)
                    : call_3d_gen<R, NP, NM, false, false, DIAG>(L, c, x, k);
    } else {
        if (L.aniso)
            return obst ? call_2d_gen<R, NP, NM, true, true, DIAG>(L, c, x, k)
                        : call_2d_gen<R, NP, NM, true, false, DIAG>(L, c, x, k);
        return obst ? call_2d_gen<R, NP, NM, false, true, DIAG>(L, c, x, k)
                    : call_2d_gen<R, NP, NM, false, false, DIAG>(L, c, x, k);
    }
}

template <typename R, bool D3, bool DIAG>
int call_step_gen(const StepLaunch& L, const Coef<R>& c, const CoefX<R>& x, KernelCall& k) {
    if (L.nphases == 2 && L.nmu == 1) return call_gen_flags<R, 2, 1, D3, DIAG>(L, c, x, k);
    if (L.nphases == 2 && L.nmu == 2) return call_gen_flags<R, 2, 2, D3, DIAG>(L, c, x, k);
    if (L.nphases == 3 && L.nmu == 1) return call_gen_flags<R, 3, 1, D3, DIAG>(L, c, x, k);
    if (L.nphases == 3 && L.nmu == 2) return call_gen_flags<R, 3, 2, D3, DIAG>(L, c, x, k);
    return MP_E_PARAM;
}

template <typename R, bool D3, bool DIAG>
int call_step_dim(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    if (L.nphases == 2 && L.nmu == 1) return call_flags<R, 2, 1, D3, DIAG>(L, c, k);
    if (L.nphases == 2 && L.nmu == 2) return call_flags<R, 2, 2, D3, DIAG>(L, c, k);
    if (L.nphases == 3 && L.nmu == 1) return call_flags<R, 3, 1, D3, DIAG>(L, c, k);
    if (L.nphases == 3 && L.nmu == 2) return call_flags<R, 3, 2, D3, DIAG>(L, c, k);
    return MP_E_PARAM;
}

}  // namespace mp
