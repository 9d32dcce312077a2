// Instances of the anti-trapping correction kernels for the extended model
// (compositions at each row's temperature, 2 x 2 susceptibility).
#include "antitrap3d.hpp"

namespace mp {

// The correction after one step of the extended model at time level *stepctr + kstep
// (T - Te = tb0 + tdn (*stepctr + kstep) + tslope * row).
template <typename R>
int at_launch_gen(const AtLaunch& L, const AtCoef<R>& c, const CoefX<R>& x, const int64_t* stepctr, int kstep,
                  double tb0, double tdn, double tslope, hipStream_t s) {
    const AtTime t{stepctr, kstep, tb0, tdn, tslope};
    return L.g.nz > 1 ? at_launch3d<R, true>(L, c, s, &x, &t) : at_launch2d<R, true>(L, c, s, &x, &t);
}

template int at_launch_gen<float>(const AtLaunch&, const AtCoef<float>&, const CoefX<float>&, const int64_t*, int,
                                  double, double, double, hipStream_t);
template int at_launch_gen<double>(const AtLaunch&, const AtCoef<double>&, const CoefX<double>&, const int64_t*, int,
                                   double, double, double, hipStream_t);
}  // namespace mp
