// Instances of the anti-trapping correction kernels (antitrap2d.hpp, antitrap3d.hpp).
#include "antitrap3d.hpp"

namespace mp {

template <typename R>
int at_launch(const AtLaunch& L, const AtCoef<R>& c, hipStream_t s) {
    return L.g.nz > 1 ? at_launch3d<R>(L, c, s) : at_launch2d<R>(L, c, s);
}

template int at_launch<float>(const AtLaunch&, const AtCoef<float>&, hipStream_t);
template int at_launch<double>(const AtLaunch&, const AtCoef<double>&, hipStream_t);
}  // namespace mp
