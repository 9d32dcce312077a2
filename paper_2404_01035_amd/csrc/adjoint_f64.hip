// Adjoint kernel instances, FP64.
#include "adjoint2d.hpp"

namespace mp {
template int adj_launch<double>(const AdjLaunch&, const AdjCoef<double>&, hipStream_t);
}  // namespace mp
