// Instances of the anti-trapping correction kernel (antitrap2d.hpp).
#include "antitrap2d.hpp"

namespace mp {
template int at_launch<float>(const AtLaunch&, const AtCoef<float>&, hipStream_t);
template int at_launch<double>(const AtLaunch&, const AtCoef<double>&, hipStream_t);
}  // namespace mp
