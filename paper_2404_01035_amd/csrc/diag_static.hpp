// The allocation-free diagnostics (mp_diagnostics_static): its scratch lives
// in a static device array of diag.hip instead of a caller workspace.
#pragma once

#include "mp_internal.hpp"

namespace mp {

// Instances mp_diagnostics_static reduces at most (one result record each in
// its static device scratch, after DIAG_BLOCKS_MAX partial records).
constexpr int DIAG_STATIC_INST = 256;

// Address of that scratch on the current device (looked up once per device).
hipError_t diag_static_scratch(double** out);

}  // namespace mp
