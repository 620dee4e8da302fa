// Process-wide round-schedule tunables (set by the autotuner through the C ABI).
#pragma once

#include "gkr_internal.hpp"

namespace gkr {

Tuning current_tuning();
void store_tuning(const Tuning& t);

}  // namespace gkr
