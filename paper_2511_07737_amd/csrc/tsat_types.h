// tsat_types.h -- plain data shared by the host store builder and the
// kernels (no HIP types).
#pragma once
#include <stdint.h>

namespace tsat {

// Static per-instance sizes.
struct InstInfo {
    int64_t C;       // clauses, empty ones included
    int64_t n_empty; // empty clauses (R = 0 for every candidate)
};

} // namespace tsat
