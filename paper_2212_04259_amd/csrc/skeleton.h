// Result of a skeleton search as held by the library (bns_skeleton handles).
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/bns.h"

struct bns_skeleton {
    int32_t n = 0;
    std::vector<uint8_t> adj;         // n x n, 1 = edge kept
    std::vector<int32_t> depth;       // n x n, removal depth or -1
    std::vector<int64_t> sepoff;      // n x n, offset of the pair's sepset in pool or -1
    std::vector<int32_t> pool;        // sepset members, ascending per pair
    std::vector<bns_depth_stats> stats;
};
