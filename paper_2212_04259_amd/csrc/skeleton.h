// Result of a skeleton search as held by the library (bns_skeleton handles).
#pragma once

#include <stdint.h>

#include <mutex>
#include <vector>

#include "../../include/bns.h"

// A search fills the compact form (removal depth per pair as int8, the
// sepsets of depth >= 1 in removal-record order); the n x n arrays are
// expanded from it once, when an accessor first needs them (expand()).
// Handles built on the host fill the arrays directly (full = true).
struct bns_skeleton {
    int32_t n = 0;
    std::vector<int8_t> rdep;         // compact: n x n, removal depth or -1
    std::vector<int64_t> rec_pair;    // compact: i n + j (i < j) of each pool record
    std::vector<int64_t> rec_off;     // compact: its offset in pool
    std::vector<int32_t> pool;        // sepset members, ascending per pair
    std::vector<bns_depth_stats> stats;
    // expanded form
    mutable std::vector<uint8_t> adj;     // n x n, 1 = edge kept
    mutable std::vector<int32_t> depth;   // n x n, removal depth or -1
    mutable std::vector<int64_t> sepoff;  // n x n, offset of the pair's sepset in pool or -1
    mutable std::once_flag once;
    bool full = false;
    void expand() const {
        if (full) return;
        std::call_once(once, [this] {
            const int64_t nn = (int64_t)n * n;
            adj.resize((size_t)nn);
            depth.resize((size_t)nn);
            sepoff.assign((size_t)nn, -1);
            for (int64_t i = 0, e = 0; i < n; ++i)
                for (int64_t j = 0; j < n; ++j, ++e) {
                    const int8_t dd = rdep[(size_t)e];
                    depth[(size_t)e] = dd;
                    adj[(size_t)e] = (dd < 0 && i != j) ? 1 : 0;
                    if (dd == 0) sepoff[(size_t)e] = 0;  // empty set
                }
            for (size_t r = 0; r < rec_pair.size(); ++r) {
                const int64_t i = rec_pair[r] / n, j = rec_pair[r] % n;
                sepoff[(size_t)(i * n + j)] = rec_off[r];
                sepoff[(size_t)(j * n + i)] = rec_off[r];
            }
        });
    }
};
