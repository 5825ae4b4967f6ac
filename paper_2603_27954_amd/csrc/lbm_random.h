// Counter-based generator of the seeded draws (tree jitter, inflow modes):
// SplitMix64 (Steele, Lea and Flood 2014); a draw in [0, 1) is the top 53
// bits of the output scaled by 2^-53.  Internal.
#pragma once
#include <stdint.h>

namespace lbm {

struct SplitMix64 {
    uint64_t s;
    uint64_t next()
    {
        s += 0x9E3779B97F4A7C15ULL;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    double uniform() { return double(next() >> 11) * 0x1.0p-53; }
};

}  // namespace lbm
