// Division of node indices by an axis length without a hardware divide:
// for a divisor d >= 1 and every x < 2^31,
//   floor(x / d) = (x * m) >> k,  k = 31 + ceil(log2 d),  m = ceil(2^k / d),
// because m d - 2^k = e < d <= 2^(k-31), so x e < 2^31 d <= 2^k and the error
// term never reaches the next integer; m < 2^32 for every d.  The host
// computes (m, k) once per grid; a kernel pays one 32x32->64 multiply and one
// shift instead of a reciprocal-based division sequence.
#pragma once

#include <stdint.h>

namespace hj {

struct DivMagic {
    uint32_t m;
    uint32_t k;
};

inline DivMagic div_magic(uint32_t d)
{
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    const uint32_t k = 31 + l;
    const uint64_t p = uint64_t(1) << k;
    return DivMagic{uint32_t((p + d - 1) / d), k};
}

}  // namespace hj
