// Check of the node-index division magic at the values where a wrong magic
// shows first: every divisor 1..3000 against every x < 3d, and divisors up to
// 2^21 (every one up to 3000, then every 37th) against multiples of d and
// their neighbours up to 2^31, the largest x below 2^31 and a stride through
// [0, 2^31).
#include <cstdio>
#include <cstdint>

#include "../paper_2507_11542_amd/csrc/hj_divmagic.h"

static int check(uint32_t d, uint32_t x)
{
    const hj::DivMagic mg = hj::div_magic(d);
    const uint32_t q = uint32_t((uint64_t(x) * mg.m) >> mg.k);
    if (q != x / d) {
        std::printf("mismatch d=%u x=%u q=%u want=%u\n", d, x, q, x / d);
        return 1;
    }
    return 0;
}

int main()
{
    const uint32_t top = 0x7fffffffu;
    long bad = 0, n = 0;
    for (uint32_t d = 1; d <= (1u << 21); d += (d < 3000 ? 1 : 37)) {
        if (d <= 3000)
            for (uint32_t x = 0; x < 3 * d; ++x, ++n) bad += check(d, x);
        for (uint64_t q = 1; q * d <= top; q = q * 3 + 1) {
            const uint32_t x = uint32_t(q * d);
            bad += check(d, x) + check(d, x - 1);
            if (x < top) bad += check(d, x + 1);
            n += 3;
        }
        bad += check(d, top);
        for (uint32_t x = d; x < top - 104729u * 7919u; x += 104729u * 7919u, ++n) bad += check(d, x);
    }
    std::printf("%ld checks, %ld mismatches\n", n, bad);
    return bad != 0;
}
