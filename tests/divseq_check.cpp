// Host check of the FP64 division sequence of the WENO weights (hj_divseq.h):
// with reciprocal estimates of relative error up to 2^-e, the quotient and
// reciprocal equal the correctly rounded a/b and 1/b (IEEE division of the
// host) over the operands the weights produce: denominators (S + eps)^2 from
// 1e-198 up, sums of three such reciprocals times 0.1, 0.6, 0.3, numerators
// 1, 0 and weighted candidate sums of either sign, and the edges of those
// ranges.  One family of denominators is a known exception and is counted
// apart: the largest double below a power of two, b = 2^k (1 - 2^-53), whose
// reciprocal lies within 2^-106 (relative) above a rounding tie; Newton
// iterates that land on the tie's lower neighbour make the final correction
// meet an exact tie, which rounds to even (one ulp low).  A WENO weight
// denominator is such a number with probability about 2^-52.
// Usage: divseq_check E COUNT (prints the mismatch counts).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <initializer_list>
#include <random>

#include "../paper_2507_11542_amd/csrc/hj_divseq.h"

static double seed_error;  // relative error of the current estimate
struct PerturbedRcp {
    double operator()(double b) const { return (1.0 / b) * (1.0 + seed_error); }
};

static long bad = 0, top = 0, n = 0;

static bool binade_top(double b)
{
    int e;
    const double m = std::frexp(std::fabs(b), &e);  // m in [0.5, 1)
    return m == std::nextafter(1.0, 0.0);
}

static void check(double a, double b, double err)
{
    seed_error = err;
    const double q = hj::div_rn_seq(a, b, PerturbedRcp());
    const double r = hj::rcp_rn_seq(b, PerturbedRcp());
    ++n;
    if (q != a / b || r != 1.0 / b) {
        if (binade_top(b)) {
            ++top;
            return;
        }
        if (bad < 10)
            std::printf("mismatch a=%.17g b=%.17g err=%g q=%.17g want %.17g r=%.17g want %.17g\n",
                        a, b, err, q, a / b, r, 1.0 / b);
        ++bad;
    }
}

int main(int argc, char **argv)
{
    const int e = argc > 1 ? std::atoi(argv[1]) : 23;
    const long count = argc > 2 ? std::atol(argv[2]) : 2000000;
    const double emax = std::ldexp(1.0, -e);
    std::mt19937_64 rng(20250711);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    auto seed = [&]() {
        const double x = u(rng);
        return x < 0.1 ? emax : (x < 0.2 ? -emax : (2.0 * u(rng) - 1.0) * emax);
    };
    for (long k = 0; k < count; ++k) {
        // (S + eps)^2 over its whole range, log-uniform: 1e-198 .. 1e200
        const double s = std::pow(10.0, -99.0 + 199.0 * u(rng));
        const double den = s * s * (1.0 + u(rng));
        check(1.0, den, seed());
        // the weight sum of three reciprocals and a blend numerator
        const double r1 = 1.0 / (std::pow(10.0, -99.0 + 198.0 * u(rng)));
        const double r2 = r1 * std::pow(10.0, -20.0 + 40.0 * u(rng));
        const double r3 = r1 * std::pow(10.0, -20.0 + 40.0 * u(rng));
        if (!std::isfinite(r2) || !std::isfinite(r3)) continue;
        const double a1 = 0.1 * r1, a2 = 0.6 * r2, a3 = 0.3 * r3;
        const double sum = a1 + a2 + a3;
        const double phi = std::pow(10.0, -60.0 + 130.0 * u(rng)) * (u(rng) < 0.5 ? -1.0 : 1.0);
        const double num = a1 * phi + a2 * phi * (1.0 + u(rng)) + a3 * phi * (2.0 * u(rng) - 1.0);
        if (std::isfinite(num) && std::isfinite(sum)) check(num, sum, seed());
        check(0.0, sum, seed());
    }
    // edges: the smallest denominators, powers of two, neighbours of 1
    const double edges[] = {1e-198, 2e-198, 0x1p-657, 1.0, std::nextafter(1.0, 2.0),
                            std::nextafter(1.0, 0.0), 0x1p600, 1e200, 3.0, 0.1};
    for (double b : edges)
        for (double a : {1.0, -1.0, 0.0, 1e-60, -3e50, 0.3, 7.0 / 3.0})
            for (double err : {0.0, emax, -emax, emax / 3.0}) check(a, b, err);
    // the exception family itself: the top double of binades over the range
    for (int k = -650; k <= 660; k += 13)
        for (double err : {emax, -emax}) check(1.0, std::ldexp(std::nextafter(1.0, 0.0), k), err);
    std::printf("%ld checks at seed error 2^-%d, %ld mismatches, %ld at binade tops\n", n, e,
                bad, top);
    return bad != 0;
}
