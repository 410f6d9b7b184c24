// FP64 division and reciprocal for the WENO weights: Newton-Raphson
// refinement of a reciprocal estimate (two steps, each squaring the relative
// error) and Markstein's final residual correction, which turns a quotient
// within an ulp and a reciprocal within half an ulp into the correctly
// rounded quotient.  This is the fused-multiply-add sequence of the general
// divide without its operand scaling and special-value fixup, so it equals
// the correctly rounded a/b where that sequence does not rescale: a nonzero
// numerator with denominator and quotient normal and their exponents well
// inside the range (or a zero numerator).  The WENO denominators are
// (S + eps)^2 >= 1e-198 and sums of such weights, the numerators 1 or
// weighted candidate sums, inside that range for any difference quotient of
// magnitude below 1e70.
//
// The estimate is a parameter so that the same sequence is checked on the
// host with estimates of a given relative error (the kernels pass the
// hardware reciprocal).
#pragma once

#if defined(__HIP__)
#define HJ_HOST_DEVICE __host__ __device__
#else
#define HJ_HOST_DEVICE
#endif

namespace hj {

template <typename Rcp>
HJ_HOST_DEVICE inline double div_rn_seq(double a, double b, Rcp rcp)
{
    const double nb = -b;
    const double r = rcp(b);
    const double y1 = __builtin_fma(r, __builtin_fma(nb, r, 1.0), r);
    const double y2 = __builtin_fma(y1, __builtin_fma(nb, y1, 1.0), y1);
    const double q = a * y2;
    return __builtin_fma(__builtin_fma(nb, q, a), y2, q);
}

template <typename Rcp>
HJ_HOST_DEVICE inline double rcp_rn_seq(double b, Rcp rcp)
{
    const double nb = -b;
    const double r = rcp(b);
    const double y1 = __builtin_fma(r, __builtin_fma(nb, r, 1.0), r);
    const double y2 = __builtin_fma(y1, __builtin_fma(nb, y1, 1.0), y1);
    return __builtin_fma(__builtin_fma(nb, y2, 1.0), y2, y2);
}

}  // namespace hj
