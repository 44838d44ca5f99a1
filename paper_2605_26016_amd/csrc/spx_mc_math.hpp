// spx_mc_math.hpp -- FP64 functions of the Monte Carlo moves (heat-bath
// inverse distribution function and the Metropolis acceptance test), written
// for the arguments the moves produce rather than for the whole double range:
//   - expm1_nonpos(y), y <= 0: y = k ln 2 + r with k = rint(y / ln 2) and
//     |r| <= ln 2 / 2 (ln 2 split so that k ln2_hi is exact for |k| < 2^11),
//     e^r - 1 as its Taylor series up to r^13 (the next term is below 2^-56
//     of the result), and 2^k (e^r - 1) + (2^k - 1) in one fused
//     multiply-add.  Arguments below -40 are clamped there: e^y is then below
//     half an ulp of 1 and the result is -1 either way.  About one ulp.
//   - exp_nonpos(y), y <= 0: the same reduction, 2^k + 2^k (e^r - 1); below
//     -746 the result is 0.  About one ulp (fewer digits once 2^k is
//     subnormal).
//   - log1p_neg(w), -1 < w <= 0 with 1 + w a normal number: for
//     |w| < 2^-20 the series w - w^2/2 + w^3/3 - w^4/4 (the next term is
//     below 2^-80 of the result); else u = 1 + w rounded and
//     ln(1 + w) = ln u + ln(1 + d / u) with d = w - (u - 1) the rounding
//     error of u, ln u by log_pos and the second term as d / u to first
//     order (|d / u| is then below 2^-34 of the result, so the hardware
//     reciprocal estimate is precise enough).  About two ulp.
// Each function states its argument range; nothing here checks it.
//
// A host build (the accuracy tests) includes spx_math.hpp first with its
// host replacements of the hardware estimates.
#pragma once

#include "spx_math.hpp"

namespace spx {

// e^r - 1 for |r| <= ln 2 / 2 (plus rounding slack)
SPX_MATH_FN double expm1_reduced(double r) {
    double q = 1.0 / 6227020800.0;     // 1/13!
    q = std::fma(q, r, 1.0 / 479001600.0);
    q = std::fma(q, r, 1.0 / 39916800.0);
    q = std::fma(q, r, 1.0 / 3628800.0);
    q = std::fma(q, r, 1.0 / 362880.0);
    q = std::fma(q, r, 1.0 / 40320.0);
    q = std::fma(q, r, 1.0 / 5040.0);
    q = std::fma(q, r, 1.0 / 720.0);
    q = std::fma(q, r, 1.0 / 120.0);
    q = std::fma(q, r, 1.0 / 24.0);
    q = std::fma(q, r, 1.0 / 6.0);
    q = std::fma(q, r, 0.5);
    return std::fma(r, r * q, r);
}

// y = k ln 2 + r, |r| <= ln 2 / 2, for -1100 < y <= 0
SPX_MATH_FN double exp_reduce(double y, int &k) {
    constexpr double kInvLn2 = 0x1.71547652b82fep+0;
    constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;   // 42 bits: k ln2_hi exact for |k| < 2^11
    constexpr double kLn2Lo = 0x1.ef35793c76730p-45;  // ln 2 - ln2_hi
    const double kd = std::rint(y * kInvLn2);
    k = (int)kd;
    return std::fma(-kd, kLn2Lo, std::fma(-kd, kLn2Hi, y));
}

// e^y - 1, y <= 0
SPX_MATH_FN double expm1_nonpos(double y) {
    int k;
    const double r = exp_reduce(std::fmax(y, -40.0), k);
    const double s = std::ldexp(1.0, k);  // 2^k, k in [-58, 0]
    return std::fma(s, expm1_reduced(r), s - 1.0);
}

// e^y, y <= 0
SPX_MATH_FN double exp_nonpos(double y) {
    int k;
    const double r = exp_reduce(std::fmax(y, -746.0), k);
    const double s = std::ldexp(1.0, k);  // 2^k, 0 below the subnormal range
    return std::fma(s, expm1_reduced(r), s);
}

// ln(1 + w), -1 < w <= 0, 1 + w normal
SPX_MATH_FN double log1p_neg(double w) {
    const double u = 1.0 + w;
    const double d = w - (u - 1.0);
    const double big = std::fma(d, SPX_EST_RCP(u), log_pos(u));
    const double p = std::fma(w, std::fma(w, std::fma(w, -0.25, 1.0 / 3.0), -0.5), 1.0);
    return w > -0x1p-20 ? w * p : big;
}

}  // namespace spx
