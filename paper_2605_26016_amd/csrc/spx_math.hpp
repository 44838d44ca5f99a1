// spx_math.hpp -- FP64 elementary functions of the thermal-noise transform
// (Box-Muller on Philox uniforms) and of the spin normalisation, written for
// the arguments they receive there rather than for the whole double range.
//
// The general-purpose device library evaluates log in double-double
// arithmetic and handles denormals, infinities and NaNs in every function;
// for a stochastic Heun step that is most of the per-spin arithmetic.  Here:
//   - log_pos: positive normal arguments (the uniforms lie in [2^-33, 1));
//     the mantissa is reduced to [sqrt(1/2), sqrt(2)) and ln m = 2 atanh(s),
//     s = (m - 1)/(m + 1), is summed as its Taylor series in s^2 <= 0.0295
//     (ten terms reach 2^-54); e ln 2 is added with ln 2 split so that
//     e ln2_hi is exact.  About one ulp.
//   - sincospi_d: sin(pi t), cos(pi t) for |t| < 2^30; t = r + n/2 with
//     |r| <= 1/4, and the Taylor series of sin(pi r) and cos(pi r) (up to
//     (pi r)^17 and (pi r)^18: the next terms are below 2^-63 of the result),
//     pi split in two doubles so that the leading term keeps full precision.
//     About one ulp.
//   - sqrt_pos, rsqrt_pos: positive normal arguments; the hardware estimate
//     (relative error near 2^-23) refined by Newton steps to about one ulp.
//   - div_pos: a / b for b positive normal, about half an ulp.
//   - atan2_nonneg: atan2(y, x) for y >= 0 (the angle between two vectors
//     from |a x b| and a.b): the ratio min/max of |x|, y in [0, 1], reduced
//     by pi/4 to |t| <= tan(pi/8), then twenty terms of the series of
//     atan t (the next term is below 2^-56 of the result); quadrants by
//     pi/2 - . and pi - . with pi split in two doubles.  About two ulp.
//   - expmap_cs: cos r and sin(r)/r from z = r^2 (the exponential map on the
//     sphere), as power series in z for z <= 1 (ten terms each, the next
//     below 2^-60), else through sqrt_pos and sincospi_d.  A few ulp.
// Each function states its argument range; nothing here checks it.
//
// A host build of this header (for the accuracy tests) may define SPX_MATH_FN,
// SPX_EST_RSQ and SPX_EST_RCP before including it.
#pragma once

#include <cmath>

#ifndef SPX_MATH_FN
#define SPX_MATH_FN __device__ __forceinline__
#endif
#ifndef SPX_EST_RSQ
#define SPX_EST_RSQ(x) __builtin_amdgcn_rsq(x)
#endif
#ifndef SPX_EST_RCP
#define SPX_EST_RCP(x) __builtin_amdgcn_rcp(x)
#endif

namespace spx {

// 1/sqrt(x), x positive normal: y <- y + y (1 - x y^2)/2, twice.
SPX_MATH_FN double rsqrt_pos(double x) {
    double y = SPX_EST_RSQ(x);
    double e = std::fma(-x * y, y, 1.0);
    y = std::fma(0.5 * y, e, y);
    e = std::fma(-x * y, y, 1.0);
    return std::fma(0.5 * y, e, y);
}

// sqrt(a), a positive normal: coupled iteration on g ~ sqrt(a) and
// h ~ 1/(2 sqrt(a)), then one residual correction g + (a - g^2) h.
SPX_MATH_FN double sqrt_pos(double a) {
    const double y = SPX_EST_RSQ(a);
    double g = a * y, h = 0.5 * y;
    const double r = std::fma(-g, h, 0.5);
    g = std::fma(g, r, g);
    h = std::fma(h, r, h);
    const double d = std::fma(-g, g, a);
    return std::fma(d, h, g);
}

// ln(u), u positive normal.
SPX_MATH_FN double log_pos(double u) {
    constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;   // ln 2 to 43 bits: e ln2_hi exact for |e| < 2^10
    constexpr double kLn2Lo = 0x1.ef35793c76730p-45;  // ln 2 - ln2_hi
    constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
    int e;
    double m = std::frexp(u, &e);  // u = m 2^e, m in [1/2, 1)
    if (m < kSqrtHalf) {
        m += m;
        --e;
    }
    const double f = m - 1.0;  // exact
    // s = f / (2 + f) to half an ulp; d + dl = 2 + f exactly
    const double d = 2.0 + f;
    const double dl = (2.0 - d) + f;
    double r = SPX_EST_RCP(d);
    r = std::fma(std::fma(-d, r, 1.0), r, r);
    r = std::fma(std::fma(-d, r, 1.0), r, r);
    double s = f * r;
    s = std::fma(std::fma(-s, d, f) - s * dl, r, s);
    // ln m = 2 s + 2 s z (1/3 + z/5 + ... + z^9/21), z = s^2
    const double z = s * s;
    double p = 1.0 / 21.0;
    p = std::fma(p, z, 1.0 / 19.0);
    p = std::fma(p, z, 1.0 / 17.0);
    p = std::fma(p, z, 1.0 / 15.0);
    p = std::fma(p, z, 1.0 / 13.0);
    p = std::fma(p, z, 1.0 / 11.0);
    p = std::fma(p, z, 1.0 / 9.0);
    p = std::fma(p, z, 1.0 / 7.0);
    p = std::fma(p, z, 1.0 / 5.0);
    p = std::fma(p, z, 1.0 / 3.0);
    const double s2 = s + s;
    const double lnm = std::fma(s2 * z, p, s2);
    const double de = (double)e;
    return std::fma(de, kLn2Hi, std::fma(de, kLn2Lo, lnm));
}

// a / b, b positive normal: reciprocal refined by two Newton steps, then
// one residual correction of the quotient.
SPX_MATH_FN double div_pos(double a, double b) {
    double r = SPX_EST_RCP(b);
    r = std::fma(std::fma(-b, r, 1.0), r, r);
    r = std::fma(std::fma(-b, r, 1.0), r, r);
    const double q = a * r;
    return std::fma(std::fma(-q, b, a), r, q);
}

// sin(pi t) and cos(pi t), |t| < 2^30.
SPX_MATH_FN void sincospi_d(double t, double &sn, double &cs) {
    // Taylor coefficients (-1)^k pi^(2k+1)/(2k+1)! and (-1)^k pi^(2k)/(2k)!
    constexpr double kPiHi = 0x1.921fb54442d18p+1, kPiLo = 0x1.1a62633145c07p-53;
    constexpr double S1 = -0x1.4abbce625be53p+2, S2 = 0x1.466bc6775aae2p+1, S3 = -0x1.32d2cce62bd86p-1,
                     S4 = 0x1.50783487ee782p-4, S5 = -0x1.e3074fde8871fp-8, S6 = 0x1.e8f434d018d63p-12,
                     S7 = -0x1.6fadb9f155744p-16, S8 = 0x1.aaec32af93359p-21;
    constexpr double C1 = -0x1.3bd3cc9be45dep+2, C2 = 0x1.03c1f081b5ac4p+2, C3 = -0x1.55d3c7e3cbffap+0,
                     C4 = 0x1.e1f506891babbp-3, C5 = -0x1.a6d1f2a204a8cp-6, C6 = 0x1.f9d38a3763cc3p-10,
                     C7 = -0x1.b6e24f44b128fp-14, C8 = 0x1.20c62c2f2d7f5p-18, C9 = -0x1.2a0c591af8314p-23;
    const double n = std::rint(t + t);   // t = r + n/2
    const double r = std::fma(-0.5, n, t);  // exact, |r| <= 1/4
    const double z = r * r;
    double ps = S8;
    ps = std::fma(ps, z, S7);
    ps = std::fma(ps, z, S6);
    ps = std::fma(ps, z, S5);
    ps = std::fma(ps, z, S4);
    ps = std::fma(ps, z, S3);
    ps = std::fma(ps, z, S2);
    ps = std::fma(ps, z, S1);
    const double sr = std::fma(r, kPiHi, r * std::fma(z, ps, kPiLo));
    double pc = C9;
    pc = std::fma(pc, z, C8);
    pc = std::fma(pc, z, C7);
    pc = std::fma(pc, z, C6);
    pc = std::fma(pc, z, C5);
    pc = std::fma(pc, z, C4);
    pc = std::fma(pc, z, C3);
    pc = std::fma(pc, z, C2);
    pc = std::fma(pc, z, C1);
    const double cr = std::fma(z, pc, 1.0);
    // pi t = pi r + q pi/2, q = n mod 4
    const int q = (int)n & 3;
    const double a = (q & 1) ? cr : sr;
    const double b = (q & 1) ? sr : cr;
    sn = (q & 2) ? -a : a;
    cs = ((q + 1) & 2) ? -b : b;
}


// atan2(y, x) for y >= 0 and (x, y) != (0, 0); result in [0, pi].
SPX_MATH_FN double atan2_nonneg(double y, double x) {
    constexpr double kPi4Hi = 0x1.921fb54442d18p-1, kPi4Lo = 0x1.1a62633145c07p-55;
    constexpr double kTanPi8 = 0x1.a827999fcef32p-2;  // sqrt 2 - 1
    const double ax = std::fabs(x);
    const double mx = std::fmax(ax, y), mn = std::fmin(ax, y);
    // r = mn / mx in [0, 1]; above tan(pi/8), atan r = pi/4 + atan((r - 1)/(r + 1))
    const bool big = mn > kTanPi8 * mx;
    const double t = big ? div_pos(mn - mx, mn + mx) : div_pos(mn, mx);
    const double z = t * t;
    // atan t = t + t z sum_{k>=1} (-1)^k z^(k-1) / (2k + 1), k up to 19
    double p = -1.0 / 39.0;
    p = std::fma(p, z, 1.0 / 37.0);
    p = std::fma(p, z, -1.0 / 35.0);
    p = std::fma(p, z, 1.0 / 33.0);
    p = std::fma(p, z, -1.0 / 31.0);
    p = std::fma(p, z, 1.0 / 29.0);
    p = std::fma(p, z, -1.0 / 27.0);
    p = std::fma(p, z, 1.0 / 25.0);
    p = std::fma(p, z, -1.0 / 23.0);
    p = std::fma(p, z, 1.0 / 21.0);
    p = std::fma(p, z, -1.0 / 19.0);
    p = std::fma(p, z, 1.0 / 17.0);
    p = std::fma(p, z, -1.0 / 15.0);
    p = std::fma(p, z, 1.0 / 13.0);
    p = std::fma(p, z, -1.0 / 11.0);
    p = std::fma(p, z, 1.0 / 9.0);
    p = std::fma(p, z, -1.0 / 7.0);
    p = std::fma(p, z, 1.0 / 5.0);
    p = std::fma(p, z, -1.0 / 3.0);
    const double at = std::fma(t * z, p, t);
    // angle of (mx, mn) in [0, pi/4]
    double th = big ? kPi4Hi + (at + kPi4Lo) : at;
    // the ratio was |x| / y: pi/2 - th
    if (y > ax) th = (2.0 * kPi4Hi - th) + 2.0 * kPi4Lo;
    // second quadrant: pi - th
    if (x < 0.0) th = (4.0 * kPi4Hi - th) + 4.0 * kPi4Lo;
    return th;
}

// cos r and sin(r) / r from z = r^2 >= 0.
SPX_MATH_FN void expmap_cs(double z, double &cs, double &sc) {
    if (z <= 1.0) {
        // cos r = sum_k (-1)^k z^k / (2k)!, sin(r)/r = sum_k (-1)^k z^k / (2k+1)!, k <= 9
        double c = 1.0 / 6402373705728000.0;  // 1/18!
        c = std::fma(c, z, -1.0 / 20922789888000.0);
        c = std::fma(c, z, 1.0 / 87178291200.0);
        c = std::fma(c, z, -1.0 / 479001600.0);
        c = std::fma(c, z, 1.0 / 3628800.0);
        c = std::fma(c, z, -1.0 / 40320.0);
        c = std::fma(c, z, 1.0 / 720.0);
        c = std::fma(c, z, -1.0 / 24.0);
        c = std::fma(c, z, 0.5);
        cs = std::fma(-c, z, 1.0);
        double q = 1.0 / 121645100408832000.0;  // 1/19!
        q = std::fma(q, z, -1.0 / 355687428096000.0);
        q = std::fma(q, z, 1.0 / 1307674368000.0);
        q = std::fma(q, z, -1.0 / 6227020800.0);
        q = std::fma(q, z, 1.0 / 39916800.0);
        q = std::fma(q, z, -1.0 / 362880.0);
        q = std::fma(q, z, 1.0 / 5040.0);
        q = std::fma(q, z, -1.0 / 120.0);
        q = std::fma(q, z, 1.0 / 6.0);
        sc = std::fma(-q, z, 1.0);
    } else {
        constexpr double kInvPi = 0x1.45f306dc9c883p-2;
        const double r = sqrt_pos(z);
        double sn;
        sincospi_d(r * kInvPi, sn, cs);
        sc = div_pos(sn, r);
    }
}

}  // namespace spx
