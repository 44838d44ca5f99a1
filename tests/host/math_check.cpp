// Host accuracy check of the device elementary functions in
// paper_2605_26016_amd/csrc/spx_math.hpp: the header is compiled for the CPU
// with the hardware estimates replaced by values carrying a relative error
// of 2^-23 (the precision stated for v_rsq_f64 / v_rcp_f64), and every result
// is compared with the x87 long-double libm value (64-bit significand).
// Prints "name max_ulp count" lines.
#include <cstdint>
#include <cstdio>
#include <cmath>
#include <random>

#define SPX_MATH_FN static inline
static inline double est_perturb(long double v, int k) {
    // alternate the sign of a 2^-23 relative error
    const long double e = ldexpl(1.0L, -23);
    return (double)(v * ((k & 1) ? 1.0L + e : 1.0L - e));
}
static int g_est_k = 0;
#define SPX_EST_RSQ(x) est_perturb(1.0L / sqrtl((long double)(x)), ++g_est_k)
#define SPX_EST_RCP(x) est_perturb(1.0L / (long double)(x), ++g_est_k)
#include "../../paper_2605_26016_amd/csrc/spx_math.hpp"
#include "../../paper_2605_26016_amd/csrc/spx_mc_math.hpp"

static double ulp_err(double got, long double ref) {
    if (ref == 0.0L) return got == 0.0 ? 0.0 : INFINITY;
    int e;
    frexpl(ref, &e);
    const long double ulp = ldexpl(1.0L, e - 53);
    return (double)(fabsl((long double)got - ref) / ulp);
}

int main() {
    const long double PI = 3.14159265358979323846264338327950288L;
    std::mt19937_64 rng(12345);
    // uniforms of the noise transform: u = (x + 1/2) 2^-32 over random and edge x
    double mlog = 0, msq = 0, mrsq = 0, msin = 0, mcos = 0;
    long n = 0;
    auto check_u = [&](uint32_t x) {
        const double u = ((double)x + 0.5) * 0x1p-32;
        const double l = spx::log_pos(u);
        mlog = fmax(mlog, ulp_err(l, logl((long double)u)));
        const double a = -2.0 * l;
        msq = fmax(msq, ulp_err(spx::sqrt_pos(a), sqrtl((long double)a)));
        double s, c;
        spx::sincospi_d(2.0 * u, s, c);
        const long double th = PI * (long double)(2.0 * u);
        // absolute error in units of 2^-53 (the results have magnitude <= 1
        // and enter the normals as r cos, r sin)
        const long double rs = sinl(th), rc = cosl(th);
        msin = fmax(msin, (double)(fabsl((long double)s - rs) / ldexpl(1.0L, -53)));
        mcos = fmax(mcos, (double)(fabsl((long double)c - rc) / ldexpl(1.0L, -53)));
        ++n;
    };
    for (uint32_t x = 0; x < 4096; ++x) check_u(x);
    for (uint32_t x = 0xFFFFFFFFu; x > 0xFFFFFFFFu - 4096; --x) check_u(x);
    const uint32_t edges[] = {0x40000000u, 0x3FFFFFFFu, 0x7FFFFFFFu, 0x80000000u, 0xB504F333u, 0xB504F334u,
                              0xC0000000u, 0x5A827999u, 0x5A82799Au};
    for (uint32_t x : edges)
        for (int d = -64; d <= 64; ++d) check_u(x + (uint32_t)d);
    for (int k = 0; k < 4000000; ++k) check_u((uint32_t)rng());
    // 1/sqrt of squared norms near 1 and of arbitrary positive values
    for (int k = 0; k < 2000000; ++k) {
        const double v = (k & 1) ? 1.0 + ldexp((double)(rng() >> 11), -53) * 0.05
                                 : ldexp(1.0 + ldexp((double)(rng() >> 11), -53), (int)(rng() % 200) - 100);
        mrsq = fmax(mrsq, ulp_err(spx::rsqrt_pos(v), 1.0L / sqrtl((long double)v)));
    }
    // a / b over random magnitudes
    double mdiv = 0;
    for (int k = 0; k < 1000000; ++k) {
        const double a = ldexp(1.0 + ldexp((double)(rng() >> 11), -53), (int)(rng() % 200) - 100) * ((k & 1) ? -1 : 1);
        const double b = ldexp(1.0 + ldexp((double)(rng() >> 11), -53), (int)(rng() % 200) - 100);
        mdiv = fmax(mdiv, ulp_err(spx::div_pos(a, b), (long double)a / (long double)b));
    }
    // angle between unit vectors from (|a x b|, a.b): random directions, pairs
    // close together (angles down to 1e-9), nearly opposite, and the octant
    // boundaries of the reduction
    std::normal_distribution<double> nd;
    double mang = 0;
    long nang = 0;
    auto check_angle = [&](double y, double x) {
        mang = fmax(mang, ulp_err(spx::atan2_nonneg(y, x), atan2l((long double)y, (long double)x)));
        ++nang;
    };
    for (int k = 0; k < 1000000; ++k) {
        double a[3] = {nd(rng), nd(rng), nd(rng)}, b[3];
        const double eps = (k % 4 == 0) ? 1.0 : ldexp(1.0, -(int)(rng() % 30));
        for (int c = 0; c < 3; ++c) b[c] = ((k % 4 == 3) ? -a[c] : a[c]) + eps * nd(rng);
        const double c0 = a[1] * b[2] - a[2] * b[1], c1 = a[2] * b[0] - a[0] * b[2], c2 = a[0] * b[1] - a[1] * b[0];
        check_angle(sqrt(c0 * c0 + c1 * c1 + c2 * c2), a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
    }
    const double tp8 = 0.41421356237309503;
    for (int d = -2000; d <= 2000; ++d) {
        const double r = tp8 + d * 1e-16, q = 1.0 + d * 1e-16;
        check_angle(r, 1.0); check_angle(1.0, r); check_angle(r, -1.0); check_angle(1.0, -r);
        check_angle(q, 1.0); check_angle(1.0, q); check_angle(q, -1.0);
    }
    check_angle(0.0, 1.0); check_angle(0.0, -1.0); check_angle(1.0, 0.0); check_angle(1.0, -0.0);
    // cos r and sin(r)/r from z = r^2: steps of the exponential map (0 to a few rad)
    // (series branch z <= 1: cos, and sin r / r relative; beyond: the
    // absolute errors of cos r and r (sin r / r) = sin r, the terms of the
    // retraction, in 2^-53 units)
    double mcs = 0, msc = 0, mcs_far = 0, msn_far = 0;
    for (int k = 0; k < 1000000; ++k) {
        const double r = (k & 1) ? ldexp((double)(rng() >> 11), -53) * 4.0 : ldexp((double)(rng() >> 11), -53 - (int)(rng() % 40));
        const double z = r * r;
        double cs, sc;
        spx::expmap_cs(z, cs, sc);
        const long double rl = sqrtl((long double)z);
        const double ecs = (double)(fabsl((long double)cs - cosl(rl)) / ldexpl(1.0L, -53));
        if (z <= 1.0) {
            mcs = fmax(mcs, ecs);
            msc = fmax(msc, ulp_err(sc, rl == 0.0L ? 1.0L : sinl(rl) / rl));
        } else {
            mcs_far = fmax(mcs_far, ecs);
            msn_far = fmax(msn_far, (double)(fabsl((long double)sc * rl - sinl(rl)) / ldexpl(1.0L, -53)));
        }
    }
    {
        double cs, sc;
        spx::expmap_cs(0.0, cs, sc);
        if (cs != 1.0 || sc != 1.0) mcs = INFINITY;
    }
    std::printf("log %.3f %ld\nsqrt %.3f %ld\nsinpi_abs %.3f %ld\ncospi_abs %.3f %ld\nrsqrt %.3f 2000000\n", mlog, n, msq,
                n, msin, n, mcos, n, mrsq);
    std::printf("div %.3f 1000000\natan2 %.3f %ld\nexpmap_cos_abs %.3f 1000000\nexpmap_sinc %.3f 1000000\n", mdiv, mang,
                nang, mcs, msc);
    std::printf("expmap_far_cos_abs %.3f 1000000\nexpmap_far_sin_abs %.3f 1000000\n", mcs_far, msn_far);
    // Monte Carlo moves: e^y - 1 and e^y for y <= 0 (random magnitudes from
    // 2^-60 to 50 / 745, both sides of every reduction boundary
    // (k + 1/2) ln 2 and the clamps), ln(1 + w) for -1 < w <= 0 (random
    // magnitudes from 2^-60 to 1 - 2^-33, and w near -1/2 where 1 + w
    // stops being exact)
    double mem1 = 0, mex = 0, ml1p = 0;
    long nem1 = 0, nex = 0, nl1p = 0;
    auto check_y = [&](double y) {
        mem1 = fmax(mem1, ulp_err(spx::expm1_nonpos(y), expm1l((long double)y)));
        ++nem1;
        if (y > -708.0) {  // normal results
            mex = fmax(mex, ulp_err(spx::exp_nonpos(y), expl((long double)y)));
            ++nex;
        }
    };
    for (int k = 0; k < 2000000; ++k) {
        const double m = 1.0 + ldexp((double)(rng() >> 11), -53);
        check_y(-ldexp(m, (int)(rng() % 66) - 60));
        check_y(-ldexp((double)(rng() >> 11), -53) * ((k & 1) ? 50.0 : 745.0));
    }
    const long double LN2 = 0.693147180559945309417232121458176568L;
    for (int k = 0; k <= 1070; ++k)
        for (int d = -8; d <= 8; ++d) {
            const double y = (double)(-(k + 0.5L) * LN2) + d * ldexp(1.0, -40) * (k + 1);
            if (y <= 0.0) check_y(y);
        }
    for (double y : {0.0, -0.0, -40.0, -39.999, -40.001, -745.0, -707.9, -1e-300, -0x1p-1074}) check_y(y);
    auto check_w = [&](double w) {
        ml1p = fmax(ml1p, ulp_err(spx::log1p_neg(w), log1pl((long double)w)));
        ++nl1p;
    };
    for (int k = 0; k < 2000000; ++k) {
        const double m = 1.0 + ldexp((double)(rng() >> 11), -53);
        const double w = -ldexp(m, -(int)(rng() % 61));
        if (w > -1.0 + 0x1p-33) check_w(w);
        check_w(-0.5 + ldexp((double)(rng() >> 11), -53) * 0x1p-10 - 0x1p-11);
    }
    for (double w : {0.0, -0x1p-60, -0.5, -0.5 + 0x1p-54, -0.5 - 0x1p-53, -1.0 + 0x1p-33, -0.75}) check_w(w);
    std::printf("expm1_nonpos %.3f %ld\nexp_nonpos %.3f %ld\nlog1p_neg %.3f %ld\n", mem1, nem1, mex, nex, ml1p,
                nl1p);
    return 0;
}
