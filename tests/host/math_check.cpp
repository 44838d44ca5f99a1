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
    std::printf("log %.3f %ld\nsqrt %.3f %ld\nsinpi_abs %.3f %ld\ncospi_abs %.3f %ld\nrsqrt %.3f 2000000\n", mlog, n, msq,
                n, msin, n, mcos, n, mrsq);
    return 0;
}
