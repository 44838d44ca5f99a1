// spx_device.hpp -- device-side building blocks of libspx.so: neighbour
// addressing on the sublattice grid, the bilinear stencil sum, on-site terms,
// the LLG right-hand side and the Philox4x32-10 thermal noise.
#pragma once

#include "spx_internal.hpp"
#include "spx_math.hpp"

namespace spx {

// Wrap or reject a cell coordinate.  Periodic axes wrap (a true modulo only
// when some offset exceeds the extent), open axes drop the neighbour
// (truncation rule for finite supercells).
__device__ __forceinline__ int wrap_coord(int c, int L, int per, int general, bool &ok) {
    if (c >= 0 && c < L) return c;
    if (!per) { ok = false; return 0; }
    if (!general) return c < 0 ? c + L : c - L;
    c %= L;
    return c < 0 ? c + L : c;
}

// Site coordinates of local index t within one sublattice.
__device__ __forceinline__ void site_xyz(const Grid &g, int t, int &x, int &y, int &z) {
    const int plane = g.Lx * g.Ly;
    z = t / plane;
    int r = t - z * plane;
    y = r / g.Lx;
    x = r - y * g.Lx;
}

// Bilinear reduced field of sublattice a at cell (x,y,z) for NIN spin states
// at once (the Heun corrector needs S^n and S~):
//   acc[k][alpha] = sum_{bonds p of a} sum_beta J_p^{alpha beta} S_k^beta(R + delta_p)
// In FP32 mode each neighbour spin is rounded to float before the product.
template <typename AccT, bool ISO, int NIN>
__device__ __forceinline__ void bil_sum(const BondTable &tb, const Grid &g, int a, int x, int y, int z,
                                        const double *const (&S)[NIN], AccT (&acc)[NIN][3]) {
#pragma unroll
    for (int k = 0; k < NIN; ++k) acc[k][0] = acc[k][1] = acc[k][2] = AccT(0);
    const int64_t N = g.N;
    const int p0 = tb.start[a], p1 = tb.start[a + 1];
    for (int p = p0; p < p1; ++p) {
        const int4 q = tb.geo[p];
        bool ok = true;
        const int xx = wrap_coord(x + q.y, g.Lx, g.per[0], g.wrap_general, ok);
        const int yy = wrap_coord(y + q.z, g.Ly, g.per[1], g.wrap_general, ok);
        const int zz = wrap_coord(z + q.w, g.Lz, g.per[2], g.wrap_general, ok);
        if (!ok) continue;
        const int64_t j = (int64_t)q.x * g.M + xx + g.Lx * (yy + g.Ly * zz);
        if constexpr (ISO) {
            AccT J;
            if constexpr (sizeof(AccT) == 4) J = tb.Jf[p]; else J = tb.Jd[p];
#pragma unroll
            for (int k = 0; k < NIN; ++k) {
                acc[k][0] += J * (AccT)S[k][j];
                acc[k][1] += J * (AccT)S[k][N + j];
                acc[k][2] += J * (AccT)S[k][2 * N + j];
            }
        } else {
            AccT J[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                if constexpr (sizeof(AccT) == 4) J[e] = tb.Jf[9 * p + e]; else J[e] = tb.Jd[9 * p + e];
            }
#pragma unroll
            for (int k = 0; k < NIN; ++k) {
                const AccT s0 = (AccT)S[k][j], s1 = (AccT)S[k][N + j], s2 = (AccT)S[k][2 * N + j];
                acc[k][0] += J[0] * s0 + J[1] * s1 + J[2] * s2;
                acc[k][1] += J[3] * s0 + J[4] * s1 + J[5] * s2;
                acc[k][2] += J[6] * s0 + J[7] * s1 + J[8] * s2;
            }
        }
    }
}

// Anisotropy field 2 K (S.n) n summed over the axes of sublattice a (FP64).
__device__ __forceinline__ void aniso_field(const Onsite &os, int a, const double s[3], double b[3]) {
    b[0] = b[1] = b[2] = 0.0;
    for (int l = 0; l < os.n_aniso; ++l) {
        const double *n = os.axis[a][l];
        const double c = 2.0 * os.K[a][l] * (s[0] * n[0] + s[1] * n[1] + s[2] * n[2]);
        b[0] += c * n[0];
        b[1] += c * n[1];
        b[2] += c * n[2];
    }
}

// LLG right-hand side f = pre [S x B + alpha S x (S x B)], pre = -gamma/(1+alpha^2).
__device__ __forceinline__ void llg_rhs(const double s[3], const double B[3], double pre, double alpha,
                                        double f[3]) {
    const double c0 = s[1] * B[2] - s[2] * B[1];
    const double c1 = s[2] * B[0] - s[0] * B[2];
    const double c2 = s[0] * B[1] - s[1] * B[0];
    const double d0 = s[1] * c2 - s[2] * c1;
    const double d1 = s[2] * c0 - s[0] * c2;
    const double d2 = s[0] * c1 - s[1] * c0;
    f[0] = pre * (c0 + alpha * d0);
    f[1] = pre * (c1 + alpha * d1);
    f[2] = pre * (c2 + alpha * d2);
}

// The direction of the LLG right-hand side, S x B + alpha S x (S x B), so
// that f = pre * llg_dir (pre folded into the step constants by callers that
// only need dt f).
__device__ __forceinline__ void llg_dir(const double s[3], const double B[3], double alpha, double g[3]) {
    const double c0 = s[1] * B[2] - s[2] * B[1];
    const double c1 = s[2] * B[0] - s[0] * B[2];
    const double c2 = s[0] * B[1] - s[1] * B[0];
    const double d0 = s[1] * c2 - s[2] * c1;
    const double d1 = s[2] * c0 - s[0] * c2;
    const double d2 = s[0] * c1 - s[1] * c0;
    g[0] = c0 + alpha * d0;
    g[1] = c1 + alpha * d1;
    g[2] = c2 + alpha * d2;
}

// N[v] = v/|v| with one reciprocal square root (about one ulp; the norm of a
// spin update is close to 1).
__device__ __forceinline__ void normalise3(double v[3]) {
    const double inv = rsqrt_pos(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] *= inv;
    v[1] *= inv;
    v[2] *= inv;
}

// Three-input exclusive or in one instruction (gfx950 v_bitop3_b32 with the
// truth table of a ^ b ^ c).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products on counter words 0 and 2; the high halves are
// mixed with the other words and the round key, the key advances by the two
// Weyl increments after every round.
__device__ __forceinline__ void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Three standard normals for site i at step n: one Philox block with
// counter (i lo, i hi ^ tag, n lo, n hi) and key (seed lo, seed hi), uniforms
// (x + 1/2) 2^-32, Box-Muller on (u0,u1) -> (eta_x, eta_y), (u2,u3) -> eta_z.
// The angle 2 pi u is evaluated as sin/cos(pi t) of t = 2u: 2u is exact, so no
// argument reduction by pi is needed.  The uniforms lie in [2^-33, 1 - 2^-33],
// so -2 ln u is a positive normal number and the functions of spx_math.hpp
// (about one ulp each) apply; the normals agree with a libm evaluation to a
// few ulp.
__device__ __forceinline__ void thermal_eta(uint64_t seed, uint64_t step, uint32_t tag, uint64_t site,
                                            double eta[3]) {
    uint32_t c0 = (uint32_t)site, c1 = (uint32_t)(site >> 32) ^ tag;
    uint32_t c2 = (uint32_t)step, c3 = (uint32_t)(step >> 32);
    philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    // (x + 1/2) 2^-32, exact (the sum has at most 33 significant bits)
    const double u0 = ldexp((double)c0 + 0.5, -32), u1 = ldexp((double)c1 + 0.5, -32);
    const double u2 = ldexp((double)c2 + 0.5, -32), u3 = ldexp((double)c3 + 0.5, -32);
    const double r0 = sqrt_pos(-2.0 * log_pos(u0));
    const double r1 = sqrt_pos(-2.0 * log_pos(u2));
    double sn, cs, sn3, cs3;
    sincospi_d(u1 + u1, sn, cs);
    sincospi_d(u3 + u3, sn3, cs3);
    eta[0] = r0 * cs;
    eta[1] = r0 * sn;
    eta[2] = r1 * cs3;
}

// Wavefront (64 lanes) sum of a double, result valid in lane 0.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

}  // namespace spx
