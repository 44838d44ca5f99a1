// spx_kernels.hip -- sparse sublattice stencil field, fused normalised-Heun
// predictor/corrector with Philox thermal noise, and the deterministic energy
// reduction, for gfx950.
//
// Launch shape: blockIdx.y is the target sublattice a (so the bond loop and
// its table loads are uniform over a block and go through the scalar unit),
// blockIdx.x * 256 + threadIdx.x is the site inside that sublattice, x fastest
// (coalesced SoA loads of the three spin planes).
#include <algorithm>

#include "spx_device.hpp"

namespace spx {

constexpr int kBlock = 256;

static dim3 site_grid(const Grid &g) {
    return dim3((unsigned)((g.M + kBlock - 1) / kBlock), (unsigned)g.n_sub, 1);
}

// ---------------------------------------------------------------- field
template <typename AccT, bool ISO, typename OutT>
__global__ __launch_bounds__(kBlock) void k_field(BondTable tb, Grid g, Onsite os,
                                                  const double *__restrict__ S,
                                                  const float *__restrict__ bdip,
                                                  OutT *__restrict__ b) {
    const int a = blockIdx.y;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= g.M) return;
    int x, y, z;
    site_xyz(g, t, x, y, z);
    const int64_t N = g.N;
    const int64_t i = (int64_t)a * g.M + t;
    AccT acc[1][3];
    const double *const src[1] = {S};
    bil_sum<AccT, ISO, 1>(tb, g, a, x, y, z, src, acc);
    const double s[3] = {S[i], S[N + i], S[2 * N + i]};
    double ba[3];
    aniso_field(os, a, s, ba);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double v = (double)acc[0][c] + ba[c] + os.bz[a][c];
        if (bdip) v += (double)bdip[c * N + i];
        b[c * N + i] = (OutT)v;
    }
}

hipError_t launch_field(int field_prec, const BondTable &tb, const Grid &g, const Onsite &os,
                        const double *S, const float *bdip, void *b, hipStream_t st) {
    const dim3 grid = site_grid(g);
    if (field_prec == 0) {
        if (tb.iso)
            k_field<double, true, double><<<grid, kBlock, 0, st>>>(tb, g, os, S, bdip, (double *)b);
        else
            k_field<double, false, double><<<grid, kBlock, 0, st>>>(tb, g, os, S, bdip, (double *)b);
    } else {
        if (tb.iso)
            k_field<float, true, float><<<grid, kBlock, 0, st>>>(tb, g, os, S, bdip, (float *)b);
        else
            k_field<float, false, float><<<grid, kBlock, 0, st>>>(tb, g, os, S, bdip, (float *)b);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- Heun
// Predictor: S~ = N[S + dt f(S, B(S) + sigma eta)].
template <typename AccT, bool ISO>
__global__ __launch_bounds__(kBlock) void k_heun_predict(BondTable tb, Grid g, Onsite os, HeunConst hc,
                                                         uint64_t step, const double *__restrict__ S,
                                                         const float *__restrict__ bdip,
                                                         double *__restrict__ St) {
    const int a = blockIdx.y;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= g.M) return;
    int x, y, z;
    site_xyz(g, t, x, y, z);
    const int64_t N = g.N;
    const int64_t i = (int64_t)a * g.M + t;
    AccT acc[1][3];
    const double *const src[1] = {S};
    bil_sum<AccT, ISO, 1>(tb, g, a, x, y, z, src, acc);
    const double s[3] = {S[i], S[N + i], S[2 * N + i]};
    double ba[3];
    aniso_field(os, a, s, ba);
    double B[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double v = (double)acc[0][c] + ba[c] + os.bz[a][c];
        if (bdip) v += (double)bdip[c * N + i];
        B[c] = v * hc.inv_mumuB[a];
    }
    if (hc.noise) {
        double eta[3];
        thermal_eta(hc.seed, noise_step(hc, step), hc.tag, (uint64_t)i, eta);
        const double sg = hc.sigma[a];
        B[0] += sg * eta[0];
        B[1] += sg * eta[1];
        B[2] += sg * eta[2];
    }
    double f[3];
    llg_rhs(s, B, hc.pre, hc.alpha, f);
    double p[3] = {s[0] + hc.dt * f[0], s[1] + hc.dt * f[1], s[2] + hc.dt * f[2]};
    normalise3(p);
    St[i] = p[0];
    St[N + i] = p[1];
    St[2 * N + i] = p[2];
}

// Corrector: S' = N[S + dt/2 (f(S) + f(S~))], f(S) recomputed from S (no
// stored field), the same eta as the predictor.
template <typename AccT, bool ISO>
__global__ __launch_bounds__(kBlock) void k_heun_correct(BondTable tb, Grid g, Onsite os, HeunConst hc,
                                                         uint64_t step, const double *__restrict__ S,
                                                         const double *__restrict__ St,
                                                         const float *__restrict__ bdipS,
                                                         const float *__restrict__ bdipT,
                                                         double *__restrict__ out) {
    const int a = blockIdx.y;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= g.M) return;
    int x, y, z;
    site_xyz(g, t, x, y, z);
    const int64_t N = g.N;
    const int64_t i = (int64_t)a * g.M + t;
    AccT acc[2][3];
    const double *const src[2] = {S, St};
    bil_sum<AccT, ISO, 2>(tb, g, a, x, y, z, src, acc);
    const double s[3] = {S[i], S[N + i], S[2 * N + i]};
    const double st[3] = {St[i], St[N + i], St[2 * N + i]};
    double ba[3], bt[3];
    aniso_field(os, a, s, ba);
    aniso_field(os, a, st, bt);
    double B0[3], B1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double v0 = (double)acc[0][c] + ba[c] + os.bz[a][c];
        double v1 = (double)acc[1][c] + bt[c] + os.bz[a][c];
        if (bdipS) v0 += (double)bdipS[c * N + i];
        if (bdipT) v1 += (double)bdipT[c * N + i];
        B0[c] = v0 * hc.inv_mumuB[a];
        B1[c] = v1 * hc.inv_mumuB[a];
    }
    if (hc.noise) {
        double eta[3];
        thermal_eta(hc.seed, noise_step(hc, step), hc.tag, (uint64_t)i, eta);
        const double sg = hc.sigma[a];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            B0[c] += sg * eta[c];
            B1[c] += sg * eta[c];
        }
    }
    double f0[3], f1[3];
    llg_rhs(s, B0, hc.pre, hc.alpha, f0);
    llg_rhs(st, B1, hc.pre, hc.alpha, f1);
    const double h = 0.5 * hc.dt;
    double p[3] = {s[0] + h * (f0[0] + f1[0]), s[1] + h * (f0[1] + f1[1]), s[2] + h * (f0[2] + f1[2])};
    normalise3(p);
    out[i] = p[0];
    out[N + i] = p[1];
    out[2 * N + i] = p[2];
}

hipError_t launch_heun_predict(int field_prec, const BondTable &tb, const Grid &g, const Onsite &os,
                               const HeunConst &hc, uint64_t step, const double *S,
                               const float *bdip, double *St, hipStream_t st) {
    const dim3 grid = site_grid(g);
    if (field_prec == 0) {
        if (tb.iso) k_heun_predict<double, true><<<grid, kBlock, 0, st>>>(tb, g, os, hc, step, S, bdip, St);
        else k_heun_predict<double, false><<<grid, kBlock, 0, st>>>(tb, g, os, hc, step, S, bdip, St);
    } else {
        if (tb.iso) k_heun_predict<float, true><<<grid, kBlock, 0, st>>>(tb, g, os, hc, step, S, bdip, St);
        else k_heun_predict<float, false><<<grid, kBlock, 0, st>>>(tb, g, os, hc, step, S, bdip, St);
    }
    return hipGetLastError();
}

hipError_t launch_heun_correct(int field_prec, const BondTable &tb, const Grid &g, const Onsite &os,
                               const HeunConst &hc, uint64_t step, const double *S, const double *St,
                               const float *bdip_S, const float *bdip_St, double *out, hipStream_t st) {
    const dim3 grid = site_grid(g);
    if (field_prec == 0) {
        if (tb.iso)
            k_heun_correct<double, true><<<grid, kBlock, 0, st>>>(tb, g, os, hc, step, S, St, bdip_S, bdip_St, out);
        else
            k_heun_correct<double, false><<<grid, kBlock, 0, st>>>(tb, g, os, hc, step, S, St, bdip_S, bdip_St, out);
    } else {
        if (tb.iso)
            k_heun_correct<float, true><<<grid, kBlock, 0, st>>>(tb, g, os, hc, step, S, St, bdip_S, bdip_St, out);
        else
            k_heun_correct<float, false><<<grid, kBlock, 0, st>>>(tb, g, os, hc, step, S, St, bdip_S, bdip_St, out);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- energy
// Per-site terms -S.b_bil/2, -S.b_Z, -S.b_ani/2, -S.b_dip/2, summed per block
// in a fixed tree; partial[block][4].
template <typename AccT, bool ISO>
__global__ __launch_bounds__(kBlock) void k_energy_partial(BondTable tb, Grid g, Onsite os,
                                                           const double *__restrict__ S,
                                                           const float *__restrict__ bdip,
                                                           const AccT *__restrict__ bil,
                                                           double *__restrict__ partial) {
    // bil != NULL: the bilinear field comes precomputed (stencil-engine pass)
    __shared__ double red[kBlock / 64][4];
    const int a = blockIdx.y;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    double e[4] = {0.0, 0.0, 0.0, 0.0};
    if (t < g.M) {
        int x, y, z;
        site_xyz(g, t, x, y, z);
        const int64_t N = g.N;
        const int64_t i = (int64_t)a * g.M + t;
        AccT acc[1][3];
        if (bil) {
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[0][c] = bil[c * N + i];
        } else {
            const double *const src[1] = {S};
            bil_sum<AccT, ISO, 1>(tb, g, a, x, y, z, src, acc);
        }
        const double s[3] = {S[i], S[N + i], S[2 * N + i]};
        double ba[3];
        aniso_field(os, a, s, ba);
        double sb = 0.0, sz = 0.0, sa = 0.0, sd = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sb += s[c] * (double)acc[0][c];
            sz += s[c] * os.bz[a][c];
            sa += s[c] * ba[c];
            if (bdip) sd += s[c] * (double)bdip[c * N + i];
        }
        e[0] = -0.5 * sb;
        e[1] = -sz;
        e[2] = -0.5 * sa;
        e[3] = -0.5 * sd;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double v = wave_sum(e[k]);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) v += red[w][threadIdx.x];
        partial[(size_t)(blockIdx.y * gridDim.x + blockIdx.x) * 4 + threadIdx.x] = v;
    }
}

// Middle level of the fixed-order reduction: block b sums partial quadruples
// [b chunk, min(n, (b + 1) chunk)) into out[b][4], so that the one-block final
// pass reads at most kEnergyL2 quadruples however large the lattice.
__global__ __launch_bounds__(kBlock) void k_energy_reduce(const double *__restrict__ partial, int n, int chunk,
                                                          double *__restrict__ out) {
    __shared__ double red[kBlock / 64][4];
    const int p0 = blockIdx.x * chunk, p1 = min(n, p0 + chunk);
    double e[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = p0 + threadIdx.x; p < p1; p += kBlock)
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] += partial[(size_t)p * 4 + k];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double v = wave_sum(e[k]);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) v += red[w][threadIdx.x];
        out[(size_t)blockIdx.x * 4 + threadIdx.x] = v;
    }
}

// Fixed-order final reduction of n partial quadruples by one block.
__global__ __launch_bounds__(kBlock) void k_energy_final(const double *__restrict__ partial, int n,
                                                         double *__restrict__ E, double *__restrict__ terms) {
    __shared__ double red[kBlock / 64][4];
    double e[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < n; p += kBlock)
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] += partial[(size_t)p * 4 + k];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double v = wave_sum(e[k]);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[4];
        for (int k = 0; k < 4; ++k) {
            tot[k] = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) tot[k] += red[w][k];
        }
        const double all = ((tot[0] + tot[1]) + tot[2]) + tot[3];
        if (E) *E = all;
        if (terms) {
            for (int k = 0; k < 4; ++k) terms[k] = tot[k];
            terms[4] = all;
        }
    }
}

int energy_partial_count(const Grid &g) {
    return (int)(((g.M + kBlock - 1) / kBlock) * g.n_sub);
}

size_t energy_partial_doubles(const Grid &g) { return (size_t)4 * ((size_t)energy_partial_count(g) + kEnergyL2); }

hipError_t launch_energy(int field_prec, const BondTable &tb, const Grid &g, const Onsite &os,
                         const double *S, const float *bdip, const void *bil, double *partial, double *E,
                         double *terms, hipStream_t st) {
    const dim3 grid = site_grid(g);
    if (field_prec == 0) {
        const double *bd = (const double *)bil;
        if (tb.iso) k_energy_partial<double, true><<<grid, kBlock, 0, st>>>(tb, g, os, S, bdip, bd, partial);
        else k_energy_partial<double, false><<<grid, kBlock, 0, st>>>(tb, g, os, S, bdip, bd, partial);
    } else {
        const float *bf = (const float *)bil;
        if (tb.iso) k_energy_partial<float, true><<<grid, kBlock, 0, st>>>(tb, g, os, S, bdip, bf, partial);
        else k_energy_partial<float, false><<<grid, kBlock, 0, st>>>(tb, g, os, S, bdip, bf, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_energy_reduce(partial, energy_partial_count(g), E, terms, st);
}

hipError_t launch_energy_reduce(double *partial, int n, double *E, double *terms, hipStream_t st) {
    if (n <= 8 * kBlock) {
        k_energy_final<<<1, kBlock, 0, st>>>(partial, n, E, terms);
        return hipGetLastError();
    }
    // two levels: at most kEnergyL2 blocks of at least 8 kBlock quadruples
    const int nb = (int)std::min<int64_t>(kEnergyL2, ((int64_t)n + 8 * kBlock - 1) / (8 * kBlock));
    const int chunk = (int)(((int64_t)n + nb - 1) / nb);
    double *mid = partial + (size_t)4 * n;
    k_energy_reduce<<<nb, kBlock, 0, st>>>(partial, n, chunk, mid);
    k_energy_final<<<1, kBlock, 0, st>>>(mid, nb, E, terms);
    return hipGetLastError();
}

// ---------------------------------------------------------------- RNG hooks
__global__ __launch_bounds__(kBlock) void k_thermal_noise(uint64_t seed, uint64_t step, uint32_t tag,
                                                          int64_t N, double *__restrict__ eta) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    double e[3];
    thermal_eta(seed, step, tag, (uint64_t)i, e);
    eta[i] = e[0];
    eta[N + i] = e[1];
    eta[2 * N + i] = e[2];
}

hipError_t launch_thermal_noise(uint64_t seed, uint64_t step, uint32_t tag, int64_t N, double *eta,
                                hipStream_t st) {
    if (N <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((N + kBlock - 1) / kBlock);
    k_thermal_noise<<<blocks, kBlock, 0, st>>>(seed, step, tag, N, eta);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_philox(const uint32_t *__restrict__ ctr,
                                                   const uint32_t *__restrict__ key, int64_t n,
                                                   uint32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t c0 = ctr[4 * i], c1 = ctr[4 * i + 1], c2 = ctr[4 * i + 2], c3 = ctr[4 * i + 3];
    philox4x32_10(c0, c1, c2, c3, key[2 * i], key[2 * i + 1]);
    out[4 * i] = c0;
    out[4 * i + 1] = c1;
    out[4 * i + 2] = c2;
    out[4 * i + 3] = c3;
}

// Streaming probe of the attainable HBM bandwidth: 16-byte accesses, four
// in flight per thread, grid-stride.  kind 0 copies src to dst, 1 reads src
// (folded into a word that is stored only if it equals a sentinel, so the
// loads stay and nothing is written), 2 fills dst.
__global__ __launch_bounds__(256) void k_stream(int kind, const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                int64_t n) {
    const int64_t st = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (kind == 0) {
        for (; i + 3 * st < n; i += 4 * st) {
            const uint4 a = src[i], b = src[i + st], c = src[i + 2 * st], d = src[i + 3 * st];
            dst[i] = a;
            dst[i + st] = b;
            dst[i + 2 * st] = c;
            dst[i + 3 * st] = d;
        }
        for (; i < n; i += st) dst[i] = src[i];
    } else if (kind == 1) {
        uint32_t x = 0;
        for (; i + 3 * st < n; i += 4 * st) {
            const uint4 a = src[i], b = src[i + st], c = src[i + 2 * st], d = src[i + 3 * st];
            x ^= (a.x ^ a.y ^ a.z ^ a.w) + (b.x ^ b.y ^ b.z ^ b.w) + (c.x ^ c.y ^ c.z ^ c.w) + (d.x ^ d.y ^ d.z ^ d.w);
        }
        for (; i < n; i += st) x ^= src[i].x ^ src[i].y ^ src[i].z ^ src[i].w;
        if (x == 0x9E3779B9u && dst) dst[0].x = x;
    } else {
        const uint4 v = make_uint4(0x3FF00000u, 0u, 0x3FF00000u, 0u);
        for (; i + 3 * st < n; i += 4 * st) {
            dst[i] = v;
            dst[i + st] = v;
            dst[i + 2 * st] = v;
            dst[i + 3 * st] = v;
        }
        for (; i < n; i += st) dst[i] = v;
    }
}

hipError_t launch_stream(int kind, const void *src, void *dst, int64_t n16, hipStream_t st) {
    if (n16 <= 0) return hipSuccess;
    const int64_t want = (n16 + 1023) / 1024;
    const unsigned blocks = (unsigned)(want < 4096 ? want : 4096);
    k_stream<<<blocks, 256, 0, st>>>(kind, (const uint4 *)src, (uint4 *)dst, n16);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, int64_t n, uint32_t *out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    k_philox<<<blocks, kBlock, 0, st>>>(ctr, key, n, out);
    return hipGetLastError();
}

}  // namespace spx
