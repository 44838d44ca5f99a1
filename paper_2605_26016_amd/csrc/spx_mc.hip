// spx_mc.hip -- heat-bath and Metropolis Monte Carlo with colour-based
// parallel updates (Methods, Monte Carlo sampling), and the magnetisation sum
// used by the thermodynamic observables (Methods, thermodynamic observables).
//
// Colouring: site (x, y, z, a) has colour (x + ky y + kz z + o_a) mod C.  The
// host picks the smallest C >= 2, then the lexicographically smallest
// (ky, kz, o_1 .. o_{n_sub-1}) (o_0 = 0, coefficients in [0, C)), such that no
// bond joins two sites of one colour.  A bond (a <- b, delta) joins sites whose
// coordinate difference along an axis is delta itself or, on a periodic
// axis, a wrapped value of it; the set of differences the lattice realises is
// enumerated per axis, so the test is exact for any extent.  One sweep is C
// launches, one per colour; every site of the colour is updated in place
// against the bilinear + Zeeman field of its neighbours, none of which is
// being written in that launch.
//
// Random numbers: one Philox4x32-10 block per (site, sweep), counter
// (i lo, i hi ^ tag, sweep lo, sweep hi), key (seed lo, seed hi), uniforms
// (x + 1/2) 2^-32, tag kMcTag.
//
// Colour-major layout.  In the natural layout the sites of one colour sit
// C apart along every row, so each launch touches every cache line of the
// state.  A call of several sweeps therefore copies the state once into rows
// ordered by colour class, [x mod C][x div C], runs every launch there and
// copies it back: a colour's sites of one row are then one contiguous run,
// and so are the runs of every neighbour class it reads.  Each class block
// carries ghost slots at both ends and the rows carry ghost rows in y and
// z (copies of the wrapped sites on periodic axes, zero across open faces),
// so the neighbour through bond p of a site in class x0 is at a fixed
// offset from the site's slot for every site, tabulated per (p, x0), and no
// site tests a boundary; a site whose ghost copies exist writes them with
// its new spin (no site of the launch reads them: they share its colour).
// The bonds are summed in the same order with the same arithmetic (a ghost
// across an open face adds an exact zero where the natural kernel skips the
// bond), and the Philox counter is the natural site index, so both layouts
// give the same bits.

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "spx_device.hpp"
#include "spx_ext.hpp"
#include "spx_mc_math.hpp"

namespace spx {

struct MCState {
    int C = 0;  // colours (0: not searched yet, -1: none found)
    int C_fail = 0;  // why the search failed (a ColourResult)
    int ky = 0, kz = 0;
    int o[kMaxSub] = {0};
    unsigned long long *d_acc = nullptr;  // accepted-move counter of the last call
    double *d_part = nullptr;             // magnetisation block partials [kMagBlocks][3]
    int64_t *d_off = nullptr;             // linear index offset of every bond (interior sites)
    int rad[3] = {0, 0, 0};               // largest |delta| of the bonds along each axis
    int64_t *d_coff = nullptr;            // colour-major slot offset per (bond, class x0), [n_bonds][C]
    double *d_cm = nullptr;               // colour-major copy of the state, 3 x n_rows x C J
    size_t cm_cap = 0;                    // doubles held by d_cm
};

void mc_destroy(MCState *m) {
    if (!m) return;
    if (m->d_acc) (void)hipFree(m->d_acc);
    if (m->d_part) (void)hipFree(m->d_part);
    if (m->d_off) (void)hipFree(m->d_off);
    if (m->d_coff) (void)hipFree(m->d_coff);
    if (m->d_cm) (void)hipFree(m->d_cm);
    delete m;
}

namespace {

constexpr uint32_t kMcTag = 0x4D430000u;
constexpr int kMcB = 256;
constexpr int kMagBlocks = 1024;

struct McColour {
    int C, ky, kz;
    int o[kMaxSub];
};

// Orthonormal frame (e1, e2) perpendicular to unit e3: e1 = normalize(e3 x a),
// a the Cartesian axis least aligned with e3 (first on ties), e2 = e3 x e1.
__device__ __forceinline__ void frame(const double e3[3], double e1[3], double e2[3]) {
    int k = 0;
    double best = fabs(e3[0]);
    if (fabs(e3[1]) < best) { best = fabs(e3[1]); k = 1; }
    if (fabs(e3[2]) < best) { k = 2; }
    const double ax[3] = {k == 0 ? 1.0 : 0.0, k == 1 ? 1.0 : 0.0, k == 2 ? 1.0 : 0.0};
    e1[0] = e3[1] * ax[2] - e3[2] * ax[1];
    e1[1] = e3[2] * ax[0] - e3[0] * ax[2];
    e1[2] = e3[0] * ax[1] - e3[1] * ax[0];
    normalise3(e1);
    e2[0] = e3[1] * e1[2] - e3[2] * e1[1];
    e2[1] = e3[2] * e1[0] - e3[0] * e1[2];
    e2[2] = e3[0] * e1[1] - e3[1] * e1[0];
}

// -sum_l K_l (s.n_l)^2
__device__ __forceinline__ double aniso_energy(const Onsite &os, int a, const double s[3]) {
    double e = 0.0;
    for (int l = 0; l < os.n_aniso; ++l) {
        const double *n = os.axis[a][l];
        const double sn = s[0] * n[0] + s[1] * n[1] + s[2] * n[2];
        e -= os.K[a][l] * sn * sn;
    }
    return e;
}

// The move of site i (natural index) in field b: one Philox block for (i,
// sweep).  Heat-bath draws the new spin from exp(beta b.s) on the sphere;
// Metropolis proposes a uniform direction and accepts it if u2 <
// exp(-beta dH) (si: the current spin).  Returns 1 for an accepted move
// (heat-bath: always).
template <int METHOD>
__device__ __forceinline__ unsigned mc_move(const Onsite &os, int a, const double b[3], const double si[3],
                                            double beta, uint64_t seed, uint64_t sweep, int64_t i, double sn[3]) {
    uint32_t c0 = (uint32_t)i, c1 = (uint32_t)((uint64_t)i >> 32) ^ kMcTag;
    uint32_t c2 = (uint32_t)sweep, c3 = (uint32_t)(sweep >> 32);
    philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double sc = 2.3283064365386963e-10;  // 2^-32
    const double u0 = ((double)c0 + 0.5) * sc, u1 = ((double)c1 + 0.5) * sc;
    if (METHOD == 0) {
        // heat-bath: cos to b from the inverse distribution function of
        // exp(x c) on [-1, 1], c = 1 + ln(1 + (1 - u0)(e^(-2x) - 1)) / x,
        // azimuth 2 pi u1 in the frame around b
        const double n2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
        double cth, e3[3] = {0.0, 0.0, 1.0};
        if (n2 > 0.0) {
            // |b| below 2^-511 is scaled by 2^600 first (exact), so that the
            // squared norm is a normal number
            const bool tiny = n2 < 0x1p-1022;
            const double sf = tiny ? 0x1p600 : 1.0;
            const double c[3] = {b[0] * sf, b[1] * sf, b[2] * sf};
            const double m2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
            const double rn = rsqrt_pos(m2);
            const double xb = beta * ((m2 * rn) * (tiny ? 0x1p-600 : 1.0));
            for (int q = 0; q < 3; ++q) e3[q] = c[q] * rn;
            cth = 1.0 + div_pos(log1p_neg((1.0 - u0) * expm1_nonpos(-2.0 * xb)), xb);
        } else {
            cth = 2.0 * u0 - 1.0;
        }
        cth = fmin(fmax(cth, -1.0), 1.0);
        double e1[3], e2[3];
        frame(e3, e1, e2);
        const double v = 1.0 - cth * cth;
        const double st = v > 0.0 ? sqrt_pos(v) : 0.0;
        double sp, cp;
        sincospi_d(2.0 * u1, sp, cp);
        for (int q = 0; q < 3; ++q) sn[q] = cth * e3[q] + st * (cp * e1[q] + sp * e2[q]);
        return 1u;
    } else {
        // Metropolis: uniform trial direction, accepted if u2 < exp(-beta dH)
        // (always when dH <= 0, since u2 < 1)
        const double u2 = ((double)c2 + 0.5) * sc;
        const double zt = 2.0 * u0 - 1.0, v = 1.0 - zt * zt;
        const double r = v > 0.0 ? sqrt_pos(v) : 0.0;
        double sp, cp;
        sincospi_d(2.0 * u1, sp, cp);
        const double tr[3] = {r * cp, r * sp, zt};
        const double dH = -((tr[0] - si[0]) * b[0] + (tr[1] - si[1]) * b[1] + (tr[2] - si[2]) * b[2]) +
                          aniso_energy(os, a, tr) - aniso_energy(os, a, si);
        const double y = -beta * dH;
        const bool ok = y >= 0.0 || u2 < exp_nonpos(y);
        for (int q = 0; q < 3; ++q) sn[q] = ok ? tr[q] : si[q];
        return ok ? 1u : 0u;
    }
}

// Workgroups are dealt to the 8 XCDs in turn (block b to XCD b mod 8); this
// renumbering gives each XCD one contiguous range of blocks instead, so the
// neighbour rows (y +- 1, z +- 1) that a block reads were mostly fetched by
// blocks of the same XCD and come from its L2.
__device__ __forceinline__ int64_t xcd_block() {
    const int64_t T = gridDim.x, b = blockIdx.x;
    const int64_t q = T / 8, r = T % 8, k = b % 8;
    return k * q + (k < r ? k : r) + b / 8;
}

// One colour of one sweep.  Thread t covers x-slot j = t % J of row (y, z, a)
// = t / J, J = ceil(Lx / C): the row's sites of colour c are x = x0 + C j.
// Bilinear field of an interior site (every neighbour inside the lattice):
// neighbour j = i + off_p, no coordinate wrapping.
template <bool ISO, int UNR>
__device__ __forceinline__ void bil_interior(const BondTable &tb, const int64_t *__restrict__ off, int64_t N, int a,
                                             int64_t i, const double *__restrict__ S, double acc[3]) {
    acc[0] = acc[1] = acc[2] = 0.0;
    const int p0 = tb.start[a], p1 = tb.start[a + 1];
#pragma unroll UNR
    for (int p = p0; p < p1; ++p) {
        const int64_t j = i + off[p];
        const double s0 = S[j], s1 = S[N + j], s2 = S[2 * N + j];
        if constexpr (ISO) {
            const double J = tb.Jd[p];
            acc[0] += J * s0;
            acc[1] += J * s1;
            acc[2] += J * s2;
        } else {
            const double *Jp = tb.Jd + 9 * p;
            acc[0] += Jp[0] * s0 + Jp[1] * s1 + Jp[2] * s2;
            acc[1] += Jp[3] * s0 + Jp[4] * s1 + Jp[5] * s2;
            acc[2] += Jp[6] * s0 + Jp[7] * s1 + Jp[8] * s2;
        }
    }
}

template <bool ISO, int METHOD, int UNR>
__global__ __launch_bounds__(kMcB) void k_mc_colour(double *__restrict__ S, BondTable tb, Grid g, Onsite os,
                                                    McColour col, int c, double beta, uint64_t seed,
                                                    uint64_t sweep, unsigned long long *__restrict__ acc,
                                                    const int64_t *__restrict__ off, int3 rad) {
    const int C = col.C;
    const int J = (g.Lx + C - 1) / C;
    const int64_t n_rows = (int64_t)g.Ly * g.Lz * g.n_sub;
    const int64_t total = n_rows * J;
    const int64_t N = g.N;
    unsigned int accepted = 0;
    for (int64_t t = xcd_block() * kMcB + threadIdx.x; t < total; t += (int64_t)gridDim.x * kMcB) {
        // slot -> (j, y, z, a); 32-bit division when the slot count fits
        // (every lattice below 2^32 slots), which is far cheaper than the
        // 64-bit routine
        int j, y, z, a;
        if (total <= (int64_t)0xffffffffll) {
            const uint32_t tt = (uint32_t)t, uJ = (uint32_t)J, uLy = (uint32_t)g.Ly, uLz = (uint32_t)g.Lz;
            const uint32_t row = tt / uJ;
            const uint32_t yz = row / uLy;
            j = (int)(tt - row * uJ);
            y = (int)(row - yz * uLy);
            a = (int)(yz / uLz);
            z = (int)(yz - (uint32_t)a * uLz);
        } else {
            const int64_t row = t / J;
            j = (int)(t % J);
            y = (int)(row % g.Ly);
            z = (int)((row / g.Ly) % g.Lz);
            a = (int)(row / ((int64_t)g.Ly * g.Lz));
        }
        int x0 = (c - col.ky * y - col.kz * z - col.o[a]) % C;
        if (x0 < 0) x0 += C;
        const int x = x0 + C * j;
        if (x >= g.Lx) continue;
        const int64_t i = (int64_t)a * g.M + x + (int64_t)g.Lx * (y + (int64_t)g.Ly * z);
        double bl[1][3];
        const bool interior = x >= rad.x && x < g.Lx - rad.x && y >= rad.y && y < g.Ly - rad.y && z >= rad.z &&
                              z < g.Lz - rad.z;
        if (interior) {
            bil_interior<ISO, UNR>(tb, off, N, a, i, S, bl[0]);
        } else {
            const double *const src[1] = {S};
            bil_sum<double, ISO, 1>(tb, g, a, x, y, z, src, bl);
        }
        const double b[3] = {bl[0][0] + os.bz[a][0], bl[0][1] + os.bz[a][1], bl[0][2] + os.bz[a][2]};
        double si[3] = {0.0, 0.0, 0.0};
        if (METHOD == 1) {
            si[0] = S[i];
            si[1] = S[N + i];
            si[2] = S[2 * N + i];
        }
        double sn[3];
        accepted += mc_move<METHOD>(os, a, b, si, beta, seed, sweep, i, sn);
        S[i] = sn[0];
        S[N + i] = sn[1];
        S[2 * N + i] = sn[2];
    }
    if (acc) {
        // integer counts: the order of the atomic additions does not matter
        unsigned int w = accepted;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) w += __shfl_down(w, off, 64);
        if ((threadIdx.x & 63) == 0 && w) atomicAdd(acc, (unsigned long long)w);
    }
}

// The padded colour-major layout.  Row (y, z, a) holds C class blocks of Jp
// = J + 2 ex slots (J = ceil(Lx / C), ex = ceil(rx / C)); slot ex + jv of
// block k is virtual x = k + C jv, so a block covers x from k - C ex to
// k + C (J + ex) - 1.  Rows run over virtual y in [-ry, Ly + ry) and z in
// [-rz, Lz + rz) (rx, ry, rz: the bonds' largest offsets).  A virtual site
// outside the lattice is a ghost: on a periodic axis a copy of its wrapped
// site, across an open face zero (it adds nothing to a field).
struct CmDims {
    int C, J, Jp, ex;       // colours, real and padded slots per class block, ghost slots per end
    int lxq, lxm;           // Lx div C, Lx mod C
    int ry, rz, Lyp, Lzp;   // ghost rows and padded row extents
    int64_t n_rows, NP;     // real rows (y, z, a) and padded doubles per component
    int64_t pitch;          // C Jp
};

// padded slot of virtual site (xv, yv, zv, a)
__device__ __forceinline__ int64_t cm_slot(const CmDims &d, int xv, int yv, int zv, int a) {
    int k = xv % d.C;
    if (k < 0) k += d.C;
    const int jv = (xv - k) / d.C;  // exact
    const int64_t pr = (yv + d.ry) + (int64_t)d.Lyp * ((zv + d.rz) + (int64_t)d.Lzp * a);
    return pr * d.pitch + (int64_t)k * d.Jp + jv + d.ex;
}

// the real coordinate of virtual coordinate v (-1: across an open face)
__device__ __forceinline__ int cm_real(int v, int L, int per) {
    if (v >= 0 && v < L) return v;
    if (!per) return -1;
    v %= L;
    return v < 0 ? v + L : v;
}

// Natural -> padded colour-major copy, one thread per padded slot (ghosts
// included), and back, one thread per site.
__global__ __launch_bounds__(kMcB) void k_mc_to_cm(const double *__restrict__ S, double *__restrict__ P, Grid g,
                                                   CmDims d) {
    for (int64_t q = (int64_t)blockIdx.x * kMcB + threadIdx.x; q < d.NP; q += (int64_t)gridDim.x * kMcB) {
        const int64_t pr = q / d.pitch;
        const int s = (int)(q - pr * d.pitch);
        const int k = s / d.Jp, jv = s - k * d.Jp - d.ex;
        const int64_t yz = pr / d.Lyp;
        const int yv = (int)(pr - yz * d.Lyp) - d.ry;
        const int a = (int)(yz / d.Lzp);
        const int zv = (int)(yz - (int64_t)a * d.Lzp) - d.rz;
        const int x = cm_real(k + d.C * jv, g.Lx, g.per[0]), y = cm_real(yv, g.Ly, g.per[1]),
                  z = cm_real(zv, g.Lz, g.per[2]);
        const bool live = (x | y | z) >= 0;
        const int64_t i = live ? (int64_t)a * g.M + x + (int64_t)g.Lx * (y + (int64_t)g.Ly * z) : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) P[c * d.NP + q] = live ? S[c * g.N + i] : 0.0;
    }
}

__global__ __launch_bounds__(kMcB) void k_mc_from_cm(const double *__restrict__ P, double *__restrict__ S, Grid g,
                                                     CmDims d) {
    for (int64_t i = (int64_t)blockIdx.x * kMcB + threadIdx.x; i < g.N; i += (int64_t)gridDim.x * kMcB) {
        const int a = (int)(i / g.M);
        int x, y, z;
        site_xyz(g, (int)(i - (int64_t)a * g.M), x, y, z);
        const int64_t q = cm_slot(d, x, y, z, a);
#pragma unroll
        for (int c = 0; c < 3; ++c) S[c * g.N + i] = P[c * d.NP + q];
    }
}

// One colour of one sweep on the padded colour-major copy P: the natural
// kernel's site loop, draw and update, every neighbour at the tabulated
// offset of its bond and class, and the new spin also written to the
// site's ghost copies.  The register allocator is left free: asking it for
// four waves per SIMD (at most 128 registers) kept the count of resident
// waves where it was but made the code slower, Metropolis with 2-5 shells
// by a third (sc 200^3).
template <bool ISO, int METHOD, int UNR>
__global__ __launch_bounds__(kMcB) void k_mc_colour_cm(double *__restrict__ P, BondTable tb, Grid g, Onsite os,
                                                      McColour col, int c, double beta, uint64_t seed,
                                                      uint64_t sweep, unsigned long long *__restrict__ acc,
                                                      const int64_t *__restrict__ coff, CmDims d) {
    const int C = col.C;
    const int J = d.J;
    const int64_t total = d.n_rows * J;
    const int64_t NP = d.NP;
    unsigned int accepted = 0;
    // slot t -> (j, y, z, a) of row t / J, and the site's class x0
    auto decode = [&](int64_t t, int &j, int &y, int &z, int &a, int64_t &row, int &x0)
                      __attribute__((always_inline)) {
        if (total <= (int64_t)0xffffffffll) {
            const uint32_t tt = (uint32_t)t, uJ = (uint32_t)J, uLy = (uint32_t)g.Ly, uLz = (uint32_t)g.Lz;
            const uint32_t rw = tt / uJ;
            const uint32_t yz = rw / uLy;
            j = (int)(tt - rw * uJ);
            y = (int)(rw - yz * uLy);
            a = (int)(yz / uLz);
            z = (int)(yz - (uint32_t)a * uLz);
            row = rw;
        } else {
            row = t / J;
            j = (int)(t % J);
            y = (int)(row % g.Ly);
            z = (int)((row / g.Ly) % g.Lz);
            a = (int)(row / ((int64_t)g.Ly * g.Lz));
        }
        x0 = (c - col.ky * y - col.kz * z - col.o[a]) % C;
        if (x0 < 0) x0 += C;
    };
    // the other virtual x of the site: x - Lx in class x0 - (Lx mod C) and
    // block slot j - (Lx div C), one less where the class folds into
    // [0, C); x + Lx likewise (-1: outside the padded block, or open x)
    auto x_images = [&](int x0, int j, int &sm, int &sp) __attribute__((always_inline)) {
        sm = sp = -1;
        if (!g.per[0]) return;
        int km = x0 - d.lxm, jm = j - d.lxq;
        if (km < 0) { km += C; --jm; }
        if (jm + d.ex >= 0) sm = km * d.Jp + jm + d.ex;
        int kp = x0 + d.lxm, jp = j + d.lxq;
        if (kp >= C) { kp -= C; ++jp; }
        if (jp + d.ex < d.Jp) sp = kp * d.Jp + jp + d.ex;
    };
    for (int64_t t = xcd_block() * kMcB + threadIdx.x; t < total; t += (int64_t)gridDim.x * kMcB) {
        int j, y, z, a, x0;
        int64_t row;
        decode(t, j, y, z, a, row, x0);
        const int x = x0 + C * j;
        if (x >= g.Lx) continue;
        // which ghost images the site has (bits: x - Lx, x + Lx, y - Ly,
        // y + Ly, z - Lz, z + Lz); their slots are worked out again after
        // the draw, only by the sites that have some
        int ghosts;
        {
            int sm, sp;
            x_images(x0, j, sm, sp);
            ghosts = (sm >= 0 ? 1 : 0) | (sp >= 0 ? 2 : 0) | (g.per[1] && y - g.Ly >= -d.ry ? 4 : 0) |
                     (g.per[1] && y < d.ry ? 8 : 0) | (g.per[2] && z - g.Lz >= -d.rz ? 16 : 0) |
                     (g.per[2] && z < d.rz ? 32 : 0);
        }
        const int64_t i = x + (int64_t)g.Lx * row;  // natural index (the Philox counter)
        const int64_t own = ((y + d.ry) + (int64_t)d.Lyp * ((z + d.rz) + (int64_t)d.Lzp * a)) * d.pitch +
                            (int64_t)x0 * d.Jp + j + d.ex;
        double bl[3] = {0.0, 0.0, 0.0};
        const int p0 = tb.start[a], p1 = tb.start[a + 1];
#pragma unroll UNR
        for (int p = p0; p < p1; ++p) {
            const int64_t q = own + coff[p * C + x0];
            const double s0 = P[q], s1 = P[NP + q], s2 = P[2 * NP + q];
            if constexpr (ISO) {
                const double Jp = tb.Jd[p];
                bl[0] += Jp * s0;
                bl[1] += Jp * s1;
                bl[2] += Jp * s2;
            } else {
                const double *Jp = tb.Jd + 9 * p;
                bl[0] += Jp[0] * s0 + Jp[1] * s1 + Jp[2] * s2;
                bl[1] += Jp[3] * s0 + Jp[4] * s1 + Jp[5] * s2;
                bl[2] += Jp[6] * s0 + Jp[7] * s1 + Jp[8] * s2;
            }
        }
        const double b[3] = {bl[0] + os.bz[a][0], bl[1] + os.bz[a][1], bl[2] + os.bz[a][2]};
        double si[3] = {0.0, 0.0, 0.0};
        if (METHOD == 1) {
            si[0] = P[own];
            si[1] = P[NP + own];
            si[2] = P[2 * NP + own];
        }
        double sn[3];
        accepted += mc_move<METHOD>(os, a, b, si, beta, seed, sweep, i, sn);
        P[own] = sn[0];
        P[NP + own] = sn[1];
        P[2 * NP + own] = sn[2];
        // ghost copies: every combination of the real and the other virtual
        // coordinates of each axis except the real site itself
        if (ghosts) {
            decode(t, j, y, z, a, row, x0);
            int xs[3] = {x0 * d.Jp + j + d.ex, -1, -1};  // slots within a row (C Jp < 2^31)
            x_images(x0, j, xs[1], xs[2]);
            const int ym = (ghosts & 4) ? y - g.Ly : INT_MIN, yp = (ghosts & 8) ? y + g.Ly : INT_MIN;
            const int zm = (ghosts & 16) ? z - g.Lz : INT_MIN, zp = (ghosts & 32) ? z + g.Lz : INT_MIN;
#pragma unroll
            for (int iz = 0; iz < 3; ++iz) {
                const int zv = iz == 0 ? z : (iz == 1 ? zm : zp);
                if (zv == INT_MIN) continue;
#pragma unroll
                for (int iy = 0; iy < 3; ++iy) {
                    const int yv = iy == 0 ? y : (iy == 1 ? ym : yp);
                    if (yv == INT_MIN) continue;
                    const int64_t rb = ((yv + d.ry) + (int64_t)d.Lyp * ((zv + d.rz) + (int64_t)d.Lzp * a)) * d.pitch;
#pragma unroll
                    for (int ix = 0; ix < 3; ++ix) {
                        if ((ix | iy | iz) == 0 || xs[ix] < 0) continue;
                        const int64_t qg = rb + xs[ix];
                        P[qg] = sn[0];
                        P[NP + qg] = sn[1];
                        P[2 * NP + qg] = sn[2];
                    }
                }
            }
        }
    }
    if (acc) {
        unsigned int w = accepted;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) w += __shfl_down(w, off, 64);
        if ((threadIdx.x & 63) == 0 && w) atomicAdd(acc, (unsigned long long)w);
    }
}

__global__ void k_mc_zero(unsigned long long *acc) { *acc = 0ull; }

// sum_i S_i: block partials (grid-stride, fixed order), then one block
__global__ __launch_bounds__(kMcB) void k_mag_partial(const double *__restrict__ S, int64_t N,
                                                      double *__restrict__ part) {
    __shared__ double red[3][kMcB / 64];
    double m[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kMcB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kMcB)
        for (int q = 0; q < 3; ++q) m[q] += S[q * N + i];
    for (int q = 0; q < 3; ++q) {
        const double v = wave_sum(m[q]);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int k = 0; k < kMcB / 64; ++k) t += red[threadIdx.x][k];
        part[blockIdx.x * 3 + threadIdx.x] = t;
    }
}

__global__ __launch_bounds__(kMcB) void k_mag_final(const double *__restrict__ part, int nb, double *__restrict__ m) {
    __shared__ double red[3][kMcB / 64];
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < nb; k += kMcB)
        for (int q = 0; q < 3; ++q) v[q] += part[k * 3 + q];
    for (int q = 0; q < 3; ++q) {
        const double s = wave_sum(v[q]);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int k = 0; k < kMcB / 64; ++k) t += red[threadIdx.x][k];
        m[threadIdx.x] = t;
    }
}

// Coordinate differences that a bond offset d realises along an axis of
// extent L: d itself where x + d stays inside, and on a periodic axis the
// wrapped difference elsewhere.
void realised(int d, int L, bool per, std::vector<int> &out) {
    out.clear();
    for (int x = 0; x < L; ++x) {
        const int t = x + d;
        int diff;
        if (t >= 0 && t < L) diff = d;
        else if (per) diff = (((t % L) + L) % L) - x;
        else continue;
        if (std::find(out.begin(), out.end(), diff) == out.end()) out.push_back(diff);
    }
}

// Candidate colourings tried at most, over all C (each candidate is checked
// against the realised bonds until one joins two sites of one colour).
constexpr long long kColourSearchBudget = 1LL << 26;

enum ColourResult { COLOUR_FOUND = 1, COLOUR_NONE = 0, COLOUR_IMPOSSIBLE = -1, COLOUR_BUDGET = -2 };

// The colouring (see the header).  COLOUR_NONE if none with C <= cmax,
// COLOUR_IMPOSSIBLE if a bond joins a site to itself (same sublattice, every
// realised difference zero on all three axes: no colouring separates them),
// COLOUR_BUDGET if the candidates up to cmax exceed kColourSearchBudget
// before one is found.
int find_colouring(const Grid &g, const std::vector<int> &ab, const std::vector<int> &dl, int cmax, McColour &out) {
    const int nb = (int)ab.size() / 2;
    struct Realised {
        int a, b;
        std::vector<int> dx, dy, dz;
    };
    std::vector<Realised> rb;
    rb.reserve(nb);
    for (int p = 0; p < nb; ++p) {
        Realised r;
        r.a = ab[2 * p];
        r.b = ab[2 * p + 1];
        realised(dl[3 * p], g.Lx, g.per[0] != 0, r.dx);
        realised(dl[3 * p + 1], g.Ly, g.per[1] != 0, r.dy);
        realised(dl[3 * p + 2], g.Lz, g.per[2] != 0, r.dz);
        if (r.dx.empty() || r.dy.empty() || r.dz.empty()) continue;
        auto has0 = [](const std::vector<int> &v) { return std::find(v.begin(), v.end(), 0) != v.end(); };
        if (r.a == r.b && has0(r.dx) && has0(r.dy) && has0(r.dz)) return COLOUR_IMPOSSIBLE;
        rb.push_back(std::move(r));
    }
    const int n_free = 2 + (g.n_sub - 1);
    long long spent = 0;
    for (int C = 2; C <= cmax; ++C) {
        long long total = 1;
        for (int k = 0; k < n_free; ++k) total *= C;
        if (spent + total > kColourSearchBudget) return COLOUR_BUDGET;
        spent += total;
        int digits[2 + kMaxSub];
        for (long long t = 0; t < total; ++t) {
            long long r = t;
            for (int k = n_free - 1; k >= 0; --k) {
                digits[k] = (int)(r % C);
                r /= C;
            }
            McColour col{};
            col.C = C;
            col.ky = digits[0];
            col.kz = digits[1];
            col.o[0] = 0;
            for (int a = 1; a < g.n_sub; ++a) col.o[a] = digits[1 + a];
            bool ok = true;
            for (const Realised &r2 : rb) {
                const int off = col.o[r2.b] - col.o[r2.a];
                for (int dz : r2.dz) {
                    for (int dy : r2.dy) {
                        for (int dx : r2.dx) {
                            const long long v = (long long)dx + (long long)col.ky * dy + (long long)col.kz * dz + off;
                            if (((v % C) + C) % C == 0) { ok = false; break; }
                        }
                        if (!ok) break;
                    }
                    if (!ok) break;
                }
                if (!ok) break;
            }
            if (ok) {
                out = col;
                return COLOUR_FOUND;
            }
        }
    }
    return COLOUR_NONE;
}

spx_status colour_error(int r, int cmax) {
    if (r == COLOUR_IMPOSSIBLE)
        return set_error(SPX_ERR_UNSUPPORTED, "no colouring exists: a bond joins a site to itself");
    if (r == COLOUR_BUDGET)
        return set_error(SPX_ERR_UNSUPPORTED, "colouring search stopped at 2^26 candidates without a result");
    return set_error(SPX_ERR_UNSUPPORTED, "no colouring with at most " + std::to_string(cmax) + " colours");
}

// The handle's Monte Carlo state (scratch; the colouring is searched on
// first use by mc_colouring).
spx_status mc_state(const HamView &v, MCState **out) {
    if (*v.mc) {
        *out = *v.mc;
        return SPX_OK;
    }
    MCState *m = new MCState();
    if (hipMalloc((void **)&m->d_acc, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void **)&m->d_part, sizeof(double) * 3 * kMagBlocks) != hipSuccess) {
        (void)hipGetLastError();
        mc_destroy(m);
        return set_error(SPX_ERR_OUT_OF_MEMORY, "hipMalloc failed for Monte Carlo scratch");
    }
    *v.mc = m;
    *out = m;
    return SPX_OK;
}

spx_status mc_colouring(spx_ham *h, const HamView &v, MCState *m) {
    if (m->C > 0) return SPX_OK;
    if (m->C < 0) return colour_error(m->C_fail, 64);
    spx_ham_info info;
    spx_status s = spx_get_info(h, &info);
    if (s != SPX_OK) return s;
    const size_t nb = (size_t)std::max(info.n_bonds, 1);
    std::vector<int32_t> ab(2 * nb), dl(3 * nb);
    std::vector<double> J(9 * nb);
    s = spx_get_bonds(h, ab.data(), dl.data(), J.data());
    if (s != SPX_OK) return s;
    std::vector<int> abi(ab.begin(), ab.begin() + 2 * (size_t)info.n_bonds);
    std::vector<int> dli(dl.begin(), dl.begin() + 3 * (size_t)info.n_bonds);
    McColour col{};
    const int r = find_colouring(v.grid, abi, dli, 64, col);
    if (r != COLOUR_FOUND) {
        m->C = -1;
        m->C_fail = r;
        return colour_error(r, 64);
    }
    m->C = col.C;
    m->ky = col.ky;
    m->kz = col.kz;
    for (int a = 0; a < kMaxSub; ++a) m->o[a] = col.o[a];
    // linear offset of every bond, indexed like the device bond table (the
    // host's bond order, grouped by target sublattice)
    const Grid &g = v.grid;
    std::vector<int64_t> off(std::max(info.n_bonds, 1), 0);
    for (int p = 0; p < info.n_bonds; ++p) {
        const int dx = dli[3 * p], dy = dli[3 * p + 1], dz = dli[3 * p + 2];
        off[p] = (int64_t)(abi[2 * p + 1] - abi[2 * p]) * g.M + dx + (int64_t)g.Lx * (dy + (int64_t)g.Ly * dz);
        m->rad[0] = std::max(m->rad[0], std::abs(dx));
        m->rad[1] = std::max(m->rad[1], std::abs(dy));
        m->rad[2] = std::max(m->rad[2], std::abs(dz));
    }
    // padded colour-major slot offset of every bond from a site of class x0:
    // neighbour x' = x + dx in class (x0 + dx) mod C, slot j + floor((x0 +
    // dx) / C), padded row pr + dy + Lyp (dz + Lzp (b - a))
    const int C = col.C, JC = (g.Lx + C - 1) / C, ex = (m->rad[0] + C - 1) / C;
    const int64_t Jp = JC + 2 * ex, pitch = C * Jp;
    const int64_t Lyp = g.Ly + 2 * m->rad[1], Lzp = g.Lz + 2 * m->rad[2];
    std::vector<int64_t> coff((size_t)std::max(info.n_bonds, 1) * C, 0);
    for (int p = 0; p < info.n_bonds; ++p) {
        const int dx = dli[3 * p], dy = dli[3 * p + 1], dz = dli[3 * p + 2];
        const int64_t dr = dy + Lyp * (dz + Lzp * (abi[2 * p + 1] - abi[2 * p]));
        for (int x0 = 0; x0 < C; ++x0) {
            const int xs = x0 + dx;
            const int cls = ((xs % C) + C) % C;
            const int dv = (xs - cls) / C;  // exact
            coff[(size_t)p * C + x0] = dr * pitch + (int64_t)(cls - x0) * Jp + dv;
        }
    }
    if (hipMalloc((void **)&m->d_off, sizeof(int64_t) * off.size()) != hipSuccess ||
        hipMemcpy(m->d_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc((void **)&m->d_coff, sizeof(int64_t) * coff.size()) != hipSuccess ||
        hipMemcpy(m->d_coff, coff.data(), sizeof(int64_t) * coff.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        if (m->d_off) (void)hipFree(m->d_off);
        if (m->d_coff) (void)hipFree(m->d_coff);
        m->d_off = nullptr;
        m->d_coff = nullptr;
        m->C = 0;
        return set_error(SPX_ERR_OUT_OF_MEMORY, "Monte Carlo bond offsets");
    }
    return SPX_OK;
}

// Dimensions of the padded colour-major copy and, on first use, its buffer.
// False (the sweeps then run in the natural layout) when a bond is longer
// than an extent, when a ghost band of a periodic axis is wider than the
// extent (a site would need copies two periods away), or when the buffer
// cannot be allocated.
bool mc_cm_buffer(const Grid &g, MCState *m, CmDims &d) {
    if (g.wrap_general) return false;
    d.C = m->C;
    d.J = (g.Lx + m->C - 1) / m->C;
    d.ex = (m->rad[0] + m->C - 1) / m->C;
    d.Jp = d.J + 2 * d.ex;
    d.lxq = g.Lx / m->C;
    d.lxm = g.Lx % m->C;
    d.ry = m->rad[1];
    d.rz = m->rad[2];
    d.Lyp = g.Ly + 2 * d.ry;
    d.Lzp = g.Lz + 2 * d.rz;
    d.pitch = (int64_t)d.C * d.Jp;
    d.n_rows = (int64_t)g.Ly * g.Lz * g.n_sub;
    d.NP = (int64_t)d.Lyp * d.Lzp * g.n_sub * d.pitch;
    if (g.per[0] && ((int64_t)d.C * d.ex > g.Lx || (int64_t)d.C * (d.J + d.ex) > 2 * (int64_t)g.Lx)) return false;
    if ((g.per[1] && d.ry > g.Ly) || (g.per[2] && d.rz > g.Lz)) return false;
    const size_t need = 3 * (size_t)d.NP;
    if (m->cm_cap >= need) return true;
    if (m->d_cm) (void)hipFree(m->d_cm);
    m->d_cm = nullptr;
    m->cm_cap = 0;
    if (hipMalloc((void **)&m->d_cm, sizeof(double) * need) != hipSuccess) {
        (void)hipGetLastError();
        m->d_cm = nullptr;
        return false;
    }
    m->cm_cap = need;
    return true;
}

}  // namespace
}  // namespace spx

using namespace spx;

extern "C" {

spx_status spx_mc_find_colouring(int32_t n_sub, const int32_t *dims, const int32_t *periodic, int32_t n_bonds,
                                 const int32_t *bond_ab, const int32_t *bond_delta, int32_t cmax, int32_t *n_colours,
                                 int32_t *coef) {
    if (!dims || !periodic || !n_colours || (n_bonds > 0 && (!bond_ab || !bond_delta)))
        return set_error(SPX_ERR_INVALID_ARG, "spx_mc_find_colouring: NULL argument");
    if (n_sub < 1 || n_sub > kMaxSub || n_bonds < 0 || cmax < 2)
        return set_error(SPX_ERR_INVALID_ARG, "spx_mc_find_colouring: n_sub in [1, 8], n_bonds >= 0, cmax >= 2");
    Grid g{};
    g.Lx = dims[0];
    g.Ly = dims[1];
    g.Lz = dims[2];
    if (g.Lx < 1 || g.Ly < 1 || g.Lz < 1) return set_error(SPX_ERR_INVALID_ARG, "dims must be >= 1");
    for (int k = 0; k < 3; ++k) g.per[k] = periodic[k] ? 1 : 0;
    g.n_sub = n_sub;
    std::vector<int> ab(bond_ab, bond_ab + 2 * (size_t)n_bonds), dl(bond_delta, bond_delta + 3 * (size_t)n_bonds);
    for (int p = 0; p < n_bonds; ++p)
        if (ab[2 * p] < 0 || ab[2 * p] >= n_sub || ab[2 * p + 1] < 0 || ab[2 * p + 1] >= n_sub)
            return set_error(SPX_ERR_INVALID_ARG, "spx_mc_find_colouring: bond sublattice out of range");
    McColour col{};
    const int r = find_colouring(g, ab, dl, cmax, col);
    if (r != COLOUR_FOUND) {
        *n_colours = 0;
        return colour_error(r, cmax);
    }
    *n_colours = col.C;
    if (coef) {
        coef[0] = col.ky;
        coef[1] = col.kz;
        for (int a = 0; a < n_sub; ++a) coef[2 + a] = col.o[a];
    }
    return SPX_OK;
}

spx_status spx_mc_colouring(spx_ham *h, int32_t *n_colours, int32_t *coef) {
    HamView v;
    spx_status s = get_ham_view(h, v);
    if (s != SPX_OK) return s;
    if (!n_colours) return set_error(SPX_ERR_INVALID_ARG, "n_colours is NULL");
    MCState *m = nullptr;
    s = mc_state(v, &m);
    if (s == SPX_OK) s = mc_colouring(h, v, m);
    if (s != SPX_OK) return s;
    *n_colours = m->C;
    if (coef) {
        coef[0] = m->ky;
        coef[1] = m->kz;
        for (int a = 0; a < v.grid.n_sub; ++a) coef[2 + a] = m->o[a];
    }
    return SPX_OK;
}

spx_status spx_mc_sweep(spx_ham *h, double *S, const spx_mc_params *p, unsigned long long *accepted, void *stream) {
    HamView v;
    spx_status s = get_ham_view(h, v);
    if (s != SPX_OK) return s;
    if (!S || !p) return set_error(SPX_ERR_INVALID_ARG, "S or params is NULL");
    if (!(p->temperature_K > 0.0)) return set_error(SPX_ERR_INVALID_ARG, "temperature must be > 0");
    if (p->n_sweeps < 0) return set_error(SPX_ERR_INVALID_ARG, "n_sweeps < 0");
    if (p->method != 0 && p->method != 1) return set_error(SPX_ERR_INVALID_ARG, "method must be 0 or 1");
    if (p->layout != 0 && p->layout != 1) return set_error(SPX_ERR_INVALID_ARG, "layout must be 0 or 1");
    if (v.dip) return set_error(SPX_ERR_UNSUPPORTED, "Monte Carlo with the dipolar term is not supported");
    if (p->method == 0 && v.onsite.n_aniso > 0)
        return set_error(SPX_ERR_UNSUPPORTED, "heat-bath needs a local energy linear in the spin (no anisotropy)");
    MCState *m = nullptr;
    s = mc_state(v, &m);
    if (s == SPX_OK) s = mc_colouring(h, v, m);
    if (s != SPX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    McColour col{};
    col.C = m->C;
    col.ky = m->ky;
    col.kz = m->kz;
    for (int a = 0; a < kMaxSub; ++a) col.o[a] = m->o[a];
    const double beta = 1.0 / (kKB * p->temperature_K);
    unsigned long long *acc = accepted ? m->d_acc : nullptr;
    if (acc) k_mc_zero<<<1, 1, 0, st>>>(acc);
    const int64_t total = (int64_t)((v.grid.Lx + col.C - 1) / col.C) * v.grid.Ly * v.grid.Lz * v.grid.n_sub;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + kMcB - 1) / kMcB, 65536));
    const bool iso = v.tab.iso != 0;
    const int3 rad = make_int3(m->rad[0], m->rad[1], m->rad[2]);
    // in place, heat-bath runs its neighbour loop two-deep (the FP64 draw
    // then keeps more waves resident: sc 200^3 one shell 21.3 against
    // 18.9e9 updates/s; one sweep with two shells 0.87 against 1.01 ms, with
    // five 11.4 against 15.1 ms); Metropolis is faster four-deep
    int max_bonds = 0;
    for (int a = 0; a < v.grid.n_sub; ++a) max_bonds = std::max(max_bonds, v.tab.start[a + 1] - v.tab.start[a]);
    const bool short_list = max_bonds <= 8;
    // The colour-major copy costs two copies of the state per call; in place,
    // every colour launch moves the whole lattice's cache lines.  A single
    // sweep of two colours runs faster in place (sc 200^3 one shell: 280
    // against 403 us); two sweeps or more colours run on the copy (five
    // shells, 20 colours, one sweep: 1.96 against 15.0 ms).
    CmDims cd{};
    const bool cm = p->layout == 0 && (p->n_sweeps >= 2 || (p->n_sweeps == 1 && col.C > 2)) &&
                    mc_cm_buffer(v.grid, m, cd);
    const unsigned pgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((cd.NP + kMcB - 1) / kMcB, 65536));
    const unsigned ngrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((v.grid.N + kMcB - 1) / kMcB, 65536));
    if (cm) k_mc_to_cm<<<pgrid, kMcB, 0, st>>>(S, m->d_cm, v.grid, cd);
    for (int n = 0; n < p->n_sweeps; ++n) {
        const uint64_t sweep = p->sweep0 + (uint64_t)n;
        for (int c = 0; c < col.C; ++c) {
            if (cm) {
                double *P = m->d_cm;
                const int64_t *co = m->d_coff;
                // neighbour-loop unroll depths as timed on sc 200^3 with 1-5
                // shells: heat-bath 2 throughout (a third faster than 4 with
                // 2-5 shells; with exchange + DMI tensors 342 against 365 us
                // per sweep at one shell), Metropolis 2 for one scalar shell
                // and 4 otherwise
                if (p->method == 0) {
                    if (iso) k_mc_colour_cm<true, 0, 2><<<grid, kMcB, 0, st>>>(P, v.tab, v.grid, v.onsite, col, c, beta, p->seed, sweep, acc, co, cd);
                    else k_mc_colour_cm<false, 0, 2><<<grid, kMcB, 0, st>>>(P, v.tab, v.grid, v.onsite, col, c, beta, p->seed, sweep, acc, co, cd);
                } else {
                    if (iso && short_list) k_mc_colour_cm<true, 1, 2><<<grid, kMcB, 0, st>>>(P, v.tab, v.grid, v.onsite, col, c, beta, p->seed, sweep, acc, co, cd);
                    else if (iso) k_mc_colour_cm<true, 1, 4><<<grid, kMcB, 0, st>>>(P, v.tab, v.grid, v.onsite, col, c, beta, p->seed, sweep, acc, co, cd);
                    else k_mc_colour_cm<false, 1, 4><<<grid, kMcB, 0, st>>>(P, v.tab, v.grid, v.onsite, col, c, beta, p->seed, sweep, acc, co, cd);
                }
                continue;
            }
            if (p->method == 0) {
                if (iso) k_mc_colour<true, 0, 2><<<grid, kMcB, 0, st>>>(S, v.tab, v.grid, v.onsite, col, c, beta, p->seed, sweep, acc, m->d_off, rad);
                else k_mc_colour<false, 0, 4><<<grid, kMcB, 0, st>>>(S, v.tab, v.grid, v.onsite, col, c, beta, p->seed, sweep, acc, m->d_off, rad);
            } else {
                if (iso) k_mc_colour<true, 1, 4><<<grid, kMcB, 0, st>>>(S, v.tab, v.grid, v.onsite, col, c, beta, p->seed, sweep, acc, m->d_off, rad);
                else k_mc_colour<false, 1, 4><<<grid, kMcB, 0, st>>>(S, v.tab, v.grid, v.onsite, col, c, beta, p->seed, sweep, acc, m->d_off, rad);
            }
        }
    }
    if (cm) k_mc_from_cm<<<ngrid, kMcB, 0, st>>>(m->d_cm, S, v.grid, cd);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && accepted)
        e = hipMemcpyAsync(accepted, m->d_acc, sizeof(unsigned long long), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return set_hip_error(e, "spx_mc_sweep");
    return SPX_OK;
}

spx_status spx_magnetization(spx_ham *h, const double *S, double *m_out, void *stream) {
    HamView v;
    spx_status s = get_ham_view(h, v);
    if (s != SPX_OK) return s;
    if (!S || !m_out) return set_error(SPX_ERR_INVALID_ARG, "S or m is NULL");
    MCState *m = nullptr;
    s = mc_state(v, &m);
    if (s != SPX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((v.grid.N + kMcB - 1) / kMcB, kMagBlocks));
    k_mag_partial<<<nb, kMcB, 0, st>>>(S, v.grid.N, m->d_part);
    k_mag_final<<<1, kMcB, 0, st>>>(m->d_part, nb, m_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "spx_magnetization");
    return SPX_OK;
}

}  // extern "C"
