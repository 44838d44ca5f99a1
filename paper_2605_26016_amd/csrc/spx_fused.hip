// spx_fused.hip -- temporally fused normalised Heun step (predictor and
// corrector in one pass over the lattice) for single-sublattice shell shapes
// of range one cell (simple cubic shells 1 and 1-3).
//
// The normalised Heun scheme of the Methods (atomistic spin dynamics) needs
// the field of the predicted state S~ at the neighbours of every site, so a
// two-sweep step writes S~ to memory and reads it back.  Here one block owns a
// column of the lattice and marches along z, keeping everything the corrector
// needs on chip:
//   - the block's 64 x NW thread grid is the predictor region: x0-1 .. x0+62
//     by y0-1 .. y0+NW-2 (one wavefront per row); the corrector writes its
//     interior, 62 x (NW-2) sites, so the one-cell ring of S~ that the
//     interior's stencil reads is predicted by this block as well;
//   - S^n planes (with a two-cell x/y halo) stream through a 4-plane LDS ring
//     in the compute type, the predicted planes S~ through another 4-plane
//     ring; each thread keeps its own site's P = S^n + dt/2 f(S^n), thermal
//     field sigma eta and FP64 S~ in registers for the one plane by which the
//     corrector trails the predictor;
//   - every predicted site, halo sites included, draws its thermal noise
//     from the Philox block of its own (wrapped) lattice index, so a halo
//     site's S~ is bit-identical to the one its own tile predicts and the
//     same eta enters both stages.
// Per step the lattice is read once (S^n) and written once (S^{n+1}): 48
// bytes per spin in FP64, against 120 for two sweeps.  The price is the
// predictor work on the halo ring, (64 NW) / (62 (NW-2)) per site.
//
// Plane schedule of one block (load index L: S^n plane z = zs - 2 + L):
//   before the loop   load planes 0, 1, 2 into ring slots 0, 1, 2;
//   iteration k       fetch plane k+1 into registers (in flight over the
//                     compute), corrector of plane L = k-3 from S~ slots
//                     (L-1, L, L+1) % 4, predictor of plane L = k-1 from S^n
//                     slots (L-1, L, L+1) % 4 into S~ slot L % 4, commit the
//                     fetched plane into slot (k+1) % 4, one barrier.
// A slot is overwritten only after the barrier that follows its last read,
// so one barrier per plane suffices.
#include <type_traits>

#include "spx_device.hpp"
#include "spx_ext.hpp"
#include "spx_stencil.hpp"

namespace spx {

namespace {

constexpr int kFX = 64;        // predictor columns per block (one wavefront)
constexpr int kFXI = kFX - 2;  // corrector columns per block
constexpr int kSW = kFX + 2;   // staged S^n columns

template <typename T, int NWT>
struct FWeights {
    T w[NWT];
};

struct FArgs {
    int Lx, Ly, Lz;
    int per[3];
    int64_t N;
    int zch, nbx, nby;
    const double *S;
    double *out;
    uint64_t step;
};

// Integrator and on-site constants of the one sublattice, packed so that the
// kernel keeps few of them in scalar registers.
struct FConst {
    double dtp, hdtp;  // dt pre and dt/2 pre, pre = -gamma/(1 + alpha^2)
    double alpha, inv, sigma;
    double bz[3];
    double K2[kMaxAniso];     // 2 K_l
    double ax[kMaxAniso][3];  // unit axes
    int n_aniso;
    int noise;
    uint64_t seed;
    uint32_t tag;
    const uint64_t *step_dev;
};

// On-site field 2 K_l (s.n_l) n_l + Zeeman; NA = the number of anisotropy axes
// (0 or 1), or -1 for up to kMaxAniso axes counted at run time.
template <int NA>
__device__ __forceinline__ void fused_onsite(const FConst &fc, const double s[3], double b[3]) {
    b[0] = fc.bz[0];
    b[1] = fc.bz[1];
    b[2] = fc.bz[2];
    constexpr int NL = NA < 0 ? kMaxAniso : NA;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        if (NA >= 0 || l < fc.n_aniso) {
            const double c = fc.K2[l] * (s[0] * fc.ax[l][0] + s[1] * fc.ax[l][1] + s[2] * fc.ax[l][2]);
            b[0] = fma(c, fc.ax[l][0], b[0]);
            b[1] = fma(c, fc.ax[l][1], b[1]);
            b[2] = fma(c, fc.ax[l][2], b[2]);
        }
    }
}

template <int KIND>
struct FShape {
    static constexpr ShapeTable t = make_shape(KIND);
};

template <typename F, int... K>
__device__ __forceinline__ void fstatic_for_impl(F &&f, std::integer_sequence<int, K...>) {
    (f(std::integral_constant<int, K>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void fstatic_for(F &&f) {
    fstatic_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Coordinate c wrapped onto [0, L) for a periodic axis (true modulo), or
// flagged invalid on an open one.
__device__ __forceinline__ int fwrap(int c, int L, int per, bool &ok) {
    if (c >= 0 && c < L) return c;
    if (!per) {
        ok = false;
        return 0;
    }
    c %= L;
    return c < 0 ? c + L : c;
}

// Bilinear field of one site from a ring of three staged planes
// (plane[dz + 1] holds the plane at offset dz), row pitch P, the site at
// offset `at` of each plane.  Isotropic shells: the neighbours of a shell are
// summed first and the sum is multiplied by the shell's coupling once.
template <int KIND, typename T, bool ISO, int P, int NWT>
__device__ __forceinline__ void fused_bil(const T *const (&plane)[3], int at, int cstride, const FWeights<T, NWT> &W,
                                          T (&bil)[3]) {
    constexpr ShapeTable tb = FShape<KIND>::t;
    constexpr int NB = tb.nb;
    if constexpr (ISO) {
        constexpr int NSH = tb.nshell;
        T sh[NSH][3];
#pragma unroll
        for (int s = 0; s < NSH; ++s) sh[s][0] = sh[s][1] = sh[s][2] = T(0);
        fstatic_for<NB>([&](auto kc) __attribute__((always_inline)) {
            constexpr ZBond bd = FShape<KIND>::t.bonds[decltype(kc)::value];
            const T *p = plane[bd.dz + 1] + at + bd.dy * P + bd.dx;
#pragma unroll
            for (int c = 0; c < 3; ++c) sh[bd.shell][c] += p[c * cstride];
        });
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T v = W.w[0] * sh[0][c];
#pragma unroll
            for (int s = 1; s < NSH; ++s) v += W.w[s] * sh[s][c];
            bil[c] = v;
        }
    } else {
        bil[0] = bil[1] = bil[2] = T(0);
        fstatic_for<NB>([&](auto kc) __attribute__((always_inline)) {
            constexpr int kb = decltype(kc)::value;
            constexpr ZBond bd = FShape<KIND>::t.bonds[kb];
            const T *p = plane[bd.dz + 1] + at + bd.dy * P + bd.dx;
            const T s0 = p[0], s1 = p[cstride], s2 = p[2 * cstride];
            const T *J = &W.w[9 * kb];
            bil[0] += J[0] * s0 + J[1] * s1 + J[2] * s2;
            bil[1] += J[3] * s0 + J[4] * s1 + J[5] * s2;
            bil[2] += J[6] * s0 + J[7] * s1 + J[8] * s2;
        });
    }
}

template <int KIND, typename T, bool ISO, int NW, int NA>
__global__ __launch_bounds__(kFX *NW) void k_heun_fused(FArgs g, FConst fc,
                                                        FWeights<T, ISO ? make_shape(KIND).nshell
                                                                        : 9 * make_shape(KIND).nb> W) {
    static_assert(make_shape(KIND).nsub == 1 && make_shape(KIND).rx <= 1 && make_shape(KIND).ry <= 1 &&
                      make_shape(KIND).dzlo >= -1 && make_shape(KIND).dzhi <= 1,
                  "the fused Heun step handles single-sublattice shapes of range one cell");
    constexpr int SH = NW + 2;        // staged S^n rows
    constexpr int SPL = kSW * SH;     // staged plane, per component
    constexpr int TPL = kFX * NW;     // predicted plane, per component
    __shared__ T ls[4][3][SPL];
    __shared__ T lt[4][3][TPL];

    const int lane = threadIdx.x & (kFX - 1);
    const int row = threadIdx.x / kFX;
    const unsigned tile = blockIdx.x;
    const int x0 = (int)(tile % (unsigned)g.nbx) * kFXI;
    const int y0 = (int)((tile / (unsigned)g.nbx) % (unsigned)g.nby) * (NW - 2);
    const int zs = (int)(tile / ((unsigned)g.nbx * (unsigned)g.nby)) * g.zch;
    const int nz = min(g.zch, g.Lz - zs);
    const int64_t N = g.N;
    const int64_t pstride = (int64_t)g.Lx * g.Ly;

    // Staging slots: slot 0 is the thread's own predictor site (staged column
    // lane + 1, row row + 1); the 2 NW + 132 halo elements of the staged
    // plane are dealt to the first threads as slot 1.
    constexpr int HN = SPL - TPL;
    static_assert(HN <= kFX * NW, "halo must fit one slot per thread");
    int scol[2], srow[2];
    scol[0] = lane + 1;
    srow[0] = row + 1;
    const bool has1 = (int)threadIdx.x < HN;
    {
        const int h = has1 ? (int)threadIdx.x : 0;
        if (h < kSW) {
            srow[1] = 0;
            scol[1] = h;
        } else if (h < 2 * kSW) {
            srow[1] = SH - 1;
            scol[1] = h - kSW;
        } else {
            const int m = h - 2 * kSW;
            srow[1] = 1 + (m >> 1);
            scol[1] = (m & 1) ? kSW - 1 : 0;
        }
    }
    int64_t xy[2];
    bool xyok[2];
    int loff[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        bool ok = true;
        const int gx = fwrap(x0 - 2 + scol[s], g.Lx, g.per[0], ok);
        const int gy = fwrap(y0 - 2 + srow[s], g.Ly, g.per[1], ok);
        xy[s] = gx + (int64_t)g.Lx * gy;
        xyok[s] = ok;
        loff[s] = srow[s] * kSW + scol[s];
    }
    // the thread's predictor site in x/y (wrapped) and its corrector role
    bool pok = true;
    const int px = fwrap(x0 - 1 + lane, g.Lx, g.per[0], pok);
    const int py = fwrap(y0 - 1 + row, g.Ly, g.per[1], pok);
    const int cx = x0 - 1 + lane, cy = y0 - 1 + row;
    const bool corr = lane >= 1 && lane <= kFX - 2 && row >= 1 && row <= NW - 2 && cx < g.Lx && cy < g.Ly;

    double pre[2][3];
    auto fetch = [&](int L) __attribute__((always_inline)) {
        bool zok = true;
        const int gz = fwrap(zs - 2 + L, g.Lz, g.per[2], zok);
        const int64_t zo = pstride * gz;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const bool ok = zok && xyok[s] && (s == 0 || has1);
            const int64_t j = xy[s] + zo;
#pragma unroll
            for (int c = 0; c < 3; ++c) pre[s][c] = ok ? g.S[c * N + j] : 0.0;
        }
    };
    auto commit = [&](int L) __attribute__((always_inline)) {
        T *const base = &ls[L & 3][0][0];
#pragma unroll
        for (int c = 0; c < 3; ++c) base[c * SPL + loff[0]] = (T)pre[0][c];
        if (has1)
#pragma unroll
            for (int c = 0; c < 3; ++c) base[c * SPL + loff[1]] = (T)pre[1][c];
    };

    // Registers that carry a plane from one iteration to a later one, in two
    // sets used by alternate iterations (the loop below is unrolled by two):
    //   own[j]: FP64 S^n of the thread's site, read by the predictor of
    //     iteration k (plane k-1, set (k-1) & 1), then refilled with plane
    //     k+1 from the fetch;
    //   cP/cH/cT[j]: the corrector's P = S^n + dt/2 f(S^n), thermal field
    //     sigma eta and FP64 S~ of plane L, read by the corrector of iteration
    //     k (plane k-3) and then overwritten by the predictor (plane k-1), both
    //     of parity (k-1) & 1.
    double own[2][3];
    double cP[2][3], cH[2][3], cT[2][3];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) cP[j][c] = cH[j][c] = cT[j][c] = 0.0;

    fetch(0);
    commit(0);
    fetch(1);
    commit(1);
#pragma unroll
    for (int c = 0; c < 3; ++c) own[1][c] = pre[0][c];
    fetch(2);
    commit(2);
#pragma unroll
    for (int c = 0; c < 3; ++c) own[0][c] = pre[0][c];
    __syncthreads();

    const uint64_t nstep = fc.noise ? (fc.step_dev ? *fc.step_dev + g.step : g.step) : 0;
    const int lastL = nz + 3;  // last S^n plane a predictor needs
    auto iter = [&](int k, double (&oS)[3], double (&P)[3], double (&H)[3], double (&Tt)[3])
                    __attribute__((always_inline)) {
        const bool more = k + 1 <= lastL;
        if (more) fetch(k + 1);
        if (k >= 5 && corr) {
            // corrector of plane L = k - 3 (z = zs + k - 5)
            const int L = k - 3;
            const T *tp[3] = {&lt[(L - 1) & 3][0][0], &lt[L & 3][0][0], &lt[(L + 1) & 3][0][0]};
            T bil[3];
            fused_bil<KIND, T, ISO, kFX>(tp, row * kFX + lane, TPL, W, bil);
            double bt[3];
            fused_onsite<NA>(fc, Tt, bt);
            double B1[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) B1[c] = ((double)bil[c] + bt[c]) * fc.inv + H[c];
            double g1[3];
            llg_dir(Tt, B1, fc.alpha, g1);
            double pn[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) pn[c] = P[c] + fc.hdtp * g1[c];
            normalise3(pn);
            const int64_t i = cx + (int64_t)g.Lx * (cy + (int64_t)g.Ly * (zs + L - 2));
#pragma unroll
            for (int c = 0; c < 3; ++c) g.out[c * N + i] = pn[c];
        }
        if (k <= lastL) {
            // predictor of plane L = k - 1 (z = zs + k - 3) over the whole region
            const int L = k - 1;
            bool ok = pok;
            const int pz = fwrap(zs + L - 2, g.Lz, g.per[2], ok);
            const T *sp[3] = {&ls[(L - 1) & 3][0][0], &ls[L & 3][0][0], &ls[(L + 1) & 3][0][0]};
            T bil[3];
            fused_bil<KIND, T, ISO, kSW>(sp, (row + 1) * kSW + lane + 1, SPL, W, bil);
            double eta[3] = {0.0, 0.0, 0.0};
            if (fc.noise) {
                const int64_t i = px + (int64_t)g.Lx * (py + (int64_t)g.Ly * pz);
                // The key and step words are uniform.  Hiding them from the
                // loop optimiser here keeps the per-round keys and the first
                // round's product of the step word as scalar instructions in
                // the loop; hoisted, their twenty-odd values spill into
                // vector-lane storage and every use becomes a vector read.
                uint64_t sd = fc.seed, ns = nstep;
                asm volatile("" : "+s"(sd), "+s"(ns));
                thermal_eta(sd, ns, fc.tag, (uint64_t)i, eta);
            }
            double ba[3];
            fused_onsite<NA>(fc, oS, ba);
            double B[3], g0[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                H[c] = fc.sigma * eta[c];
                B[c] = ((double)bil[c] + ba[c]) * fc.inv + H[c];
            }
            llg_dir(oS, B, fc.alpha, g0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Tt[c] = oS[c] + fc.dtp * g0[c];
                P[c] = oS[c] + fc.hdtp * g0[c];
            }
            normalise3(Tt);
            T *const tb = &lt[L & 3][0][0];
#pragma unroll
            for (int c = 0; c < 3; ++c) tb[c * TPL + row * kFX + lane] = ok ? (T)Tt[c] : T(0);
        }
        if (more) {
            commit(k + 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) oS[c] = pre[0][c];
        }
        __syncthreads();
    };
#pragma unroll 1
    for (int k = 2; k <= nz + 4; k += 2) {
        iter(k, own[1], cP[1], cH[1], cT[1]);
        if (k + 1 <= nz + 4) iter(k + 1, own[0], cP[0], cH[0], cT[0]);
    }
}

template <int KIND, typename T, bool ISO, int NW>
hipError_t launch_fused_kind(const ZPlan &zp, const FArgs &a0, const FConst &fc, hipStream_t st) {
    constexpr int NWT = ISO ? make_shape(KIND).nshell : 9 * make_shape(KIND).nb;
    FWeights<T, NWT> W;
    for (int k = 0; k < NWT; ++k) W.w[k] = (T)(sizeof(T) == 4 ? (double)zp.wf[k] : zp.wd[k]);
    FArgs a = a0;
    a.nbx = (a.Lx + kFXI - 1) / kFXI;
    a.nby = (a.Ly + NW - 3) / (NW - 2);
    const int nzc = (a.Lz + a.zch - 1) / a.zch;
    const int64_t ntile = (int64_t)a.nbx * a.nby * nzc;
    if (ntile > 0x7fffffff) return hipErrorInvalidValue;
    if (fc.n_aniso == 0) k_heun_fused<KIND, T, ISO, NW, 0><<<(unsigned)ntile, kFX * NW, 0, st>>>(a, fc, W);
    else if (fc.n_aniso == 1) k_heun_fused<KIND, T, ISO, NW, 1><<<(unsigned)ntile, kFX * NW, 0, st>>>(a, fc, W);
    else k_heun_fused<KIND, T, ISO, NW, -1><<<(unsigned)ntile, kFX * NW, 0, st>>>(a, fc, W);
    return hipGetLastError();
}

// Rows per block: 16 wavefronts for FP32 nearest neighbours (106 KB of LDS,
// 125 VGPRs: four waves per SIMD) or 8 (zp.frows, chosen by the autotuner);
// 8 otherwise (FP64 planes take twice the LDS; the 26-neighbour shape needs
// more than 128 VGPRs).
template <typename T, bool ISO>
hipError_t launch_fused_t(const ZPlan &zp, const FArgs &a, const FConst &fc, hipStream_t st) {
    switch (zp.kind) {
    case SHAPE_SC_NN:
        if constexpr (sizeof(T) == 4) {
            if (zp.frows == 8) return launch_fused_kind<SHAPE_SC_NN, T, ISO, 8>(zp, a, fc, st);
            return launch_fused_kind<SHAPE_SC_NN, T, ISO, 16>(zp, a, fc, st);
        }
        return launch_fused_kind<SHAPE_SC_NN, T, ISO, 8>(zp, a, fc, st);
    case SHAPE_SC_3SH:
        if constexpr (ISO) return launch_fused_kind<SHAPE_SC_3SH, T, ISO, 8>(zp, a, fc, st);
        break;
    default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace

int fused_rows(const ZPlan &zp) {
    return (zp.kind == SHAPE_SC_NN && zp.prec == 1 && zp.frows != 8) ? 16 : 8;
}

bool fused_heun_supported(const ZPlan &zp, const Grid &g) {
    if (!zp.valid || g.n_sub != 1) return false;
    if (zp.kind == SHAPE_SC_NN) return true;
    return zp.kind == SHAPE_SC_3SH && zp.iso;
}

hipError_t heun_fused(const ZPlan &zp, const Grid &g, const Onsite &os, const HeunConst &hc, uint64_t step,
                      const double *S, double *out, hipStream_t st) {
    if (!fused_heun_supported(zp, g) || zp.zch < 1) return hipErrorInvalidValue;
    FArgs a{};
    a.Lx = g.Lx;
    a.Ly = g.Ly;
    a.Lz = g.Lz;
    for (int k = 0; k < 3; ++k) a.per[k] = g.per[k];
    a.N = g.N;
    a.zch = zp.zch;
    a.S = S;
    a.out = out;
    a.step = step;
    FConst fc{};
    fc.dtp = hc.dt * hc.pre;
    fc.hdtp = 0.5 * hc.dt * hc.pre;
    fc.alpha = hc.alpha;
    fc.inv = hc.inv_mumuB[0];
    fc.sigma = hc.sigma[0];
    fc.n_aniso = os.n_aniso;
    for (int l = 0; l < os.n_aniso && l < kMaxAniso; ++l) {
        fc.K2[l] = 2.0 * os.K[0][l];
        for (int c = 0; c < 3; ++c) fc.ax[l][c] = os.axis[0][l][c];
    }
    // the Zeeman term enters B = (b_bil + b_ani + b_Z) / (mu mu_B): it is
    // carried in the on-site sum, added after the anisotropy
    for (int c = 0; c < 3; ++c) fc.bz[c] = os.bz[0][c];
    fc.noise = hc.noise;
    fc.seed = hc.seed;
    fc.tag = hc.tag;
    fc.step_dev = hc.step_dev;
    if (zp.prec == 0) {
        if (zp.iso) return launch_fused_t<double, true>(zp, a, fc, st);
        return launch_fused_t<double, false>(zp, a, fc, st);
    }
    if (zp.iso) return launch_fused_t<float, true>(zp, a, fc, st);
    return launch_fused_t<float, false>(zp, a, fc, st);
}

}  // namespace spx
