// spx_gneb.hip -- batched geodesic nudged elastic band (GNEB) with velocity
// projection and the exponential-map retraction, for many images of many
// ragged lattices in one set of persistent launches (Methods, static
// optimisation and minimum-energy paths).
//
// Instances whose bond table has a z-march shell shape run an iteration as
// two passes of the stencil engine over their images, with no stored force:
//   pass A2 (all images)      field, energy, distance to the next image and,
//                             for interior images, the nine sums a.a, a.b,
//                             b.b, F.a, F.b, v.a, v.b, v.F, F.F with a, b the
//                             projected differences to the next and previous
//                             image (the improved tangent is w+ a + w- b, so
//                             its dot products follow from these once the
//                             energy weights w+- are known); one set per tile
//   reduce  (per image)       fixed order
//   scalars (per instance)    climbing image, tangent weights
//   scalars (per instance)    tau.tau, F.tau, v.tau, c_n, VP projection
//   pass C2 (interior images) field again, F_gneb = F + c_n tau^, VP velocity,
//                             exp-map step into the other buffer
//   reduce + scalars          max |F_gneb|, CI switch, convergence, buffer flip
// which moves 96 + 120 = 216 bytes per spin-image-iteration (pass A2 reads
// S_n, S_n-1, S_n+1 and v; pass C2 reads S_n, S_n-1, S_n+1 and writes v, S').
// Other instances (any bond table) use items: every (instance, image,
// 256-site tile) is one item of a flat list and each per-site pass is one
// grid-stride launch over the items of all instances:
//   pass A  (all images)      field, energy, projected force F, distance terms
//                             (the field from a batched z-march pass when the
//                             table has an FP64 shape, else gathered)
//   reduce  (per image)       E_n, d(Y_n, Y_n+1)^2           fixed order
//   scalars (per instance)    climbing image, tangent weights
//   pass B  (movable images)  tangent tau, dots v.F F.F tau.tau F.tau v.tau
//   reduce  (per image)
//   scalars (per instance)    c_n, VP projection v.F/F.F from image sums
//   pass C  (movable images)  F_gneb = F + c_n tau^, VP velocity, exp-map step
//   reduce + scalars          max |F_gneb|, CI switch, convergence, buffer flip
// and, for string-method instances (mode 4), the geodesic reparameterisation
//   distances (all images)    d(Y_n, Y_n+1)^2 of the displaced path
//   brackets  (per instance)  arc-length targets, bracketing image k, fraction f
//   interpolation             every spin of image n on the arc Y_k -> Y_k+1
// All per-instance control state lives on the device, so an iteration needs
// no host synchronisation and can be captured once in a hipGraph.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "spx_device.hpp"
#include "spx_ext.hpp"

namespace spx {
namespace {

constexpr int kGB = 256;  // sites per item / threads per block
constexpr int kMaxImages = 4096;  // images per instance (arc-length table in LDS)

// per-image statistics
// (the two-pass first pass fills IS_E .. IS_FF in this order; pass B fills
// IS_VF .. IS_VT)
enum { IS_E = 0, IS_D2, IS_AA, IS_AB, IS_BB, IS_FA, IS_FB, IS_VA, IS_VB, IS_VF, IS_FF, IS_TT, IS_FT, IS_VT, IS_COEF,
       IS_TN, IS_WP, IS_WM, IS_RD2, IS_RK, IS_RF, IS_FM, IS_N };
constexpr int kPassA2Values = IS_FF - IS_E + 1;
// Partial values of item or tile k start at partial[k * kPS] for every pass,
// so passes of different instances that run at the same time never overlap.
constexpr int kPS = kPassA2Values;
// per-instance state (ST_RDONE: the reparameterisation has seen ST_DONE)
enum { ST_PROJ = 0, ST_MAXF, ST_CI, ST_CION, ST_ITER, ST_DONE, ST_CUR, ST_RDONE, ST_N };
// mode of an instance (the ci_mode parameter)
enum { MODE_STRING = 4 };

struct GInst {
    Grid g;
    BondTable tb;
    const Onsite *os;     // device copy
    int n_img;
    int item0;            // first item (all images) of this instance
    int items_per_img;
    double *Y[2];         // image buffers [n_img][3][N]; Y[0] is the caller's
    double *V;            // velocities
    double *F;            // projected physical force, then nothing else
    double *img;          // [n_img][IS_N]
    double *st;           // [ST_N]
    double k, dt, mass, ci_on_below, tol;
    int ci_mode;
    const double *alpha;  // target arc-length fractions of the images [n_img]
    // bilinear field of every image from the batched z-march pass
    // ([n_img][3][N], FP64); NULL: pass A gathers the neighbours itself
    const double *Bbil;
    // > 0: the instance runs the two z-march passes, which leave one partial
    // set per tile (this many per image) in the image's first item slots; the
    // item passes skip it
    int zt_per_img;
};

struct GItem {
    int inst, img, site0, pad;
};

__device__ __forceinline__ double block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kGB / 64; ++k) t += red[k];
    return t;  // valid in thread 0
}

__device__ __forceinline__ double block_max(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kGB / 64; ++k) t = fmax(t, red[k]);
    return t;
}

__device__ __forceinline__ void ld3(const double *p, int64_t N, int64_t i, double v[3]) {
    v[0] = p[i];
    v[1] = p[N + i];
    v[2] = p[2 * N + i];
}

// geodesic angle atan2(|a x b|, a.b) (= arccos(a.b), accurate near 0 and pi)
__device__ __forceinline__ double angle3(const double a[3], const double b[3]) {
    const double c0 = a[1] * b[2] - a[2] * b[1];
    const double c1 = a[2] * b[0] - a[0] * b[2];
    const double c2 = a[0] * b[1] - a[1] * b[0];
    const double cc = c0 * c0 + c1 * c1 + c2 * c2;
    return atan2_nonneg(cc > 0.0 ? sqrt_pos(cc) : 0.0, a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
}

// Point at fraction t of the great-circle arc from a to b (unit vectors):
// cos(t w) a + sin(t w) e with e the unit tangent of b at a and w the angle
// between them.  Parallel spins (tangent part below 1e-10, a.b > 0) give a;
// antiparallel ones rotate by pi about normalize(a x e_k), e_k the Cartesian
// axis least aligned with a (first on ties).
__device__ __forceinline__ void geodesic_point(const double a[3], const double b[3], double t, double p[3]) {
    const double dot = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    double w[3] = {b[0] - dot * a[0], b[1] - dot * a[1], b[2] - dot * a[2]};
    const double wn2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double e[3], ang;
    if (wn2 < 1e-20) {  // |w| below 1e-10
        if (dot > 0) {
            for (int q = 0; q < 3; ++q) p[q] = a[q];
            return;
        }
        int kx = 0;
        double best = fabs(a[0]);
        if (fabs(a[1]) < best) { best = fabs(a[1]); kx = 1; }
        if (fabs(a[2]) < best) { kx = 2; }
        double ek[3] = {0, 0, 0};
        ek[kx] = 1.0;
        double ax[3] = {a[1] * ek[2] - a[2] * ek[1], a[2] * ek[0] - a[0] * ek[2], a[0] * ek[1] - a[1] * ek[0]};
        const double an = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
        for (int q = 0; q < 3; ++q) ax[q] /= an;
        e[0] = ax[1] * a[2] - ax[2] * a[1];
        e[1] = ax[2] * a[0] - ax[0] * a[2];
        e[2] = ax[0] * a[1] - ax[1] * a[0];
        ang = M_PI;
    } else {
        const double rn = rsqrt_pos(wn2);
        for (int q = 0; q < 3; ++q) e[q] = w[q] * rn;
        ang = atan2_nonneg(wn2 * rn, dot);
    }
    double cs, sn;  // of t ang, as sin and cos of pi (t ang / pi)
    sincospi_d(t * ang * (1.0 / M_PI), sn, cs);
    for (int q = 0; q < 3; ++q) p[q] = cs * a[q] + sn * e[q];
    normalise3(p);
}

// ---------------------------------------------------------------- pass A
__global__ __launch_bounds__(kGB) void k_gneb_a(const GInst *__restrict__ inst, const GItem *__restrict__ items,
                                                int n_items, double *__restrict__ partial) {
    __shared__ double red[kGB / 64];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const GItem itm = items[it];
        const GInst &G = inst[itm.inst];
        if (G.zt_per_img > 0) continue;  // done by the fused z-march pass (uniform over the block)
        double e = 0.0, d2 = 0.0;
        const bool active = G.st[ST_DONE] == 0.0;
        if (active) {
            const int cur = (int)G.st[ST_CUR];
            const int64_t N = G.g.N;
            const int64_t t = (int64_t)itm.site0 + threadIdx.x;
            if (t < N) {
                const double *S = G.Y[cur] + (int64_t)itm.img * 3 * N;
                const int a = (int)(t / G.g.M);
                int x, y, z;
                site_xyz(G.g, (int)(t - (int64_t)a * G.g.M), x, y, z);
                double acc[1][3];
                if (G.Bbil) {
                    const double *Bb = G.Bbil + (int64_t)itm.img * 3 * N;
                    ld3(Bb, N, t, acc[0]);
                } else {
                    const double *const src[1] = {S};
                    if (G.tb.iso) bil_sum<double, true, 1>(G.tb, G.g, a, x, y, z, src, acc);
                    else bil_sum<double, false, 1>(G.tb, G.g, a, x, y, z, src, acc);
                }
                double s[3], ba[3];
                ld3(S, N, t, s);
                aniso_field(*G.os, a, s, ba);
                double b[3];
                double sb = 0, sz = 0, sa = 0;
                for (int c = 0; c < 3; ++c) {
                    b[c] = acc[0][c] + ba[c] + G.os->bz[a][c];
                    sb += s[c] * acc[0][c];
                    sz += s[c] * G.os->bz[a][c];
                    sa += s[c] * ba[c];
                }
                e = -0.5 * sb - sz - 0.5 * sa;
                if (itm.img > 0 && itm.img < G.n_img - 1) {
                    const double bs = b[0] * s[0] + b[1] * s[1] + b[2] * s[2];
                    double *F = G.F + (int64_t)itm.img * 3 * N;
                    for (int c = 0; c < 3; ++c) F[c * N + t] = b[c] - bs * s[c];
                }
                if (itm.img < G.n_img - 1) {
                    double s2[3];
                    ld3(S + 3 * N, N, t, s2);
                    const double th = angle3(s, s2);
                    d2 = th * th;
                }
            }
        }
        const double es = block_sum(e, red);
        const double ds = block_sum(d2, red);
        if (threadIdx.x == 0) {
            partial[(size_t)it * kPS] = es;
            partial[(size_t)it * kPS + 1] = ds;
        }
    }
}

// per-image fixed-order reduction of `nv` partial values per item into
// img[IS_base + v]; one block per (instance, image) with a flat index
// Gates of the reparameterisation kernels: GATE_STRING runs them for string
// instances that have not finished, GATE_ALL for every instance (an explicit
// redistribution); the GNEB passes use GATE_ITER (unconverged instances).
enum { GATE_ITER = 0, GATE_STRING = 1, GATE_ALL = 2 };
__device__ __forceinline__ bool gate_open(const GInst &G, int gate) {
    if (gate == GATE_ALL) return true;
    if (gate == GATE_STRING) return G.ci_mode == MODE_STRING && G.st[ST_RDONE] == 0.0;
    return G.st[ST_DONE] == 0.0;
}

// Work index w -> item, images fastest: within each instance (whose items
// are stored image-major) the n_img items of one site block follow each
// other, and blocks take their work in XCD-contiguous ranges, so the
// neighbouring image that an item reads besides its own was mostly just read
// by the item before it, on the same XCD, and comes from its L2.  The
// instance of w is that of item w: both orders cover the same range per
// instance.
__device__ __forceinline__ int image_fastest_item(const GInst *__restrict__ inst, const GItem *__restrict__ items,
                                                  int w) {
    const GInst &G = inst[items[w].inst];
    const int local = w - G.item0, tile = local / G.n_img, img = local - tile * G.n_img;
    return G.item0 + img * G.items_per_img + tile;
}
__device__ __forceinline__ int xcd_block_index() {
    const int T = (int)gridDim.x, b = (int)blockIdx.x;
    const int q = T / 8, r = T % 8, k = b % 8;
    return k * q + (k < r ? k : r) + b / 8;
}

// nv_items / nv_tiles: partial values per item of the item passes / per tile
// of the two-pass instances (0: this reduction does not apply to them);
// items_only: the pass reduced was an item pass for every instance.
__global__ __launch_bounds__(kGB) void k_gneb_reduce(const GInst *__restrict__ inst, const int2 *__restrict__ imgs,
                                                     const double *__restrict__ partial, int nv_items, int nv_tiles,
                                                     int base, int only_movable, int gate, int take_max,
                                                     int items_only) {
    __shared__ double red[kGB / 64];
    const int2 ii = imgs[blockIdx.x];
    const GInst &G = inst[ii.x];
    if (!gate_open(G, gate)) return;
    if (only_movable && (ii.y == 0 || ii.y == G.n_img - 1)) return;
    const bool tiles = G.zt_per_img > 0 && !items_only;
    const int nv = tiles ? nv_tiles : nv_items;
    if (nv == 0) return;
    const int first = G.item0 + ii.y * G.items_per_img;
    const int count = tiles ? G.zt_per_img : G.items_per_img;
    for (int v = 0; v < nv; ++v) {
        double s = 0.0;
        for (int k = threadIdx.x; k < count; k += kGB) {
            const double x = partial[(size_t)(first + k) * kPS + v];
            s = take_max ? fmax(s, x) : s + x;
        }
        const double t = take_max ? block_max(s, red) : block_sum(s, red);
        if (threadIdx.x == 0) G.img[ii.y * IS_N + base + v] = t;
    }
}

// climbing image and tangent weights (Henkelman-Jonsson improved tangent);
// one block per instance, threads over the images
__global__ __launch_bounds__(kGB) void k_gneb_scalars1(const GInst *__restrict__ inst) {
    __shared__ double rv[kGB / 64];
    __shared__ int ri[kGB / 64];
    const GInst &G = inst[blockIdx.x];
    if (G.st[ST_DONE] != 0.0) return;
    double *im = G.img;
    const int M = G.n_img;
    for (int n = 1 + (int)threadIdx.x; n < M - 1; n += kGB) {
        double wp = 0.0, wm = 0.0;
        if (G.ci_mode != 3) {  // minimisation: no tangent, so no projection and no spring
            const double Ep = im[(n + 1) * IS_N + IS_E], Em = im[(n - 1) * IS_N + IS_E], E0 = im[n * IS_N + IS_E];
            if (Ep > E0 && E0 > Em) { wp = 1.0; wm = 0.0; }
            else if (Ep < E0 && E0 < Em) { wp = 0.0; wm = 1.0; }
            else {
                const double dmax = fmax(fabs(Ep - E0), fabs(Em - E0));
                const double dmin = fmin(fabs(Ep - E0), fabs(Em - E0));
                if (Ep > Em) { wp = dmax; wm = dmin; } else { wp = dmin; wm = dmax; }
            }
        }
        im[n * IS_N + IS_WP] = wp;
        im[n * IS_N + IS_WM] = wm;
    }
    // climbing image: the first movable image of highest energy
    int ci = -1;
    if (G.ci_mode == 2 || (G.ci_mode == 1 && G.st[ST_CION] != 0.0)) {
        double best = 0.0;
        for (int n = 1 + (int)threadIdx.x; n < M - 1; n += kGB) {
            const double e = im[n * IS_N + IS_E];
            if (ci < 0 || e > best) { best = e; ci = n; }
        }
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_down(best, off, 64);
            const int oi = __shfl_down(ci, off, 64);
            if (oi >= 0 && (ci < 0 || ob > best || (ob == best && oi < ci))) { best = ob; ci = oi; }
        }
        if (lane == 0) { rv[w] = best; ri[w] = ci; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 1; q < kGB / 64; ++q)
                if (ri[q] >= 0 && (ci < 0 || rv[q] > best || (rv[q] == best && ri[q] < ci))) { best = rv[q]; ci = ri[q]; }
        }
    }
    if (threadIdx.x == 0) G.st[ST_CI] = (double)ci;
}

// tangent of image n at site t (projected on the tangent plane, unnormalised)
__device__ __forceinline__ void tangent_at(const GInst &G, const double *S, int64_t N, int64_t t, double wp,
                                           double wm, const double s[3], double tau[3]) {
    double sp[3], sm[3];
    ld3(S + 3 * N, N, t, sp);
    ld3(S - 3 * N, N, t, sm);
    for (int c = 0; c < 3; ++c) tau[c] = wp * (sp[c] - s[c]) + wm * (s[c] - sm[c]);
    const double ts = tau[0] * s[0] + tau[1] * s[1] + tau[2] * s[2];
    for (int c = 0; c < 3; ++c) tau[c] -= ts * s[c];
}

// ---------------------------------------------------------------- pass B
__global__ __launch_bounds__(kGB) void k_gneb_b(const GInst *__restrict__ inst, const GItem *__restrict__ items,
                                                int n_items, double *__restrict__ partial) {
    __shared__ double red[kGB / 64];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const GItem itm = items[it];
        const GInst &G = inst[itm.inst];
        if (G.zt_per_img > 0) continue;  // two-pass instance (uniform over the block)
        double v5[5] = {0, 0, 0, 0, 0};
        const bool movable = itm.img > 0 && itm.img < G.n_img - 1;
        if (G.st[ST_DONE] == 0.0 && movable) {
            const int64_t N = G.g.N;
            const int64_t t = (int64_t)itm.site0 + threadIdx.x;
            if (t < N) {
                const int cur = (int)G.st[ST_CUR];
                const double *S = G.Y[cur] + (int64_t)itm.img * 3 * N;
                const double *im = G.img + itm.img * IS_N;
                double s[3], tau[3], f[3], v[3];
                ld3(S, N, t, s);
                tangent_at(G, S, N, t, im[IS_WP], im[IS_WM], s, tau);
                ld3(G.F + (int64_t)itm.img * 3 * N, N, t, f);
                // (string method: the velocities stay zero and are not read)
                if (G.ci_mode == MODE_STRING) v[0] = v[1] = v[2] = 0.0;
                else ld3(G.V + (int64_t)itm.img * 3 * N, N, t, v);
                // in the order of the image slots IS_VF, IS_FF, IS_TT, IS_FT, IS_VT
                for (int c = 0; c < 3; ++c) {
                    v5[0] += v[c] * f[c];
                    v5[1] += f[c] * f[c];
                    v5[2] += tau[c] * tau[c];
                    v5[3] += f[c] * tau[c];
                    v5[4] += v[c] * tau[c];
                }
            }
        }
        for (int q = 0; q < 5; ++q) {
            const double r = block_sum(v5[q], red);
            if (threadIdx.x == 0) partial[(size_t)it * kPS + q] = r;
        }
    }
}

// GNEB coefficients c_n and the VP projection from the image sums:
// F_gneb = F + c_n tau^, c_n = -2 F.tau^ on the climbing image, else
// -F.tau^ + k (d_n - d_{n-1});  v.F_gneb and F_gneb.F_gneb follow in closed form.
// One block per instance, threads over the images, fixed-order block sums.
__global__ __launch_bounds__(kGB) void k_gneb_scalars2(const GInst *__restrict__ inst) {
    __shared__ double red[kGB / 64];
    const GInst &G = inst[blockIdx.x];
    if (G.st[ST_DONE] != 0.0) return;
    double *im = G.img;
    const int ci = (int)G.st[ST_CI];
    double P = 0.0, Q = 0.0;
    for (int n = 1 + (int)threadIdx.x; n + 1 < G.n_img; n += kGB) {
        double *r = im + n * IS_N;
        if (G.zt_per_img > 0) {
            // two-pass instance: tau = w+ a + w- b
            const double wp = r[IS_WP], wm = r[IS_WM];
            r[IS_TT] = wp * wp * r[IS_AA] + 2.0 * wp * wm * r[IS_AB] + wm * wm * r[IS_BB];
            r[IS_FT] = wp * r[IS_FA] + wm * r[IS_FB];
            r[IS_VT] = wp * r[IS_VA] + wm * r[IS_VB];
        }
        const double tn = sqrt(r[IS_TT]);
        r[IS_TN] = tn;
        const double ft = tn > 0.0 ? r[IS_FT] / tn : 0.0;
        const double vt = tn > 0.0 ? r[IS_VT] / tn : 0.0;
        double c;
        if (n == ci) c = -2.0 * ft;
        else if (G.ci_mode == MODE_STRING) c = -ft;  // only the reported force is projected
        else c = -ft + G.k * (sqrt(im[n * IS_N + IS_D2]) - sqrt(im[(n - 1) * IS_N + IS_D2]));
        if (!(tn > 0.0)) c = 0.0;
        r[IS_COEF] = c;
        P += r[IS_VF] + c * vt;
        Q += r[IS_FF] + 2.0 * c * ft + c * c;
    }
    const double Ps = block_sum(P, red);
    const double Qs = block_sum(Q, red);
    if (threadIdx.x == 0) G.st[ST_PROJ] = (G.ci_mode != MODE_STRING && Ps > 0.0 && Qs > 0.0) ? Ps / Qs : 0.0;
}

// ---------------------------------------------------------------- pass C
__global__ __launch_bounds__(kGB) void k_gneb_c(const GInst *__restrict__ inst, const GItem *__restrict__ items,
                                                int n_items, double *__restrict__ partial) {
    __shared__ double red[kGB / 64];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const GItem itm = items[it];
        const GInst &G = inst[itm.inst];
        if (G.zt_per_img > 0) continue;  // two-pass instance (uniform over the block)
        double fm = 0.0;
        const bool movable = itm.img > 0 && itm.img < G.n_img - 1;
        if (G.st[ST_DONE] == 0.0 && movable) {
            const int64_t N = G.g.N;
            const int64_t t = (int64_t)itm.site0 + threadIdx.x;
            if (t < N) {
                const int cur = (int)G.st[ST_CUR];
                const int64_t off = (int64_t)itm.img * 3 * N;
                const double *S = G.Y[cur] + off;
                const double *im = G.img + itm.img * IS_N;
                double s[3], tau[3], f[3];
                ld3(S, N, t, s);
                tangent_at(G, S, N, t, im[IS_WP], im[IS_WM], s, tau);
                ld3(G.F + off, N, t, f);
                const double tn = im[IS_TN], c = im[IS_COEF];
                const double proj = G.st[ST_PROJ];
                double u[3];
                double f2 = 0.0;
                const bool string = G.ci_mode == MODE_STRING;
                for (int q = 0; q < 3; ++q) {
                    const double th = tn > 0.0 ? tau[q] / tn : 0.0;
                    const double ft = f[q] + c * th;
                    f2 += ft * ft;
                    // string method: displacement by the projected physical
                    // force itself, no velocity memory
                    const double v = string ? 0.0 : proj * ft + (G.dt / G.mass) * ft;
                    if (!string) G.V[off + q * N + t] = v;  // string method: V stays zero
                    u[q] = string ? G.dt * f[q] : G.dt * v;
                }
                fm = sqrt(f2);
                if (!string) {
                    const double us = u[0] * s[0] + u[1] * s[1] + u[2] * s[2];
                    for (int q = 0; q < 3; ++q) u[q] -= us * s[q];
                }
                // exponential map cos|u| S + sin|u| u/|u|, then renormalise
                const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                double o[3];
                if (un == 0.0) {
                    o[0] = s[0]; o[1] = s[1]; o[2] = s[2];
                } else {
                    const double cs = cos(un), sn = sin(un) / un;
                    for (int q = 0; q < 3; ++q) o[q] = cs * s[q] + sn * u[q];
                    normalise3(o);
                }
                double *Sn = G.Y[cur ^ 1] + off;
                for (int q = 0; q < 3; ++q) Sn[q * N + t] = o[q];
            }
        }
        const double r = block_max(fm, red);
        if (threadIdx.x == 0) partial[(size_t)it * kPS] = r;
    }
}

// max |F_gneb| per instance (from the per-image maxima), climbing-image
// switch, convergence, buffer flip
__global__ __launch_bounds__(kGB) void k_gneb_finish(const GInst *__restrict__ inst) {
    __shared__ double red[kGB / 64];
    const GInst &G = inst[blockIdx.x];
    if (G.st[ST_DONE] != 0.0) return;
    double m = 0.0;
    for (int n = 1 + (int)threadIdx.x; n + 1 < G.n_img; n += kGB) m = fmax(m, G.img[n * IS_N + IS_FM]);
    const double mx = block_max(m, red);
    if (threadIdx.x == 0) {
        G.st[ST_MAXF] = mx;
        G.st[ST_ITER] += 1.0;
        G.st[ST_CUR] = 1.0 - G.st[ST_CUR];
        const bool ci_ready = G.ci_mode != 1 || G.st[ST_CION] != 0.0;
        if (G.ci_mode == 1 && G.st[ST_CION] == 0.0 && mx < G.ci_on_below) G.st[ST_CION] = 1.0;
        if (G.tol > 0.0 && mx < G.tol && ci_ready) G.st[ST_DONE] = 1.0;
    }
}

// bring the state back to the caller's buffer Y[0] (after an odd number of flips)
__global__ __launch_bounds__(kGB) void k_gneb_copyback(const GInst *__restrict__ inst, const GItem *__restrict__ items,
                                                       int n_items) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const GItem itm = items[it];
        const GInst &G = inst[itm.inst];
        if (G.st[ST_CUR] == 0.0) continue;
        const int64_t N = G.g.N;
        const int64_t t = (int64_t)itm.site0 + threadIdx.x;
        if (t >= N) continue;
        const int64_t off = (int64_t)itm.img * 3 * N;
        for (int q = 0; q < 3; ++q) G.Y[0][off + q * N + t] = G.Y[1][off + q * N + t];
    }
}

__global__ void k_gneb_cur_reset(const GInst *__restrict__ inst, int n_inst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_inst) inst[k].st[ST_CUR] = 0.0;
}

// Geodesic initial path from the end images of Y[0]: image n at t = n/(n_img-1)
// on each spin's great circle; antiparallel pairs rotate about
// normalize(S_A x e_k), e_k the Cartesian axis least aligned with S_A.  Also
// copies the end images into Y[1] and clears the velocities.
__global__ __launch_bounds__(kGB) void k_gneb_geodesic(const GInst *__restrict__ inst, const GItem *__restrict__ items,
                                                       int n_items) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const GItem itm = items[it];
        const GInst &G = inst[itm.inst];
        const int64_t N = G.g.N;
        const int64_t t = (int64_t)itm.site0 + threadIdx.x;
        if (t >= N) continue;
        const int64_t off = (int64_t)itm.img * 3 * N;
        const int last = G.n_img - 1;
        double a[3], b[3], p[3];
        ld3(G.Y[0], N, t, a);
        ld3(G.Y[0] + (int64_t)last * 3 * N, N, t, b);
        if (itm.img == 0 || itm.img == last) {
            const double *src = itm.img == 0 ? a : b;
            for (int q = 0; q < 3; ++q) p[q] = src[q];
        } else {
            geodesic_point(a, b, (double)itm.img / (double)last, p);
        }
        for (int q = 0; q < 3; ++q) {
            G.Y[0][off + q * N + t] = p[q];
            G.Y[1][off + q * N + t] = p[q];
            G.V[off + q * N + t] = 0.0;
        }
    }
}

// ------------------------------------------ geodesic reparameterisation
// d(Y_n, Y_n+1)^2 of the current buffer, per item (image n < n_img - 1)
__global__ __launch_bounds__(kGB) void k_gneb_rdist(const GInst *__restrict__ inst, const GItem *__restrict__ items,
                                                    int n_items, double *__restrict__ partial, int gate) {
    __shared__ double red[kGB / 64];
    for (int w = xcd_block_index(); w < n_items; w += gridDim.x) {
        const int it = image_fastest_item(inst, items, w);
        const GItem itm = items[it];
        const GInst &G = inst[itm.inst];
        double d2 = 0.0;
        if (gate_open(G, gate) && itm.img < G.n_img - 1) {
            const int64_t N = G.g.N;
            const int64_t t = (int64_t)itm.site0 + threadIdx.x;
            if (t < N) {
                const double *S = G.Y[(int)G.st[ST_CUR]] + (int64_t)itm.img * 3 * N;
                double s[3], s2[3];
                ld3(S, N, t, s);
                ld3(S + 3 * N, N, t, s2);
                const double th = angle3(s, s2);
                d2 = th * th;
            }
        }
        const double ds = block_sum(d2, red);
        if (threadIdx.x == 0) partial[(size_t)it * kPS] = ds;
    }
}

// Arc-length coordinates s_n (cumulative distances, summed in image order
// in LDS), targets alpha_n s_last, and for every movable image the last image
// k <= n_img - 2 with s_k <= target and the fraction f = (target - s_k) /
// (s_k+1 - s_k) in [0, 1].  One block per instance, threads over the images.
__global__ __launch_bounds__(kGB) void k_gneb_rscalars(const GInst *__restrict__ inst, int gate) {
    __shared__ double sc[kMaxImages];
    const GInst &G = inst[blockIdx.x];
    if (!gate_open(G, gate)) return;
    double *im = G.img;
    const int M = G.n_img;
    for (int n = (int)threadIdx.x; n + 1 < M; n += kGB) sc[n + 1] = sqrt(im[n * IS_N + IS_RD2]);
    __syncthreads();
    if (threadIdx.x == 0) {
        sc[0] = 0.0;
        for (int n = 1; n < M; ++n) sc[n] += sc[n - 1];
    }
    __syncthreads();
    const double total = sc[M - 1];
    for (int n = 1 + (int)threadIdx.x; n + 1 < M; n += kGB) {
        const double target = G.alpha[n] * total;
        int kk = 0;
        while (kk + 1 < M - 1 && sc[kk + 1] <= target) ++kk;
        const double gap = sc[kk + 1] - sc[kk];
        double f = gap > 0.0 ? (target - sc[kk]) / gap : 0.0;
        f = fmin(fmax(f, 0.0), 1.0);
        im[n * IS_N + IS_RK] = (double)kk;
        im[n * IS_N + IS_RF] = f;
    }
}

// New path into the other buffer: movable image n at fraction f of every
// spin's arc from Y_k to Y_k+1; end images copied.  An explicit
// redistribution clears the velocities; string-method instances never write
// them (they stay zero from set-up or the last parameter change).
__global__ __launch_bounds__(kGB) void k_gneb_reparam(const GInst *__restrict__ inst, const GItem *__restrict__ items,
                                                      int n_items, int gate) {
    for (int w = xcd_block_index(); w < n_items; w += gridDim.x) {
        const GItem itm = items[image_fastest_item(inst, items, w)];
        const GInst &G = inst[itm.inst];
        if (!gate_open(G, gate)) continue;
        const int64_t N = G.g.N;
        const int64_t t = (int64_t)itm.site0 + threadIdx.x;
        if (t >= N) continue;
        const int cur = (int)G.st[ST_CUR];
        const int64_t off = (int64_t)itm.img * 3 * N;
        double p[3];
        if (itm.img == 0 || itm.img == G.n_img - 1) {
            ld3(G.Y[cur] + off, N, t, p);
        } else {
            const double *im = G.img + itm.img * IS_N;
            const int kk = (int)im[IS_RK];
            double a[3], b[3];
            ld3(G.Y[cur] + (int64_t)kk * 3 * N, N, t, a);
            ld3(G.Y[cur] + (int64_t)(kk + 1) * 3 * N, N, t, b);
            geodesic_point(a, b, im[IS_RF], p);
        }
        double *Yn = G.Y[cur ^ 1] + off;
        for (int q = 0; q < 3; ++q) Yn[q * N + t] = p[q];
        if (gate == GATE_ALL)
            for (int q = 0; q < 3; ++q) G.V[off + q * N + t] = 0.0;
    }
}

__global__ void k_gneb_rflip(const GInst *__restrict__ inst, int n_inst, int gate) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_inst) return;
    const GInst &G = inst[k];
    if (!gate_open(G, gate)) return;
    G.st[ST_CUR] = 1.0 - G.st[ST_CUR];
    if (gate == GATE_STRING) G.st[ST_RDONE] = G.st[ST_DONE];
}

// per-instance state reset (iteration counter, CI switch, convergence)
__global__ void k_gneb_reset(const GInst *__restrict__ inst, int n_inst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_inst) return;
    for (int q = 0; q < ST_N; ++q) inst[k].st[q] = 0.0;
    inst[k].st[ST_CI] = -1.0;
}

unsigned grid_for(int n_items) {
    return (unsigned)std::max(1, std::min(n_items, 8192));
}

}  // namespace
}  // namespace spx

using namespace spx;

struct spx_gneb {
    int n_inst = 0;
    std::vector<GInst> hinst;
    std::vector<int> n_img;
    std::vector<double *> caller;
    GInst *d_inst = nullptr;
    GItem *d_items = nullptr;
    int n_items = 0;
    int2 *d_imgs = nullptr;   // (instance, image) of every image
    int n_imgs = 0;
    double *d_partial = nullptr;
    std::vector<void *> owned;  // library allocations
    float *d_tvals = nullptr;   // reaction coordinates for the learned init
    int max_img = 0;
    hipGraphExec_t graph = nullptr;
    hipStream_t cap_stream = nullptr;  // library-owned capture stream (the caller's may be the null stream)
    int use_graph = 1;
    // Parallel branches of the captured iteration: one stream per instance,
    // a fork event and per-instance join events for each of the two passes.
    std::vector<hipStream_t> side;
    hipEvent_t fork_ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> join_ev[2];
    bool branch = false;  // set while an iteration is being captured with branches
    std::vector<ZPlan> zplan;  // per instance: FP64 z-march plan (used when its Bbil or zt_per_img is set)
    std::vector<Onsite> hos;   // per instance: host copy of the on-site tables (fused first pass)
};

namespace {

spx_status gneb_alloc(spx_gneb *g, void **p, size_t bytes, const char *what) {
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return set_error(SPX_ERR_OUT_OF_MEMORY, std::string("hipMalloc failed for ") + what);
    }
    g->owned.push_back(*p);
    return SPX_OK;
}

void gneb_free(spx_gneb *g) {
    if (g->graph) (void)hipGraphExecDestroy(g->graph);
    g->graph = nullptr;
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    g->cap_stream = nullptr;
    for (hipStream_t s : g->side)
        if (s) (void)hipStreamDestroy(s);
    g->side.clear();
    for (int p = 0; p < 2; ++p) {
        if (g->fork_ev[p]) (void)hipEventDestroy(g->fork_ev[p]);
        g->fork_ev[p] = nullptr;
        for (hipEvent_t e : g->join_ev[p])
            if (e) (void)hipEventDestroy(e);
        g->join_ev[p].clear();
    }
    for (void *p : g->owned) (void)hipFree(p);
    g->owned.clear();
}

// Arguments of the two z-march passes of instance k.
GnebPassArgs pass_args(const spx_gneb *g, int k) {
    const GInst &G = g->hinst[k];
    GnebPassArgs a{};
    a.n_img = G.n_img;
    a.item0 = G.item0;
    a.items_per_img = G.items_per_img;
    a.Y0 = G.Y[0];
    a.Y1 = G.Y[1];
    a.V = G.V;
    a.cur = G.st + ST_CUR;
    a.done = G.st + ST_DONE;
    a.img = G.img;
    a.st = G.st;
    a.slots = GnebSlots{IS_N, IS_WP, IS_WM, IS_TN, IS_COEF, ST_PROJ};
    a.dt = G.dt;
    a.mass = G.mass;
    a.string = G.ci_mode == MODE_STRING ? 1 : 0;
    a.partial = g->d_partial;
    return a;
}

// Enqueue the geodesic reparameterisation of the instances the gate admits.
hipError_t enqueue_reparam(spx_gneb *g, int gate, hipStream_t st) {
    const unsigned gi = grid_for(g->n_items);
    const unsigned gs = (unsigned)((g->n_inst + 63) / 64);
    k_gneb_rdist<<<gi, kGB, 0, st>>>(g->d_inst, g->d_items, g->n_items, g->d_partial, gate);
    k_gneb_reduce<<<g->n_imgs, kGB, 0, st>>>(g->d_inst, g->d_imgs, g->d_partial, 1, 1, IS_RD2, 0, gate, 0, 1);
    k_gneb_rscalars<<<g->n_inst, kGB, 0, st>>>(g->d_inst, gate);
    k_gneb_reparam<<<gi, kGB, 0, st>>>(g->d_inst, g->d_items, g->n_items, gate);
    k_gneb_rflip<<<gs, 64, 0, st>>>(g->d_inst, g->n_inst, gate);
    return hipGetLastError();
}

// Enqueue one GNEB iteration (all instances) on stream st.
GnebPassArgs pass_args(const spx_gneb *g, int k);

// Enqueue one z-march pass of every instance that has one: in turn on st,
// or, while g->branch is set (capture), each instance on its own stream
// between a fork from st and a join back into it, so that the graph runs
// the instances' passes side by side and the small lattices' blocks fill
// the chip beside the large one's.  The instances share no buffer.
constexpr int kMaxBranches = 8;
template <typename F>
hipError_t per_instance(spx_gneb *g, int pass, hipStream_t st, F launch) {
    if (!g->branch) {
        for (int k = 0; k < g->n_inst; ++k) {
            const hipError_t e = launch(k, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    hipError_t e = hipEventRecord(g->fork_ev[pass], st);
    for (int k = 0; k < g->n_inst && e == hipSuccess; ++k) {
        e = hipStreamWaitEvent(g->side[k], g->fork_ev[pass], 0);
        if (e == hipSuccess) e = launch(k, g->side[k]);
        if (e == hipSuccess) e = hipEventRecord(g->join_ev[pass][k], g->side[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, g->join_ev[pass][k], 0);
    }
    return e;
}

hipError_t enqueue_iteration(spx_gneb *g, hipStream_t st) {
    const unsigned gi = grid_for(g->n_items);
    bool any_items = false;  // an instance that runs the item passes
    for (const GInst &G : g->hinst) any_items = any_items || G.zt_per_img == 0;
    hipError_t e0 = per_instance(g, 0, st, [&](int k, hipStream_t s) {
        const GInst &G = g->hinst[k];
        if (G.zt_per_img > 0) return zmarch_gneb_pass(0, g->zplan[k], G.g, g->hos[k], pass_args(g, k), s);
        if (G.Bbil)
            return zmarch_bil_images(g->zplan[k], G.g, G.n_img, G.Y[0], G.Y[1], G.st + ST_CUR, G.st + ST_DONE,
                                     (double *)G.Bbil, s);
        return hipSuccess;
    });
    if (e0 != hipSuccess) return e0;
    if (any_items) k_gneb_a<<<gi, kGB, 0, st>>>(g->d_inst, g->d_items, g->n_items, g->d_partial);
    k_gneb_reduce<<<g->n_imgs, kGB, 0, st>>>(g->d_inst, g->d_imgs, g->d_partial, 2, kPassA2Values, IS_E, 0, GATE_ITER,
                                             0, 0);
    k_gneb_scalars1<<<g->n_inst, kGB, 0, st>>>(g->d_inst);
    if (any_items) {
        k_gneb_b<<<gi, kGB, 0, st>>>(g->d_inst, g->d_items, g->n_items, g->d_partial);
        k_gneb_reduce<<<g->n_imgs, kGB, 0, st>>>(g->d_inst, g->d_imgs, g->d_partial, 5, 0, IS_VF, 1, GATE_ITER, 0, 0);
    }
    k_gneb_scalars2<<<g->n_inst, kGB, 0, st>>>(g->d_inst);
    if (any_items) k_gneb_c<<<gi, kGB, 0, st>>>(g->d_inst, g->d_items, g->n_items, g->d_partial);
    hipError_t e1 = per_instance(g, 1, st, [&](int k, hipStream_t s) {
        const GInst &G = g->hinst[k];
        if (G.zt_per_img == 0) return hipSuccess;
        return zmarch_gneb_pass(1, g->zplan[k], G.g, g->hos[k], pass_args(g, k), s);
    });
    if (e1 != hipSuccess) return e1;
    k_gneb_reduce<<<g->n_imgs, kGB, 0, st>>>(g->d_inst, g->d_imgs, g->d_partial, 1, 1, IS_FM, 1, GATE_ITER, 1, 0);
    k_gneb_finish<<<g->n_inst, kGB, 0, st>>>(g->d_inst);
    bool any_string = false;
    for (const GInst &G : g->hinst) any_string = any_string || G.ci_mode == MODE_STRING;
    if (any_string) {
        hipError_t e = enqueue_reparam(g, GATE_STRING, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace

extern "C" {

spx_status spx_gneb_create(spx_ham *const *H, int32_t n_inst, double *const *images, const int32_t *n_img,
                           const spx_gneb_params *p, void *stream, spx_gneb **out) {
    if (!out) return set_error(SPX_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!H || !images || !n_img || !p || n_inst < 1) return set_error(SPX_ERR_INVALID_ARG, "bad GNEB arguments");
    if (!(p->vp_dt > 0.0) || !(p->vp_mass > 0.0) || !(p->spring_k >= 0.0))
        return set_error(SPX_ERR_INVALID_ARG, "vp_dt, vp_mass must be > 0 and spring_k >= 0");
    if (p->ci_mode < 0 || p->ci_mode > 4) return set_error(SPX_ERR_INVALID_ARG, "ci_mode must be 0 .. 4");
    hipStream_t st = (hipStream_t)stream;
    spx_gneb *g = new spx_gneb();
    g->n_inst = n_inst;
    std::vector<GItem> items;
    std::vector<int2> imgs;
    std::vector<Onsite> onsites(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        HamView v;
        spx_status s = get_ham_view(H[k], v);
        if (s != SPX_OK) { delete g; return s; }
        if (v.field_prec != SPX_FP64) {
            delete g;
            return set_error(SPX_ERR_INVALID_ARG, "GNEB needs Hamiltonians with field_prec SPX_FP64");
        }
        if (v.dip) {
            delete g;
            return set_error(SPX_ERR_UNSUPPORTED, "GNEB with the dipolar term is not supported");
        }
        if (v.pl) {
            delete g;
            return set_error(SPX_ERR_UNSUPPORTED, "GNEB needs a lattice Hamiltonian, not a pair list");
        }
        if (n_img[k] < 3 || n_img[k] > kMaxImages || !images[k]) {
            delete g;
            return set_error(SPX_ERR_INVALID_ARG, "each GNEB instance needs 3 .. 4096 images and a buffer");
        }
        GInst gi{};
        gi.g = v.grid;
        gi.tb = v.tab;
        gi.n_img = n_img[k];
        gi.items_per_img = (int)((v.grid.N + kGB - 1) / kGB);
        gi.item0 = (int)items.size();
        gi.k = p->spring_k;
        gi.dt = p->vp_dt;
        gi.mass = p->vp_mass;
        gi.ci_mode = p->ci_mode;
        gi.ci_on_below = p->ci_on_below;
        gi.tol = p->tol_force;
        onsites[k] = v.onsite;
        g->hos.push_back(v.onsite);
        // the batched z-march field pass needs an FP64 plan of the table
        gi.Bbil = nullptr;
        g->zplan.push_back(v.zp64 ? *v.zp64 : ZPlan{});
        if (v.zp64) g->zplan.back().zch = 16;
        for (int n = 0; n < n_img[k]; ++n) {
            imgs.push_back(make_int2(k, n));
            for (int b = 0; b < gi.items_per_img; ++b) items.push_back(GItem{k, n, b * kGB, 0});
        }
        g->hinst.push_back(gi);
        g->n_img.push_back(n_img[k]);
        g->caller.push_back(images[k]);
    }
    if (items.size() > (size_t)INT32_MAX / 8) {
        delete g;
        return set_error(SPX_ERR_INVALID_ARG, "too many GNEB work items");
    }
    g->n_items = (int)items.size();
    g->n_imgs = (int)imgs.size();
    spx_status s = SPX_OK;
    Onsite *d_os = nullptr;
    s = gneb_alloc(g, (void **)&d_os, sizeof(Onsite) * n_inst, "GNEB on-site tables");
    for (int k = 0; k < n_inst && s == SPX_OK; ++k) {
        GInst &gi = g->hinst[k];
        const size_t n3 = (size_t)3 * gi.g.N * gi.n_img;
        gi.os = d_os + k;
        gi.Y[0] = images[k];
        if ((s = gneb_alloc(g, (void **)&gi.Y[1], n3 * sizeof(double), "GNEB image buffer")) != SPX_OK) break;
        if ((s = gneb_alloc(g, (void **)&gi.V, n3 * sizeof(double), "GNEB velocities")) != SPX_OK) break;
        if ((s = gneb_alloc(g, (void **)&gi.img, sizeof(double) * IS_N * gi.n_img, "GNEB image stats")) != SPX_OK) break;
        if ((s = gneb_alloc(g, (void **)&gi.st, sizeof(double) * ST_N, "GNEB state")) != SPX_OK) break;
        if ((s = gneb_alloc(g, (void **)&gi.alpha, sizeof(double) * gi.n_img, "GNEB image spacing")) != SPX_OK) break;
        const ZPlan &zp = g->zplan[k];
        gi.zt_per_img = 0;
        gi.F = nullptr;
        if (zp.valid && zp.prec == 0) g->zplan[k].txw = zmarch_gneb_width(zp, gi.g);
        if (zp.valid && zp.prec == 0 && zmarch_gneb_tiles(zp, gi.g) <= gi.items_per_img) {
            gi.zt_per_img = zmarch_gneb_tiles(zp, gi.g);  // the two z-march passes; no stored force
        } else {
            g->zplan[k].txw = 64;
            if ((s = gneb_alloc(g, (void **)&gi.F, n3 * sizeof(double), "GNEB forces")) != SPX_OK) break;
            if (zp.valid &&
                (s = gneb_alloc(g, (void **)&gi.Bbil, n3 * sizeof(double), "GNEB bilinear field")) != SPX_OK)
                break;
        }
    }
    if (s == SPX_OK) s = gneb_alloc(g, (void **)&g->d_inst, sizeof(GInst) * n_inst, "GNEB instances");
    if (s == SPX_OK) s = gneb_alloc(g, (void **)&g->d_items, sizeof(GItem) * items.size(), "GNEB items");
    if (s == SPX_OK) s = gneb_alloc(g, (void **)&g->d_imgs, sizeof(int2) * imgs.size(), "GNEB image list");
    if (s == SPX_OK)
        s = gneb_alloc(g, (void **)&g->d_partial, sizeof(double) * kPassA2Values * items.size(), "GNEB partials");
    for (int k = 0; k < n_inst; ++k) g->max_img = std::max(g->max_img, n_img[k]);
    if (s == SPX_OK) s = gneb_alloc(g, (void **)&g->d_tvals, sizeof(float) * g->max_img * n_inst, "GNEB t values");
    if (s != SPX_OK) {
        gneb_free(g);
        delete g;
        return s;
    }
    // equal arc-length spacing until spx_gneb_set_spacing says otherwise
    std::vector<std::vector<double>> alpha0(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        alpha0[k].resize(n_img[k]);
        for (int n = 0; n < n_img[k]; ++n) alpha0[k][n] = (double)n / (double)(n_img[k] - 1);
    }
    hipError_t e = hipMemcpyAsync(d_os, onsites.data(), sizeof(Onsite) * n_inst, hipMemcpyHostToDevice, st);
    for (int k = 0; k < n_inst && e == hipSuccess; ++k)
        e = hipMemcpyAsync((void *)g->hinst[k].alpha, alpha0[k].data(), sizeof(double) * n_img[k],
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_inst, g->hinst.data(), sizeof(GInst) * n_inst, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_items, items.data(), sizeof(GItem) * items.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_imgs, imgs.data(), sizeof(int2) * imgs.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        k_gneb_reset<<<(n_inst + 63) / 64, 64, 0, st>>>(g->d_inst, n_inst);
        e = hipGetLastError();
    }
    // both buffers start from the caller's images, velocities at rest
    for (int k = 0; k < n_inst && e == hipSuccess; ++k) {
        const GInst &gi = g->hinst[k];
        const size_t bytes = sizeof(double) * 3 * gi.g.N * gi.n_img;
        e = hipMemcpyAsync(gi.Y[1], gi.Y[0], bytes, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemsetAsync(gi.V, 0, bytes, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        gneb_free(g);
        delete g;
        return set_hip_error(e, "spx_gneb_create");
    }
    register_handle(g);
    *out = g;
    return SPX_OK;
}

spx_status spx_gneb_destroy(spx_gneb *g) {
    if (!handle_alive(g)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_gneb handle");
    unregister_handle(g);
    (void)hipDeviceSynchronize();
    gneb_free(g);
    delete g;
    return SPX_OK;
}

spx_status spx_gneb_init_path(spx_gneb *g, int32_t method, spx_net *net, const float *params, void *stream) {
    if (!handle_alive(g)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_gneb handle");
    if (method != 0 && method != 1) return set_error(SPX_ERR_INVALID_ARG, "method must be 0 (geodesic) or 1 (learned)");
    if (method == 1) {
        if (!net_alive(net) || !params) return set_error(SPX_ERR_INVALID_ARG, "learned init needs a network and parameters");
        for (const GInst &gi : g->hinst)
            if (gi.g.n_sub != 1) return set_error(SPX_ERR_UNSUPPORTED, "learned init needs single-sublattice lattices");
    }
    hipStream_t st = (hipStream_t)stream;
    k_gneb_reset<<<(g->n_inst + 63) / 64, 64, 0, st>>>(g->d_inst, g->n_inst);
    k_gneb_geodesic<<<grid_for(g->n_items), kGB, 0, st>>>(g->d_inst, g->d_items, g->n_items);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "spx_gneb_init_path");
    if (method == 1) {
        for (int k = 0; k < g->n_inst; ++k) {
            const GInst &gi = g->hinst[k];
            const int nm = gi.n_img - 2;
            const int64_t N = gi.g.N;
            std::vector<float> tv(nm);
            for (int n = 0; n < nm; ++n) tv[n] = (float)(n + 1) / (float)(gi.n_img - 1);
            float *d_t = g->d_tvals + (size_t)k * g->max_img;
            e = hipMemcpyAsync(d_t, tv.data(), sizeof(float) * nm, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return set_hip_error(e, "spx_gneb_init_path (learned)");
            const int32_t dims[3] = {gi.g.Lx, gi.g.Ly, gi.g.Lz};
            double *Sg = gi.Y[0] + 3 * N;  // images 1 .. n_img-2, corrected in place
            spx_status s = net_apply(net, params, dims, nm, Sg, gi.Y[0], gi.Y[0] + (int64_t)(gi.n_img - 1) * 3 * N, 1,
                                     d_t, Sg, st);
            if (s != SPX_OK) return s;
            e = hipMemcpyAsync(gi.Y[1] + 3 * N, Sg, sizeof(double) * 3 * N * nm, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return set_hip_error(e, "spx_gneb_init_path (learned)");
        }
    }
    return SPX_OK;
}

spx_status spx_gneb_step(spx_gneb *g, int32_t n_iter, void *stream) {
    if (!handle_alive(g)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_gneb handle");
    if (n_iter < 0) return set_error(SPX_ERR_INVALID_ARG, "n_iter < 0");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (g->use_graph && n_iter > 1 && !g->graph) {
        // One iteration captured once on a private stream; the graph is then
        // launched on whatever stream the caller passes.  Capture failure
        // (graphs unsupported) leaves direct launches in place.
        if (!g->cap_stream) e = hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking);
        // with two to kMaxBranches instances, their passes become parallel
        // branches (streams and events of default priority, made once)
        const bool branches = g->n_inst > 1 && g->n_inst <= kMaxBranches;
        if (e == hipSuccess && branches && g->side.empty()) {
            g->side.assign(g->n_inst, nullptr);
            for (int p = 0; p < 2; ++p) g->join_ev[p].assign(g->n_inst, nullptr);
            for (int k = 0; k < g->n_inst && e == hipSuccess; ++k) {
                e = hipStreamCreateWithFlags(&g->side[k], hipStreamNonBlocking);
                for (int p = 0; p < 2 && e == hipSuccess; ++p)
                    e = hipEventCreateWithFlags(&g->join_ev[p][k], hipEventDisableTiming);
            }
            for (int p = 0; p < 2 && e == hipSuccess; ++p)
                e = hipEventCreateWithFlags(&g->fork_ev[p], hipEventDisableTiming);
        }
        hipGraph_t graph;
        if (e == hipSuccess) e = hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            g->branch = branches;
            hipError_t e2 = enqueue_iteration(g, g->cap_stream);
            g->branch = false;
            e = hipStreamEndCapture(g->cap_stream, &graph);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) {
                e = hipGraphInstantiate(&g->graph, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
            }
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            g->graph = nullptr;
            g->use_graph = 0;
            e = hipSuccess;
        }
    }
    for (int it = 0; it < n_iter && e == hipSuccess; ++it) {
        if (g->graph) e = hipGraphLaunch(g->graph, st);
        else e = enqueue_iteration(g, st);
    }
    if (e == hipSuccess) {
        k_gneb_copyback<<<grid_for(g->n_items), kGB, 0, st>>>(g->d_inst, g->d_items, g->n_items);
        k_gneb_cur_reset<<<(g->n_inst + 63) / 64, 64, 0, st>>>(g->d_inst, g->n_inst);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return set_hip_error(e, "spx_gneb_step");
    return SPX_OK;
}

spx_status spx_gneb_get_stats(spx_gneb *g, int32_t inst, double *E, double *dist, double *max_force,
                              int32_t *ci_index, int32_t *ci_on, int32_t *iterations, int32_t *converged,
                              void *stream) {
    if (!handle_alive(g)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_gneb handle");
    if (inst < 0 || inst >= g->n_inst) return set_error(SPX_ERR_INVALID_ARG, "instance out of range");
    hipStream_t st = (hipStream_t)stream;
    const GInst &gi = g->hinst[inst];
    std::vector<double> im(IS_N * gi.n_img), s(ST_N);
    hipError_t e = hipMemcpyAsync(im.data(), gi.img, sizeof(double) * im.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s.data(), gi.st, sizeof(double) * ST_N, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_hip_error(e, "spx_gneb_get_stats");
    for (int n = 0; n < gi.n_img; ++n) {
        if (E) E[n] = im[n * IS_N + IS_E];
        if (dist && n + 1 < gi.n_img) dist[n] = std::sqrt(im[n * IS_N + IS_D2]);
    }
    if (max_force) *max_force = s[ST_MAXF];
    if (ci_index) *ci_index = (int32_t)s[ST_CI];
    if (ci_on) *ci_on = (int32_t)s[ST_CION];
    if (iterations) *iterations = (int32_t)s[ST_ITER];
    if (converged) *converged = (int32_t)s[ST_DONE];
    return SPX_OK;
}

spx_status spx_gneb_set_spacing(spx_gneb *g, int32_t inst, const double *alpha, void *stream) {
    if (!handle_alive(g)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_gneb handle");
    if (inst < 0 || inst >= g->n_inst) return set_error(SPX_ERR_INVALID_ARG, "instance out of range");
    if (!alpha) return set_error(SPX_ERR_INVALID_ARG, "alpha is NULL");
    const GInst &gi = g->hinst[inst];
    if (alpha[0] != 0.0 || alpha[gi.n_img - 1] != 1.0)
        return set_error(SPX_ERR_INVALID_ARG, "alpha must start at 0 and end at 1");
    for (int n = 0; n + 1 < gi.n_img; ++n)
        if (!(alpha[n + 1] >= alpha[n])) return set_error(SPX_ERR_INVALID_ARG, "alpha must be nondecreasing");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync((void *)gi.alpha, alpha, sizeof(double) * gi.n_img, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_hip_error(e, "spx_gneb_set_spacing");
    return SPX_OK;
}

spx_status spx_gneb_redistribute(spx_gneb *g, void *stream) {
    if (!handle_alive(g)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_gneb handle");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = enqueue_reparam(g, GATE_ALL, st);
    if (e == hipSuccess) {
        k_gneb_copyback<<<grid_for(g->n_items), kGB, 0, st>>>(g->d_inst, g->d_items, g->n_items);
        k_gneb_cur_reset<<<(g->n_inst + 63) / 64, 64, 0, st>>>(g->d_inst, g->n_inst);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return set_hip_error(e, "spx_gneb_redistribute");
    return SPX_OK;
}

spx_status spx_gneb_set_params(spx_gneb *g, const spx_gneb_params *p, void *stream) {
    if (!handle_alive(g)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_gneb handle");
    if (!p) return set_error(SPX_ERR_INVALID_ARG, "params is NULL");
    if (!(p->vp_dt > 0.0) || !(p->vp_mass > 0.0) || !(p->spring_k >= 0.0) || !(p->tol_force >= 0.0))
        return set_error(SPX_ERR_INVALID_ARG, "vp_dt, vp_mass must be > 0; spring_k, tol_force >= 0");
    if (p->ci_mode < 0 || p->ci_mode > 4) return set_error(SPX_ERR_INVALID_ARG, "ci_mode must be 0 .. 4");
    hipStream_t st = (hipStream_t)stream;
    for (GInst &gi : g->hinst) {
        gi.k = p->spring_k;
        gi.dt = p->vp_dt;
        gi.mass = p->vp_mass;
        gi.ci_mode = p->ci_mode;
        gi.ci_on_below = p->ci_on_below;
        gi.tol = p->tol_force;
    }
    // the iteration graph depends on whether any instance runs the string method
    if (g->graph) (void)hipGraphExecDestroy(g->graph);
    g->graph = nullptr;
    hipError_t e = hipMemcpyAsync(g->d_inst, g->hinst.data(), sizeof(GInst) * g->n_inst, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        k_gneb_reset<<<(g->n_inst + 63) / 64, 64, 0, st>>>(g->d_inst, g->n_inst);
        e = hipGetLastError();
    }
    for (int k = 0; k < g->n_inst && e == hipSuccess; ++k) {
        const GInst &gi = g->hinst[k];
        e = hipMemsetAsync(gi.V, 0, sizeof(double) * 3 * gi.g.N * gi.n_img, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_hip_error(e, "spx_gneb_set_params");
    return SPX_OK;
}

spx_status spx_gneb_set_graph(spx_gneb *g, int32_t enable) {
    if (!handle_alive(g)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_gneb handle");
    g->use_graph = enable ? 1 : 0;
    if (!enable && g->graph) {
        (void)hipGraphExecDestroy(g->graph);
        g->graph = nullptr;
    }
    return SPX_OK;
}

}  // extern "C"
