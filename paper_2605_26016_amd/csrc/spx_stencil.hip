// spx_stencil.hip -- z-marching LDS stencil engine for structured shell
// patterns on gfx950: effective field, Heun predictor and Heun corrector.
//
// A block (512 threads by default) owns a 64 x 8 column tile (64 lanes along
// x, one wavefront per y row) and a chunk of z planes.  It streams input
// planes z' upward: each plane (all sublattices, 3 components, with the x/y
// halo of the shape) is read once from global memory -- periodic wrap or zero
// fill at open faces done here, so the compute loop has no boundary logic --
// into registers while the previous plane is being computed, then written to
// a double-buffered LDS slot, converted to the compute type (float in mixed
// mode).  Each thread stages its own interior sites first and keeps their
// FP64 spins in a small register ring until its epilogue needs them.
//
// Every bond (compile-time offset, runtime coupling) pushes J S_b(x+dx, y+dy,
// z') into a register accumulator of output plane z' - dz; with isotropic
// shells the bonds that share J are summed first (shared partial sums, one
// multiply per use).  The accumulators of the D = dzhi - dzlo + 1 pending
// output planes form a register ring that shifts by one slot per input plane,
// so every bond's slot (dzhi - dz) is a compile-time register.  An output
// plane is final once its highest input plane has been pushed; one copy of
// the epilogue then adds the on-site terms in FP64 and runs the Heun stage
// for the thread's sites (the predictor across its sublattice sites phase by
// phase, the correctors site by site), with the corrector's stored stage
// fetched one plane ahead.
#include <type_traits>
#include <vector>

#include "spx_device.hpp"
#include "spx_ext.hpp"
#include "spx_stencil.hpp"

namespace spx {

namespace {

// Tile shape and plane staging (compile-time; the defaults were the fastest
// of the measured alternatives on the bcc 5-shell and sc NN workloads).
#ifndef SPX_ZM_TYT
#define SPX_ZM_TYT 8
#endif
#ifndef SPX_ZM_YB
#define SPX_ZM_YB 1
#endif
#ifndef SPX_ZM_PREFETCH
#define SPX_ZM_PREFETCH 1
#endif
constexpr int kTX = 64;   // tile width in x (one wavefront per thread row)
constexpr int kTYT = SPX_ZM_TYT;   // thread rows per block
constexpr int kYB = SPX_ZM_YB;     // y sites per thread
// 1: the next input plane is fetched into registers before the current
// plane's compute and written to LDS after it (global latency overlapped);
// single-input modes only (two staged inputs would double those registers)
constexpr bool kPrefetch = SPX_ZM_PREFETCH != 0;

constexpr int kThreads = kTX * kTYT;  // default block: kTX x kTYT threads, tile height kTYT kYB

// ZM_CORRECT: recompute the fields of S^n and S~; ZM_CORRECT_STORED: read the
// predictor's FP32 bilinear field of S^n; ZM_CORRECT_P: read the predictor's
// partial update P = S^n + dt/2 f(S^n) and its noise eta (FP64; or draw eta
// again when it was not stored), so that the corrector evaluates only f(S~).
// ZM_BIL: store only the FP32 bilinear field (the split Heun mode's stencil
// pass; the Heun stages then run as elementwise kernels).
// ZM_MIN_FORCE: the force pass of the static minimisers in the epilogue
// (force projected on the spin's tangent plane, its max norm and the dot
// products of the method), reduced to one partial set per block.
// ZM_ENERGY: the energy terms -S.b_bil/2, -S.b_Z, -S.b_ani/2, -S.b_dip/2 of the
// thread's sites summed in the epilogue (the field is never stored), reduced
// to one quadruple per tile in a fixed order.
// ZM_GNEB_A2 / ZM_GNEB_C2: the two passes of a GNEB iteration that keeps no
// stored force.  A2 (every image): energy terms, squared distance to the next
// image and, for interior images, the nine image sums from which the
// improved tangent's dot products follow once its energy weights are known
// (a = P(S_n+1 - S_n), b = P(S_n - S_n-1), P the projection on the spin's
// tangent plane: a.a, a.b, b.b, F.a, F.b, v.a, v.b, v.F, F.F), eleven
// partials per tile.  C2 (interior images): the force again from the field,
// the tangent w+ a + w- b, the spring / climbing-image force, the velocity
// projection step and the exponential-map retraction into the other image
// buffer, the velocity store and max |F_gneb| per tile.
enum ZMode { ZM_FIELD = 0, ZM_PREDICT = 1, ZM_CORRECT = 2, ZM_CORRECT_STORED = 3, ZM_CORRECT_P = 4, ZM_BIL = 5,
             ZM_MIN_FORCE = 7, ZM_ENERGY = 8, ZM_GNEB_A2 = 9, ZM_GNEB_C2 = 10 };

// Block size of a mode on a shape.  The GNEB passes run 256-thread blocks
// (two per CU at their register use) whose tile width is chosen per lattice
// (zp.txw: 64 x 4, 32 x 8 or 16 x 16 sites, so that x extents such as 48 and
// 96 fill every lane); the two-cell 4-shell shape needs all 256 registers
// there and keeps the default block.  The other modes use the engine default
// and 64-wide tiles.
constexpr bool zm_gneb(int mode) { return mode == ZM_GNEB_A2 || mode == ZM_GNEB_C2; }
constexpr int zm_block(int mode, int kind) { return zm_gneb(mode) && kind != SHAPE_SC_4SH ? 256 : kThreads; }

// Tiles of one image for a block size and tile width.
int zm_tiles(const Grid &g, int zch, int block, int txw) {
    const int rows = block / txw * kYB;
    return ((g.Lx + txw - 1) / txw) * ((g.Ly + rows - 1) / rows) * ((g.Lz + zch - 1) / zch);
}

template <typename T, int NW>
struct ZWeights {
    T w[NW];
};

struct ZArgs {
    int Lx, Ly, Lz;
    int per[3];
    int M;
    int64_t N;
    int zch;
    const double *S0;  // S^n (or the state of a field evaluation)
    const double *S1;  // S~ (corrector)
    double *out;       // S~ (predictor) or S^{n+1} (corrector)
    void *bout;        // field output (field mode)
    float *bstore;     // predictor: FP32 bilinear field of S^n (may be NULL)
    const float *bload;  // stored-field corrector: that field
    double *pstore;    // predictor: P = S^n + dt/2 f(S^n) (may be NULL)
    double *estore;    // predictor: eta of this step (may be NULL; T > 0 only)
    const double *pload, *eload;  // ZM_CORRECT_P: P and eta; predictor: eta if not NULL
    const float *bdip0, *bdip1;  // dipolar fields of S0 / S1 (may be NULL)
    uint64_t step;
    // image batch (field modes): blockIdx.z = image * nzc + z chunk, images
    // bstride elements apart; S0alt replaces S0 when *sel != 0; the whole
    // launch is a no-op when *skip != 0
    int nzc, nimg;
    int64_t bstride;
    // 1: tiles are dealt to the XCDs in contiguous runs (set by the launcher
    // when every tile of the grid is resident at once, or with imgfast)
    int xcd;
    // 1: the image index is the fastest of the tile decomposition
    int imgfast;
    const double *S0alt;
    const double *sel, *skip;
    // ZM_MIN_FORCE: force [3][N]; partials of the modes that reduce per tile
    double *gF;
    double *gpart;
    int gitem0, gipi;
    // ZM_MIN_FORCE (force in gF, partials [tile][6] in gpart): the method's
    // velocity (0) or previous step and force (1, 2), the L-BFGS history
    // rings and the minimiser state (candidate slot)
    const double *mV, *mUp, *mFp;
    double *mSh, *mYh;
    const double *mst;
    int mmethod, mcand_idx;
    // ZM_GNEB_A2 / C2: launch image k is image gimg0 + k of gntot; velocities
    // gV [gntot][3][N]; C2 writes to O0, or O1 when *sel != 0; per-image
    // scalars gims[n * gis.n + {wp, wm, tn, coef}], the VP projection at
    // gst[gis.proj]; the VP step and mass; string method (no velocity)
    int gimg0, gntot;
    double *gV;
    double *O0, *O1;
    const double *gims, *gst;
    GnebSlots gis;
    double gdt, gmass;
    int gstring;
};

// Shape table as a static constant, so that every bond read in an unrolled
// loop is a constant expression.
template <int KIND>
struct ShapeC {
    static constexpr ShapeTable t = make_shape(KIND);
};

template <int KIND>
struct SumC {
    static constexpr SumTable t = make_sums(KIND);
    static_assert(t.ok, "shape exceeds the partial-sum table");
};

// Compile-time loop: f(std::integral_constant<int, k>) for k = 0 .. N-1.
template <typename F, int... K>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, K...>) {
    (f(std::integral_constant<int, K>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ int zwrap(int c, int L, int per, bool &ok) {
    if (c >= 0 && c < L) return c;
    if (!per) { ok = false; return 0; }
    c %= L;
    return c < 0 ? c + L : c;
}

template <int KIND, typename T, bool ISO, int MODE, int TXW>
__global__ __launch_bounds__(zm_block(MODE, KIND)) void k_zmarch(ZArgs g, Onsite os, HeunConst hc,
                                                           ZWeights<T, ISO ? make_shape(KIND).nshell : 9 * make_shape(KIND).nb> W) {
    // block size and tile shape of this instantiation (they shadow the
    // engine-wide defaults): TXW lanes along x, the other threads along y
    constexpr int kThreads = zm_block(MODE, KIND);
    constexpr int kTX = TXW;
    constexpr int kTYE = kThreads / TXW * kYB;
    static_assert(kThreads % TXW == 0 && (TXW & (TXW - 1)) == 0, "tile width: a power of two dividing the block");
    constexpr int NSUB = ShapeC<KIND>::t.nsub, NB = ShapeC<KIND>::t.nb;
    constexpr int RX = ShapeC<KIND>::t.rx, RY = ShapeC<KIND>::t.ry;
    constexpr int DZLO = ShapeC<KIND>::t.dzlo, DZHI = ShapeC<KIND>::t.dzhi;
    constexpr int D = DZHI - DZLO + 1;
    constexpr int NIN = (MODE == ZM_CORRECT) ? 2 : 1;
    constexpr int PW = kTX + 2 * RX, PH = kTYE + 2 * RY;
    constexpr int PLANE = PW * PH;
    __shared__ T lds[2][NIN][NSUB][3][PLANE];

    const int tx = threadIdx.x & (kTX - 1);
    const int ty = threadIdx.x / kTX;
    if (g.skip && *g.skip != 0.0) return;  // uniform over the grid
    // 1-D grid of (x tile, y tile, z chunk, image) tiles, x fastest.  Blocks
    // are dealt to the 8 XCDs round-robin; with g.xcd each XCD instead gets
    // one contiguous run of tiles, so the tiles that share halo rows and
    // march through the same planes at the same time share that XCD's L2.
    // With g.imgfast the image index runs fastest instead, so that the
    // launches of one spatial tile over all images are adjacent: with the
    // contiguous XCD order they run together on one XCD, and the neighbouring
    // images that each block reads besides its own come from that L2.
    const unsigned nbx = (unsigned)((g.Lx + kTX - 1) / kTX), nby = (unsigned)((g.Ly + kTYE - 1) / kTYE);
    const unsigned ntile = gridDim.x;
    unsigned tile = blockIdx.x;
    if (g.xcd && (ntile & 7u) == 0) tile = (tile & 7u) * (ntile >> 3) + (tile >> 3);
    unsigned stile;  // spatial tile of the image: x tile + nbx (y tile + nby z chunk)
    int img;
    if (g.imgfast) {
        img = (int)(tile % (unsigned)g.nimg);
        stile = tile / (unsigned)g.nimg;
    } else {
        const unsigned per_img = nbx * nby * (unsigned)g.nzc;
        img = (int)(tile / per_img);
        stile = tile - (unsigned)img * per_img;
    }
    const int x0 = (int)(stile % nbx) * kTX;
    const int y0 = (int)((stile / nbx) % nby) * kTYE;
    const int zs = (int)(stile / (nbx * nby)) * g.zch;
    // image offset of the launch's image in its buffer (the GNEB second pass
    // launches over the interior images only: launch image k is image
    // gimg0 + k)
    const int64_t boff = (int64_t)(img + g.gimg0) * g.bstride;
    const int nout = min(g.zch, g.Lz - zs);
    const int nq = nout + D - 1;
    const int64_t N = g.N;
    const double *S0 = ((g.sel && *g.sel != 0.0) ? g.S0alt : g.S0) + boff;
    // LDS inputs: the field of S0 (and of S1 for the recomputing corrector);
    // the stored-field corrector needs only the field of S1 = S~
    const double *src[2] = {(MODE == ZM_CORRECT_STORED || MODE == ZM_CORRECT_P) ? g.S1 : S0, g.S1};

    T acc[D][kYB][NSUB][3][NIN];
#pragma unroll
    for (int s = 0; s < D; ++s)
#pragma unroll
        for (int yb = 0; yb < kYB; ++yb)
#pragma unroll
            for (int a = 0; a < NSUB; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int k = 0; k < NIN; ++k) acc[s][yb][a][c][k] = T(0);

    // Per-site FP64 inputs of the epilogue other than the spin itself,
    // fetched one march iteration before their use so that their latency
    // hides behind a plane's stencil: CORRECT_P reads P and eta, PREDICT
    // reads eta when the noise comes from a pre-pass.
    constexpr bool kEpiPre = MODE == ZM_CORRECT_P || MODE == ZM_PREDICT || MODE == ZM_MIN_FORCE ||
                             MODE == ZM_GNEB_A2 || MODE == ZM_GNEB_C2;
    constexpr int NE = MODE == ZM_GNEB_A2 ? 9
                       : (MODE == ZM_CORRECT_P || MODE == ZM_MIN_FORCE || MODE == ZM_GNEB_C2) ? 6
                       : MODE == ZM_PREDICT ? 3 : 1;
    // image of the launch in its instance (GNEB two-pass modes)
    const int gimg = img + g.gimg0;
    // ZM_GNEB_C2: the image's tangent weights w+-, c_n / |tau| (the spring or
    // climbing-image coefficient over the tangent norm) and the velocity
    // factor (VP projection + dt / m), uniform over the block
    double gwp = 0.0, gwm = 0.0, gcn = 0.0, gvf = 0.0;
    if constexpr (MODE == ZM_GNEB_C2) {
        const double *im = g.gims + (int64_t)gimg * g.gis.n;
        gwp = im[g.gis.wp];
        gwm = im[g.gis.wm];
        const double tn = im[g.gis.tn];
        gcn = tn > 0.0 ? im[g.gis.coef] / tn : 0.0;
        gvf = g.gst[g.gis.proj] + g.gdt / g.gmass;
    }
    // kDeep: the staged plane and the epilogue inputs are fetched two march
    // iterations ahead into two register sets, whose names stay static
    // because the march loop is unrolled by two (passes whose iterations wait
    // on memory longer than they compute; about 30 more registers, which the
    // two-cell 4-shell shape does not have)
    constexpr bool kDeep =
        kPrefetch && NIN == 1 && (MODE == ZM_GNEB_A2 || MODE == ZM_GNEB_C2) && KIND != SHAPE_SC_4SH;
    constexpr int NSET = kDeep ? 2 : 1;
    double epi[NSET][kYB][NSUB][NE];
    auto fetch_epi = [&](int o, auto es) __attribute__((always_inline)) {
        constexpr int E = decltype(es)::value;
        if (o < 0 || o >= nout) return;  // uniform over the block
        if (MODE == ZM_PREDICT && !(hc.noise && g.eload)) return;
        if (MODE == ZM_MIN_FORCE && g.mmethod == 3) return;   // Adam reads nothing here
        const int x = x0 + tx;
        static_for<NSUB>([&](auto ac) __attribute__((always_inline)) {
            constexpr int a = decltype(ac)::value;
#pragma unroll
            for (int yb = 0; yb < kYB; ++yb) {
                const int y = y0 + ty * kYB + yb;
                if (x >= g.Lx || y >= g.Ly) continue;
                const int64_t i = (int64_t)a * g.M + x + (int64_t)g.Lx * (y + (int64_t)g.Ly * (zs + o));
                double *e = epi[E][yb][a];
                if constexpr (MODE == ZM_CORRECT_P) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) e[c] = g.pload[c * N + i];
                    if (hc.noise && g.eload)
#pragma unroll
                        for (int c = 0; c < 3; ++c) e[3 + c] = g.eload[c * N + i];
                } else if constexpr (MODE == ZM_PREDICT) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) e[c] = g.eload[c * N + i];
                } else if constexpr (MODE == ZM_GNEB_A2 || MODE == ZM_GNEB_C2) {
                    // the neighbouring images (zero where there is none)
                    // and, for A2, the interior image's velocity
                    const bool nx = gimg < g.gntot - 1, pv = gimg > 0;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        e[c] = nx ? S0[g.bstride + c * N + i] : 0.0;
                        e[3 + c] = pv ? S0[c * N + i - g.bstride] : 0.0;
                    }
                    if constexpr (MODE == ZM_GNEB_A2) {
                        const bool vel = nx && pv && !g.gstring;
#pragma unroll
                        for (int c = 0; c < 3; ++c) e[6 + c] = vel ? g.gV[(int64_t)gimg * g.bstride + c * N + i] : 0.0;
                    }
                } else if constexpr (MODE == ZM_MIN_FORCE) {
                    if (g.mmethod == 0) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) e[c] = g.mV[c * N + i];
                    } else {
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            e[c] = g.mUp[c * N + i];
                            e[3 + c] = g.mFp[c * N + i];
                        }
                    }
                }
            }
        });
    };

    // Staged elements of a plane.  Slots 0 .. NI-1 of thread (tx, ty) are
    // its own interior sites (sublattice a, row yb), so the FP64 spins of the
    // sites it finishes pass through its registers; slots NI .. NLD-1 hold
    // the x/y halo ring, dealt over the block's threads.  The x/y source
    // offsets and wrap/zero decisions do not depend on the plane and are
    // computed once here; per plane only z is added.
    constexpr int HS = PLANE - kTX * kTYE;  // halo elements per sublattice
    constexpr int RX2 = 2 * RX > 0 ? 2 * RX : 1;
    constexpr int NI = NSUB * kYB;
    constexpr int NH = (NSUB * HS + kThreads - 1) / kThreads;
    constexpr int NLD = NI + NH;
    int64_t xy_off[NLD];
    int lds_off[NLD];
    unsigned xy_ok = 0;    // bit t: element inside the lattice in x/y (after wrap)
    unsigned slot_ok = 0;  // bit t: slot t holds an element of the plane
#pragma unroll
    for (int t = 0; t < NLD; ++t) {
        int sub, cy, cx;
        bool have = true;
        if (t < NI) {
            sub = t / kYB;
            cy = ty * kYB + t % kYB + RY;
            cx = tx + RX;
        } else {
            const int h = threadIdx.x + (t - NI) * kThreads;
            have = h < NSUB * HS;
            sub = h / HS;
            int m = h - sub * HS;
            if (m < RY * PW) {  // rows above the tile
                cy = m / PW;
                cx = m - cy * PW;
            } else if ((m -= RY * PW) < kTYE * 2 * RX) {  // left / right columns
                cy = RY + m / RX2;
                const int k = m - (cy - RY) * RX2;
                cx = k < RX ? k : kTX + k;
            } else {  // rows below the tile
                m -= kTYE * 2 * RX;
                cy = RY + kTYE + m / PW;
                cx = m - (cy - RY - kTYE) * PW;
            }
        }
        xy_off[t] = 0;
        lds_off[t] = 0;
        if (have) {
            slot_ok |= 1u << t;
            bool ok = true;
            const int gx = zwrap(x0 - RX + cx, g.Lx, g.per[0], ok);
            const int gy = zwrap(y0 - RY + cy, g.Ly, g.per[1], ok);
            xy_off[t] = (int64_t)sub * g.M + gx + (int64_t)g.Lx * gy;
            lds_off[t] = sub * 3 * PLANE + cy * PW + cx;
            if (ok) xy_ok |= 1u << t;
        }
    }
    const int64_t plane_stride = (int64_t)g.Lx * g.Ly;
    T *const lds_flat = &lds[0][0][0][0][0];
    constexpr int BUF_STRIDE = NIN * NSUB * 3 * PLANE, IN_STRIDE = NSUB * 3 * PLANE;
    // plane q (z = zs + DZLO + q) in two halves: fetch into registers, then
    // commit to LDS buffer `buf`
    double pre[NSET][NLD][NIN][3];
    // FP64 spins of the thread's own sites for the last DZHI + 1 staged
    // planes: own[0] holds the plane that the current iteration finishes
    constexpr bool kOwn = kPrefetch && NIN == 1 && MODE != ZM_BIL;
    double own[kOwn ? DZHI + 1 : 1][NI][3];
    auto keep_own = [&](auto ps) __attribute__((always_inline)) {
        constexpr int P = decltype(ps)::value;
        if constexpr (kOwn) {
#pragma unroll
            for (int r = 0; r < DZHI; ++r)
#pragma unroll
                for (int k = 0; k < NI; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) own[r][k][c] = own[r + 1][k][c];
#pragma unroll
            for (int k = 0; k < NI; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) own[DZHI][k][c] = pre[P][k][0][c];
        }
    };
    auto fetch_plane = [&](int q, auto ps) __attribute__((always_inline)) {
        constexpr int P = decltype(ps)::value;
        bool zok = true;
        const int gz = zwrap(zs + DZLO + q, g.Lz, g.per[2], zok);
        const int64_t zoff = plane_stride * gz;
#pragma unroll
        for (int t = 0; t < NLD; ++t) {
            const bool ok = zok && ((xy_ok >> t) & 1u);
            const int64_t j = xy_off[t] + zoff;
#pragma unroll
            for (int k = 0; k < NIN; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) pre[P][t][k][c] = ok ? src[k][c * N + j] : 0.0;
        }
    };
    auto commit_plane = [&](int buf, auto ps) __attribute__((always_inline)) {
        constexpr int P = decltype(ps)::value;
#pragma unroll
        for (int t = 0; t < NLD; ++t) {
            if (t < NI || ((slot_ok >> t) & 1u)) {
#pragma unroll
                for (int k = 0; k < NIN; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        lds_flat[buf * BUF_STRIDE + k * IN_STRIDE + c * PLANE + lds_off[t]] = (T)pre[P][t][k][c];
            }
        }
    };
    // global -> LDS copy of input plane q into buffer `buf` in one pass
    auto load_plane = [&](int q, int buf) {
        bool zok = true;
        const int gz = zwrap(zs + DZLO + q, g.Lz, g.per[2], zok);
        const int64_t zoff = plane_stride * gz;
#pragma unroll
        for (int t = 0; t < NLD; ++t) {
            if (t < NI || ((slot_ok >> t) & 1u)) {
                const bool ok = zok && ((xy_ok >> t) & 1u);
                const int64_t j = xy_off[t] + zoff;
#pragma unroll
                for (int k = 0; k < NIN; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        lds_flat[buf * BUF_STRIDE + k * IN_STRIDE + c * PLANE + lds_off[t]] =
                            ok ? (T)src[k][c * N + j] : T(0);
            }
        }
    };

    // Corrector epilogue of one site (sublattice a, index j) whose bilinear
    // field sums are v[in][c].  One copy serves every site of the thread;
    // the caller selects the site's values from the register rings.
    auto finish_corr = [&](auto ac, int64_t j, const T (&v)[NIN][3], const double (&e)[NE], const double (&so)[3])
                           __attribute__((always_inline)) {
        constexpr int a = decltype(ac)::value;
        double st[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) st[c] = (kOwn && MODE != ZM_CORRECT) ? so[c] : g.S1[c * N + j];
        double bt[3];
        aniso_field(os, a, st, bt);
        double B1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double v1 = (double)v[NIN - 1][c] + bt[c] + os.bz[a][c];
            if (g.bdip1) v1 += (double)g.bdip1[c * N + j];
            B1[c] = v1 * hc.inv_mumuB[a];
        }
        const double hdt = 0.5 * hc.dt;
        double pn[3];
        if constexpr (MODE == ZM_CORRECT_P) {
            // P = S^n + dt/2 f(S^n) comes from the predictor; eta too, or it
            // is drawn again here (the same Philox block)
            if (hc.noise) {
                double eta[3];
                if (g.eload) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) eta[c] = e[3 + c];
                } else {
                    thermal_eta(hc.seed, noise_step(hc, g.step), hc.tag, (uint64_t)j, eta);
                }
                const double sg = hc.sigma[a];
#pragma unroll
                for (int c = 0; c < 3; ++c) B1[c] += sg * eta[c];
            }
            double f1[3];
            llg_rhs(st, B1, hc.pre, hc.alpha, f1);
#pragma unroll
            for (int c = 0; c < 3; ++c) pn[c] = e[c] + hdt * f1[c];
        } else {
            double sv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) sv[c] = g.S0[c * N + j];
            double ba[3];
            aniso_field(os, a, sv, ba);
            double B0[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double bil0 = MODE == ZM_CORRECT ? (double)v[0][c] : (double)g.bload[c * N + j];
                double v0 = bil0 + ba[c] + os.bz[a][c];
                if (g.bdip0) v0 += (double)g.bdip0[c * N + j];
                B0[c] = v0 * hc.inv_mumuB[a];
            }
            if (hc.noise) {
                double eta[3];
                thermal_eta(hc.seed, noise_step(hc, g.step), hc.tag, (uint64_t)j, eta);
                const double sg = hc.sigma[a];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    B0[c] += sg * eta[c];
                    B1[c] += sg * eta[c];
                }
            }
            double f0[3], f1[3];
            llg_rhs(sv, B0, hc.pre, hc.alpha, f0);
            llg_rhs(st, B1, hc.pre, hc.alpha, f1);
#pragma unroll
            for (int c = 0; c < 3; ++c) pn[c] = sv[c] + hdt * (f0[c] + f1[c]);
        }
        normalise3(pn);
#pragma unroll
        for (int c = 0; c < 3; ++c) g.out[c * N + j] = pn[c];
    };

    // Field / predictor epilogue of the thread's NSUB sites (one per
    // sublattice) in row y of plane z, whose bilinear field sums are
    // v[a][in][c].  The work runs phase
    // by phase across the sites, with no branch inside a phase, so that the
    // sites' independent FP64 and Philox chains interleave; sites outside
    // the lattice (valid = false) compute on a clamped index and store nothing.
    double eE[4] = {0.0, 0.0, 0.0, 0.0};  // ZM_ENERGY: the thread's four energy terms
    // ZM_GNEB_C2: the thread's max |F_gneb|.  ZM_GNEB_A2: the thread's energy,
    // squared distance and nine image sums (a.a, a.b, b.b, F.a, F.b, v.a, v.b,
    // v.F, F.F) live in its own LDS column rather than in registers
    double gX[1] = {0.0};
    double *gacc = nullptr;  // [11][kThreads], ZM_GNEB_A2 only
    if constexpr (MODE == ZM_GNEB_A2) {
        __shared__ double gacc_lds[11 * kThreads];
        gacc = gacc_lds;
#pragma unroll
        for (int k = 0; k < 11; ++k) gacc[k * kThreads + threadIdx.x] = 0.0;
    }
    // ZM_MIN_FORCE: max |F|, v.F, F.F, s.s, s.y, y.y of the thread's sites
    double mred[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    auto finish_row = [&](int x, int y, int z, bool valid, const T (&v)[NSUB][NIN][3],
                          const double (&e)[NSUB][NE], const double (&so)[NSUB][3]) __attribute__((always_inline)) {
        int64_t i[NSUB], ir[NSUB];
#pragma unroll
        for (int a = 0; a < NSUB; ++a) {
            i[a] = (int64_t)a * g.M + x + (int64_t)g.Lx * (y + (int64_t)g.Ly * z);
            ir[a] = valid ? i[a] : 0;
        }
        if constexpr (MODE == ZM_BIL) {
            T *const bo = (T *)g.bout + boff;
            if (valid)
#pragma unroll
                for (int a = 0; a < NSUB; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c) bo[c * N + i[a]] = v[a][0][c];
            return;
        }
        if constexpr (MODE == ZM_MIN_FORCE) {
            if (!valid) return;
            const int method = g.mmethod;
            const int cand = (int)g.mst[g.mcand_idx];
#pragma unroll
            for (int a = 0; a < NSUB; ++a) {
                const double *sp = so[a];
                double ba[3];
                aniso_field(os, a, sp, ba);
                double b[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) b[c] = (double)v[a][0][c] + ba[c] + os.bz[a][c];
                const double bs = b[0] * sp[0] + b[1] * sp[1] + b[2] * sp[2];
                double f[3], f2 = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    f[c] = b[c] - bs * sp[c];
                    f2 += f[c] * f[c];
                    g.gF[c * N + i[a]] = f[c];
                }
                mred[0] = fmax(mred[0], sqrt(f2));
                mred[2] += f2;
                if (method == 0) {
                    mred[1] += e[a][0] * f[0] + e[a][1] * f[1] + e[a][2] * f[2];
                } else if (method == 1 || method == 2) {
                    // step and force change, both projected on the tangent plane of s
                    double sv[3], yv[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        sv[c] = e[a][c];
                        yv[c] = e[a][3 + c];
                    }
                    const double ds = sv[0] * sp[0] + sv[1] * sp[1] + sv[2] * sp[2];
                    const double dy = yv[0] * sp[0] + yv[1] * sp[1] + yv[2] * sp[2];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        sv[c] -= ds * sp[c];
                        yv[c] -= dy * sp[c];
                        yv[c] -= f[c];
                    }
                    mred[3] += sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2];
                    mred[4] += sv[0] * yv[0] + sv[1] * yv[1] + sv[2] * yv[2];
                    mred[5] += yv[0] * yv[0] + yv[1] * yv[1] + yv[2] * yv[2];
                    if (method == 2) {
                        double *Sj = g.mSh + (int64_t)cand * 3 * N, *Yj = g.mYh + (int64_t)cand * 3 * N;
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            Sj[c * N + i[a]] = sv[c];
                            Yj[c * N + i[a]] = yv[c];
                        }
                    }
                }
            }
            return;
        }
        if constexpr (MODE == ZM_GNEB_A2 || MODE == ZM_GNEB_C2) {
            if (!valid) return;
            const bool interior = gimg > 0 && gimg < g.gntot - 1, has_next = gimg < g.gntot - 1;
#pragma unroll
            for (int a = 0; a < NSUB; ++a) {
                const double *sp = so[a];
                double ba[3];
                aniso_field(os, a, sp, ba);
                double b[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) b[c] = (double)v[a][0][c] + ba[c] + os.bz[a][c];
                if constexpr (MODE == ZM_GNEB_A2) {
                    double sb = 0.0, sz = 0.0, sa = 0.0;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        sb += sp[c] * (double)v[a][0][c];
                        sz += sp[c] * os.bz[a][c];
                        sa += sp[c] * ba[c];
                    }
                    gacc[threadIdx.x] += -0.5 * sb - sz - 0.5 * sa;
                    if (has_next) {
                        const double *q = e[a];
                        const double c0 = sp[1] * q[2] - sp[2] * q[1], c1 = sp[2] * q[0] - sp[0] * q[2],
                                     c2 = sp[0] * q[1] - sp[1] * q[0];
                        const double cc = c0 * c0 + c1 * c1 + c2 * c2;
                        const double th =
                            atan2_nonneg(cc > 0.0 ? sqrt_pos(cc) : 0.0, sp[0] * q[0] + sp[1] * q[1] + sp[2] * q[2]);
                        gacc[kThreads + threadIdx.x] += th * th;
                    }
                }
                if (!interior) continue;
                const double bs = b[0] * sp[0] + b[1] * sp[1] + b[2] * sp[2];
                double F[3], ap[3], bp[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    F[c] = b[c] - bs * sp[c];
                    ap[c] = e[a][c] - sp[c];
                    bp[c] = sp[c] - e[a][3 + c];
                }
                const double as = ap[0] * sp[0] + ap[1] * sp[1] + ap[2] * sp[2];
                const double bss = bp[0] * sp[0] + bp[1] * sp[1] + bp[2] * sp[2];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    ap[c] -= as * sp[c];
                    bp[c] -= bss * sp[c];
                }
                if constexpr (MODE == ZM_GNEB_A2) {
                    // the velocity, fetched a plane ahead (zero for the
                    // string method)
                    const double vv[3] = {e[a][6], e[a][7], e[a][8]};
                    double d9[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        d9[0] += ap[c] * ap[c];
                        d9[1] += ap[c] * bp[c];
                        d9[2] += bp[c] * bp[c];
                        d9[3] += F[c] * ap[c];
                        d9[4] += F[c] * bp[c];
                        d9[5] += vv[c] * ap[c];
                        d9[6] += vv[c] * bp[c];
                        d9[7] += vv[c] * F[c];
                        d9[8] += F[c] * F[c];
                    }
#pragma unroll
                    for (int k = 0; k < 9; ++k) gacc[(2 + k) * kThreads + threadIdx.x] += d9[k];
                } else {
                    // F_gneb = F + c_n tau / |tau|, VP step, exponential map
                    double u[3], vn[3], f2 = 0.0;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const double tau = gwp * ap[c] + gwm * bp[c];
                        const double ft = F[c] + gcn * tau;
                        f2 += ft * ft;
                        vn[c] = g.gstring ? 0.0 : gvf * ft;
                        u[c] = g.gstring ? g.gdt * F[c] : g.gdt * vn[c];
                    }
                    // max |F_gneb|^2 here, its square root once per tile
                    gX[0] = fmax(gX[0], f2);
                    if (!g.gstring) {
                        double *V = g.gV + (int64_t)gimg * g.bstride;
#pragma unroll
                        for (int c = 0; c < 3; ++c) V[c * N + i[a]] = vn[c];
                        const double us = u[0] * sp[0] + u[1] * sp[1] + u[2] * sp[2];
#pragma unroll
                        for (int c = 0; c < 3; ++c) u[c] -= us * sp[c];
                    }
                    // exp_S(u) = cos|u| S + (sin|u| / |u|) u, renormalised;
                    // u = 0 leaves S as it is
                    const double uz = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                    double cs, sc;
                    expmap_cs(uz, cs, sc);
                    double o[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) o[c] = cs * sp[c] + sc * u[c];
                    normalise3(o);
#pragma unroll
                    for (int c = 0; c < 3; ++c) o[c] = uz == 0.0 ? sp[c] : o[c];
                    double *On = ((g.sel && *g.sel != 0.0) ? g.O1 : g.O0) + (int64_t)gimg * g.bstride;
#pragma unroll
                    for (int c = 0; c < 3; ++c) On[c * N + i[a]] = o[c];
                }
            }
            return;
        }
        if constexpr (MODE == ZM_ENERGY) {
            if (!valid) return;
#pragma unroll
            for (int a = 0; a < NSUB; ++a) {
                double ba[3];
                aniso_field(os, a, so[a], ba);
                double sb = 0.0, sz = 0.0, sa = 0.0, sd = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    sb += so[a][c] * (double)v[a][0][c];
                    sz += so[a][c] * os.bz[a][c];
                    sa += so[a][c] * ba[c];
                    if (g.bdip0) sd += so[a][c] * (double)g.bdip0[c * N + i[a]];
                }
                eE[0] += -0.5 * sb;
                eE[1] += -sz;
                eE[2] += -0.5 * sa;
                eE[3] += -0.5 * sd;
            }
            return;
        }
        // field and predictor: phase by phase across the sites.  Optional
        // per-site inputs are each gathered under one uniform branch
        double d0[NSUB][3] = {};
        if (g.bdip0)
#pragma unroll
            for (int a = 0; a < NSUB; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) d0[a][c] = (double)g.bdip0[c * N + ir[a]];
        double eta[NSUB][3] = {};
        if constexpr (MODE != ZM_FIELD) {
            if (hc.noise) {
                if (MODE == ZM_PREDICT && g.eload) {
#pragma unroll
                    for (int a = 0; a < NSUB; ++a)
#pragma unroll
                        for (int c = 0; c < 3; ++c) eta[a][c] = e[a][c];
                } else {
                    const uint64_t ns = noise_step(hc, g.step);
#pragma unroll
                    for (int a = 0; a < NSUB; ++a) thermal_eta(hc.seed, ns, hc.tag, (uint64_t)i[a], eta[a]);
                }
            }
        }
        double out[NSUB][3];
        {
            // the spin of the state whose field this is: the thread's own
            // staged value
            double sv[NSUB][3], ba[NSUB][3];
#pragma unroll
            for (int a = 0; a < NSUB; ++a) {
#pragma unroll
                for (int c = 0; c < 3; ++c) sv[a][c] = kOwn ? so[a][c] : g.S0[c * N + ir[a]];
                aniso_field(os, a, sv[a], ba[a]);
            }
            if constexpr (MODE == ZM_FIELD) {
                if (valid)
#pragma unroll
                    for (int a = 0; a < NSUB; ++a)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            ((T *)g.bout)[c * N + i[a]] = (T)((double)v[a][0][c] + ba[a][c] + os.bz[a][c] + d0[a][c]);
                return;
            } else if constexpr (MODE == ZM_PREDICT) {
                double f[NSUB][3];
#pragma unroll
                for (int a = 0; a < NSUB; ++a) {
                    double B[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        B[c] = ((double)v[a][0][c] + ba[a][c] + os.bz[a][c] + d0[a][c]) * hc.inv_mumuB[a] +
                               hc.sigma[a] * eta[a][c];
                    llg_rhs(sv[a], B, hc.pre, hc.alpha, f[a]);
#pragma unroll
                    for (int c = 0; c < 3; ++c) out[a][c] = sv[a][c] + hc.dt * f[a][c];
                    normalise3(out[a]);
                }
                if (valid) {
                    const double hdt = 0.5 * hc.dt;
#pragma unroll
                    for (int a = 0; a < NSUB; ++a)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            if (g.bstore) g.bstore[c * N + i[a]] = (float)v[a][0][c];
                            if (g.estore && hc.noise) g.estore[c * N + i[a]] = eta[a][c];
                            if (g.pstore) g.pstore[c * N + i[a]] = sv[a][c] + hdt * f[a][c];
                        }
                }
            }
        }
        if (valid)
#pragma unroll
            for (int a = 0; a < NSUB; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) g.out[c * N + i[a]] = out[a][c];
    };

    // acc[k] holds output plane o = q - (D-1) + k after input plane q has been
    // pushed; input plane q feeds slot k = dzhi - dz of every bond.
    // Register sets: with kDeep, iteration q stages plane q + 2 into set
    // q & 1 and commits plane q + 1 from set (q + 1) & 1; the epilogue inputs
    // of output plane o live in set o & 1.  Otherwise one set, one ahead.
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    if constexpr (kPrefetch && NIN == 1) {
        fetch_plane(0, I0{});
        commit_plane(0, I0{});
        keep_own(I0{});
        if constexpr (kDeep) {
            if (1 < nq) fetch_plane(1, I1{});
        }
    } else {
        load_plane(0, 0);
    }
    if constexpr (kEpiPre) {
        if constexpr (kDeep) {
            fetch_epi(1 - D, std::integral_constant<int, (1 - D) & 1>{});
            fetch_epi(2 - D, std::integral_constant<int, (2 - D) & 1>{});
        } else {
            fetch_epi(-(D - 1), I0{});
        }
    }
    __syncthreads();
    auto march = [&](int q, auto qp) __attribute__((always_inline)) {
        // QP = q & 1 with kDeep, else 0
        constexpr int QP = decltype(qp)::value;
        // register set of this iteration's output plane o = q - (D - 1)
        constexpr int ES = kDeep ? (QP ^ ((D - 1) & 1)) : 0;
        const int buf = kDeep ? QP : (q & 1);
        if constexpr (kDeep) {
            if (q + 2 < nq) fetch_plane(q + 2, qp);
        } else if constexpr (kPrefetch && NIN == 1) {
            if (q + 1 < nq) fetch_plane(q + 1, I0{});
        } else {
            if (q + 1 < nq) load_plane(q + 1, buf ^ 1);
        }
        if constexpr (ISO) {
            // isotropic couplings: shared partial sums, then one FMA per use
            constexpr int NSUM = SumC<KIND>::t.nsum;
            static_for<NSUM>([&](auto kc) __attribute__((always_inline)) {
                constexpr int ks = decltype(kc)::value;
                constexpr ZSum sm = SumC<KIND>::t.sums[ks];
                static_for<kYB>([&](auto ybc) __attribute__((always_inline)) {
                    constexpr int yb = decltype(ybc)::value;
                    static_for<NIN>([&](auto inc) __attribute__((always_inline)) {
                        constexpr int in = decltype(inc)::value;
                        T v[3] = {T(0), T(0), T(0)};
                        static_for<sm.n>([&](auto mc) __attribute__((always_inline)) {
                            constexpr int m = decltype(mc)::value;
                            const int off = (ty * kYB + yb + sm.dy[m] + RY) * PW + tx + sm.dx[m] + RX;
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                const T sv = lds[buf][in][sm.b[m]][c][off];
                                v[c] = m == 0 ? sv : v[c] + sv;
                            }
                        });
                        static_for<sm.nu>([&](auto uc) __attribute__((always_inline)) {
                            constexpr ZUse u = SumC<KIND>::t.uses[sm.u0 + decltype(uc)::value];
                            constexpr int slot = DZHI - u.dz;
                            const T J = W.w[u.shell];
#pragma unroll
                            for (int c = 0; c < 3; ++c) acc[slot][yb][u.a][c][in] += J * v[c];
                        });
                    });
                });
                // scheduling fence where the next sum reads another source
                // sublattice: sums over one sublattice share their staged
                // reads, and only that sublattice's values are live at a time
                // (after every sum when two states are staged)
                if constexpr (ks + 1 < NSUM) {
                    if constexpr (NIN == 2 || SumC<KIND>::t.sums[ks + 1].b[0] != sm.b[0]) {
#pragma unroll
                        for (int s2 = 0; s2 < D; ++s2)
#pragma unroll
                            for (int yb = 0; yb < kYB; ++yb)
#pragma unroll
                                for (int a2 = 0; a2 < NSUB; ++a2)
#pragma unroll
                                    for (int c = 0; c < 3; ++c)
#pragma unroll
                                        for (int in = 0; in < NIN; ++in)
                                            asm volatile("" : "+v"(acc[s2][yb][a2][c][in]));
                        asm volatile("" ::: "memory");
                    }
                }
            });
        } else {
        static_for<NB>([&](auto kc) __attribute__((always_inline)) {
            constexpr int kb = decltype(kc)::value;
            constexpr ZBond bd = ShapeC<KIND>::t.bonds[kb];
            constexpr int slot = DZHI - bd.dz;
            static_for<kYB>([&](auto ybc) __attribute__((always_inline)) {
                constexpr int yb = decltype(ybc)::value;
                const int off = (ty * kYB + yb + bd.dy + RY) * PW + tx + bd.dx + RX;
                static_for<NIN>([&](auto inc) __attribute__((always_inline)) {
                    constexpr int in = decltype(inc)::value;
                    const T s0 = lds[buf][in][bd.b][0][off];
                    const T s1 = lds[buf][in][bd.b][1][off];
                    const T s2 = lds[buf][in][bd.b][2][off];
                    const T *J = &W.w[9 * kb];
                    acc[slot][yb][bd.a][0][in] += J[0] * s0 + J[1] * s1 + J[2] * s2;
                    acc[slot][yb][bd.a][1][in] += J[3] * s0 + J[4] * s1 + J[5] * s2;
                    acc[slot][yb][bd.a][2][in] += J[6] * s0 + J[7] * s1 + J[8] * s2;
                });
            });
            // scheduling fence between source rows (b, dy): the pending sums
            // are forced out and the next row's staged values are read after
            // it, so only one row of staged values is live at a time (fewer
            // registers, more resident waves)
            if constexpr (kb + 1 < NB) {
                constexpr ZBond nx = ShapeC<KIND>::t.bonds[kb + 1];
                if constexpr (nx.b != bd.b || nx.dy != bd.dy) {
#pragma unroll
                    for (int s2 = 0; s2 < D; ++s2)
#pragma unroll
                        for (int yb = 0; yb < kYB; ++yb)
#pragma unroll
                            for (int a2 = 0; a2 < NSUB; ++a2)
#pragma unroll
                                for (int c = 0; c < 3; ++c)
#pragma unroll
                                    for (int in = 0; in < NIN; ++in) asm volatile("" : "+v"(acc[s2][yb][a2][c][in]));
                    asm volatile("" ::: "memory");
                }
            }
        });
        }
        // output plane q - (D-1) (slot 0) has received all of its inputs
        const int o = q - (D - 1);
        constexpr bool kCorr = MODE == ZM_CORRECT_P || MODE == ZM_CORRECT || MODE == ZM_CORRECT_STORED;
        if constexpr (kCorr) {
        if (o >= 0 && o < nout) {
            const int x = x0 + tx;
            // sublattices unrolled (the on-site tables are indexed by a at
            // compile time), rows by a runtime loop with register selects
            static_for<NSUB>([&](auto ac) __attribute__((always_inline)) {
                constexpr int a = decltype(ac)::value;
                // rows go through one copy of the epilogue: row yb's values
                // are always in slot 0, shifted down after each row
                T fin[kYB][NIN][3];
                double ef[kYB][NE], sf[kYB][3];
#pragma unroll
                for (int yb = 0; yb < kYB; ++yb) {
#pragma unroll
                    for (int in = 0; in < NIN; ++in)
#pragma unroll
                        for (int c = 0; c < 3; ++c) fin[yb][in][c] = acc[0][yb][a][c][in];
#pragma unroll
                    for (int k = 0; k < NE; ++k) ef[yb][k] = kEpiPre ? epi[ES][yb][a][k] : 0.0;
#pragma unroll
                    for (int c = 0; c < 3; ++c) sf[yb][c] = kOwn ? own[0][a * kYB + yb][c] : 0.0;
                }
#pragma unroll 1
                for (int yb = 0; yb < kYB; ++yb) {
                    const int y = y0 + ty * kYB + yb;
                    if (x < g.Lx && y < g.Ly)
                        finish_corr(ac, (int64_t)a * g.M + x + (int64_t)g.Lx * (y + (int64_t)g.Ly * (zs + o)), fin[0],
                                    ef[0], sf[0]);
#pragma unroll
                    for (int k = 0; k + 1 < kYB; ++k) {
#pragma unroll
                        for (int in = 0; in < NIN; ++in)
#pragma unroll
                            for (int c = 0; c < 3; ++c) fin[k][in][c] = fin[k + 1][in][c];
#pragma unroll
                        for (int m = 0; m < NE; ++m) ef[k][m] = ef[k + 1][m];
#pragma unroll
                        for (int c = 0; c < 3; ++c) sf[k][c] = sf[k + 1][c];
                    }
                }
            });
        }
        } else {
        if (o >= 0 && o < nout) {
            const int x = x0 + tx;
            // rows go through one copy of the epilogue: row yb's values are
            // always in slot 0 of these arrays, shifted down after each row
            T fin[kYB][NSUB][NIN][3];
            double ef[kYB][NSUB][NE], sf[kYB][NSUB][3];
#pragma unroll
            for (int yb = 0; yb < kYB; ++yb)
#pragma unroll
                for (int a = 0; a < NSUB; ++a) {
#pragma unroll
                    for (int in = 0; in < NIN; ++in)
#pragma unroll
                        for (int c = 0; c < 3; ++c) fin[yb][a][in][c] = acc[0][yb][a][c][in];
#pragma unroll
                    for (int k = 0; k < NE; ++k) ef[yb][a][k] = kEpiPre ? epi[ES][yb][a][k] : 0.0;
#pragma unroll
                    for (int c = 0; c < 3; ++c) sf[yb][a][c] = kOwn ? own[0][a * kYB + yb][c] : 0.0;
                }
#pragma unroll 1
            for (int yb = 0; yb < kYB; ++yb) {
                const int y = y0 + ty * kYB + yb;
                finish_row(x, y, zs + o, x < g.Lx && y < g.Ly, fin[0], ef[0], sf[0]);
#pragma unroll
                for (int k = 0; k + 1 < kYB; ++k)
#pragma unroll
                    for (int a = 0; a < NSUB; ++a) {
#pragma unroll
                        for (int in = 0; in < NIN; ++in)
#pragma unroll
                            for (int c = 0; c < 3; ++c) fin[k][a][in][c] = fin[k + 1][a][in][c];
#pragma unroll
                        for (int m = 0; m < NE; ++m) ef[k][a][m] = ef[k + 1][a][m];
#pragma unroll
                        for (int c = 0; c < 3; ++c) sf[k][a][c] = sf[k + 1][a][c];
                    }
            }
        }
        }
        // rotate the ring: slot k <- k+1, the top slot starts a new plane
#pragma unroll
        for (int k = 0; k + 1 < D; ++k)
#pragma unroll
            for (int yb = 0; yb < kYB; ++yb)
#pragma unroll
                for (int a = 0; a < NSUB; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
#pragma unroll
                        for (int in = 0; in < NIN; ++in) acc[k][yb][a][c][in] = acc[k + 1][yb][a][c][in];
#pragma unroll
        for (int yb = 0; yb < kYB; ++yb)
#pragma unroll
            for (int a = 0; a < NSUB; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int in = 0; in < NIN; ++in) acc[D - 1][yb][a][c][in] = T(0);
        if constexpr (kPrefetch && NIN == 1) {
            constexpr int CP = kDeep ? (QP ^ 1) : 0;  // set holding plane q + 1
            if (q + 1 < nq) commit_plane(buf ^ 1, std::integral_constant<int, CP>{});
            keep_own(std::integral_constant<int, CP>{});  // every iteration, so that own[0] stays aligned
        }
        // the per-site inputs of a later output plane are in flight across
        // the barrier and the next iteration's stencil (two of them with
        // kDeep: output o + 2 reuses the set that o just released)
        if constexpr (kEpiPre) {
            if constexpr (kDeep) fetch_epi(q - D + 3, std::integral_constant<int, ES>{});
            else fetch_epi(q - D + 2, I0{});
        }
        __syncthreads();
    };
    if constexpr (kDeep) {
#pragma unroll 1
        for (int q = 0; q < nq; q += 2) {
            march(q, I0{});
            if (q + 1 < nq) march(q + 1, I1{});
        }
    } else {
#pragma unroll 1
        for (int q = 0; q < nq; ++q) march(q, I0{});
    }
    if constexpr (MODE == ZM_MIN_FORCE) {
        // fixed-order block reductions (the first a maximum), one set per tile
        __shared__ double mr[6][kThreads / 64];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double v = mred[k];
            if (k == 0) {
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
            } else {
                v = wave_sum(v);
            }
            if ((threadIdx.x & 63) == 0) mr[k][threadIdx.x >> 6] = v;
        }
        __syncthreads();
        if (threadIdx.x < 6) {
            const int k = threadIdx.x;
            double t = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) t = k == 0 ? fmax(t, mr[k][w]) : t + mr[k][w];
            g.gpart[(size_t)tile * 6 + k] = t;
        }
    }
    if constexpr (MODE == ZM_GNEB_A2 || MODE == ZM_GNEB_C2) {
        // fixed-order block sums (A2: energy, squared distance and the nine
        // image sums) or maximum (C2: max |F_gneb|), one set per tile
        constexpr int NV = MODE == ZM_GNEB_A2 ? 11 : 1;
        __shared__ double gred[NV][kThreads / 64];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double v = MODE == ZM_GNEB_C2 ? sqrt(gX[0]) : gacc[k * kThreads + threadIdx.x];
            if constexpr (MODE == ZM_GNEB_C2) {
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
            } else {
                v = wave_sum(v);
            }
            if ((threadIdx.x & 63) == 0) gred[k][threadIdx.x >> 6] = v;
        }
        __syncthreads();
        if (threadIdx.x < NV) {
            double t = 0.0;
            for (int w = 0; w < kThreads / 64; ++w)
                t = MODE == ZM_GNEB_C2 ? fmax(t, gred[threadIdx.x][w]) : t + gred[threadIdx.x][w];
            g.gpart[((size_t)g.gitem0 + (size_t)gimg * g.gipi + stile) * 11 + threadIdx.x] = t;
        }
    }
    if constexpr (MODE == ZM_ENERGY) {
        // fixed-order block sums of the four terms, one quadruple per tile
        __shared__ double ered[4][kThreads / 64];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double v = wave_sum(eE[k]);
            if ((threadIdx.x & 63) == 0) ered[k][threadIdx.x >> 6] = v;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            double t = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) t += ered[threadIdx.x][w];
            g.gpart[(size_t)tile * 4 + threadIdx.x] = t;
        }
    }
}

// Thermal noise of one Heun step for every site (Heun mode 4: generated by
// this elementwise pass, read by both stages).
__global__ __launch_bounds__(256) void k_noise_pre(HeunConst hc, uint64_t step, int64_t N, double *__restrict__ eta) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    double e[3];
    thermal_eta(hc.seed, noise_step(hc, step), hc.tag, (uint64_t)i, e);
    eta[i] = e[0];
    eta[N + i] = e[1];
    eta[2 * N + i] = e[2];
}

// Split Heun stages (elementwise over the sites of sublattice blockIdx.y):
// the bilinear field comes from the ZM_BIL pass, on-site terms and the
// integration are FP64.
// Predictor: S~ = N[S + dt f(S)], P = S + dt/2 f(S), eta stored for the corrector.
__global__ __launch_bounds__(256) void k_heun_pre(int64_t M, int64_t N, Onsite os, HeunConst hc, uint64_t step,
                                                  const double *__restrict__ S, const float *__restrict__ bil,
                                                  const float *__restrict__ bdip, double *__restrict__ St,
                                                  double *__restrict__ P, double *__restrict__ eta_out) {
    const int a = blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= M) return;
    const int64_t i = (int64_t)a * M + t;
    const double s[3] = {S[i], S[N + i], S[2 * N + i]};
    double ba[3];
    aniso_field(os, a, s, ba);
    double B[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double v = (double)bil[c * N + i] + ba[c] + os.bz[a][c];
        if (bdip) v += (double)bdip[c * N + i];
        B[c] = v * hc.inv_mumuB[a];
    }
    if (hc.noise) {
        double eta[3];
        thermal_eta(hc.seed, noise_step(hc, step), hc.tag, (uint64_t)i, eta);
        const double sg = hc.sigma[a];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            B[c] += sg * eta[c];
            eta_out[c * N + i] = eta[c];
        }
    }
    double f[3];
    llg_rhs(s, B, hc.pre, hc.alpha, f);
    const double hdt = 0.5 * hc.dt;
    double p[3] = {s[0] + hc.dt * f[0], s[1] + hc.dt * f[1], s[2] + hc.dt * f[2]};
    normalise3(p);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        P[c * N + i] = s[c] + hdt * f[c];
        St[c * N + i] = p[c];
    }
}

// Corrector: S' = N[P + dt/2 f(S~)] with the predictor's eta.
__global__ __launch_bounds__(256) void k_heun_post(int64_t M, int64_t N, Onsite os, HeunConst hc,
                                                   const double *__restrict__ St, const float *__restrict__ bil,
                                                   const float *__restrict__ bdip, const double *__restrict__ P,
                                                   const double *__restrict__ eta, double *__restrict__ out) {
    const int a = blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= M) return;
    const int64_t i = (int64_t)a * M + t;
    const double s[3] = {St[i], St[N + i], St[2 * N + i]};
    double bt[3];
    aniso_field(os, a, s, bt);
    double B[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double v = (double)bil[c * N + i] + bt[c] + os.bz[a][c];
        if (bdip) v += (double)bdip[c * N + i];
        B[c] = v * hc.inv_mumuB[a];
    }
    if (hc.noise) {
        const double sg = hc.sigma[a];
#pragma unroll
        for (int c = 0; c < 3; ++c) B[c] += sg * eta[c * N + i];
    }
    double f[3];
    llg_rhs(s, B, hc.pre, hc.alpha, f);
    const double hdt = 0.5 * hc.dt;
    double p[3] = {P[i] + hdt * f[0], P[N + i] + hdt * f[1], P[2 * N + i] + hdt * f[2]};
    normalise3(p);
    out[i] = p[0];
    out[N + i] = p[1];
    out[2 * N + i] = p[2];
}

// Compute units of the current device (queried once per process).
int device_cus() {
    static int n = 0;
    if (n == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            return 0;
        n = v;
    }
    return n;
}

template <int KIND, typename T, bool ISO, int MODE, int TXW>
hipError_t launch_tile(const ZPlan &zp, const ZArgs &a0, const Onsite &os, const HeunConst &hc, hipStream_t st) {
    constexpr int NB = make_shape(KIND).nb;
    constexpr int NW = ISO ? make_shape(KIND).nshell : 9 * NB;
    constexpr int kBlock = zm_block(MODE, KIND), kRows = kBlock / TXW * kYB;
    ZWeights<T, NW> W;
    for (int k = 0; k < NW; ++k) W.w[k] = (T)(sizeof(T) == 4 ? (double)zp.wf[k] : zp.wd[k]);
    const int64_t ntile = (int64_t)((a0.Lx + TXW - 1) / TXW) * ((a0.Ly + kRows - 1) / kRows) * a0.nzc * a0.nimg;
    if (ntile > 0x7fffffff) return hipErrorInvalidValue;
    // a grid whose tiles are all resident at once (two blocks per CU) gets
    // the XCD-contiguous tile order: the x/y halo rows shared by concurrent
    // neighbouring tiles are then fetched into one L2 once (measured: the
    // bcc 128^3 bilinear pass fetches 2.25x fewer bytes).  Larger grids keep
    // the round-robin order, which measured faster there.
    ZArgs a = a0;
    const int ncu = device_cus();
    a.xcd = (a0.imgfast || (ncu > 0 && ntile <= 2 * (int64_t)ncu)) ? 1 : 0;
    k_zmarch<KIND, T, ISO, MODE, TXW><<<(unsigned)ntile, kBlock, 0, st>>>(a, os, hc, W);
    return hipGetLastError();
}

template <int KIND, typename T, bool ISO, int MODE>
hipError_t launch_kind(const ZPlan &zp, const ZArgs &a, const Onsite &os, const HeunConst &hc, hipStream_t st) {
    if constexpr (zm_gneb(MODE)) {
        if (zp.txw == 32) return launch_tile<KIND, T, ISO, MODE, 32>(zp, a, os, hc, st);
        if (zp.txw == 16) return launch_tile<KIND, T, ISO, MODE, 16>(zp, a, os, hc, st);
    }
    if (zp.txw != kTX) return hipErrorInvalidValue;
    return launch_tile<KIND, T, ISO, MODE, kTX>(zp, a, os, hc, st);
}

template <typename T, bool ISO, int MODE>
hipError_t launch_mode(const ZPlan &zp, const ZArgs &a, const Onsite &os, const HeunConst &hc, hipStream_t st) {
    switch (zp.kind) {
    case SHAPE_SC_NN: return launch_kind<SHAPE_SC_NN, T, ISO, MODE>(zp, a, os, hc, st);
    case SHAPE_SC_3SH:
        if constexpr (ISO) return launch_kind<SHAPE_SC_3SH, T, ISO, MODE>(zp, a, os, hc, st);
        break;
    case SHAPE_SC_4SH:
        if constexpr (ISO) return launch_kind<SHAPE_SC_4SH, T, ISO, MODE>(zp, a, os, hc, st);
        break;
    case SHAPE_BCC_5SH:
        if constexpr (ISO && sizeof(T) == 4) return launch_kind<SHAPE_BCC_5SH, T, ISO, MODE>(zp, a, os, hc, st);
        break;
    default: break;
    }
    return hipErrorInvalidValue;
}

template <int MODE>
hipError_t launch_any(const ZPlan &zp, const ZArgs &a, const Onsite &os, const HeunConst &hc, hipStream_t st) {
    if (zp.prec == 0) {
        if (zp.iso) return launch_mode<double, true, MODE>(zp, a, os, hc, st);
        return launch_mode<double, false, MODE>(zp, a, os, hc, st);
    }
    if (zp.iso) return launch_mode<float, true, MODE>(zp, a, os, hc, st);
    return launch_mode<float, false, MODE>(zp, a, os, hc, st);
}

ZArgs make_args(const ZPlan &zp, const Grid &g) {
    ZArgs a{};
    a.Lx = g.Lx;
    a.Ly = g.Ly;
    a.Lz = g.Lz;
    for (int k = 0; k < 3; ++k) a.per[k] = g.per[k];
    a.M = g.M;
    a.N = g.N;
    a.zch = zp.zch;
    a.nzc = (g.Lz + zp.zch - 1) / zp.zch;
    a.nimg = 1;
    return a;
}

}  // namespace

// ---------------------------------------------------------------- host planning
bool zmarch_plan(int prec, int n_sub, const int *bond_a, const int *bond_b, const int *bond_d,
                 const double *bond_J, int n_bonds, bool iso, ZPlan &zp) {
    zp = ZPlan{};
    if (prec != 0 && prec != 1) return false;
    for (int kind = 0; kind < SHAPE_COUNT; ++kind) {
        const ShapeTable t = make_shape(kind);
        if (t.nsub != n_sub) continue;
        // supported instantiations (LDS budget): tensors only on SC_NN, FP64 not on bcc
        if (!iso && kind != SHAPE_SC_NN) continue;
        if (prec == 0 && kind == SHAPE_BCC_5SH) continue;
        // isotropic tables: one coupling per shell (every bond of a shell must
        // carry the same J); tensor tables: one 3x3 block per bond
        const int nwb = (iso ? 1 : 9) * t.nb;
        std::vector<double> w(nwb, 0.0);
        bool ok = true;
        for (int p = 0; p < n_bonds && ok; ++p) {
            int hit = -1;
            for (int k = 0; k < t.nb; ++k) {
                const ZBond &z = t.bonds[k];
                if (z.a == bond_a[p] && z.b == bond_b[p] && z.dx == bond_d[3 * p] && z.dy == bond_d[3 * p + 1] &&
                    z.dz == bond_d[3 * p + 2]) {
                    hit = k;
                    break;
                }
            }
            if (hit < 0) { ok = false; break; }
            if (iso) w[hit] += bond_J[9 * p];
            else
                for (int e = 0; e < 9; ++e) w[9 * hit + e] += bond_J[9 * p + e];
        }
        if (!ok) continue;
        int nw = nwb;
        if (iso) {
            std::vector<double> ws(t.nshell, 0.0);
            std::vector<int> seen(t.nshell, 0);
            for (int k = 0; k < t.nb && ok; ++k) {
                const int sh = t.bonds[k].shell;
                if (!seen[sh]) { ws[sh] = w[k]; seen[sh] = 1; }
                else if (w[k] != ws[sh]) ok = false;
            }
            if (!ok) continue;
            w = ws;
            nw = t.nshell;
        }
        zp.kind = kind;
        zp.prec = prec;
        zp.iso = iso ? 1 : 0;
        zp.nw = nw;
        for (int k = 0; k < nw; ++k) {
            zp.wd[k] = w[k];
            zp.wf[k] = (float)w[k];
        }
        zp.zch = 8;
        zp.valid = true;
        return true;
    }
    return false;
}

hipError_t zmarch_field(const ZPlan &zp, const Grid &g, const Onsite &os, const double *S, const float *bdip,
                        void *b, hipStream_t st) {
    ZArgs a = make_args(zp, g);
    a.S0 = S;
    a.bout = b;
    a.bdip0 = bdip;
    HeunConst hc{};
    return launch_any<ZM_FIELD>(zp, a, os, hc, st);
}

hipError_t zmarch_energy(const ZPlan &zp, const Grid &g, const Onsite &os, const double *S, const float *bdip,
                         double *partial, hipStream_t st) {
    ZArgs a = make_args(zp, g);
    a.S0 = S;
    a.bdip0 = bdip;
    a.gpart = partial;
    HeunConst hc{};
    return launch_any<ZM_ENERGY>(zp, a, os, hc, st);
}

hipError_t zmarch_bil(const ZPlan &zp, const Grid &g, const double *S, float *bil, hipStream_t st) {
    if (zp.prec != 1) return hipErrorInvalidValue;
    ZArgs a = make_args(zp, g);
    a.S0 = S;
    a.bout = bil;
    Onsite os{};
    HeunConst hc{};
    return launch_any<ZM_BIL>(zp, a, os, hc, st);
}

hipError_t zmarch_min_force(const ZPlan &zp, const Grid &g, const Onsite &os, const double *S, double *F,
                            const double *V, const double *Up, const double *Fp, double *Sh, double *Yh,
                            const double *state, int done_idx, int cand_idx, int method, double *partial,
                            hipStream_t st) {
    if (zp.prec != 0) return hipErrorInvalidValue;
    ZArgs a = make_args(zp, g);
    a.S0 = S;
    a.skip = state + done_idx;  // the minimiser has converged: no-op
    a.gF = F;
    a.gpart = partial;
    a.mV = V;
    a.mUp = Up;
    a.mFp = Fp;
    a.mSh = Sh;
    a.mYh = Yh;
    a.mst = state;
    a.mmethod = method;
    a.mcand_idx = cand_idx;
    HeunConst hc{};
    if (zp.iso) return launch_mode<double, true, ZM_MIN_FORCE>(zp, a, os, hc, st);
    return launch_mode<double, false, ZM_MIN_FORCE>(zp, a, os, hc, st);
}

int zmarch_tiles(const ZPlan &zp, const Grid &g) { return zm_tiles(g, zp.zch, kThreads, kTX); }

int zmarch_gneb_tiles(const ZPlan &zp, const Grid &g) {
    return zm_tiles(g, zp.zch, zm_block(ZM_GNEB_A2, zp.kind), zp.txw);
}

int zmarch_gneb_width(const ZPlan &zp, const Grid &g) {
    // the width with the fewest padded sites in x and y (the wider on ties)
    int best = kTX;
    int64_t area = -1;
    for (int w = kTX; w >= 16; w >>= 1) {
        const int rows = zm_block(ZM_GNEB_A2, zp.kind) / w * kYB;
        const int64_t a = (int64_t)((g.Lx + w - 1) / w) * w * (((g.Ly + rows - 1) / rows) * rows);
        if (area < 0 || a < area) {
            area = a;
            best = w;
        }
    }
    return best;
}

hipError_t zmarch_gneb_pass(int pass, const ZPlan &zp, const Grid &g, const Onsite &os, const GnebPassArgs &ga,
                            hipStream_t st) {
    if (zp.prec != 0 || ga.n_img < 3 || zmarch_gneb_tiles(zp, g) > ga.items_per_img) return hipErrorInvalidValue;
    ZArgs a = make_args(zp, g);
    a.bstride = 3 * g.N;
    a.gntot = ga.n_img;
    // the second pass runs over the interior images only
    a.gimg0 = pass == 0 ? 0 : 1;
    a.nimg = pass == 0 ? ga.n_img : ga.n_img - 2;
    a.S0 = ga.Y0;
    a.S0alt = ga.Y1;
    a.sel = ga.cur;
    a.skip = ga.done;
    a.O0 = ga.Y1;
    a.O1 = ga.Y0;
    a.gV = ga.V;
    a.gims = ga.img;
    a.gst = ga.st;
    a.gis = ga.slots;
    a.gdt = ga.dt;
    a.gmass = ga.mass;
    a.gstring = ga.string;
    a.gpart = ga.partial;
    a.gitem0 = ga.item0;
    a.gipi = ga.items_per_img;
    a.imgfast = 1;
    HeunConst hc{};
    if (pass == 0) {
        if (zp.iso) return launch_mode<double, true, ZM_GNEB_A2>(zp, a, os, hc, st);
        return launch_mode<double, false, ZM_GNEB_A2>(zp, a, os, hc, st);
    }
    if (zp.iso) return launch_mode<double, true, ZM_GNEB_C2>(zp, a, os, hc, st);
    return launch_mode<double, false, ZM_GNEB_C2>(zp, a, os, hc, st);
}

hipError_t zmarch_bil_images(const ZPlan &zp, const Grid &g, int n_img, const double *S0, const double *S0alt,
                             const double *sel, const double *skip, double *bil, hipStream_t st) {
    if (zp.prec != 0 || n_img <= 0) return hipErrorInvalidValue;
    ZArgs a = make_args(zp, g);
    a.S0 = S0;
    a.S0alt = S0alt ? S0alt : S0;
    a.sel = sel;
    a.skip = skip;
    a.nimg = n_img;
    a.bstride = 3 * g.N;
    a.bout = bil;
    Onsite os{};
    HeunConst hc{};
    return launch_any<ZM_BIL>(zp, a, os, hc, st);
}

hipError_t heun_split_pre(const Grid &g, const Onsite &os, const HeunConst &hc, uint64_t step, const double *S,
                          const float *bil, const float *bdip, double *St, double *P, double *eta, hipStream_t st) {
    dim3 grid((unsigned)((g.M + 255) / 256), (unsigned)g.n_sub);
    k_heun_pre<<<grid, 256, 0, st>>>(g.M, g.N, os, hc, step, S, bil, bdip, St, P, eta);
    return hipGetLastError();
}

hipError_t heun_split_post(const Grid &g, const Onsite &os, const HeunConst &hc, const double *St, const float *bil,
                           const float *bdip, const double *P, const double *eta, double *out, hipStream_t st) {
    dim3 grid((unsigned)((g.M + 255) / 256), (unsigned)g.n_sub);
    k_heun_post<<<grid, 256, 0, st>>>(g.M, g.N, os, hc, St, bil, bdip, P, eta, out);
    return hipGetLastError();
}

hipError_t zmarch_noise(const HeunConst &hc, uint64_t step, int64_t N, double *eta, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    k_noise_pre<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(hc, step, N, eta);
    return hipGetLastError();
}

hipError_t zmarch_predict(const ZPlan &zp, const Grid &g, const Onsite &os, const HeunConst &hc, uint64_t step,
                          const double *S, const float *bdip, double *St, float *bstore, double *pstore,
                          double *estore, const double *eload, hipStream_t st) {
    ZArgs a = make_args(zp, g);
    a.eload = eload;
    a.S0 = S;
    a.out = St;
    a.bdip0 = bdip;
    a.bstore = bstore;
    a.pstore = pstore;
    a.estore = estore;
    a.step = step;
    return launch_any<ZM_PREDICT>(zp, a, os, hc, st);
}

hipError_t zmarch_correct(const ZPlan &zp, const Grid &g, const Onsite &os, const HeunConst &hc, uint64_t step,
                          const double *S, const double *St, const float *bdipS, const float *bdipT,
                          const float *bload, const double *pload, const double *eload, double *out,
                          hipStream_t st) {
    ZArgs a = make_args(zp, g);
    a.S0 = S;
    a.S1 = St;
    a.out = out;
    a.bdip0 = bdipS;
    a.bdip1 = bdipT;
    a.bload = bload;
    a.pload = pload;
    a.eload = eload;
    a.step = step;
    if (pload) return launch_any<ZM_CORRECT_P>(zp, a, os, hc, st);  // eload NULL: noise drawn again
    if (bload) return launch_any<ZM_CORRECT_STORED>(zp, a, os, hc, st);
    return launch_any<ZM_CORRECT>(zp, a, os, hc, st);
}

}  // namespace spx
