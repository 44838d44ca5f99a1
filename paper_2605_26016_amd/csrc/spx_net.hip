// spx_net.hip -- the learned GNEB initial-path corrector: a 4-layer 3^3
// convolution network (10 -> 16 -> 16 -> 16 -> 3 channels, zero padding,
// SiLU between layers) with hand-written FP32 forward, backward and Adam
// kernels.  Input per image: the geodesic guess S_g, the two end images S_A,
// S_B and the reaction coordinate t (10 channels); output u (3 channels) is
// projected on the tangent plane of S_g and applied by the exponential map
// S_hat = exp_{S_g}(P u) (the retraction of the Methods' minimum-energy-path
// section).  Training loss: mean over images and sites of |S_hat - S*|^2.
//
// Activations are [batch][channel][z][y][x] FP32.  Convolutions are direct:
// a 256-thread block owns an 8 x 8 x 4 output tile, stages the (10 x 10 x 6)
// input halo tile of every input channel in LDS (SiLU applied on load) and
// reads the weights through the scalar cache (uniform over the block).  The
// input gradient is the same convolution with transposed, flipped weights;
// weight gradients use one (out, in) channel pair per thread over the block's
// sites, then a fixed-order reduction over blocks (deterministic).
//
// A layer may be dilated by d (tap k reads offset (k - 1) d per axis, which
// widens the receptive field of the four layers from 9 to 1 + 2 (d1 + d2 +
// d3 + d4) cells).  The sites of one phase (px, py, pz) in [0, d)^3, at
// (px + d sx, py + d sy, pz + d sz), only read each other, so a dilated
// layer runs as the same 3^3 tiles over every phase's sub-grid of
// ceil(L / d) sites per axis: tiles stay in sub-grid coordinates and only
// the global addressing is strided.
//
// Inference may instead run every layer as a BF16 implicit GEMM on the
// matrix cores (spx_net_set_precision): for 16 output sites x 16 output
// channels (inputs and outputs padded to 16 channels), K runs over pairs of
// taps x 16 input channels, 14 v_mfma_f32_16x16x32_bf16 per layer with FP32
// accumulation.  The activations between layers are stored as BF16 with the
// channels innermost (32 bytes per site), each layer's epilogue applying
// the next layer's SiLU, so a tile is staged in LDS by 16-byte copies and a
// lane's operand fragment (8 channels of one site and tap) is one 16-byte
// read; the weight fragments of a layer are packed from the FP32 parameters
// by a small kernel before the layer runs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "spx_device.hpp"
#include "spx_ext.hpp"

namespace spx {
namespace {

constexpr int kTXn = 8, kTYn = 8, kTZn = 4;  // output tile
constexpr int kHX = kTXn + 2, kHY = kTYn + 2, kHZ = kTZn + 2;
constexpr int kHalo = kHX * kHY * kHZ;
constexpr int kNT = 256;

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

struct NetDims {
    int Lx, Ly, Lz;
    int64_t P;
    int dil;         // dilation of the layer
    int Sx, Sy, Sz;  // sub-grid extents ceil(L / dil)
};

// Tile of this block: origin (x0, y0, z0) in sub-grid coordinates and the
// phase (px, py, pz).  blockIdx.x = bx + nbx (by + nby (px + dil py)),
// blockIdx.y = bz + nbz pz.
struct NetTile {
    int x0, y0, z0, px, py, pz;
};
__device__ __forceinline__ NetTile tile_origin_at(const NetDims &d, int bx, int by) {
    const int nbx = (d.Sx + kTXn - 1) / kTXn, nby = (d.Sy + kTYn - 1) / kTYn, nbz = (d.Sz + kTZn - 1) / kTZn;
    NetTile t;
    int r = bx;
    t.x0 = (r % nbx) * kTXn;
    r /= nbx;
    t.y0 = (r % nby) * kTYn;
    r /= nby;
    t.px = r % d.dil;
    t.py = r / d.dil;
    t.z0 = (by % nbz) * kTZn;
    t.pz = by / nbz;
    return t;
}
__device__ __forceinline__ NetTile tile_origin(const NetDims &d) {
    return tile_origin_at(d, (int)blockIdx.x, (int)blockIdx.y);
}

// Stage CIN input channels of image blockIdx.z with a 1-cell zero halo (in
// sub-grid cells: d sites in the lattice).
template <int CIN, bool SILU_IN>
__device__ __forceinline__ void stage_tile(const float *__restrict__ in, const NetDims &d, const NetTile &t,
                                           float (*tile)[kHalo]) {
    const float *src = in + (int64_t)blockIdx.z * CIN * d.P;
    for (int idx = threadIdx.x; idx < CIN * kHalo; idx += kNT) {
        const int ci = idx / kHalo, r = idx - ci * kHalo;
        const int hx = r % kHX, hy = (r / kHX) % kHY, hz = r / (kHX * kHY);
        const int gx = t.px + d.dil * (t.x0 + hx - 1), gy = t.py + d.dil * (t.y0 + hy - 1),
                  gz = t.pz + d.dil * (t.z0 + hz - 1);
        float v = 0.0f;
        if (gx >= 0 && gy >= 0 && gz >= 0 && gx < d.Lx && gy < d.Ly && gz < d.Lz) {
            v = src[ci * d.P + gx + (int64_t)d.Lx * (gy + (int64_t)d.Ly * gz)];
            if (SILU_IN) v = silu(v);
        }
        tile[ci][r] = v;
    }
}

// out[co] = bias[co] + sum_ci sum_k W[co][ci][k] a[ci](p + k - 1)   (bias may be NULL)
// MUL_GRAD: the result is multiplied by silu'(zmul) (input-gradient pass).
template <int CIN, int COUT, bool SILU_IN, bool MUL_GRAD>
__global__ __launch_bounds__(kNT) void k_conv(const float *__restrict__ in, const float *__restrict__ W,
                                              const float *__restrict__ bias, const float *__restrict__ zmul,
                                              float *__restrict__ out, NetDims d) {
    __shared__ float tile[CIN][kHalo];
    const NetTile tl = tile_origin(d);
    stage_tile<CIN, SILU_IN>(in, d, tl, tile);
    __syncthreads();
    const int tx = threadIdx.x % kTXn, ty = (threadIdx.x / kTXn) % kTYn, tz = threadIdx.x / (kTXn * kTYn);
    float acc[COUT];
#pragma unroll
    for (int co = 0; co < COUT; ++co) acc[co] = bias ? bias[co] : 0.0f;
    for (int ci = 0; ci < CIN; ++ci) {
#pragma unroll
        for (int k = 0; k < 27; ++k) {
            const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
            const float v = tile[ci][(tx + kx) + kHX * ((ty + ky) + kHY * (tz + kz))];
#pragma unroll
            for (int co = 0; co < COUT; ++co) acc[co] += W[(co * CIN + ci) * 27 + k] * v;
        }
    }
    const int x = tl.px + d.dil * (tl.x0 + tx), y = tl.py + d.dil * (tl.y0 + ty), z = tl.pz + d.dil * (tl.z0 + tz);
    if (x >= d.Lx || y >= d.Ly || z >= d.Lz) return;
    const int64_t p = x + (int64_t)d.Lx * (y + (int64_t)d.Ly * z);
    float *dst = out + (int64_t)blockIdx.z * COUT * d.P;
#pragma unroll
    for (int co = 0; co < COUT; ++co) {
        float v = acc[co];
        if (MUL_GRAD) v *= silu_grad(zmul[(int64_t)blockIdx.z * COUT * d.P + co * d.P + p]);
        dst[co * d.P + p] = v;
    }
}

// Wt[ci][co][k] = W[co][ci][26 - k]: weights of the input-gradient convolution.
__global__ void k_transpose_flip(const float *__restrict__ W, float *__restrict__ Wt, int cin, int cout) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cin * cout * 27) return;
    const int k = i % 27, co = (i / 27) % cout, ci = i / (27 * cout);
    Wt[i] = W[(co * cin + ci) * 27 + (26 - k)];
}

// Per-block weight/bias gradient partials:
//   dW[co][ci][k] = sum_p g[co](p) a[ci](p + (k - 1) d),  db[co] = sum_p g[co](p)
// over the block's output tile; partial[blk][COUT*CIN*27 + COUT].
template <int CIN, int COUT, bool SILU_IN>
__global__ __launch_bounds__(kNT) void k_conv_wgrad(const float *__restrict__ in, const float *__restrict__ g,
                                                    double *__restrict__ partial, NetDims d) {
    __shared__ float tile[CIN][kHalo];
    __shared__ float gt[COUT][kTXn * kTYn * kTZn];
    const NetTile tl = tile_origin(d);
    stage_tile<CIN, SILU_IN>(in, d, tl, tile);
    const float *gsrc = g + (int64_t)blockIdx.z * COUT * d.P;
    for (int idx = threadIdx.x; idx < COUT * kNT; idx += kNT) {
        const int co = idx / kNT, s = idx % kNT;
        const int x = tl.px + d.dil * (tl.x0 + s % kTXn), y = tl.py + d.dil * (tl.y0 + (s / kTXn) % kTYn),
                  z = tl.pz + d.dil * (tl.z0 + s / (kTXn * kTYn));
        float v = 0.0f;
        if (x < d.Lx && y < d.Ly && z < d.Lz) v = gsrc[co * d.P + x + (int64_t)d.Lx * (y + (int64_t)d.Ly * z)];
        gt[co][s] = v;
    }
    __syncthreads();
    const int nw = COUT * CIN * 27 + COUT;
    const size_t blk = (size_t)blockIdx.z * gridDim.x * gridDim.y + (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    // FP64 accumulation: the product of two floats is exact in double, so the
    // weight-gradient sums carry no FP32 rounding of their own (only that of
    // the FP32 activations and back-propagated fields they multiply)
    double *dst = partial + blk * nw;
    const int t = threadIdx.x;
    if (t < COUT * CIN) {
        const int co = t / CIN, ci = t % CIN;
        double acc[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) acc[k] = 0.0;
        for (int s = 0; s < kNT; ++s) {
            const double gv = (double)gt[co][s];
            const int sx = s % kTXn, sy = (s / kTXn) % kTYn, sz = s / (kTXn * kTYn);
#pragma unroll
            for (int k = 0; k < 27; ++k) {
                const int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
                acc[k] = fma(gv, (double)tile[ci][(sx + kx) + kHX * ((sy + ky) + kHY * (sz + kz))], acc[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < 27; ++k) dst[(co * CIN + ci) * 27 + k] = acc[k];
    }
    if (t < COUT) {
        double sb = 0.0;
        for (int s = 0; s < kNT; ++s) sb += (double)gt[t][s];
        dst[COUT * CIN * 27 + t] = sb;
    }
}

// Fixed-order FP64 sum of n_blk partial vectors of length nw, rounded to
// float once.
__global__ void k_sum_partials(const double *__restrict__ partial, int n_blk, int nw, float *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw) return;
    double s = 0.0;
    for (int b = 0; b < n_blk; ++b) s += partial[(size_t)b * nw + i];
    out[i] = (float)s;
}

// Network input: channels (S_g, S_A, S_B, t) as FP32.
// ab_stride: 3P for per-image end images, 0 when all images share them.
__global__ void k_net_input(const double *__restrict__ Sg, const double *__restrict__ SA,
                            const double *__restrict__ SB, const float *__restrict__ t, float *__restrict__ x,
                            int64_t P, int64_t ab_stride) {
    const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    const int b = blockIdx.y;
    if (p >= P) return;
    float *xb = x + (int64_t)b * 10 * P;
    const int64_t o = (int64_t)b * 3 * P, oab = (int64_t)b * ab_stride;
    for (int c = 0; c < 3; ++c) {
        xb[c * P + p] = (float)Sg[o + c * P + p];
        xb[(3 + c) * P + p] = (float)SA[oab + c * P + p];
        xb[(6 + c) * P + p] = (float)SB[oab + c * P + p];
    }
    xb[9 * P + p] = t[b];
}

// S_hat = exp_{S_g}(P_perp u) (FP64); with S* also the loss partial per block
// and d loss / d u for the backward pass (loss = mean over batch and sites).
__global__ __launch_bounds__(kNT) void k_net_head(const float *__restrict__ u, const double *__restrict__ Sg,
                                                  const double *__restrict__ Sstar, double *__restrict__ Shat,
                                                  float *__restrict__ gu, double *__restrict__ loss_part, int64_t P,
                                                  double inv_count) {
    __shared__ double red[kNT / 64];
    const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    const int b = blockIdx.y;
    double l = 0.0;
    if (p < P) {
        const int64_t o = (int64_t)b * 3 * P;
        double s[3], r[3];
        for (int c = 0; c < 3; ++c) {
            s[c] = Sg[o + c * P + p];
            r[c] = (double)u[o + c * P + p];
        }
        const double rs = r[0] * s[0] + r[1] * s[1] + r[2] * s[2];
        double w[3] = {r[0] - rs * s[0], r[1] - rs * s[1], r[2] - rs * s[2]};
        const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        double sinc, c2;  // sin(th)/th, (cos th - sinc)/th^2 with series near 0
        if (th < 1e-4) {
            const double t2 = th * th;
            sinc = 1.0 - t2 / 6.0 + t2 * t2 / 120.0;
            c2 = -1.0 / 3.0 + t2 / 30.0;
        } else {
            sinc = sin(th) / th;
            c2 = (cos(th) - sinc) / (th * th);
        }
        const double ct = cos(th);
        double h[3] = {ct * s[0] + sinc * w[0], ct * s[1] + sinc * w[1], ct * s[2] + sinc * w[2]};
        normalise3(h);
        if (Shat)
            for (int c = 0; c < 3; ++c) Shat[o + c * P + p] = h[c];
        if (Sstar) {
            double gs[3];
            for (int c = 0; c < 3; ++c) {
                const double dlt = h[c] - Sstar[o + c * P + p];
                l += dlt * dlt;
                gs[c] = 2.0 * dlt * inv_count;
            }
            const double ug = w[0] * gs[0] + w[1] * gs[1] + w[2] * gs[2];
            const double sg = s[0] * gs[0] + s[1] * gs[1] + s[2] * gs[2];
            double gw[3];
            for (int c = 0; c < 3; ++c) gw[c] = sinc * gs[c] + c2 * ug * w[c] - sinc * sg * w[c];
            const double gws = gw[0] * s[0] + gw[1] * s[1] + gw[2] * s[2];
            for (int c = 0; c < 3; ++c) gu[o + c * P + p] = (float)(gw[c] - gws * s[c]);
        }
    }
    if (loss_part) {
        const double t = wave_sum(l);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0;
            for (int w = 0; w < kNT / 64; ++w) a += red[w];
            loss_part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = a;
        }
    }
}

__global__ void k_loss_final(const double *__restrict__ part, int n, double scale, double *__restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *loss = s * scale;
}

// ---------------------------------------------------------------- BF16 MFMA form
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kTapPairs = 14;  // 27 taps in pairs, the last padded

// v_mfma_f32_16x16x32_bf16, one wavefront: lane l holds A[l % 16][8 (l / 16) + j]
// and B[8 (l / 16) + j][l % 16], j = 0..7; accumulator i of lane l is
// D[4 (l / 16) + i][l % 16].
__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Weight fragments of one layer: frag[tp][lane][j] = W[co][ci][tap] with
// co = lane % 16, tap = 2 tp + (lane / 32), ci = 8 ((lane / 16) & 1) + j
// (zero for co >= cout, ci >= cin or tap 27), rounded to BF16.
__global__ void k_wfrag(const float *__restrict__ W, int cin, int cout, bf16x8 *__restrict__ frag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kTapPairs * 64) return;
    const int tp = i / 64, lane = i % 64;
    const int co = lane % 16, tap = 2 * tp + (lane >> 5), ci0 = 8 * ((lane >> 4) & 1);
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int ci = ci0 + j;
        const float w = (co < cout && ci < cin && tap < 27) ? W[(co * cin + ci) * 27 + tap] : 0.0f;
        v[j] = (__bf16)w;
    }
    frag[i] = v;
}

// The BF16 form keeps each layer's input as BF16 activations with the 16
// channels innermost, a[b][p][16] (32 bytes per site; layer 0: the 10 input
// channels and six zeros), so that staging a tile is a copy of 32 bytes per
// halo site.  Each layer's epilogue writes the next layer's input,
// BF16(SiLU(z)); the last writes its FP32 pre-activation u [b][3][p] for the
// head.

// layer-0 input: (S_g, S_A, S_B, t) rounded to float, then to BF16
__global__ void k_net_input_bf16(const double *__restrict__ Sg, const double *__restrict__ SA,
                                 const double *__restrict__ SB, const float *__restrict__ t,
                                 bf16x8 *__restrict__ xa, int64_t P, int64_t ab_stride) {
    const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    const int b = blockIdx.y;
    if (p >= P) return;
    const int64_t o = (int64_t)b * 3 * P, oab = (int64_t)b * ab_stride;
    float v[16];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v[c] = (float)Sg[o + c * P + p];
        v[3 + c] = (float)SA[oab + c * P + p];
        v[6 + c] = (float)SB[oab + c * P + p];
    }
    v[9] = t[b];
#pragma unroll
    for (int c = 10; c < 16; ++c) v[c] = 0.0f;
    bf16x8 lo, hi;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        lo[j] = (__bf16)v[j];
        hi[j] = (__bf16)v[8 + j];
    }
    bf16x8 *dst = xa + ((int64_t)b * P + p) * 2;
    dst[0] = lo;
    dst[1] = hi;
}

// Workgroups are dealt to the 8 XCDs in turn by linear id (x fastest).  This
// renumbering gives each XCD one contiguous range of the grid instead, so the
// d^3 phase tiles of one region, consecutive in x, run on one XCD: the
// strided halo rows they read and the partial cache lines they write meet in
// its L2.  The grid holds fewer than 2^31 blocks.
struct GridBlock {
    int x, y, z;
};
__device__ __forceinline__ GridBlock xcd_grid_block() {
    const uint32_t gx = gridDim.x, gy = gridDim.y, T = gx * gy * gridDim.z;
    const uint32_t b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const uint32_t q = T / 8, r = T % 8, k = b % 8;
    const uint32_t l = k * q + (k < r ? k : r) + b / 8;
    return GridBlock{(int)(l % gx), (int)((l / gx) % gy), (int)(l / (gx * gy))};
}

// The BF16 halo tile in LDS: 32 bytes per site (16 channels), x rows of 10
// sites (320 bytes).  The two 16-byte halves of a site are stored swapped
// where bit 2 of its halo x is set, so that the 8 lanes (x = 0..7) that read
// one half each in an A-operand load cover eight different 16-byte bank
// groups instead of four (measured: 36% fewer bank-conflict cycles; the
// layer's time is set elsewhere and did not move).
constexpr int kRowB = kHX * 32, kPlaneB = kHY * kRowB, kTileB = kHZ * kPlaneB;
__host__ __device__ constexpr int swz(int hx) { return (hx >> 2) & 1; }

// byte offset of the y and z parts of tap (kx, ky, kz) = (tap % 3, tap / 3 %
// 3, tap / 9) in the tile, and its kx; the padded tap 27 reads offset 0 (its
// weights are zero)
constexpr int tap_bytes(int tap) { return tap >= 27 ? 0 : kRowB * ((tap / 3) % 3) + kPlaneB * (tap / 9); }
constexpr int tap_kx(int tap) { return tap >= 27 ? 0 : tap % 3; }

// SiLU with the hardware reciprocal: its result is rounded to BF16 next
__device__ __forceinline__ float silu_bf16(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// out[co] = bias[co] + sum_ci sum_k W[co][ci][k] a[ci](p + (k - 1) d), BF16
// operands, FP32 accumulation; the block's 8 x 8 x 4 tile is 16 groups of 16
// sites (two y rows of one z plane), four per wavefront.  LAST: write the
// FP32 pre-activation of the COUT channels to u [b][COUT][p]; otherwise
// BF16(SiLU) of all 16 channels to the next activation buffer.  Either goes
// through LDS first, site-major, so that each thread then writes one site.
template <int COUT, bool LAST>
__global__ __launch_bounds__(kNT) void k_conv_mfma(const bf16x8 *__restrict__ in, const bf16x8 *__restrict__ frag,
                                                   const float *__restrict__ bias, void *__restrict__ out,
                                                   NetDims d) {
    static_assert(kHX == 10 && kHY * kHZ == 60 && kNT >= 240, "staging map assumes the 10 x 10 x 6 halo");
    static_assert(kTileB >= kNT * 32, "the epilogue reuses the tile");
    __shared__ __attribute__((aligned(16))) char lds[kTileB];
    const GridBlock g = xcd_grid_block();
    const NetTile tl = tile_origin_at(d, g.x, g.y);
    const int t = threadIdx.x;
    // staging: thread t < 240 copies the 16-byte chunk c = t % 20 (halo x =
    // c / 2, channels 8 (c % 2) .. + 7) of halo rows t / 20 + 12 k, k = 0..4
    // (row = hy + kHY hz); sites outside the lattice are zero
    if (t < 240) {
        const int c = t % 20, hx = c >> 1, half = c & 1, r0 = t / 20;
        const int gx = tl.px + d.dil * (tl.x0 + hx - 1);
        const bool okx = gx >= 0 && gx < d.Lx;
        const bf16x8 *src = in + (int64_t)g.z * d.P * 2 + half;
        bf16x8 v[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int hr = r0 + 12 * k, hy = hr % kHY, hz = hr / kHY;
            const int gy = tl.py + d.dil * (tl.y0 + hy - 1), gz = tl.pz + d.dil * (tl.z0 + hz - 1);
            const bool ok = okx && gy >= 0 && gy < d.Ly && gz >= 0 && gz < d.Lz;
            const int64_t o = ok ? (gx + (int64_t)d.Lx * (gy + (int64_t)d.Ly * gz)) * 2 : 0;
            v[k] = src[o];
            if (!ok) v[k] = bf16x8{};
        }
#pragma unroll
        for (int k = 0; k < 5; ++k)
            *reinterpret_cast<bf16x8 *>(lds + (r0 + 12 * k) * kRowB + 32 * hx + 16 * (half ^ swz(hx))) = v[k];
    }
    __syncthreads();
    const int lane = t & 63, wave = t >> 6, row = lane & 15, grp = lane >> 4;
    // lane's A operand: site (x, y, z) = (row % 8, row / 8 + 2 m, wave) of
    // group m, channels 8 (grp % 2) .. + 7; lanes 32..63 take the pair's
    // second tap.  abx[kx]: the byte address of that half at tap offset kx
    // in x (the y and z offsets of a tap add to it)
    int abx[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int hx = (row & 7) + k;
        abx[k] = 32 * hx + kRowB * (row >> 3) + kPlaneB * wave + 16 * ((grp & 1) ^ swz(hx));
    }
    const bool second = grp >= 2;
    f32x4 acc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[m] = f32x4{};
#pragma unroll
    for (int tp = 0; tp < kTapPairs; ++tp) {
        const bf16x8 b = frag[tp * 64 + lane];
        const int a = second ? abx[tap_kx(2 * tp + 1)] + tap_bytes(2 * tp + 1) : abx[tap_kx(2 * tp)] + tap_bytes(2 * tp);
#pragma unroll
        for (int m = 0; m < 4; ++m)
            acc[m] = mfma16(*reinterpret_cast<const bf16x8 *>(lds + a + 2 * kRowB * m), b, acc[m]);
    }
    // accumulator i of lane l: site 16 mb + 4 grp + i of the tile (mb = 4
    // wave + m), channel co = l % 16
    const int co = lane & 15;
    __syncthreads();  // every wavefront is done with the tile
    // thread t then writes site t: group mb = t / 16, r = t % 16
    const int mb = t >> 4, r = t & 15;
    const int x = tl.px + d.dil * (tl.x0 + (r & 7)), y = tl.py + d.dil * (tl.y0 + 2 * (mb & 3) + (r >> 3)),
              z = tl.pz + d.dil * (tl.z0 + (mb >> 2));
    const bool inside = x < d.Lx && y < d.Ly && z < d.Lz;
    const int64_t p = x + (int64_t)d.Lx * (y + (int64_t)d.Ly * z);
    if constexpr (LAST) {
        float(*ot)[4] = reinterpret_cast<float(*)[4]>(lds);  // ot[site][co]
        if (co < COUT) {
            const float bco = bias[co];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) ot[16 * (4 * wave + m) + 4 * grp + i][co] = acc[m][i] + bco;
        }
        __syncthreads();
        if (inside) {
            float *u = static_cast<float *>(out) + (int64_t)g.z * COUT * d.P + p;
#pragma unroll
            for (int c = 0; c < COUT; ++c) u[(int64_t)c * d.P] = ot[t][c];
        }
    } else {
        // ot[site][8 channel pairs]; the two 16-byte halves of site s are
        // swapped when bit 3 of s is set, which spreads the one-half reads
        // of consecutive sites over the bank groups (of bits 2 and 3, bit 3
        // measured fewer conflict cycles).  Lanes co and co ^ 1 trade one
        // value so that each writes a channel pair of one site: the even
        // lane sites 4 grp + i, the odd lane 4 grp + i + 1.
        bf16x2(*ot)[8] = reinterpret_cast<bf16x2(*)[8]>(lds);
        const float bco = bias[co];
        const bool odd = co & 1;
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int i = 0; i < 4; i += 2) {
                const float v0 = silu_bf16(acc[m][i] + bco), v1 = silu_bf16(acc[m][i + 1] + bco);
                const float got =
                    __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(odd ? v0 : v1), 0xB1, 0xF, 0xF, false));
                const int st = 16 * (4 * wave + m) + 4 * grp + i + (odd ? 1 : 0);
                const bf16x2 pr = odd ? bf16x2{(__bf16)got, (__bf16)v1} : bf16x2{(__bf16)v0, (__bf16)got};
                ot[st][(co >> 1) ^ (st & 8 ? 4 : 0)] = pr;
            }
        __syncthreads();
        if (inside) {
            const int sw = t & 8 ? 1 : 0;
            const bf16x8 lo = *reinterpret_cast<const bf16x8 *>(lds + 32 * t + 16 * sw);
            const bf16x8 hi = *reinterpret_cast<const bf16x8 *>(lds + 32 * t + 16 * (1 - sw));
            bf16x8 *dst = static_cast<bf16x8 *>(out) + ((int64_t)g.z * d.P + p) * 2;
            dst[0] = lo;
            dst[1] = hi;
        }
    }
}

// Lane-layout check of the 16x16x32 BF16 MFMA: D = A B for A [16][32],
// B [32][16], D [16][16] row-major FP32 (values exact in BF16).
__global__ void k_mfma16_probe(const float *__restrict__ A, const float *__restrict__ B, float *__restrict__ D) {
    const int l = threadIdx.x;
    bf16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = (__bf16)A[(l % 16) * 32 + 8 * (l / 16) + j];
        b[j] = (__bf16)B[(8 * (l / 16) + j) * 16 + l % 16];
    }
    const f32x4 c = mfma16(a, b, f32x4{});
#pragma unroll
    for (int i = 0; i < 4; ++i) D[(4 * (l / 16) + i) * 16 + l % 16] = c[i];
}

// Adam (Kingma & Ba) on n parameters, step t >= 1.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

constexpr int kC[5] = {10, 16, 16, 16, 3};
constexpr int kMaxDilation = 64;

struct NetWork {
    int64_t cap_P = 0;
    int cap_B = 0;
    float *x = nullptr, *z[4] = {nullptr, nullptr, nullptr, nullptr};
    float *g[4] = {nullptr, nullptr, nullptr, nullptr};
    float *wt = nullptr;        // transposed weights of one layer
    double *part = nullptr;     // weight-gradient partials (FP64)
    size_t part_cap = 0;
    double *lpart = nullptr;
    size_t lpart_cap = 0;
    bf16x8 *frag = nullptr;     // BF16 MFMA weight fragments, [4 layers][14][64]
    bf16x8 *act[2] = {nullptr, nullptr};  // BF16 activations [B][P][16] (two 8-channel halves), ping-pong
    size_t act_cap = 0;                   // sites x images each holds
};

}  // namespace spx

using namespace spx;

struct spx_net {
    NetWork w;
    int dil[4] = {1, 1, 1, 1};  // per-layer dilation
    int prec = SPX_FP32;        // forward (inference) arithmetic: SPX_FP32 or SPX_BF16_MFMA
};

namespace {

int64_t net_nparams() {
    int64_t n = 0;
    for (int l = 0; l < 4; ++l) n += (int64_t)kC[l + 1] * kC[l] * 27 + kC[l + 1];
    return n;
}
int64_t layer_off(int l) {
    int64_t n = 0;
    for (int q = 0; q < l; ++q) n += (int64_t)kC[q + 1] * kC[q] * 27 + kC[q + 1];
    return n;
}

void net_free(NetWork &w) {
    for (void *p : {(void *)w.x, (void *)w.z[0], (void *)w.z[1], (void *)w.z[2], (void *)w.z[3], (void *)w.g[0],
                    (void *)w.g[1], (void *)w.g[2], (void *)w.g[3], (void *)w.wt, (void *)w.part, (void *)w.lpart,
                    (void *)w.frag, (void *)w.act[0], (void *)w.act[1]})
        if (p) (void)hipFree(p);
    w = NetWork{};
}

spx_status net_reserve(NetWork &w, int64_t P, int B, bool train) {
    if (P <= w.cap_P && B <= w.cap_B && (!train || w.g[0])) return SPX_OK;
    net_free(w);
    auto al = [](void **p, size_t bytes) {
        if (hipMalloc(p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return false;
        }
        return true;
    };
    bool ok = al((void **)&w.x, sizeof(float) * 10 * P * B);
    for (int l = 0; l < 4 && ok; ++l) ok = al((void **)&w.z[l], sizeof(float) * kC[l + 1] * P * B);
    for (int l = 0; l < 4 && ok && train; ++l) ok = al((void **)&w.g[l], sizeof(float) * kC[l + 1] * P * B);
    if (ok && train) ok = al((void **)&w.wt, sizeof(float) * 16 * 16 * 27);
    if (!ok) {
        net_free(w);
        return set_error(SPX_ERR_OUT_OF_MEMORY, "hipMalloc failed for network activations");
    }
    w.cap_P = P;
    w.cap_B = B;
    return SPX_OK;
}

// The dims of layer l: the lattice with that layer's dilation.
NetDims layer_dims(const NetDims &d, const int dil[4], int l) {
    NetDims e = d;
    e.dil = dil[l];
    e.Sx = (d.Lx + e.dil - 1) / e.dil;
    e.Sy = (d.Ly + e.dil - 1) / e.dil;
    e.Sz = (d.Lz + e.dil - 1) / e.dil;
    return e;
}

// Blocks of a layer: the tiles of one phase's sub-grid times the d^3 phases.
dim3 conv_grid(const NetDims &d, int B) {
    const int nbx = (d.Sx + kTXn - 1) / kTXn, nby = (d.Sy + kTYn - 1) / kTYn, nbz = (d.Sz + kTZn - 1) / kTZn;
    return dim3((unsigned)(nbx * nby * d.dil * d.dil), (unsigned)(nbz * d.dil), (unsigned)B);
}

// forward through the four layers as BF16 implicit GEMMs (inference), from
// the input states to the FP32 pre-activation u = z[3]
hipError_t net_forward_layers_mfma(NetWork &w, const float *params, const NetDims &d, const int dil[4], int B,
                                   const double *Sg, const double *SA, const double *SB, const float *t,
                                   int64_t ab_stride, hipStream_t st) {
    if (!w.frag) {
        hipError_t e = hipMalloc((void **)&w.frag, sizeof(bf16x8) * 4 * kTapPairs * 64);
        if (e != hipSuccess) return e;
    }
    const size_t need = (size_t)d.P * B;
    if (need > w.act_cap) {
        for (int k = 0; k < 2; ++k) {
            if (w.act[k]) (void)hipFree(w.act[k]);
            w.act[k] = nullptr;
        }
        w.act_cap = 0;
        for (int k = 0; k < 2; ++k) {
            hipError_t e = hipMalloc((void **)&w.act[k], sizeof(bf16x8) * 2 * need);
            if (e != hipSuccess) return e;
        }
        w.act_cap = need;
    }
    const int fb = (kTapPairs * 64 + 255) / 256;
    for (int l = 0; l < 4; ++l)
        k_wfrag<<<fb, 256, 0, st>>>(params + layer_off(l), kC[l], kC[l + 1], w.frag + l * kTapPairs * 64);
    const dim3 pg((unsigned)((d.P + kNT - 1) / kNT), (unsigned)B);
    k_net_input_bf16<<<pg, kNT, 0, st>>>(Sg, SA, SB, t, w.act[0], d.P, ab_stride);
    const NetDims d0 = layer_dims(d, dil, 0), d1 = layer_dims(d, dil, 1), d2 = layer_dims(d, dil, 2),
                  d3 = layer_dims(d, dil, 3);
    const float *b0 = params + layer_off(0) + 16 * 10 * 27, *b1 = params + layer_off(1) + 16 * 16 * 27;
    const float *b2 = params + layer_off(2) + 16 * 16 * 27, *b3 = params + layer_off(3) + 3 * 16 * 27;
    for (const NetDims *e : {&d0, &d1, &d2, &d3}) {
        const dim3 g = conv_grid(*e, B);
        if ((uint64_t)g.x * g.y * g.z >= ((uint64_t)1 << 31)) return hipErrorInvalidConfiguration;
    }
    bf16x8 *f = w.frag;
    k_conv_mfma<16, false><<<conv_grid(d0, B), kNT, 0, st>>>(w.act[0], f, b0, w.act[1], d0);
    k_conv_mfma<16, false><<<conv_grid(d1, B), kNT, 0, st>>>(w.act[1], f + kTapPairs * 64, b1, w.act[0], d1);
    k_conv_mfma<16, false><<<conv_grid(d2, B), kNT, 0, st>>>(w.act[0], f + 2 * kTapPairs * 64, b2, w.act[1], d2);
    k_conv_mfma<3, true><<<conv_grid(d3, B), kNT, 0, st>>>(w.act[1], f + 3 * kTapPairs * 64, b3, w.z[3], d3);
    return hipGetLastError();
}

// forward through the four layers; z[l] are pre-activations
hipError_t net_forward_layers(NetWork &w, const float *params, const NetDims &d, const int dil[4], int B,
                              hipStream_t st) {
    const NetDims d0 = layer_dims(d, dil, 0), d1 = layer_dims(d, dil, 1), d2 = layer_dims(d, dil, 2),
                  d3 = layer_dims(d, dil, 3);
    const float *W0 = params + layer_off(0), *W1 = params + layer_off(1);
    const float *W2 = params + layer_off(2), *W3 = params + layer_off(3);
    k_conv<10, 16, false, false><<<conv_grid(d0, B), kNT, 0, st>>>(w.x, W0, W0 + 16 * 10 * 27, nullptr, w.z[0], d0);
    k_conv<16, 16, true, false><<<conv_grid(d1, B), kNT, 0, st>>>(w.z[0], W1, W1 + 16 * 16 * 27, nullptr, w.z[1], d1);
    k_conv<16, 16, true, false><<<conv_grid(d2, B), kNT, 0, st>>>(w.z[1], W2, W2 + 16 * 16 * 27, nullptr, w.z[2], d2);
    k_conv<16, 3, true, false><<<conv_grid(d3, B), kNT, 0, st>>>(w.z[2], W3, W3 + 3 * 16 * 27, nullptr, w.z[3], d3);
    return hipGetLastError();
}

spx_status check_dims(const int32_t *dims, int32_t batch, NetDims &d) {
    if (!dims || dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || batch < 1)
        return set_error(SPX_ERR_INVALID_ARG, "bad network dims or batch");
    d.Lx = dims[0];
    d.Ly = dims[1];
    d.Lz = dims[2];
    d.P = (int64_t)dims[0] * dims[1] * dims[2];
    d.dil = 1;
    d.Sx = d.Lx;
    d.Sy = d.Ly;
    d.Sz = d.Lz;
    if (d.P * batch > ((int64_t)1 << 31)) return set_error(SPX_ERR_INVALID_ARG, "network batch too large");
    return SPX_OK;
}

}  // namespace

namespace spx {
// used by the GNEB learned initial path
spx_status net_apply(spx_net *net, const float *params, const int32_t dims[3], int32_t batch, const double *Sg,
                     const double *SA, const double *SB, int shared_ends, const float *t, double *Shat,
                     hipStream_t st) {
    NetDims d;
    spx_status s = check_dims(dims, batch, d);
    if (s != SPX_OK) return s;
    if ((s = net_reserve(net->w, d.P, batch, false)) != SPX_OK) return s;
    const dim3 pg((unsigned)((d.P + kNT - 1) / kNT), (unsigned)batch);
    const int64_t ab_stride = shared_ends ? 0 : 3 * d.P;
    hipError_t e;
    if (net->prec == SPX_BF16_MFMA) {
        e = net_forward_layers_mfma(net->w, params, d, net->dil, batch, Sg, SA, SB, t, ab_stride, st);
    } else {
        k_net_input<<<pg, kNT, 0, st>>>(Sg, SA, SB, t, net->w.x, d.P, ab_stride);
        e = net_forward_layers(net->w, params, d, net->dil, batch, st);
    }
    if (e == hipSuccess) {
        k_net_head<<<pg, kNT, 0, st>>>(net->w.z[3], Sg, nullptr, Shat, nullptr, nullptr, d.P, 0.0);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return set_hip_error(e, "network forward");
    return SPX_OK;
}
bool net_alive(spx_net *net) { return handle_alive(net); }
}  // namespace spx

extern "C" {

int64_t spx_net_nparams(void) { return net_nparams(); }

spx_status spx_net_create(const int32_t *channels, spx_net **out) {
    if (!out) return set_error(SPX_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (channels)
        for (int l = 0; l < 5; ++l)
            if (channels[l] != kC[l])
                return set_error(SPX_ERR_UNSUPPORTED, "only the 10-16-16-16-3 network is built");
    spx_net *n = new spx_net();
    register_handle(n);
    *out = n;
    return SPX_OK;
}

spx_status spx_net_set_dilation(spx_net *net, const int32_t *dil) {
    if (!handle_alive(net)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_net handle");
    if (!dil) return set_error(SPX_ERR_INVALID_ARG, "dil is NULL");
    for (int l = 0; l < 4; ++l)
        if (dil[l] < 1 || dil[l] > kMaxDilation)
            return set_error(SPX_ERR_INVALID_ARG, "each dilation must be 1 .. 64");
    for (int l = 0; l < 4; ++l) net->dil[l] = dil[l];
    return SPX_OK;
}

spx_status spx_net_set_precision(spx_net *net, int32_t prec) {
    if (!handle_alive(net)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_net handle");
    if (prec != SPX_FP32 && prec != SPX_BF16_MFMA)
        return set_error(SPX_ERR_INVALID_ARG, "the network runs in SPX_FP32 or SPX_BF16_MFMA");
    net->prec = prec;
    return SPX_OK;
}

spx_status spx_mfma16_probe(const float *A, const float *B, float *D, void *stream) {
    if (!A || !B || !D) return set_error(SPX_ERR_INVALID_ARG, "NULL argument");
    k_mfma16_probe<<<1, 64, 0, (hipStream_t)stream>>>(A, B, D);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "spx_mfma16_probe");
    return SPX_OK;
}

spx_status spx_net_destroy(spx_net *net) {
    if (!handle_alive(net)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_net handle");
    unregister_handle(net);
    (void)hipDeviceSynchronize();
    net_free(net->w);
    delete net;
    return SPX_OK;
}

spx_status spx_net_forward(spx_net *net, const float *params, const int32_t *dims, int32_t batch, const double *Sg,
                           const double *SA, const double *SB, const float *t, double *Shat, void *stream) {
    if (!handle_alive(net)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_net handle");
    if (!params || !Sg || !SA || !SB || !t || !Shat) return set_error(SPX_ERR_INVALID_ARG, "NULL argument");
    return net_apply(net, params, dims, batch, Sg, SA, SB, 0, t, Shat, (hipStream_t)stream);
}

spx_status spx_net_backward(spx_net *net, const float *params, const int32_t *dims, int32_t batch, const double *Sg,
                            const double *SA, const double *SB, const float *t, const double *Sstar, float *grad,
                            double *loss, void *stream) {
    if (!handle_alive(net)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_net handle");
    if (!params || !Sg || !SA || !SB || !t || !Sstar || !grad) return set_error(SPX_ERR_INVALID_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    NetDims d;
    spx_status s = check_dims(dims, batch, d);
    if (s != SPX_OK) return s;
    NetWork &w = net->w;
    if ((s = net_reserve(w, d.P, batch, true)) != SPX_OK) return s;
    NetDims dl[4];
    size_t max_blk = 0;
    for (int l = 0; l < 4; ++l) {
        dl[l] = layer_dims(d, net->dil, l);
        const dim3 g = conv_grid(dl[l], batch);
        max_blk = std::max(max_blk, (size_t)g.x * g.y * g.z);
    }
    const size_t need = max_blk * (16 * 16 * 27 + 16);
    const dim3 pg((unsigned)((d.P + kNT - 1) / kNT), (unsigned)batch);
    const size_t nl = (size_t)pg.x * pg.y;
    if (need > w.part_cap) {
        if (w.part) (void)hipFree(w.part);
        if (hipMalloc((void **)&w.part, need * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            w.part = nullptr;
            w.part_cap = 0;
            return set_error(SPX_ERR_OUT_OF_MEMORY, "hipMalloc failed for gradient partials");
        }
        w.part_cap = need;
    }
    if (nl > w.lpart_cap) {
        if (w.lpart) (void)hipFree(w.lpart);
        if (hipMalloc((void **)&w.lpart, nl * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            w.lpart = nullptr;
            w.lpart_cap = 0;
            return set_error(SPX_ERR_OUT_OF_MEMORY, "hipMalloc failed for loss partials");
        }
        w.lpart_cap = nl;
    }
    k_net_input<<<pg, kNT, 0, st>>>(Sg, SA, SB, t, w.x, d.P, 3 * d.P);
    hipError_t e = net_forward_layers(w, params, d, net->dil, batch, st);
    if (e != hipSuccess) return set_hip_error(e, "network backward (forward pass)");
    const double inv_count = 1.0 / ((double)d.P * batch);
    k_net_head<<<pg, kNT, 0, st>>>(w.z[3], Sg, Sstar, nullptr, w.g[3], w.lpart, d.P, inv_count);
    if (loss) k_loss_final<<<1, 1, 0, st>>>(w.lpart, (int)nl, inv_count, loss);
    // layer 4 (16 -> 3), 3 (16 -> 16), 2 (16 -> 16), 1 (10 -> 16)
    for (int l = 3; l >= 0; --l) {
        const int cin = kC[l], cout = kC[l + 1];
        const int nw = cout * cin * 27 + cout;
        const float *Wl = params + layer_off(l);
        float *gl = grad + layer_off(l);
        const float *ain = l == 0 ? w.x : w.z[l - 1];
        const NetDims &d_l = dl[l];
        const dim3 gr = conv_grid(d_l, batch);
        const size_t n_blk = (size_t)gr.x * gr.y * gr.z;
        if (l == 3) k_conv_wgrad<16, 3, true><<<gr, kNT, 0, st>>>(ain, w.g[3], w.part, d_l);
        else if (l == 0) k_conv_wgrad<10, 16, false><<<gr, kNT, 0, st>>>(ain, w.g[0], w.part, d_l);
        else k_conv_wgrad<16, 16, true><<<gr, kNT, 0, st>>>(ain, w.g[l], w.part, d_l);
        k_sum_partials<<<(nw + 255) / 256, 256, 0, st>>>(w.part, (int)n_blk, nw, gl);
        if (l > 0) {
            // g_{l-1} = silu'(z_{l-1}) * conv(g_l, W^T flipped)
            k_transpose_flip<<<(cin * cout * 27 + 255) / 256, 256, 0, st>>>(Wl, w.wt, cin, cout);
            // the transposed convolution of layer l has layer l's dilation
            if (l == 3) k_conv<3, 16, false, true><<<gr, kNT, 0, st>>>(w.g[3], w.wt, nullptr, w.z[2], w.g[2], d_l);
            else k_conv<16, 16, false, true><<<gr, kNT, 0, st>>>(w.g[l], w.wt, nullptr, w.z[l - 1], w.g[l - 1], d_l);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return set_hip_error(e, "network backward");
    }
    return SPX_OK;
}

spx_status spx_net_adam_step(float *params, const float *grad, float *m, float *v, int64_t n, int64_t step,
                             double lr, double b1, double b2, double eps, void *stream) {
    if (!params || !grad || !m || !v || n < 0 || step < 1) return set_error(SPX_ERR_INVALID_ARG, "bad Adam arguments");
    const float c1 = (float)(1.0 - std::pow(b1, (double)step)), c2 = (float)(1.0 - std::pow(b2, (double)step));
    k_adam<<<(unsigned)((n + kNT - 1) / kNT), kNT, 0, (hipStream_t)stream>>>(params, grad, m, v, n, (float)lr,
                                                                            (float)b1, (float)b2, (float)eps, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "spx_net_adam_step");
    return SPX_OK;
}

}  // extern "C"
