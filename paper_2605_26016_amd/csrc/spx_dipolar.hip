// spx_dipolar.hip -- open-boundary dipolar field by zero-padded FFT
// convolution (Methods, reciprocal-space convolution for long-range dipolar
// fields) on gfx950.
//
// The dipole tensor T(r) = (mu0/4pi) mu_B^2 (3 rhat rhat - 1)/r^3 is sampled
// on a grid of P_a >= 2 L_a - 1 points per axis (P_a a power of two) holding
// every displacement in [-(L_a-1), L_a-1]; its six-component real spectrum is
// built once in FP64 (scaled by mu^2 and by the 1/(Px Py Pz) of the
// unnormalised inverse).  Per evaluation the three spin components go through
// a pruned FP32 transform pipeline that never touches the zero padding:
//   x: R2C (hipFFT, rows of length Px) on the Ly x Lz occupied rows only;
//   y: column FFT of length Py reading the Ly occupied rows (the rest are
//      zero by construction), on the Lz occupied planes only;
//   z: column FFT of length Pz reading the Lz occupied planes;
// then the 3x3 spectral product, and the inverse transforms in reverse order
// keeping only the outputs inside the lattice (z < Lz, then y < Ly, then the
// C2R rows and x < Lx).  Linear (aperiodic) convolution = open boundaries.
// The column FFTs: for P = 512 a register radix-8 kernel (three passes, two
// LDS exchanges, 8 columns per block); for other P an LDS radix-2 kernel (a
// block stages P rows x W adjacent columns, bit-reverses on load, runs log2 P
// in-place butterfly stages).  Both write only the rows that are kept.
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "spx_ext.hpp"

namespace spx {

struct DipolarPlan {
    int L[3];              // x, y, z cells
    int P[3];              // padded extents (powers of two >= 2L - 1)
    int H;                 // Px / 2 + 1 complex points per x row
    int64_t N;             // sites
    int64_t n_cplx;        // Pz * Py * H spectrum points per component
    float *R = nullptr;    // [3][Lz][Ly][Px] real rows (padded spins in, field rows out)
    float2 *X = nullptr;   // [3][Lz][Ly][H] after the x transform
    float2 *Y = nullptr;   // [3][Lz][Py][H] after the y transform
    float2 *Z = nullptr;   // [3][Pz][Py][H] full spectrum (Pz != 512; 512 uses the fused z pass)
    float *kern = nullptr; // [6][Pz][Py][H] real dipole spectrum xx, xy, xz, yy, yz, zz
    // Pz = 512: the spectrum in the fused z pass's order instead,
    // [column group][kz < nkz][6][16 columns] (nkz = 257 with z parity, else 512)
    float *kernb = nullptr;
    int nkz = 0;
    // the third cell vector is along z and the first two have no z part: the
    // sampled tensor is even (xx, xy, yy, zz) or odd (xz, yz) under dz -> -dz,
    // so is its spectrum under kz -> Pz - kz, and the fused z pass reads only
    // kz <= Pz / 2 (half the spectrum traffic)
    bool zsym = false;
    float2 *tw_y = nullptr, *tw_z = nullptr;  // exp(-2 pi i k / P), k < P
    float2 *tw_x = nullptr;                    // Px = 512: the x rows run in k_xfft512_*
    hipfftHandle fwd = 0, inv = 0;
    bool fwd_ok = false, inv_ok = false;
};

namespace {

constexpr int kB = 256;
constexpr int kColThreads = 256;
constexpr int kMaxLds = 65536;

// (mu0/4pi) mu_B^2 in meV nm^3 from SI values (CODATA 2018).
double dipole_prefactor() {
    const double mu0_over_4pi = 1.0e-7;      // T m / A
    const double muB_SI = 9.2740100783e-24;  // J / T
    const double meV_in_J = 1.602176634e-22;
    return mu0_over_4pi * muB_SI * muB_SI / meV_in_J * 1.0e27;
}

int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

int log2i(int p) {
    int l = 0;
    while ((1 << l) < p) ++l;
    return l;
}

// columns per block of the column FFT: a power of two <= 16 whose staged tile
// (P x W complex) plus the twiddle table fits the LDS budget
int col_width(int P) {
    int w = 16;
    while (w > 1 && (size_t)P * w * sizeof(float2) + (size_t)(P / 2) * sizeof(float2) > (size_t)kMaxLds) w >>= 1;
    return w;
}

// displacement of padded index k on an axis of L cells and P points, or
// INT_MIN inside the gap between +(L-1) and -(L-1)
__device__ __forceinline__ int pad_disp(int k, int L, int P) {
    if (k < L) return k;
    if (k > P - L) return k - P;
    return -0x7fffffff;
}

// One component (a,b) of the real-space dipole tensor on the padded grid, FP64.
__global__ void k_dipole_component(int Lx, int Ly, int Lz, int Px, int Py, int Pz, double c00, double c01,
                                   double c02, double c10, double c11, double c12, double c20, double c21,
                                   double c22, int ca, int cb, double pref, double *__restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (idx >= (int64_t)Px * Py * Pz) return;
    const int kx = (int)(idx % Px), ky = (int)((idx / Px) % Py), kz = (int)(idx / ((int64_t)Px * Py));
    const int ix = pad_disp(kx, Lx, Px), iy = pad_disp(ky, Ly, Py), iz = pad_disp(kz, Lz, Pz);
    double v = 0.0;
    if (ix != -0x7fffffff && iy != -0x7fffffff && iz != -0x7fffffff) {
        const double dx = ix, dy = iy, dz = iz;
        const double r[3] = {dx * c00 + dy * c10 + dz * c20, dx * c01 + dy * c11 + dz * c21,
                             dx * c02 + dy * c12 + dz * c22};
        const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (r2 > 0.0) {
            const double rn = sqrt(r2);
            const double inv3 = 1.0 / (r2 * rn);
            v = pref * (3.0 * r[ca] * r[cb] / r2 - (ca == cb ? 1.0 : 0.0)) * inv3;
        }
    }
    out[idx] = v;
}

__global__ void k_take_real(const double2 *__restrict__ in, int64_t n, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) out[i] = (float)in[i].x;
}

// FP32 x rows of the occupied (y, z) lines, zero beyond x = Lx.
// One block per padded x row (c, line = y + Ly z): the occupied Lx values
// converted to FP32, zero up to Px.
__global__ __launch_bounds__(kB) void k_pad_rows(const double *__restrict__ S, int Lx, int Px, int64_t rows,
                                                 int64_t N, float *__restrict__ R) {
    const int64_t row = blockIdx.x;
    const int64_t c = row / rows, line = row - c * rows;
    const double *src = S + c * N + line * Lx;
    float *dst = R + row * Px;
    for (int x = threadIdx.x; x < Px; x += kB) dst[x] = x < Lx ? (float)src[x] : 0.0f;
}

// One block per row: the occupied Lx values of padded row (c, line) into b.
__global__ __launch_bounds__(kB) void k_crop_rows(const float *__restrict__ R, int Lx, int Px, int64_t rows,
                                                  int64_t N, float *__restrict__ b) {
    const int64_t row = blockIdx.x;
    const int64_t c = row / rows, line = row - c * rows;
    const float *src = R + row * Px;
    float *dst = b + c * N + line * Lx;
    for (int x = threadIdx.x; x < Lx; x += kB) dst[x] = src[x];
}

// b^_a = sum_b T^_ab S^_b at every frequency (T^ real symmetric).
__global__ void k_spectral_mult(float2 *__restrict__ spec, const float *__restrict__ kern, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const float2 sx = spec[i], sy = spec[n + i], sz = spec[2 * n + i];
    const float txx = kern[i], txy = kern[n + i], txz = kern[2 * n + i];
    const float tyy = kern[3 * n + i], tyz = kern[4 * n + i], tzz = kern[5 * n + i];
    spec[i] = make_float2(txx * sx.x + txy * sy.x + txz * sz.x, txx * sx.y + txy * sy.y + txz * sz.y);
    spec[n + i] = make_float2(txy * sx.x + tyy * sy.x + tyz * sz.x, txy * sx.y + tyy * sy.y + tyz * sz.y);
    spec[2 * n + i] = make_float2(txz * sx.x + tyz * sy.x + tzz * sz.x, txz * sx.y + tyz * sy.y + tzz * sz.y);
}

// Column FFT of length P = 2^logP over W adjacent columns of batch
// blockIdx.y.  Element (row r, column j) of a batch sits at
// base + r * J + j; rows r >= nin are zero; only rows r < nout are written.
// INV: exp(+2 pi i ...) (unnormalised).
template <bool INV>
__global__ __launch_bounds__(kColThreads) void k_colfft(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                        int logP, int wl, int nin, int nout, int64_t J,
                                                        int64_t in_bs, int64_t out_bs,
                                                        const float2 *__restrict__ tw) {
    extern __shared__ float2 sm[];
    const int P = 1 << logP, W = 1 << wl;
    float2 *a = sm;
    float2 *twl = sm + (size_t)P * W;
    const int tid = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * W;
    const int w = (int)((J - j0) < W ? (J - j0) : W);
    const int64_t b = blockIdx.y;
    const float2 *src = in + b * in_bs + j0;
    float2 *dst = out + b * out_bs + j0;
    for (int k = tid; k < P / 2; k += kColThreads) {
        const float2 t = tw[k];
        twl[k] = INV ? make_float2(t.x, -t.y) : t;
    }
    for (int idx = tid; idx < P * W; idx += kColThreads) {
        const int r = idx >> wl, c = idx & (W - 1);
        float2 v = make_float2(0.0f, 0.0f);
        if (r < nin && c < w) v = src[(int64_t)r * J + c];
        const int rr = (int)(__brev((unsigned)r) >> (32 - logP));
        a[(rr << wl) + c] = v;
    }
    __syncthreads();
    const int nbf = (P / 2) * W;
    for (int s = 0; s < logP; ++s) {
        const int half = 1 << s;
        for (int k = tid; k < nbf; k += kColThreads) {
            const int c = k & (W - 1);
            const int bf = k >> wl;
            const int pos = bf & (half - 1);
            const int i = ((bf >> s) << (s + 1)) + pos;
            const float2 t = twl[pos << (logP - s - 1)];
            const float2 u = a[(i << wl) + c];
            const float2 x = a[((i + half) << wl) + c];
            const float2 v = make_float2(x.x * t.x - x.y * t.y, x.x * t.y + x.y * t.x);
            a[(i << wl) + c] = make_float2(u.x + v.x, u.y + v.y);
            a[((i + half) << wl) + c] = make_float2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
    for (int idx = tid; idx < nout * W; idx += kColThreads) {
        const int r = idx >> wl, c = idx & (W - 1);
        if (c < w) dst[(int64_t)r * J + c] = a[idx];
    }
}

// ---- 512-point column FFT in registers (512 = 8 x 8 x 8) -----------------
// 64 threads per column, each holding 8 values; three radix-8 passes in
// registers with two exchanges through LDS.  With n = 64 a + b and
// k = c + 8 (g + 8 h), b = 8 e + f:
//   y_b[c]    = W512^{b c} sum_a x[64 a + b] W8^{a c}
//   z_cf[g]   = W64^{f g}  sum_e y_{8e+f}[c] W8^{e g}
//   X[c+8g+64h] =          sum_f z_cf[g] W8^{f h}.
constexpr int kW512Log = 4;
constexpr int kW512 = 1 << kW512Log;   // columns per block
constexpr int kT512 = 64 * kW512;      // threads per block
constexpr int kPitch = kW512 + 1;      // LDS float2 per position (one pad against bank conflicts)

template <bool INV>
__device__ __forceinline__ float2 cmulw(float2 x, float2 w) {
    // x * w (forward) or x * conj(w) (inverse)
    if (INV) return make_float2(x.x * w.x + x.y * w.y, x.y * w.x - x.x * w.y);
    return make_float2(x.x * w.x - x.y * w.y, x.x * w.y + x.y * w.x);
}

// in-place 8-point DFT, natural order in and out
template <bool INV>
__device__ __forceinline__ void dft8(float2 v[8]) {
    const float h = 0.70710678118654752f;
    // two 4-point DFTs of the even and odd samples
    float2 E[4], O[4];
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        const float2 a0 = v[part], a1 = v[part + 2], a2 = v[part + 4], a3 = v[part + 6];
        const float2 s02 = make_float2(a0.x + a2.x, a0.y + a2.y), d02 = make_float2(a0.x - a2.x, a0.y - a2.y);
        const float2 s13 = make_float2(a1.x + a3.x, a1.y + a3.y), d13 = make_float2(a1.x - a3.x, a1.y - a3.y);
        // W4 d13: -i d13 forward, +i d13 inverse
        const float2 wd = INV ? make_float2(-d13.y, d13.x) : make_float2(d13.y, -d13.x);
        float2 *T = part ? O : E;
        T[0] = make_float2(s02.x + s13.x, s02.y + s13.y);
        T[1] = make_float2(d02.x + wd.x, d02.y + wd.y);
        T[2] = make_float2(s02.x - s13.x, s02.y - s13.y);
        T[3] = make_float2(d02.x - wd.x, d02.y - wd.y);
    }
    // W8^k O[k], k = 0..3
    const float2 o1 = INV ? make_float2(h * (O[1].x - O[1].y), h * (O[1].x + O[1].y))
                          : make_float2(h * (O[1].x + O[1].y), h * (O[1].y - O[1].x));
    const float2 o2 = INV ? make_float2(-O[2].y, O[2].x) : make_float2(O[2].y, -O[2].x);
    const float2 o3 = INV ? make_float2(-h * (O[3].x + O[3].y), h * (O[3].x - O[3].y))
                          : make_float2(h * (O[3].y - O[3].x), -h * (O[3].x + O[3].y));
    const float2 t[4] = {O[0], o1, o2, o3};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = make_float2(E[k].x + t[k].x, E[k].y + t[k].y);
        v[k + 4] = make_float2(E[k].x - t[k].x, E[k].y - t[k].y);
    }
}

// 512-point FFT of one column held by 64 threads: on entry v[a] = x[64 a + qin]
// (qin = the column position this thread loaded), on exit v[h] = X[c + 8 g + 64 h]
// with c = q / 8, g = q % 8.  lds holds 512 x kPitch float2; w = column slot.
template <bool INV>
__device__ __forceinline__ void fft512(float2 v[8], float2 *lds, int qin, int q, int w,
                                       const float2 *__restrict__ tw) {
    dft8<INV>(v);
    __syncthreads();  // the previous user of lds has finished reading it
#pragma unroll
    for (int c = 0; c < 8; ++c) lds[(c * 64 + qin) * kPitch + w] = c ? cmulw<INV>(v[c], tw[(qin * c) & 511]) : v[c];
    __syncthreads();
    const int c2 = q >> 3, f = q & 7;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = lds[(c2 * 64 + 8 * e + f) * kPitch + w];
    dft8<INV>(v);
    __syncthreads();
#pragma unroll
    for (int g = 0; g < 8; ++g) lds[(c2 * 64 + 8 * g + f) * kPitch + w] = cmulw<INV>(v[g], tw[(8 * f * g) & 511]);
    __syncthreads();
#pragma unroll
    for (int ff = 0; ff < 8; ++ff) v[ff] = lds[(c2 * 64 + 8 * f + ff) * kPitch + w];
    dft8<INV>(v);
}

// The same transform with its two exchanges in two LDS buffers (A, then B):
// each exchange is write, barrier, read, and a buffer is written again only
// after the barrier that followed its last read, so two barriers per
// transform suffice (against four with one buffer).
template <bool INV>
__device__ __forceinline__ void fft512_2buf(float2 v[8], float2 *ldsA, float2 *ldsB, int qin, int q, int w,
                                            const float2 *__restrict__ tw) {
    dft8<INV>(v);
#pragma unroll
    for (int c = 0; c < 8; ++c) ldsA[(c * 64 + qin) * kPitch + w] = c ? cmulw<INV>(v[c], tw[(qin * c) & 511]) : v[c];
    __syncthreads();
    const int c2 = q >> 3, f = q & 7;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = ldsA[(c2 * 64 + 8 * e + f) * kPitch + w];
    dft8<INV>(v);
#pragma unroll
    for (int g = 0; g < 8; ++g) ldsB[(c2 * 64 + 8 * g + f) * kPitch + w] = cmulw<INV>(v[g], tw[(8 * f * g) & 511]);
    __syncthreads();
#pragma unroll
    for (int ff = 0; ff < 8; ++ff) v[ff] = ldsB[(c2 * 64 + 8 * f + ff) * kPitch + w];
    dft8<INV>(v);
}

template <bool INV>
__global__ __launch_bounds__(kT512) void k_colfft512(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                     int nin, int nout, int64_t J, int64_t in_bs, int64_t out_bs,
                                                     const float2 *__restrict__ tw512) {
    __shared__ float2 lds[512 * kPitch];
    const int t = threadIdx.x;
    const int w = t & (kW512 - 1), q = t >> kW512Log;  // column in the tile, thread of the column
    // Rows of J complex values are not 128-byte multiples, so a block's row
    // segments straddle lines it shares with the next column group: blocks
    // are renumbered so that each XCD takes one contiguous range of them
    // (workgroups are dealt to the 8 XCDs in turn) and shared lines meet in
    // one L2.
    int64_t bx, b;
    {
        const int64_t T = (int64_t)gridDim.x * gridDim.y, id = blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
        const int64_t qn = T / 8, rn = T % 8, k = id % 8;
        const int64_t v = k * qn + (k < rn ? k : rn) + id / 8;
        bx = v % gridDim.x;
        b = v / gridDim.x;
    }
    const int64_t j = bx * kW512 + w;
    const bool col = j < J;
    const float2 *src = in + b * in_bs + j;
    float2 *dst = out + b * out_bs + j;
    float2 v[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int r = 64 * a + q;
        v[a] = (col && r < nin) ? src[(int64_t)r * J] : make_float2(0.0f, 0.0f);
    }
    fft512<INV>(v, lds, q, q, w, tw512);
    if (col) {
        const int base = (q >> 3) + 8 * (q & 7);
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int r = base + 64 * h;
            if (r < nout) dst[(int64_t)r * J] = v[h];
        }
    }
}

// x rows for Px = 512: two real rows (A, B) of one pair transformed as one
// complex 512-point FFT z = a + i b, whose spectrum Z gives both halves,
// A[k] = (Z[k] + conj Z[512 - k]) / 2 and B[k] = (Z[k] - conj Z[512 - k]) / 2i
// for k <= 256.  Global reads and writes run along the rows (consecutive
// lanes, consecutive x or k: thread t serves pair t / 64, position t % 64);
// the values pass to and from fft512's column-slot layout through LDS.
// Row r = (c, line) of the pair index holds spins S[r Lx + x] (x < Lx, zero
// to 512) and spectrum X[r H + k] (H = 257).
__global__ __launch_bounds__(kT512) void k_xfft512_fwd(const double *__restrict__ S, float2 *__restrict__ X, int Lx,
                                                       int64_t nrows, const float2 *__restrict__ tw512) {
    __shared__ float2 lds[512 * kPitch];
    const int t = threadIdx.x;
    const int64_t pair0 = (int64_t)blockIdx.x * kW512;
    {
        const int wp = t >> 6, n0 = t & 63;
        const int64_t ra = 2 * (pair0 + wp), rb = ra + 1;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int n = 64 * a + n0;
            const float re = (n < Lx && ra < nrows) ? (float)S[ra * Lx + n] : 0.0f;
            const float im = (n < Lx && rb < nrows) ? (float)S[rb * Lx + n] : 0.0f;
            lds[n * kPitch + wp] = make_float2(re, im);
        }
    }
    __syncthreads();
    const int w = t & (kW512 - 1), q = t >> kW512Log;
    float2 v[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) v[a] = lds[(64 * a + q) * kPitch + w];
    fft512<false>(v, lds, q, q, w, tw512);
    __syncthreads();
    const int qq = (q >> 3) + 8 * (q & 7);
#pragma unroll
    for (int h = 0; h < 8; ++h) lds[(qq + 64 * h) * kPitch + w] = v[h];
    __syncthreads();
    {
        const int wp = t >> 6, k0 = t & 63;
        const int64_t ra = 2 * (pair0 + wp), rb = ra + 1;
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            const int k = k0 + 64 * m;
            if (k > 256) break;
            const float2 zk = lds[k * kPitch + wp], zm = lds[((512 - k) & 511) * kPitch + wp];
            if (ra < nrows) X[ra * 257 + k] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            if (rb < nrows) X[rb * 257 + k] = make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
        }
    }
}

// The inverse: Z[n] = A[n] + i B[n] over all 512 bins from the stored half
// (A[512 - k] = conj A[k]; the imaginary parts of bins 0 and 256 dropped, as
// for a real inverse transform), one unnormalised inverse FFT, and rows
// x < Lx of z = a + i b written to the field.
__global__ __launch_bounds__(kT512) void k_xfft512_inv(const float2 *__restrict__ X, float *__restrict__ b, int Lx,
                                                       int64_t nrows, const float2 *__restrict__ tw512) {
    __shared__ float2 lds[512 * kPitch];
    const int t = threadIdx.x;
    const int64_t pair0 = (int64_t)blockIdx.x * kW512;
    {
        const int wp = t >> 6, n0 = t & 63;
        const int64_t ra = 2 * (pair0 + wp), rb = ra + 1;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int n = 64 * a + n0;
            const int k = n <= 256 ? n : 512 - n;
            float2 A = ra < nrows ? X[ra * 257 + k] : make_float2(0.0f, 0.0f);
            float2 B = rb < nrows ? X[rb * 257 + k] : make_float2(0.0f, 0.0f);
            if (k == 0 || k == 256) {
                A.y = 0.0f;
                B.y = 0.0f;
            } else if (n > 256) {
                A.y = -A.y;
                B.y = -B.y;
            }
            lds[n * kPitch + wp] = make_float2(A.x - B.y, A.y + B.x);
        }
    }
    __syncthreads();
    const int w = t & (kW512 - 1), q = t >> kW512Log;
    float2 v[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) v[a] = lds[(64 * a + q) * kPitch + w];
    fft512<true>(v, lds, q, q, w, tw512);
    __syncthreads();
    const int qq = (q >> 3) + 8 * (q & 7);
#pragma unroll
    for (int h = 0; h < 8; ++h) lds[(qq + 64 * h) * kPitch + w] = v[h];
    __syncthreads();
    {
        const int wp = t >> 6, n0 = t & 63;
        const int64_t ra = 2 * (pair0 + wp), rb = ra + 1;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int n = 64 * a + n0;
            if (n >= Lx) break;
            const float2 z = lds[n * kPitch + wp];
            if (ra < nrows) b[ra * Lx + n] = z.x;
            if (rb < nrows) b[rb * Lx + n] = z.y;
        }
    }
}

// The dipole spectrum reordered for the fused z pass: block g of 16 columns
// reads kernb[g][kz][c][0..15] for its kz, one contiguous run per kz.
__global__ void k_kern_block(const float *__restrict__ kern, float *__restrict__ kernb, int64_t J, int64_t n_cplx,
                             int nkz, int64_t total) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int w = (int)(q % kW512);
    int64_t r = q / kW512;
    const int c = (int)(r % 6);
    r /= 6;
    const int kz = (int)(r % nkz);
    const int64_t g = r / nkz;
    const int64_t j = g * kW512 + w;
    kernb[q] = j < J ? kern[c * n_cplx + (int64_t)kz * J + j] : 0.0f;
}

// z transform, spectral product and inverse z transform fused for Pz = 512:
// each block takes 8 (y, kx) columns of the three components (rows z < Lz of
// Y, zero above), transforms them forward, multiplies by the dipole spectrum
// at its 512 kz and transforms back, writing rows z < Lz in place.  The
// forward result sits in the thread that needs it for the inverse's first
// pass (row c + 8 g + 64 h = 64 h + qin with qin = c + 8 g).
__global__ __launch_bounds__(kT512) void k_zconv512(float2 *__restrict__ Y, const float *__restrict__ kernb, int Lz,
                                                    int64_t J, int nkz, const float2 *__restrict__ tw512,
                                                    int zsym) {
    __shared__ float2 ldsA[512 * kPitch], ldsB[512 * kPitch];
    const int t = threadIdx.x;
    const int w = t & (kW512 - 1), q = t >> kW512Log;
    const int64_t j = (int64_t)blockIdx.x * kW512 + w;
    const bool col = j < J;
    const int64_t cs = (int64_t)Lz * J;
    // all three components' loads in flight before the first transform
    float2 v[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int r = 64 * a + q;
            v[c][a] = (col && r < Lz) ? Y[c * cs + (int64_t)r * J + j] : make_float2(0.0f, 0.0f);
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) fft512_2buf<false>(v[c], ldsA, ldsB, q, q, w, tw512);
    const int qq = (q >> 3) + 8 * (q & 7);
    if (col) {
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            // kz and 512 - kz read the same stored entries (sign flip for xz, yz)
            const int kz = qq + 64 * h;
            const bool mirror = zsym && kz > 256;
            const float sgn = mirror ? -1.0f : 1.0f;
            const float *kb = kernb + (((int64_t)blockIdx.x * nkz + (mirror ? 512 - kz : kz)) * 6) * kW512 + w;
            const float txx = kb[0], txy = kb[kW512], txz = sgn * kb[2 * kW512];
            const float tyy = kb[3 * kW512], tyz = sgn * kb[4 * kW512], tzz = kb[5 * kW512];
            const float2 sx = v[0][h], sy = v[1][h], sz = v[2][h];
            v[0][h] = make_float2(txx * sx.x + txy * sy.x + txz * sz.x, txx * sx.y + txy * sy.y + txz * sz.y);
            v[1][h] = make_float2(txy * sx.x + tyy * sy.x + tyz * sz.x, txy * sx.y + tyy * sy.y + tyz * sz.y);
            v[2][h] = make_float2(txz * sx.x + tyz * sy.x + tzz * sz.x, txz * sx.y + tyz * sy.y + tzz * sz.y);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        fft512_2buf<true>(v[c], ldsA, ldsB, qq, q, w, tw512);
        if (col) {
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                const int r = qq + 64 * h;
                if (r < Lz) Y[c * cs + (int64_t)r * J + j] = v[c][h];
            }
        }
    }
}

unsigned nblocks(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

spx_status fft_fail(hipfftResult r, const char *where) {
    return set_error(SPX_ERR_FFT, std::string(where) + ": hipFFT error " + std::to_string((int)r));
}

template <bool INV>
hipError_t colfft(const float2 *in, float2 *out, int P, int nin, int nout, int64_t J, int64_t nbatch, int64_t in_bs,
                  int64_t out_bs, const float2 *tw, hipStream_t st) {
    if (P == 512) {
        dim3 grid((unsigned)((J + kW512 - 1) / kW512), (unsigned)nbatch);
        k_colfft512<INV><<<grid, kT512, 0, st>>>(in, out, nin, nout, J, in_bs, out_bs, tw);
        return hipGetLastError();
    }
    const int W = col_width(P);  // P >= 2 (padded extents are at least 2)
    const size_t smem = ((size_t)P * W + P / 2) * sizeof(float2);
    dim3 grid((unsigned)((J + W - 1) / W), (unsigned)nbatch);
    k_colfft<INV><<<grid, kColThreads, smem, st>>>(in, out, log2i(P), log2i(W), nin, nout, J, in_bs, out_bs, tw);
    return hipGetLastError();
}

}  // namespace

void destroy_dipolar(DipolarPlan *p) {
    if (!p) return;
    if (p->fwd_ok) hipfftDestroy(p->fwd);
    if (p->inv_ok) hipfftDestroy(p->inv);
    for (void *q : {(void *)p->R, (void *)p->X, (void *)p->Y, (void *)p->Z, (void *)p->kern, (void *)p->kernb, (void *)p->tw_y,
                    (void *)p->tw_z, (void *)p->tw_x})
        if (q) (void)hipFree(q);
    delete p;
}

spx_status create_dipolar(const int32_t dims[3], const double cell[9], double mu, hipStream_t st,
                          DipolarPlan **out, int64_t *ws_bytes) {
    for (int k = 0; k < 3; ++k)
        if (dims[k] < 1 || dims[k] > 2048)
            return set_error(SPX_ERR_UNSUPPORTED, "dipolar FFT path: extents must be 1 .. 2048 per axis");
    DipolarPlan *p = new DipolarPlan();
    for (int k = 0; k < 3; ++k) {
        p->L[k] = dims[k];
        p->P[k] = next_pow2(2 * dims[k] - 1 < 2 ? 2 : 2 * dims[k] - 1);
    }
    const int Lx = p->L[0], Ly = p->L[1], Lz = p->L[2], Px = p->P[0], Py = p->P[1], Pz = p->P[2];
    p->H = Px / 2 + 1;
    p->N = (int64_t)Lx * Ly * Lz;
    p->n_cplx = (int64_t)Pz * Py * p->H;
    const int64_t rows = (int64_t)Ly * Lz;
    auto alloc = [&](void **ptr, size_t bytes, const char *what) -> spx_status {
        if (hipMalloc(ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *ptr = nullptr;
            return set_error(SPX_ERR_OUT_OF_MEMORY, std::string("hipMalloc failed for ") + what);
        }
        *ws_bytes += (int64_t)bytes;
        return SPX_OK;
    };
    spx_status s;
    if ((Px != 512 && (s = alloc((void **)&p->R, sizeof(float) * 3 * rows * Px, "dipolar rows")) != SPX_OK) ||
        (Px == 512 && (s = alloc((void **)&p->tw_x, sizeof(float2) * 512, "dipolar twiddles")) != SPX_OK) ||
        (s = alloc((void **)&p->X, sizeof(float2) * 3 * rows * p->H, "dipolar x spectra")) != SPX_OK ||
        (s = alloc((void **)&p->Y, sizeof(float2) * 3 * (int64_t)Lz * Py * p->H, "dipolar xy spectra")) != SPX_OK ||
        (Pz != 512 && (s = alloc((void **)&p->Z, sizeof(float2) * 3 * p->n_cplx, "dipolar spectra")) != SPX_OK) ||
        (s = alloc((void **)&p->kern, sizeof(float) * 6 * p->n_cplx, "dipole spectrum")) != SPX_OK ||
        (s = alloc((void **)&p->tw_y, sizeof(float2) * Py, "dipolar twiddles")) != SPX_OK ||
        (s = alloc((void **)&p->tw_z, sizeof(float2) * Pz, "dipolar twiddles")) != SPX_OK) {
        destroy_dipolar(p);
        return s;
    }
    // twiddle tables exp(-2 pi i k / P), k < P, from FP64
    std::vector<float2> ty(Py), tz(Pz);
    for (int k = 0; k < Py; ++k)
        ty[k] = make_float2((float)std::cos(2.0 * M_PI * k / Py), (float)(-std::sin(2.0 * M_PI * k / Py)));
    for (int k = 0; k < Pz; ++k)
        tz[k] = make_float2((float)std::cos(2.0 * M_PI * k / Pz), (float)(-std::sin(2.0 * M_PI * k / Pz)));
    hipError_t e = hipMemcpyAsync(p->tw_y, ty.data(), sizeof(float2) * ty.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->tw_z, tz.data(), sizeof(float2) * tz.size(), hipMemcpyHostToDevice, st);
    std::vector<float2> tx(Px == 512 ? 512 : 0);
    for (size_t k = 0; k < tx.size(); ++k)
        tx[k] = make_float2((float)std::cos(2.0 * M_PI * k / 512), (float)(-std::sin(2.0 * M_PI * k / 512)));
    if (e == hipSuccess && Px == 512)
        e = hipMemcpyAsync(p->tw_x, tx.data(), sizeof(float2) * tx.size(), hipMemcpyHostToDevice, st);
    // kernel spectrum, one tensor component at a time in FP64
    const int64_t n_real = (int64_t)Px * Py * Pz;
    double *treal = nullptr;
    double2 *tcplx = nullptr;
    if ((s = alloc((void **)&treal, sizeof(double) * n_real, "dipole tensor (setup)")) != SPX_OK) {
        destroy_dipolar(p);
        return s;
    }
    if ((s = alloc((void **)&tcplx, sizeof(double2) * p->n_cplx, "dipole tensor spectrum (setup)")) != SPX_OK) {
        (void)hipFree(treal);
        destroy_dipolar(p);
        return s;
    }
    *ws_bytes -= (int64_t)(sizeof(double) * n_real + sizeof(double2) * p->n_cplx);
    hipfftHandle dplan;
    hipfftResult fr = hipfftPlan3d(&dplan, Pz, Py, Px, HIPFFT_D2Z);
    if (fr != HIPFFT_SUCCESS) {
        (void)hipFree(treal);
        (void)hipFree(tcplx);
        destroy_dipolar(p);
        return fft_fail(fr, "dipolar setup plan");
    }
    hipfftSetStream(dplan, st);
    const double pref = dipole_prefactor() * mu * mu / (double)n_real;
    const int comps[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    // z parity of the sampled tensor: no coupling of the z axis with x, y in the
    // cell matrix (either storage order)
    p->zsym = cell[2] == 0.0 && cell[5] == 0.0 && cell[6] == 0.0 && cell[7] == 0.0;
    for (int c = 0; c < 6 && s == SPX_OK && e == hipSuccess; ++c) {
        k_dipole_component<<<nblocks(n_real), kB, 0, st>>>(Lx, Ly, Lz, Px, Py, Pz, cell[0], cell[1], cell[2], cell[3],
                                                            cell[4], cell[5], cell[6], cell[7], cell[8], comps[c][0],
                                                            comps[c][1], pref, treal);
        fr = hipfftExecD2Z(dplan, treal, (hipfftDoubleComplex *)tcplx);
        if (fr != HIPFFT_SUCCESS) { s = fft_fail(fr, "dipolar setup transform"); break; }
        k_take_real<<<nblocks(p->n_cplx), kB, 0, st>>>(tcplx, p->n_cplx, p->kern + c * p->n_cplx);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipfftDestroy(dplan);
    (void)hipFree(treal);
    (void)hipFree(tcplx);
    if (s == SPX_OK && e != hipSuccess) s = set_hip_error(e, "dipolar setup");
    if (s != SPX_OK) {
        destroy_dipolar(p);
        return s;
    }
    if (Pz == 512) {
        // the fused z pass's order; the [6][Pz][Py][H] spectrum is then no
        // longer needed
        const int64_t plane = (int64_t)Py * p->H, ngroup = (plane + kW512 - 1) / kW512;
        p->nkz = p->zsym ? 257 : 512;
        const int64_t total = ngroup * p->nkz * 6 * kW512;
        if ((s = alloc((void **)&p->kernb, sizeof(float) * total, "dipole spectrum (z pass order)")) != SPX_OK) {
            destroy_dipolar(p);
            return s;
        }
        k_kern_block<<<nblocks(total), kB, 0, st>>>(p->kern, p->kernb, plane, p->n_cplx, p->nkz, total);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            destroy_dipolar(p);
            return set_hip_error(e, "dipolar spectrum reorder");
        }
        (void)hipFree(p->kern);
        p->kern = nullptr;
        *ws_bytes -= (int64_t)(sizeof(float) * 6 * p->n_cplx);
    }
    if (Px == 512) {  // the x rows run in k_xfft512_fwd / k_xfft512_inv
        *out = p;
        return SPX_OK;
    }
    // batched FP32 x-row transforms of the occupied lines of the three components
    int n[1] = {Px};
    int rembed[1] = {Px}, cembed[1] = {p->H};
    const int batch = (int)(3 * rows);
    fr = hipfftPlanMany(&p->fwd, 1, n, rembed, 1, Px, cembed, 1, p->H, HIPFFT_R2C, batch);
    if (fr != HIPFFT_SUCCESS) {
        destroy_dipolar(p);
        return fft_fail(fr, "dipolar R2C plan");
    }
    p->fwd_ok = true;
    fr = hipfftPlanMany(&p->inv, 1, n, cembed, 1, p->H, rembed, 1, Px, HIPFFT_C2R, batch);
    if (fr != HIPFFT_SUCCESS) {
        destroy_dipolar(p);
        return fft_fail(fr, "dipolar C2R plan");
    }
    p->inv_ok = true;
    *out = p;
    return SPX_OK;
}

spx_status eval_dipolar(DipolarPlan *p, const double *S, float *bdip, hipStream_t st) {
    if (!p) return set_error(SPX_ERR_INVALID_ARG, "dipolar path not set up");
    const int Lx = p->L[0], Ly = p->L[1], Lz = p->L[2], Px = p->P[0], Py = p->P[1], Pz = p->P[2], H = p->H;
    const int64_t rows = (int64_t)Ly * Lz;
    // x rows: pairs of rows, 16 pairs per block
    const unsigned xgrid = (unsigned)(((3 * rows + 1) / 2 + kW512 - 1) / kW512);
    hipError_t e;
    if (Px == 512) {
        k_xfft512_fwd<<<xgrid, kT512, 0, st>>>(S, p->X, Lx, 3 * rows, p->tw_x);
        e = hipGetLastError();
        if (e != hipSuccess) return set_hip_error(e, "dipolar x rows");
    } else {
        k_pad_rows<<<(unsigned)(3 * rows), kB, 0, st>>>(S, Lx, Px, rows, p->N, p->R);
        e = hipGetLastError();
        if (e != hipSuccess) return set_hip_error(e, "dipolar pad");
        hipfftSetStream(p->fwd, st);
        hipfftResult fr = hipfftExecR2C(p->fwd, p->R, (hipfftComplex *)p->X);
        if (fr != HIPFFT_SUCCESS) return fft_fail(fr, "dipolar R2C");
    }
    const int64_t plane = (int64_t)Py * H;
    // y: X [3 Lz][Ly rows][H] -> Y [3 Lz][Py][H]
    e = colfft<false>(p->X, p->Y, Py, Ly, Py, H, 3 * (int64_t)Lz, (int64_t)Ly * H, plane, p->tw_y, st);
    if (Pz == 512) {
        // z transform, product and inverse z transform in one pass over Y
        if (e == hipSuccess) {
            k_zconv512<<<(unsigned)((plane + kW512 - 1) / kW512), kT512, 0, st>>>(p->Y, p->kernb, Lz, plane, p->nkz,
                                                                                p->tw_z, p->zsym ? 1 : 0);
            e = hipGetLastError();
        }
    } else {
        // z: Y [3][Lz planes][Py H] -> Z [3][Pz][Py H]
        if (e == hipSuccess)
            e = colfft<false>(p->Y, p->Z, Pz, Lz, Pz, plane, 3, (int64_t)Lz * plane, p->n_cplx, p->tw_z, st);
        if (e == hipSuccess) {
            k_spectral_mult<<<nblocks(p->n_cplx), kB, 0, st>>>(p->Z, p->kern, p->n_cplx);
            e = hipGetLastError();
        }
        // inverse z keeps planes z < Lz
        if (e == hipSuccess)
            e = colfft<true>(p->Z, p->Y, Pz, Pz, Lz, plane, 3, p->n_cplx, (int64_t)Lz * plane, p->tw_z, st);
    }
    // inverse y keeps rows y < Ly
    if (e == hipSuccess)
        e = colfft<true>(p->Y, p->X, Py, Py, Ly, H, 3 * (int64_t)Lz, plane, (int64_t)Ly * H, p->tw_y, st);
    if (e != hipSuccess) return set_hip_error(e, "dipolar column transforms");
    if (Px == 512) {
        k_xfft512_inv<<<xgrid, kT512, 0, st>>>(p->X, bdip, Lx, 3 * rows, p->tw_x);
        e = hipGetLastError();
        if (e != hipSuccess) return set_hip_error(e, "dipolar x rows");
        return SPX_OK;
    }
    hipfftSetStream(p->inv, st);
    hipfftResult fr = hipfftExecC2R(p->inv, (hipfftComplex *)p->X, p->R);
    if (fr != HIPFFT_SUCCESS) return fft_fail(fr, "dipolar C2R");
    k_crop_rows<<<(unsigned)(3 * rows), kB, 0, st>>>(p->R, Lx, Px, rows, p->N, bdip);
    e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "dipolar crop");
    return SPX_OK;
}

}  // namespace spx
