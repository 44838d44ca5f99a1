// spx_noalloc.hip -- spx_energy_noalloc: the energy of spx_energy for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// spx_energy reduces through a partial buffer the Hamiltonian handle owns
// and, with the z-march engine, a field buffer it allocates at its first call.
// This variant gathers each site's neighbours itself and keeps its partial
// sums in one file-scope device array, `scratch`, of kMaxBlocks quadruples
// (128 KiB) per device: the partial pass runs min(ceil(N / 256), kMaxBlocks)
// blocks, each striding over the lattice in a fixed order, and one block adds
// their quadruples in a fixed order.  Every quadruple the final pass reads is
// written by the same call, so nothing needs clearing between calls; calls
// that overlap on one device (two streams) race on the array.
#include <mutex>

#include "spx_device.hpp"
#include "spx_ext.hpp"

namespace spx {

constexpr int kNaBlock = 256;
constexpr int kMaxBlocks = 4096;

static __device__ __align__(256) double scratch[4 * kMaxBlocks];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (the array's name is a host-side stand-in, not that address).
spx_status scratch_address(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_hip_error(e, "spx_energy_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(SPX_ERR_UNSUPPORTED, "spx_energy_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                 "spx_energy_noalloc: hipGetSymbolAddress(scratch)");
        }
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return SPX_OK;
}

// Per-site terms -S.b_bil/2, -S.b_Z, -S.b_ani/2 of sites i = b 256 + t +
// k gridDim 256 (all sublattices), summed per thread in that order, then over
// the block in a fixed tree; part[b][4] (the dipolar slot is 0).
template <typename AccT, bool ISO>
__global__ __launch_bounds__(kNaBlock) void k_energy_strided(BondTable tb, Grid g, Onsite os,
                                                             const double *__restrict__ S, double *__restrict__ part) {
    __shared__ double red[kNaBlock / 64][3];
    const int64_t N = g.N;
    double e[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kNaBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kNaBlock) {
        const int a = (int)(i / g.M);
        const int t = (int)(i - (int64_t)a * g.M);
        int x, y, z;
        site_xyz(g, t, x, y, z);
        AccT acc[1][3];
        const double *const src[1] = {S};
        bil_sum<AccT, ISO, 1>(tb, g, a, x, y, z, src, acc);
        const double s[3] = {S[i], S[N + i], S[2 * N + i]};
        double ba[3];
        aniso_field(os, a, s, ba);
        double sb = 0.0, sz = 0.0, sa = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sb += s[c] * (double)acc[0][c];
            sz += s[c] * os.bz[a][c];
            sa += s[c] * ba[c];
        }
        e[0] += -0.5 * sb;
        e[1] += -sz;
        e[2] += -0.5 * sa;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = wave_sum(e[k]);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0.0;
        if (threadIdx.x < 3)
            for (int w = 0; w < kNaBlock / 64; ++w) v += red[w][threadIdx.x];
        part[(size_t)blockIdx.x * 4 + threadIdx.x] = v;
    }
}

// Fixed-order sum of nb partial quadruples by one block: E = total, terms =
// (bilinear, Zeeman, anisotropy, dipolar = 0, total).
__global__ __launch_bounds__(kNaBlock) void k_energy_strided_final(const double *__restrict__ part, int nb,
                                                                   double *__restrict__ E,
                                                                   double *__restrict__ terms) {
    __shared__ double red[kNaBlock / 64][4];
    double e[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < nb; p += kNaBlock)
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] += part[(size_t)p * 4 + k];
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
            for (int w = 0; w < kNaBlock / 64; ++w) tot[k] += red[w][k];
        }
        const double all = ((tot[0] + tot[1]) + tot[2]) + tot[3];
        if (E) *E = all;
        if (terms) {
            for (int k = 0; k < 4; ++k) terms[k] = tot[k];
            terms[4] = all;
        }
    }
}

}  // namespace
}  // namespace spx

using namespace spx;

extern "C" spx_status spx_energy_noalloc(spx_ham *h, const double *S, double *E, double *terms, void *stream) {
    HamView v;
    spx_status s = get_ham_view(h, v);
    if (s != SPX_OK) return s;
    if (!S || (!E && !terms)) return set_error(SPX_ERR_INVALID_ARG, "S is NULL or no output given");
    if (v.pl) return set_error(SPX_ERR_UNSUPPORTED, "spx_energy_noalloc: pair-list Hamiltonians use spx_energy");
    if (v.dip) return set_error(SPX_ERR_UNSUPPORTED, "spx_energy_noalloc: the dipolar term needs spx_energy");
    const int64_t N = v.grid.N;
    const int64_t want = (N + kNaBlock - 1) / kNaBlock;
    const int nb = (int)(want < kMaxBlocks ? want : kMaxBlocks);
    if (nb < 1 || nb > kMaxBlocks)
        return set_error(SPX_ERR_INVALID_ARG, "spx_energy_noalloc: partial blocks outside the 4096 of the scratch");
    double *part = nullptr;
    if ((s = scratch_address(&part)) != SPX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    // the MFMA backends evaluate energies with the FP32 gather, as spx_energy
    if (v.field_prec == SPX_FP64) {
        if (v.tab.iso) k_energy_strided<double, true><<<nb, kNaBlock, 0, st>>>(v.tab, v.grid, v.onsite, S, part);
        else k_energy_strided<double, false><<<nb, kNaBlock, 0, st>>>(v.tab, v.grid, v.onsite, S, part);
    } else {
        if (v.tab.iso) k_energy_strided<float, true><<<nb, kNaBlock, 0, st>>>(v.tab, v.grid, v.onsite, S, part);
        else k_energy_strided<float, false><<<nb, kNaBlock, 0, st>>>(v.tab, v.grid, v.onsite, S, part);
    }
    k_energy_strided_final<<<1, kNaBlock, 0, st>>>(part, nb, E, terms);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "spx_energy_noalloc");
    return SPX_OK;
}
