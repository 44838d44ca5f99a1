// spx_dipolar.hip -- open-boundary dipolar field by zero-padded FFT
// convolution (Methods, reciprocal-space convolution for long-range dipolar
// fields) on gfx950 with hipFFT.
//
// The dipole tensor T(r) = (mu0/4pi) mu_B^2 (3 rhat rhat - 1)/r^3 is sampled
// on a grid of 2L per axis holding every displacement in [-(L-1), L-1]; the
// zero-padded spin planes are transformed (batched FP32 R2C), multiplied by
// the six-component real spectrum of T (built once in FP64, scaled by mu^2 and
// by the 1/N_pad of the unnormalised inverse), transformed back (C2R) and
// cropped.  Linear (aperiodic) convolution = open boundaries.
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstring>

#include "spx_ext.hpp"

namespace spx {

struct DipolarPlan {
    int L[3];              // x, y, z cells
    int P[3];              // padded extents 2L
    int64_t n_real;        // padded real points per component
    int64_t n_cplx;        // complex points per component (2Lz * 2Ly * (Lx+1))
    int64_t N;             // sites
    float *pad = nullptr;      // [3][n_real] real grid (pad in, field out)
    float2 *spec = nullptr;    // [3][n_cplx] spin spectra, then field spectra
    float *kern = nullptr;     // [6][n_cplx] real dipole spectrum xx, xy, xz, yy, yz, zz
    hipfftHandle fwd = 0, inv = 0;
    bool fwd_ok = false, inv_ok = false;
    void *work = nullptr;
};

namespace {

constexpr int kB = 256;

// (mu0/4pi) mu_B^2 in meV nm^3 from SI values (CODATA 2018).
double dipole_prefactor() {
    const double mu0_over_4pi = 1.0e-7;      // T m / A
    const double muB_SI = 9.2740100783e-24;  // J / T
    const double meV_in_J = 1.602176634e-22;
    return mu0_over_4pi * muB_SI * muB_SI / meV_in_J * 1.0e27;
}

__device__ __forceinline__ int pad_disp(int k, int L) { return k < L ? k : k - 2 * L; }

// One component (a,b) of the real-space dipole tensor on the padded grid, FP64.
__global__ void k_dipole_component(int Lx, int Ly, int Lz, double c00, double c01, double c02, double c10,
                                   double c11, double c12, double c20, double c21, double c22, int ca,
                                   int cb, double pref, double *__restrict__ out) {
    const int64_t Px = 2 * Lx, Py = 2 * Ly, Pz = 2 * Lz;
    const int64_t idx = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (idx >= Px * Py * Pz) return;
    const int kx = (int)(idx % Px), ky = (int)((idx / Px) % Py), kz = (int)(idx / (Px * Py));
    double v = 0.0;
    if (kx != Lx && ky != Ly && kz != Lz) {
        const double dx = pad_disp(kx, Lx), dy = pad_disp(ky, Ly), dz = pad_disp(kz, Lz);
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

__global__ void k_take_real(const double2 *__restrict__ in, int64_t n, double scale, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) out[i] = (float)(in[i].x * scale);
}

// Zero-padded FP32 copies of the three spin planes.
__global__ void k_pad(const double *__restrict__ S, int Lx, int Ly, int Lz, int64_t N, int64_t n_real,
                      float *__restrict__ pad) {
    const int64_t Px = 2 * Lx, Py = 2 * Ly;
    const int64_t idx = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (idx >= n_real) return;
    const int kx = (int)(idx % Px), ky = (int)((idx / Px) % Py), kz = (int)(idx / (Px * Py));
    const bool in = kx < Lx && ky < Ly && kz < Lz;
    const int64_t i = in ? (kx + (int64_t)Lx * (ky + (int64_t)Ly * kz)) : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) pad[c * n_real + idx] = in ? (float)S[c * N + i] : 0.0f;
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

__global__ void k_crop(const float *__restrict__ pad, int Lx, int Ly, int Lz, int64_t N, int64_t n_real,
                       float *__restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= N) return;
    const int x = (int)(i % Lx), y = (int)((i / Lx) % Ly), z = (int)(i / ((int64_t)Lx * Ly));
    const int64_t k = x + (int64_t)(2 * Lx) * (y + (int64_t)(2 * Ly) * z);
#pragma unroll
    for (int c = 0; c < 3; ++c) b[c * N + i] = pad[c * n_real + k];
}

unsigned nblocks(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

spx_status fft_fail(hipfftResult r, const char *where) {
    return set_error(SPX_ERR_FFT, std::string(where) + ": hipFFT error " + std::to_string((int)r));
}

}  // namespace

void destroy_dipolar(DipolarPlan *p) {
    if (!p) return;
    if (p->fwd_ok) hipfftDestroy(p->fwd);
    if (p->inv_ok) hipfftDestroy(p->inv);
    if (p->pad) (void)hipFree(p->pad);
    if (p->spec) (void)hipFree(p->spec);
    if (p->kern) (void)hipFree(p->kern);
    delete p;
}

spx_status create_dipolar(const int32_t dims[3], const double cell[9], double mu, hipStream_t st,
                          DipolarPlan **out, int64_t *ws_bytes) {
    DipolarPlan *p = new DipolarPlan();
    for (int k = 0; k < 3; ++k) {
        p->L[k] = dims[k];
        p->P[k] = 2 * dims[k];
    }
    p->N = (int64_t)dims[0] * dims[1] * dims[2];
    p->n_real = (int64_t)p->P[0] * p->P[1] * p->P[2];
    p->n_cplx = (int64_t)p->P[2] * p->P[1] * (p->P[0] / 2 + 1);
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
    if ((s = alloc((void **)&p->pad, sizeof(float) * 3 * p->n_real, "dipolar padded grid")) != SPX_OK ||
        (s = alloc((void **)&p->spec, sizeof(float2) * 3 * p->n_cplx, "dipolar spectra")) != SPX_OK ||
        (s = alloc((void **)&p->kern, sizeof(float) * 6 * p->n_cplx, "dipole spectrum")) != SPX_OK) {
        destroy_dipolar(p);
        return s;
    }
    // kernel spectrum, one tensor component at a time in FP64
    double *treal = nullptr;
    double2 *tcplx = nullptr;
    if ((s = alloc((void **)&treal, sizeof(double) * p->n_real, "dipole tensor (setup)")) != SPX_OK) {
        destroy_dipolar(p);
        return s;
    }
    if ((s = alloc((void **)&tcplx, sizeof(double2) * p->n_cplx, "dipole tensor spectrum (setup)")) != SPX_OK) {
        (void)hipFree(treal);
        destroy_dipolar(p);
        return s;
    }
    *ws_bytes -= (int64_t)(sizeof(double) * p->n_real + sizeof(double2) * p->n_cplx);
    hipfftHandle dplan;
    int n[3] = {p->P[2], p->P[1], p->P[0]};
    hipfftResult fr = hipfftPlan3d(&dplan, n[0], n[1], n[2], HIPFFT_D2Z);
    if (fr != HIPFFT_SUCCESS) {
        (void)hipFree(treal);
        (void)hipFree(tcplx);
        destroy_dipolar(p);
        return fft_fail(fr, "dipolar setup plan");
    }
    hipfftSetStream(dplan, st);
    const double pref = dipole_prefactor() * mu * mu / (double)p->n_real;
    const int comps[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int c = 0; c < 6 && s == SPX_OK; ++c) {
        k_dipole_component<<<nblocks(p->n_real), kB, 0, st>>>(
            p->L[0], p->L[1], p->L[2], cell[0], cell[1], cell[2], cell[3], cell[4], cell[5], cell[6], cell[7],
            cell[8], comps[c][0], comps[c][1], pref, treal);
        fr = hipfftExecD2Z(dplan, treal, (hipfftDoubleComplex *)tcplx);
        if (fr != HIPFFT_SUCCESS) { s = fft_fail(fr, "dipolar setup transform"); break; }
        k_take_real<<<nblocks(p->n_cplx), kB, 0, st>>>(tcplx, p->n_cplx, 1.0, p->kern + c * p->n_cplx);
    }
    hipError_t e = hipStreamSynchronize(st);
    hipfftDestroy(dplan);
    (void)hipFree(treal);
    (void)hipFree(tcplx);
    if (s == SPX_OK && e != hipSuccess) s = set_hip_error(e, "dipolar setup");
    if (s != SPX_OK) {
        destroy_dipolar(p);
        return s;
    }
    // batched FP32 transforms of the three components
    int inembed[3] = {n[0], n[1], n[2]};
    int onembed[3] = {n[0], n[1], n[2] / 2 + 1};
    fr = hipfftPlanMany(&p->fwd, 3, n, inembed, 1, (int)p->n_real, onembed, 1, (int)p->n_cplx, HIPFFT_R2C, 3);
    if (fr != HIPFFT_SUCCESS) {
        destroy_dipolar(p);
        return fft_fail(fr, "dipolar R2C plan");
    }
    p->fwd_ok = true;
    fr = hipfftPlanMany(&p->inv, 3, n, onembed, 1, (int)p->n_cplx, inembed, 1, (int)p->n_real, HIPFFT_C2R, 3);
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
    k_pad<<<nblocks(p->n_real), kB, 0, st>>>(S, p->L[0], p->L[1], p->L[2], p->N, p->n_real, p->pad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "dipolar pad");
    hipfftSetStream(p->fwd, st);
    hipfftResult fr = hipfftExecR2C(p->fwd, p->pad, (hipfftComplex *)p->spec);
    if (fr != HIPFFT_SUCCESS) return fft_fail(fr, "dipolar R2C");
    k_spectral_mult<<<nblocks(p->n_cplx), kB, 0, st>>>(p->spec, p->kern, p->n_cplx);
    e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "dipolar spectral product");
    hipfftSetStream(p->inv, st);
    fr = hipfftExecC2R(p->inv, (hipfftComplex *)p->spec, p->pad);
    if (fr != HIPFFT_SUCCESS) return fft_fail(fr, "dipolar C2R");
    k_crop<<<nblocks(p->N), kB, 0, st>>>(p->pad, p->L[0], p->L[1], p->L[2], p->N, p->n_real, bdip);
    e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "dipolar crop");
    return SPX_OK;
}

}  // namespace spx
