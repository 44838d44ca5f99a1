// spx_internal.hpp -- types shared by the host runtime and the HIP kernels of
// libspx.so.  Not part of the public ABI (see include/spx.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spx {

constexpr int kMaxSub = 8;     // sublattices per cell
constexpr int kMaxAniso = 4;   // anisotropy axes per sublattice

// Physical constants, CODATA 2018.
constexpr double kMuB = 5.7883818060e-2;        // Bohr magneton, meV/T
constexpr double kKB = 8.617333262e-2;          // Boltzmann, meV/K
constexpr double kGammaPerFs = 1.76085963023e-4; // electron gyromagnetic ratio, rad/(fs T)

// Directed-bond table grouped by target sublattice: bonds start[a] ..
// start[a+1]-1 act on sublattice a.  geo[p] = (source sublattice, dx, dy, dz).
// J is one scalar per bond when iso != 0, else a row-major 3x3 tensor.
struct BondTable {
    const int4 *geo;
    const float *Jf;   // FP32 copy of the couplings
    const double *Jd;  // FP64 couplings
    int start[kMaxSub + 1];
    int iso;
};

// Lattice extents.  M = Lx*Ly*Lz sites per sublattice, N = n_sub*M.
struct Grid {
    int Lx, Ly, Lz;
    int per[3];
    int n_sub;
    int M;
    int64_t N;
    int wrap_general;  // 1 if some |delta| exceeds an extent (needs a true modulo)
};

// On-site terms, evaluated in FP64 in every precision mode.
struct Onsite {
    int n_aniso;
    double K[kMaxSub][kMaxAniso];
    double axis[kMaxSub][kMaxAniso][3];
    double bz[kMaxSub][3];   // Zeeman reduced field mu_a mu_B B (meV)
};

// Per-call integrator constants.
struct HeunConst {
    double dt;                     // fs
    double pre;                    // -gamma/(1+alpha^2), rad/(fs T)
    double alpha;
    double inv_mumuB[kMaxSub];     // 1/(mu_a mu_B), T/meV
    double sigma[kMaxSub];         // thermal field amplitude, T
    uint64_t seed;
    uint32_t tag;
    int noise;                     // 0: T = 0, no RNG calls
    // optional device step counter (graph replay): the noise step is
    // *step_dev + the kernel's step argument when step_dev is not NULL
    const uint64_t *step_dev;
};

__device__ __forceinline__ uint64_t noise_step(const HeunConst &hc, uint64_t step) {
    return hc.step_dev ? *hc.step_dev + step : step;
}

// ---- kernel launchers (spx_kernels.hip) ------------------------------------
// field_prec: 0 FP64 (b double), 1 FP32 (b float).  bdip may be NULL.
hipError_t launch_field(int field_prec, const BondTable &tb, const Grid &g, const Onsite &os,
                        const double *S, const float *bdip, void *b, hipStream_t st);
hipError_t launch_heun_predict(int field_prec, const BondTable &tb, const Grid &g,
                               const Onsite &os, const HeunConst &hc, uint64_t step,
                               const double *S, const float *bdip, double *St, hipStream_t st);
hipError_t launch_heun_correct(int field_prec, const BondTable &tb, const Grid &g,
                               const Onsite &os, const HeunConst &hc, uint64_t step,
                               const double *S, const double *St, const float *bdip_S,
                               const float *bdip_St, double *out, hipStream_t st);
// Energy partials: partial[block][4] (bil, Z, ani, dip), then a fixed-order
// final reduction into E (1 double) and terms (5 doubles, may be NULL).
int energy_partial_count(const Grid &g);
// Second-level quadruples of the energy reduction, stored after the first level.
constexpr int kEnergyL2 = 1024;
// Doubles of the energy partial buffer (both levels).
size_t energy_partial_doubles(const Grid &g);
// bil: precomputed bilinear field (double for field_prec 0, float otherwise)
// or NULL to gather the neighbours.
// The fixed-order reduction of n partial quadruples (a middle level of at most
// kEnergyL2 blocks when n > 8 kBlock, written after them at partial + 4 n)
// into E and terms.
hipError_t launch_energy_reduce(double *partial, int n, double *E, double *terms, hipStream_t st);
hipError_t launch_energy(int field_prec, const BondTable &tb, const Grid &g, const Onsite &os,
                         const double *S, const float *bdip, const void *bil, double *partial, double *E,
                         double *terms, hipStream_t st);
hipError_t launch_thermal_noise(uint64_t seed, uint64_t step, uint32_t tag, int64_t N, double *eta,
                                hipStream_t st);
// Streaming bandwidth probe over n16 16-byte words (kind 0 copy, 1 read, 2 write).
hipError_t launch_stream(int kind, const void *src, void *dst, int64_t n16, hipStream_t st);
hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, int64_t n, uint32_t *out,
                         hipStream_t st);

}  // namespace spx
