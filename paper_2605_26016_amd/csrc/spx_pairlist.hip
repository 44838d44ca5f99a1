// spx_pairlist.hip -- pair-list Hamiltonian (Methods, pair-list backend):
// explicit couplings for lattices without translational symmetry (chemical
// disorder, defects, site-resolved couplings).  Entry p couples target site
// i_p to source site j_p with J_p (scalar or 3x3); the reduced bilinear field
// is b_i = sum_{p: i_p = i} J_p S_{j_p}, plus site-resolved Zeeman
// mu_i mu_B B and uniaxial anisotropy 2 K_i (S_i.n_i) n_i.
//
// Layout: the entries are sorted by target site into CSR rows (stable: a
// site's entries keep their list order, which is the summation order), with
// the sources (32-bit) and couplings in row order; per-site moments and
// anisotropies are plain arrays.  One thread per target site gathers its row.  FP32 mode
// rounds every neighbour spin and coupling to float and accumulates in FP32,
// with the on-site terms added in FP64 before the result is rounded.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "spx_device.hpp"
#include "spx_ext.hpp"

namespace spx {

struct PairList {
    int64_t N = 0, P = 0;
    int tensor = 0, prec = 0;
    bool has_K = false;
    double B[3] = {0, 0, 0};
    int64_t *row = nullptr;  // [N + 1]
    int32_t *col = nullptr;  // [P] sources in row order (sites < 2^31)
    double *Jd = nullptr;    // [P] or [P][9]
    float *Jf = nullptr;
    double *mu = nullptr;    // [N]
    double *K = nullptr;     // [N]
    double *axis = nullptr;  // [N][3]
    double *St = nullptr, *f0 = nullptr;  // Heun predictor state and first stage
    double *part = nullptr;  // energy partials [kPlBlocks][3]
    std::vector<void *> owned;
};

namespace {

constexpr int kPlB = 256;
constexpr int kPlBlocks = 1024;

struct PlView {
    int64_t N;
    const int64_t *row;
    const int32_t *col;
    const double *Jd;
    const float *Jf;
    const double *mu, *K, *axis;
    double B[3];
    int has_K;
};

PlView view(const PairList *p) {
    PlView v;
    v.N = p->N;
    v.row = p->row;
    v.col = p->col;
    v.Jd = p->Jd;
    v.Jf = p->Jf;
    v.mu = p->mu;
    v.K = p->K;
    v.axis = p->axis;
    for (int c = 0; c < 3; ++c) v.B[c] = p->B[c];
    v.has_K = p->has_K ? 1 : 0;
    return v;
}

// Workgroups are dealt to the 8 XCDs in turn; this renumbering gives each
// XCD one contiguous range of the grid's blocks, so that the sites a block
// gathers from the rows next to its own were mostly fetched into the same L2
// by the blocks beside it.
__device__ __forceinline__ int64_t xcd_site_block() {
    const int64_t T = gridDim.x, b = blockIdx.x;
    const int64_t q = T / 8, r = T % 8, k = b % 8;
    return k * q + (k < r ? k : r) + b / 8;
}

// bilinear field of site i (AccT precision), result in FP64
template <typename AccT, bool TENSOR>
__device__ __forceinline__ void pl_bil(const PlView &v, const double *__restrict__ S, int64_t i, double out[3]) {
    const int64_t N = v.N;
    AccT acc[3] = {AccT(0), AccT(0), AccT(0)};
    const int64_t p0 = v.row[i], p1 = v.row[i + 1];
    // unrolled so that several entries' index loads, and then their spin
    // loads, are in flight together instead of one dependent pair per entry;
    // six deep (timed on sc 200^3 nearest-neighbour rows of six: FP32 field
    // 220 -> 208 us and FP64 294 -> 248 us against four deep; eight deep
    // was slower than four), other row lengths finish in the remainder loop
#pragma unroll 6
    for (int64_t p = p0; p < p1; ++p) {
        const int64_t j = v.col[p];
        const AccT s0 = (AccT)S[j], s1 = (AccT)S[N + j], s2 = (AccT)S[2 * N + j];
        if constexpr (TENSOR) {
            AccT J[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                if constexpr (sizeof(AccT) == 4) J[e] = v.Jf[9 * p + e]; else J[e] = v.Jd[9 * p + e];
            }
            acc[0] += J[0] * s0 + J[1] * s1 + J[2] * s2;
            acc[1] += J[3] * s0 + J[4] * s1 + J[5] * s2;
            acc[2] += J[6] * s0 + J[7] * s1 + J[8] * s2;
        } else {
            AccT J;
            if constexpr (sizeof(AccT) == 4) J = v.Jf[p]; else J = v.Jd[p];
            acc[0] += J * s0;
            acc[1] += J * s1;
            acc[2] += J * s2;
        }
    }
    for (int c = 0; c < 3; ++c) out[c] = (double)acc[c];
}

// on-site field of site i at spin s: Zeeman + anisotropy (FP64)
__device__ __forceinline__ void pl_onsite(const PlView &v, int64_t i, const double s[3], double out[3]) {
    const double m = v.mu[i] * kMuB;
    for (int c = 0; c < 3; ++c) out[c] = m * v.B[c];
    if (v.has_K) {
        const double *n = v.axis + 3 * i;
        const double c2 = 2.0 * v.K[i] * (s[0] * n[0] + s[1] * n[1] + s[2] * n[2]);
        for (int c = 0; c < 3; ++c) out[c] += c2 * n[c];
    }
}

template <typename AccT, typename OutT, bool TENSOR>
__global__ __launch_bounds__(kPlB) void k_pl_field(PlView v, const double *__restrict__ S, OutT *__restrict__ b) {
    const int64_t N = v.N;
    for (int64_t i = xcd_site_block() * kPlB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kPlB) {
        double bl[3], on[3];
        pl_bil<AccT, TENSOR>(v, S, i, bl);
        double s[3] = {0.0, 0.0, 0.0};  // the site's own spin: read only for the anisotropy
        if (v.has_K)
            for (int c = 0; c < 3; ++c) s[c] = S[c * N + i];
        pl_onsite(v, i, s, on);
        for (int c = 0; c < 3; ++c) b[c * N + i] = (OutT)(bl[c] + on[c]);
    }
}

struct PlHeun {
    double dt, alpha, pre, sig0;  // sig0 = sqrt(2 alpha k_B T / (gamma mu_B dt)); sigma_i = sig0 / sqrt(mu_i)
    uint64_t seed, step;
    uint32_t tag;
    int noise;
};

// stage 0: S~ = N[S + dt f(S)], keeps f(S); stage 1: S <- N[S + dt/2 (f0 + f(S~))]
template <typename AccT, bool TENSOR, int STAGE>
__global__ __launch_bounds__(kPlB) void k_pl_heun(PlView v, PlHeun hc, double *__restrict__ S,
                                                  double *__restrict__ St, double *__restrict__ f0) {
    const int64_t N = v.N;
    for (int64_t i = xcd_site_block() * kPlB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kPlB) {
        const double *X = STAGE == 0 ? S : St;
        double x[3] = {X[i], X[N + i], X[2 * N + i]};
        double bl[3], on[3], B[3];
        pl_bil<AccT, TENSOR>(v, X, i, bl);
        pl_onsite(v, i, x, on);
        const double inv = 1.0 / (v.mu[i] * kMuB);
        for (int c = 0; c < 3; ++c) B[c] = (bl[c] + on[c]) * inv;
        if (hc.noise) {
            double eta[3];
            thermal_eta(hc.seed, hc.step, hc.tag, (uint64_t)i, eta);
            const double sig = hc.sig0 / sqrt(v.mu[i]);
            for (int c = 0; c < 3; ++c) B[c] += sig * eta[c];
        }
        double f[3];
        llg_rhs(x, B, hc.pre, hc.alpha, f);
        double p[3];
        if (STAGE == 0) {
            for (int c = 0; c < 3; ++c) {
                f0[c * N + i] = f[c];
                p[c] = S[c * N + i] + hc.dt * f[c];
            }
            normalise3(p);
            for (int c = 0; c < 3; ++c) St[c * N + i] = p[c];
        } else {
            for (int c = 0; c < 3; ++c) p[c] = S[c * N + i] + 0.5 * hc.dt * (f0[c * N + i] + f[c]);
            normalise3(p);
            for (int c = 0; c < 3; ++c) S[c * N + i] = p[c];
        }
    }
}

template <typename AccT, bool TENSOR>
__global__ __launch_bounds__(kPlB) void k_pl_energy(PlView v, const double *__restrict__ S, double *__restrict__ part) {
    __shared__ double red[3][kPlB / 64];
    const int64_t N = v.N;
    double e[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kPlB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kPlB) {
        const double s[3] = {S[i], S[N + i], S[2 * N + i]};
        double bl[3];
        pl_bil<AccT, TENSOR>(v, S, i, bl);
        e[0] += -0.5 * (s[0] * bl[0] + s[1] * bl[1] + s[2] * bl[2]);
        const double m = v.mu[i] * kMuB;
        e[1] += -m * (s[0] * v.B[0] + s[1] * v.B[1] + s[2] * v.B[2]);
        if (v.has_K) {
            const double *n = v.axis + 3 * i;
            const double sn = s[0] * n[0] + s[1] * n[1] + s[2] * n[2];
            e[2] += -v.K[i] * sn * sn;
        }
    }
    for (int q = 0; q < 3; ++q) {
        const double w = wave_sum(e[q]);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int k = 0; k < kPlB / 64; ++k) t += red[threadIdx.x][k];
        part[blockIdx.x * 3 + threadIdx.x] = t;
    }
}

__global__ __launch_bounds__(kPlB) void k_pl_energy_final(const double *__restrict__ part, int nb, double *E,
                                                          double *terms) {
    __shared__ double red[3][kPlB / 64];
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < nb; k += kPlB)
        for (int q = 0; q < 3; ++q) v[q] += part[k * 3 + q];
    for (int q = 0; q < 3; ++q) {
        const double w = wave_sum(v[q]);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[3];
        for (int q = 0; q < 3; ++q) {
            t[q] = 0.0;
            for (int k = 0; k < kPlB / 64; ++k) t[q] += red[q][k];
        }
        const double tot = t[0] + t[1] + t[2];
        if (E) *E = tot;
        if (terms) {
            terms[0] = t[0];
            terms[1] = t[1];
            terms[2] = t[2];
            terms[3] = 0.0;
            terms[4] = tot;
        }
    }
}

unsigned blocks_for(int64_t N) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + kPlB - 1) / kPlB, kPlBlocks));
}

}  // namespace

void pl_destroy(PairList *p) {
    if (!p) return;
    for (void *q : p->owned) (void)hipFree(q);
    delete p;
}

spx_status pl_create(const spx_pairlist_desc *d, int prec, hipStream_t st, PairList **out) {
    *out = nullptr;
    if (d->n_sites < 1 || d->n_pairs < 0) return set_error(SPX_ERR_INVALID_ARG, "n_sites must be >= 1, n_pairs >= 0");
    if (d->n_sites > (int64_t)INT32_MAX) return set_error(SPX_ERR_INVALID_ARG, "more than 2^31-1 sites");
    if (d->n_pairs > 0 && (!d->target || !d->source || !d->J))
        return set_error(SPX_ERR_INVALID_ARG, "target, source or J is NULL");
    if (d->K && !d->K_axis) return set_error(SPX_ERR_INVALID_ARG, "K given without K_axis");
    const int64_t N = d->n_sites, P = d->n_pairs;
    const int tensor = d->tensor ? 1 : 0;
    std::vector<int64_t> row(N + 1, 0);
    for (int64_t p = 0; p < P; ++p) {
        if (d->target[p] < 0 || d->target[p] >= N || d->source[p] < 0 || d->source[p] >= N)
            return set_error(SPX_ERR_INVALID_ARG, "pair " + std::to_string(p) + " names a site out of range");
        ++row[d->target[p] + 1];
    }
    for (int64_t i = 0; i < N; ++i) row[i + 1] += row[i];
    std::vector<int32_t> col(std::max<int64_t>(P, 1));
    std::vector<int64_t> fill(row.begin(), row.end() - 1);
    const int nj = tensor ? 9 : 1;
    std::vector<double> Jd(std::max<int64_t>(P * nj, 1));
    std::vector<float> Jf(Jd.size());
    for (int64_t p = 0; p < P; ++p) {
        const int64_t q = fill[d->target[p]]++;
        col[q] = (int32_t)d->source[p];
        for (int e = 0; e < nj; ++e) {
            Jd[q * nj + e] = d->J[p * nj + e];
            Jf[q * nj + e] = (float)d->J[p * nj + e];
        }
    }
    std::vector<double> mu(N, 1.0), K, axis;
    for (int64_t i = 0; i < N; ++i) {
        if (d->mu) mu[i] = d->mu[i];
        if (!(mu[i] > 0.0)) return set_error(SPX_ERR_INVALID_ARG, "moments mu must be positive");
    }
    if (d->K) {
        K.assign(d->K, d->K + N);
        axis.assign(d->K_axis, d->K_axis + 3 * N);
    }
    PairList *pl = new PairList();
    pl->N = N;
    pl->P = P;
    pl->tensor = tensor;
    pl->prec = prec;
    pl->has_K = d->K != nullptr;
    for (int c = 0; c < 3; ++c) pl->B[c] = d->B_ext[c];
    auto alloc = [&](void **ptr, size_t bytes) -> bool {
        if (hipMalloc(ptr, std::max<size_t>(bytes, 8)) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        pl->owned.push_back(*ptr);
        return true;
    };
    bool ok = alloc((void **)&pl->row, sizeof(int64_t) * (N + 1)) && alloc((void **)&pl->col, sizeof(int32_t) * col.size()) &&
              alloc((void **)&pl->Jd, sizeof(double) * Jd.size()) && alloc((void **)&pl->Jf, sizeof(float) * Jf.size()) &&
              alloc((void **)&pl->mu, sizeof(double) * N) && alloc((void **)&pl->St, sizeof(double) * 3 * N) &&
              alloc((void **)&pl->f0, sizeof(double) * 3 * N) && alloc((void **)&pl->part, sizeof(double) * 3 * kPlBlocks);
    if (ok && pl->has_K) ok = alloc((void **)&pl->K, sizeof(double) * N) && alloc((void **)&pl->axis, sizeof(double) * 3 * N);
    if (!ok) {
        pl_destroy(pl);
        return set_error(SPX_ERR_OUT_OF_MEMORY, "hipMalloc failed for the pair list");
    }
    hipError_t e = hipMemcpyAsync(pl->row, row.data(), sizeof(int64_t) * (N + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pl->col, col.data(), sizeof(int32_t) * col.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pl->Jd, Jd.data(), sizeof(double) * Jd.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pl->Jf, Jf.data(), sizeof(float) * Jf.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pl->mu, mu.data(), sizeof(double) * N, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && pl->has_K) {
        e = hipMemcpyAsync(pl->K, K.data(), sizeof(double) * N, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(pl->axis, axis.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        pl_destroy(pl);
        return set_hip_error(e, "spx_setup_pairlist: upload");
    }
    *out = pl;
    return SPX_OK;
}

hipError_t pl_field(const PairList *p, const double *S, void *b, hipStream_t st) {
    const PlView v = view(p);
    const unsigned g = blocks_for(p->N);
    if (p->prec == SPX_FP32) {
        if (p->tensor) k_pl_field<float, float, true><<<g, kPlB, 0, st>>>(v, S, (float *)b);
        else k_pl_field<float, float, false><<<g, kPlB, 0, st>>>(v, S, (float *)b);
    } else {
        if (p->tensor) k_pl_field<double, double, true><<<g, kPlB, 0, st>>>(v, S, (double *)b);
        else k_pl_field<double, double, false><<<g, kPlB, 0, st>>>(v, S, (double *)b);
    }
    return hipGetLastError();
}

hipError_t pl_energy(const PairList *p, const double *S, double *E, double *terms, hipStream_t st) {
    const PlView v = view(p);
    const unsigned g = blocks_for(p->N);
    if (p->prec == SPX_FP32) {
        if (p->tensor) k_pl_energy<float, true><<<g, kPlB, 0, st>>>(v, S, p->part);
        else k_pl_energy<float, false><<<g, kPlB, 0, st>>>(v, S, p->part);
    } else {
        if (p->tensor) k_pl_energy<double, true><<<g, kPlB, 0, st>>>(v, S, p->part);
        else k_pl_energy<double, false><<<g, kPlB, 0, st>>>(v, S, p->part);
    }
    k_pl_energy_final<<<1, kPlB, 0, st>>>(p->part, (int)g, E, terms);
    return hipGetLastError();
}

hipError_t pl_heun(PairList *p, double *S, double alpha, double dt, double pre, double sig0, uint64_t seed,
                   uint64_t step0, uint32_t tag, int noise, int n_steps, hipStream_t st) {
    const PlView v = view(p);
    const unsigned g = blocks_for(p->N);
    for (int k = 0; k < n_steps; ++k) {
        const PlHeun hc{dt, alpha, pre, sig0, seed, step0 + (uint64_t)k, tag, noise};
#define SPX_PL_STAGE(ACC, TEN)                                                              \
    k_pl_heun<ACC, TEN, 0><<<g, kPlB, 0, st>>>(v, hc, S, p->St, p->f0);                     \
    k_pl_heun<ACC, TEN, 1><<<g, kPlB, 0, st>>>(v, hc, S, p->St, p->f0);
        if (p->prec == SPX_FP32) {
            if (p->tensor) { SPX_PL_STAGE(float, true) } else { SPX_PL_STAGE(float, false) }
        } else {
            if (p->tensor) { SPX_PL_STAGE(double, true) } else { SPX_PL_STAGE(double, false) }
        }
#undef SPX_PL_STAGE
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace spx
