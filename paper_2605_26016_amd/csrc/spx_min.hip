// spx_min.hip -- static minimisers on the product of unit spheres (Methods,
// static optimisation): velocity projection, Barzilai-Borwein, L-BFGS and
// Adam, each with the exponential-map or the normalised retraction.
//
// One iteration (every scalar lives on the device, so a call needs no host
// synchronisation):
//   field    b = total effective field of S (the Hamiltonian's FP64 field)
//   force    F = b - (b.S) S per spin; block partials of max |F|, v.F, F.F and,
//            with s = P(u_prev), y = P(F_prev) - F (P: projection on the
//            current tangent planes), s.s, s.y, y.y; L-BFGS writes (s, y) into
//            the candidate slot of its history ring
//   scalars  VP projection v.F/F.F, BB step s.s/s.y, L-BFGS: keep the pair if
//            s.y > 0 (rho = 1/s.y), ring bookkeeping
//   L-BFGS   two-loop recursion, newest to oldest then back, one fused pass
//            (axpy of the previous step + dot of the next) per stored pair;
//            the pairs are projected on the current tangent planes on the fly
//   update   step u (per method), tangent projection, length cap, retraction;
//            keeps u and F for the next iteration
//   finish   iteration count, convergence flag (max |F| < tol_force)
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "spx_device.hpp"
#include "spx_ext.hpp"

namespace spx {
namespace {

constexpr int kMinB = 256;
constexpr int kMinBlocks = 1024;
constexpr int kMaxHist = 32;
constexpr int kNP = 6;  // partials per block: max|F|, v.F, F.F, s.s, s.y, y.y

// device scalars
enum { MS_ITER = 0, MS_NP, MS_NEWEST, MS_DONE, MS_MAXF, MS_PROJ, MS_ALPHA, MS_GAMMA, MS_CAND, MS_RED, MS_N = 16 };

struct MinArgs {
    int64_t N;
    int method, retraction, hist;
    double dt, mass, b1, b2, eps, max_step, tol;
    double *F, *V, *W, *Fp, *Up, *Sh, *Yh, *q;
    double *part;    // [kMinBlocks][kNP]
    double *st;      // [MS_N]
    double *rho;     // [hist + 1]
    double *al;      // [hist]
    int nb;          // blocks of the elementwise passes
    int npart;       // partial sets the scalar pass reduces (nb, or the z-march tiles of the fused force pass)
};

__device__ __forceinline__ double blk_sum(double v, double *red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kMinB / 64; ++k) t += red[k];
    return t;
}

__device__ __forceinline__ double blk_max(double v, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kMinB / 64; ++k) t = fmax(t, red[k]);
    return t;
}

__device__ __forceinline__ void ld3(const double *p, int64_t N, int64_t i, double v[3]) {
    v[0] = p[i];
    v[1] = p[N + i];
    v[2] = p[2 * N + i];
}

__device__ __forceinline__ void proj3(const double s[3], double v[3]) {
    const double d = v[0] * s[0] + v[1] * s[1] + v[2] * s[2];
    for (int c = 0; c < 3; ++c) v[c] -= d * s[c];
}

// history slot of the t-th newest pair (ring of hist + 1 slots)
__device__ __forceinline__ int slot_of(const MinArgs &a, int t) {
    const int R = a.hist + 1;
    return (((int)a.st[MS_NEWEST] - t) % R + R) % R;
}

// ------------------------------------------------------------------ force
__global__ __launch_bounds__(kMinB) void k_min_force(MinArgs a, const double *__restrict__ S,
                                                     const double *__restrict__ b) {
    __shared__ double red[kMinB / 64];
    if (a.st[MS_DONE] != 0.0) return;
    const int64_t N = a.N;
    const bool pair = a.method == 1 || a.method == 2;
    const int cand = (int)a.st[MS_CAND];
    double mf = 0.0, vf = 0.0, ff = 0.0, ss = 0.0, sy = 0.0, yy = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kMinB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kMinB) {
        double s[3], bb[3], f[3];
        ld3(S, N, i, s);
        ld3(b, N, i, bb);
        const double bs = bb[0] * s[0] + bb[1] * s[1] + bb[2] * s[2];
        double f2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            f[c] = bb[c] - bs * s[c];
            f2 += f[c] * f[c];
            a.F[c * N + i] = f[c];
        }
        mf = fmax(mf, sqrt(f2));
        ff += f2;
        if (a.method == 0) {
            double v[3];
            ld3(a.V, N, i, v);
            vf += v[0] * f[0] + v[1] * f[1] + v[2] * f[2];
        } else if (pair) {
            double sv[3], yv[3];
            ld3(a.Up, N, i, sv);
            ld3(a.Fp, N, i, yv);
            proj3(s, sv);
            proj3(s, yv);
            for (int c = 0; c < 3; ++c) yv[c] -= f[c];
            ss += sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2];
            sy += sv[0] * yv[0] + sv[1] * yv[1] + sv[2] * yv[2];
            yy += yv[0] * yv[0] + yv[1] * yv[1] + yv[2] * yv[2];
            if (a.method == 2) {
                double *Sj = a.Sh + (int64_t)cand * 3 * N, *Yj = a.Yh + (int64_t)cand * 3 * N;
                for (int c = 0; c < 3; ++c) {
                    Sj[c * N + i] = sv[c];
                    Yj[c * N + i] = yv[c];
                }
            }
        }
    }
    const double r0 = blk_max(mf, red);
    const double r1 = blk_sum(vf, red);
    const double r2 = blk_sum(ff, red);
    const double r3 = blk_sum(ss, red);
    const double r4 = blk_sum(sy, red);
    const double r5 = blk_sum(yy, red);
    if (threadIdx.x == 0) {
        double *p = a.part + (size_t)blockIdx.x * kNP;
        p[0] = r0; p[1] = r1; p[2] = r2; p[3] = r3; p[4] = r4; p[5] = r5;
    }
}

// ---------------------------------------------------------------- scalars
__global__ __launch_bounds__(kMinB) void k_min_scalars(MinArgs a) {
    __shared__ double red[kMinB / 64];
    if (a.st[MS_DONE] != 0.0) return;
    double v[kNP];
    for (int k = 0; k < kNP; ++k) v[k] = 0.0;
    for (int bl = threadIdx.x; bl < a.npart; bl += kMinB) {
        const double *p = a.part + (size_t)bl * kNP;
        v[0] = fmax(v[0], p[0]);
        for (int k = 1; k < kNP; ++k) v[k] += p[k];
    }
    const double mf = blk_max(v[0], red);
    const double vf = blk_sum(v[1], red);
    const double ff = blk_sum(v[2], red);
    const double ss = blk_sum(v[3], red);
    const double sy = blk_sum(v[4], red);
    const double yy = blk_sum(v[5], red);
    if (threadIdx.x != 0) return;
    double *st = a.st;
    const double k = st[MS_ITER];
    st[MS_MAXF] = mf;
    st[MS_PROJ] = (vf > 0.0 && ff > 0.0) ? vf / ff : 0.0;
    st[MS_ALPHA] = (k > 0.0 && sy > 0.0) ? ss / sy : a.dt;
    if (a.method == 2 && k > 0.0 && sy > 0.0) {
        const int cand = (int)st[MS_CAND];
        a.rho[cand] = 1.0 / sy;
        st[MS_NEWEST] = (double)cand;
        st[MS_NP] = fmin(st[MS_NP] + 1.0, (double)a.hist);
        (void)yy;
    }
}

// ------------------------------------------------------- L-BFGS two-loop
// First loop, step t (0 = newest): q <- q - al[t-1] P(y_{t-1}) (t > 0), then
// the partial of P(s_t).q; t == 0 starts from q = -F and also takes the
// partials of P(s_0).P(y_0) and P(y_0).P(y_0) for the initial scale.
__global__ __launch_bounds__(kMinB) void k_lb_loop1(MinArgs a, const double *__restrict__ S, int t) {
    __shared__ double red[kMinB / 64];
    if (a.st[MS_DONE] != 0.0 || a.st[MS_NP] == 0.0) return;
    const int np = (int)a.st[MS_NP];
    if (t > np) return;
    const int64_t N = a.N;
    const int jp = t > 0 ? slot_of(a, t - 1) : 0;
    const int j = t < np ? slot_of(a, t) : 0;
    const double alp = t > 0 ? a.al[t - 1] : 0.0;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kMinB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kMinB) {
        double s[3], qv[3];
        ld3(S, N, i, s);
        if (t == 0) {
            for (int c = 0; c < 3; ++c) qv[c] = -a.F[c * N + i];
        } else {
            double yv[3];
            ld3(a.q, N, i, qv);
            ld3(a.Yh + (int64_t)jp * 3 * N, N, i, yv);
            proj3(s, yv);
            for (int c = 0; c < 3; ++c) qv[c] -= alp * yv[c];
        }
        for (int c = 0; c < 3; ++c) a.q[c * N + i] = qv[c];
        if (t < np) {
            double sv[3];
            ld3(a.Sh + (int64_t)j * 3 * N, N, i, sv);
            proj3(s, sv);
            d0 += sv[0] * qv[0] + sv[1] * qv[1] + sv[2] * qv[2];
            if (t == 0) {
                double yv[3];
                ld3(a.Yh + (int64_t)j * 3 * N, N, i, yv);
                proj3(s, yv);
                d1 += sv[0] * yv[0] + sv[1] * yv[1] + sv[2] * yv[2];
                d2 += yv[0] * yv[0] + yv[1] * yv[1] + yv[2] * yv[2];
            }
        }
    }
    const double r0 = blk_sum(d0, red);
    const double r1 = blk_sum(d1, red);
    const double r2 = blk_sum(d2, red);
    if (threadIdx.x == 0) {
        double *p = a.part + (size_t)blockIdx.x * kNP;
        p[0] = r0; p[1] = r1; p[2] = r2;
    }
}

// reduce the partials of loop step t: al[t] = rho_t (s.q); at t == 0 also
// gamma = (s.y)/(y.y) of the newest pair
__global__ __launch_bounds__(kMinB) void k_lb_alpha(MinArgs a, int t) {
    __shared__ double red[kMinB / 64];
    if (a.st[MS_DONE] != 0.0 || a.st[MS_NP] == 0.0) return;
    const int np = (int)a.st[MS_NP];
    if (t >= np) return;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    for (int bl = threadIdx.x; bl < a.nb; bl += kMinB) {
        const double *p = a.part + (size_t)bl * kNP;
        v0 += p[0];
        v1 += p[1];
        v2 += p[2];
    }
    const double r0 = blk_sum(v0, red);
    const double r1 = blk_sum(v1, red);
    const double r2 = blk_sum(v2, red);
    if (threadIdx.x == 0) {
        a.al[t] = a.rho[slot_of(a, t)] * r0;
        if (t == 0) a.st[MS_GAMMA] = r1 / r2;
    }
}

// Second loop, step t from np-1 (oldest) down to 0: r <- r + (al[t+1] - be)
// P(s_{t+1}) for the previous step (t + 1 < np; r = gamma q first), then the
// partial of P(y_t).r.  Called with t = np_max - 1 .. -1; t == -1 applies the
// last update only.
__global__ __launch_bounds__(kMinB) void k_lb_loop2(MinArgs a, const double *__restrict__ S, int t) {
    __shared__ double red[kMinB / 64];
    if (a.st[MS_DONE] != 0.0 || a.st[MS_NP] == 0.0) return;
    const int np = (int)a.st[MS_NP];
    if (t >= np) return;
    const int64_t N = a.N;
    const bool first = t == np - 1;
    const int jp = first ? 0 : slot_of(a, t + 1);
    const double coef = first ? 0.0 : a.al[t + 1] - a.st[MS_RED];
    const double gamma = a.st[MS_GAMMA];
    const int j = t >= 0 ? slot_of(a, t) : 0;
    double d0 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kMinB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kMinB) {
        double s[3], r[3];
        ld3(S, N, i, s);
        ld3(a.q, N, i, r);
        if (first) {
            for (int c = 0; c < 3; ++c) r[c] *= gamma;
        } else {
            double sv[3];
            ld3(a.Sh + (int64_t)jp * 3 * N, N, i, sv);
            proj3(s, sv);
            for (int c = 0; c < 3; ++c) r[c] += coef * sv[c];
        }
        for (int c = 0; c < 3; ++c) a.q[c * N + i] = r[c];
        if (t >= 0) {
            double yv[3];
            ld3(a.Yh + (int64_t)j * 3 * N, N, i, yv);
            proj3(s, yv);
            d0 += yv[0] * r[0] + yv[1] * r[1] + yv[2] * r[2];
        }
    }
    const double r0 = blk_sum(d0, red);
    if (threadIdx.x == 0) a.part[(size_t)blockIdx.x * kNP] = r0;
}

// be = rho_t (y_t . r) into MS_RED
__global__ __launch_bounds__(kMinB) void k_lb_beta(MinArgs a, int t) {
    __shared__ double red[kMinB / 64];
    if (a.st[MS_DONE] != 0.0 || a.st[MS_NP] == 0.0) return;
    const int np = (int)a.st[MS_NP];
    if (t < 0 || t >= np) return;
    double v0 = 0.0;
    for (int bl = threadIdx.x; bl < a.nb; bl += kMinB) v0 += a.part[(size_t)bl * kNP];
    const double r0 = blk_sum(v0, red);
    if (threadIdx.x == 0) a.st[MS_RED] = a.rho[slot_of(a, t)] * r0;
}

// ----------------------------------------------------------------- update
__global__ __launch_bounds__(kMinB) void k_min_update(MinArgs a, double *__restrict__ S) {
    if (a.st[MS_DONE] != 0.0) return;
    const int64_t N = a.N;
    const double proj = a.st[MS_PROJ], alpha = a.st[MS_ALPHA];
    const bool have_pairs = a.st[MS_NP] != 0.0;
    const double t = a.st[MS_ITER] + 1.0;
    const double c1 = 1.0 - pow(a.b1, t), c2 = 1.0 - pow(a.b2, t);
    for (int64_t i = (int64_t)blockIdx.x * kMinB + threadIdx.x; i < N; i += (int64_t)gridDim.x * kMinB) {
        double s[3], f[3], u[3];
        ld3(S, N, i, s);
        ld3(a.F, N, i, f);
        if (a.method == 0) {
            for (int c = 0; c < 3; ++c) {
                const double v = proj * f[c] + (a.dt / a.mass) * f[c];
                a.V[c * N + i] = v;
                u[c] = a.dt * v;
            }
        } else if (a.method == 1) {
            for (int c = 0; c < 3; ++c) u[c] = alpha * f[c];
        } else if (a.method == 2) {
            if (have_pairs)
                for (int c = 0; c < 3; ++c) u[c] = -a.q[c * N + i];
            else
                for (int c = 0; c < 3; ++c) u[c] = a.dt * f[c];
        } else {
            for (int c = 0; c < 3; ++c) {
                const double g = -f[c];
                const double m = a.b1 * a.V[c * N + i] + (1.0 - a.b1) * g;
                const double w = a.b2 * a.W[c * N + i] + (1.0 - a.b2) * g * g;
                a.V[c * N + i] = m;
                a.W[c * N + i] = w;
                u[c] = -a.dt * (m / c1) / (sqrt(w / c2) + a.eps);
            }
        }
        proj3(s, u);
        double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        if (a.max_step > 0.0 && un > a.max_step) {
            for (int c = 0; c < 3; ++c) u[c] *= a.max_step / un;
            un = a.max_step;
        }
        double o[3];
        if (a.retraction == 0) {
            if (un == 0.0) {
                for (int c = 0; c < 3; ++c) o[c] = s[c];
            } else {
                const double cs = cos(un), sn = sin(un) / un;
                for (int c = 0; c < 3; ++c) o[c] = cs * s[c] + sn * u[c];
                normalise3(o);
            }
        } else {
            for (int c = 0; c < 3; ++c) o[c] = s[c] + u[c];
            normalise3(o);
        }
        for (int c = 0; c < 3; ++c) {
            S[c * N + i] = o[c];
            a.Up[c * N + i] = u[c];
            a.Fp[c * N + i] = f[c];
        }
    }
}

__global__ void k_min_finish(MinArgs a) {
    double *st = a.st;
    if (st[MS_DONE] != 0.0) return;
    st[MS_ITER] += 1.0;
    // candidate slot of the next pair: after the newest (ring of hist + 1)
    st[MS_CAND] = st[MS_NP] == 0.0 ? 0.0 : (double)(((int)st[MS_NEWEST] + 1) % (a.hist + 1));
    if (a.tol > 0.0 && st[MS_MAXF] < a.tol) st[MS_DONE] = 1.0;
}

__global__ void k_min_zero(double *p, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = 0.0;
}

}  // namespace
}  // namespace spx

using namespace spx;

struct spx_min {
    spx_ham *h = nullptr;
    MinArgs a{};
    double *b = nullptr;
    std::vector<void *> owned;
    // the force pass runs inside the FP64 z-march field evaluation when the
    // Hamiltonian has a z-march shape and no dipolar term
    bool fused = false;
    ZPlan zp;
    Grid g{};
    Onsite os{};
    int ntile = 0;
};

namespace {

void min_free(spx_min *m) {
    for (void *p : m->owned) (void)hipFree(p);
    m->owned.clear();
}

hipError_t min_zero_state(spx_min *m, hipStream_t st) {
    const MinArgs &a = m->a;
    const int64_t n3 = 3 * a.N;
    double *blocks[] = {a.V, a.W, a.Fp, a.Up, a.q};
    for (double *p : blocks) k_min_zero<<<1024, 256, 0, st>>>(p, n3);
    k_min_zero<<<1024, 256, 0, st>>>(a.Sh, n3 * (a.hist + 1));
    k_min_zero<<<1024, 256, 0, st>>>(a.Yh, n3 * (a.hist + 1));
    k_min_zero<<<1, 64, 0, st>>>(a.st, MS_N);
    k_min_zero<<<1, 64, 0, st>>>(a.rho, a.hist + 1);
    k_min_zero<<<1, 64, 0, st>>>(a.al, a.hist);
    return hipGetLastError();
}

}  // namespace

extern "C" {

spx_status spx_min_create(spx_ham *h, const spx_min_params *p, void *stream, spx_min **out) {
    if (!out) return set_error(SPX_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    HamView v;
    spx_status s = get_ham_view(h, v);
    if (s != SPX_OK) return s;
    if (!p) return set_error(SPX_ERR_INVALID_ARG, "params is NULL");
    if (v.field_prec != SPX_FP64) return set_error(SPX_ERR_INVALID_ARG, "minimisers need field_prec SPX_FP64");
    if (p->method < 0 || p->method > 3) return set_error(SPX_ERR_INVALID_ARG, "method must be 0 .. 3");
    if (p->retraction != 0 && p->retraction != 1) return set_error(SPX_ERR_INVALID_ARG, "retraction must be 0 or 1");
    if (!(p->dt > 0.0) || (p->method == 0 && !(p->mass > 0.0)))
        return set_error(SPX_ERR_INVALID_ARG, "dt (and, for velocity projection, mass) must be > 0");
    if (p->method == 2 && (p->history < 1 || p->history > kMaxHist))
        return set_error(SPX_ERR_INVALID_ARG, "L-BFGS history must be 1 .. 32");
    if (!(p->max_step >= 0.0) || !(p->tol_force >= 0.0))
        return set_error(SPX_ERR_INVALID_ARG, "max_step and tol_force must be >= 0");
    spx_min *m = new spx_min();
    m->h = h;
    MinArgs &a = m->a;
    a.N = v.grid.N;
    a.method = p->method;
    a.retraction = p->retraction;
    a.hist = p->method == 2 ? p->history : 1;
    a.dt = p->dt;
    a.mass = p->mass;
    a.b1 = p->beta1;
    a.b2 = p->beta2;
    a.eps = p->eps;
    a.max_step = p->max_step;
    a.tol = p->tol_force;
    a.nb = (int)std::max<int64_t>(1, std::min<int64_t>((a.N + kMinB - 1) / kMinB, kMinBlocks));
    a.npart = a.nb;
    if (v.zp64 && !v.dip && !v.pl) {
        m->fused = true;
        m->zp = *v.zp64;
        m->zp.zch = 16;
        m->g = v.grid;
        m->os = v.onsite;
        m->ntile = zmarch_tiles(m->zp, v.grid);
    }
    const size_t n3 = (size_t)3 * a.N;
    auto alloc = [&](double **ptr, size_t count) -> bool {
        if (hipMalloc((void **)ptr, sizeof(double) * std::max<size_t>(count, 1)) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        m->owned.push_back(*ptr);
        return true;
    };
    bool ok = alloc(&m->b, n3) && alloc(&a.F, n3) && alloc(&a.V, n3) && alloc(&a.W, n3) && alloc(&a.Fp, n3) &&
              alloc(&a.Up, n3) && alloc(&a.q, n3) && alloc(&a.Sh, n3 * (a.hist + 1)) &&
              alloc(&a.Yh, n3 * (a.hist + 1)) && alloc(&a.part, (size_t)std::max(kMinBlocks, m->ntile) * kNP) && alloc(&a.st, MS_N) &&
              alloc(&a.rho, a.hist + 1) && alloc(&a.al, a.hist);
    if (!ok) {
        min_free(m);
        delete m;
        return set_error(SPX_ERR_OUT_OF_MEMORY, "hipMalloc failed for minimiser state");
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = min_zero_state(m, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        min_free(m);
        delete m;
        return set_hip_error(e, "spx_min_create");
    }
    register_handle(m);
    *out = m;
    return SPX_OK;
}

spx_status spx_min_step(spx_min *m, double *S, int32_t n_iter, void *stream) {
    if (!handle_alive(m)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_min handle");
    if (!S || n_iter < 0) return set_error(SPX_ERR_INVALID_ARG, "S is NULL or n_iter < 0");
    hipStream_t st = (hipStream_t)stream;
    const MinArgs &a = m->a;
    const unsigned nb = (unsigned)a.nb;
    for (int it = 0; it < n_iter; ++it) {
        if (m->fused) {
            hipError_t e = zmarch_min_force(m->zp, m->g, m->os, S, a.F, a.V, a.Up, a.Fp, a.Sh, a.Yh, a.st, MS_DONE,
                                            MS_CAND, a.method, a.part, st);
            if (e != hipSuccess) return set_hip_error(e, "spx_min_step: force pass");
            MinArgs af = a;
            af.npart = m->ntile;
            k_min_scalars<<<1, kMinB, 0, st>>>(af);
        } else {
            spx_status s = spx_eval_field(m->h, S, m->b, stream);
            if (s != SPX_OK) return s;
            k_min_force<<<nb, kMinB, 0, st>>>(a, S, m->b);
            k_min_scalars<<<1, kMinB, 0, st>>>(a);
        }
        if (a.method == 2) {
            // t = hist only applies the last axpy of a full history
            for (int t = 0; t <= a.hist; ++t) {
                k_lb_loop1<<<nb, kMinB, 0, st>>>(a, S, t);
                if (t < a.hist) k_lb_alpha<<<1, kMinB, 0, st>>>(a, t);
            }
            for (int t = a.hist - 1; t >= -1; --t) {
                k_lb_loop2<<<nb, kMinB, 0, st>>>(a, S, t);
                k_lb_beta<<<1, kMinB, 0, st>>>(a, t);
            }
        }
        k_min_update<<<nb, kMinB, 0, st>>>(a, S);
        k_min_finish<<<1, 1, 0, st>>>(a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return set_hip_error(e, "spx_min_step");
    }
    return SPX_OK;
}

spx_status spx_min_get_stats(spx_min *m, double *max_force, int32_t *iterations, int32_t *converged, void *stream) {
    if (!handle_alive(m)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_min handle");
    double st[MS_N];
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(st, m->a.st, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_hip_error(e, "spx_min_get_stats");
    if (max_force) *max_force = st[MS_MAXF];
    if (iterations) *iterations = (int32_t)st[MS_ITER];
    if (converged) *converged = (int32_t)st[MS_DONE];
    return SPX_OK;
}

spx_status spx_min_reset(spx_min *m, void *stream) {
    if (!handle_alive(m)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_min handle");
    hipError_t e = min_zero_state(m, (hipStream_t)stream);
    if (e != hipSuccess) return set_hip_error(e, "spx_min_reset");
    return SPX_OK;
}

spx_status spx_min_destroy(spx_min *m) {
    if (!handle_alive(m)) return set_error(SPX_ERR_BAD_HANDLE, "invalid spx_min handle");
    unregister_handle(m);
    (void)hipDeviceSynchronize();
    min_free(m);
    delete m;
    return SPX_OK;
}

}  // extern "C"
