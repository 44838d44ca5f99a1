// spx_api.hip -- host runtime and C ABI of libspx.so: descriptor validation,
// neighbour-shell enumeration into directed-bond kernel tables, workspace
// management, and dispatch of the field / energy / Heun kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/spx.h"
#include "spx_ext.hpp"
#include "spx_internal.hpp"

using namespace spx;

// ---------------------------------------------------------------- errors
namespace {
thread_local std::string g_last_error;

spx_status fail(spx_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

spx_status hip_fail(hipError_t e, const char *where) {
    return fail(SPX_ERR_HIP, std::string(where) + ": " + hipGetErrorName(e) + " (" +
                                 hipGetErrorString(e) + ")");
}

std::mutex g_reg_mu;
std::unordered_set<const void *> g_handles;

void reg_add(const void *p) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_handles.insert(p);
}
bool reg_has(const void *p) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    return p != nullptr && g_handles.count(p) != 0;
}
void reg_del(const void *p) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_handles.erase(p);
}
}  // namespace

namespace spx {
void register_handle(const void *p) { reg_add(p); }
bool handle_alive(const void *p) { return reg_has(p); }
void unregister_handle(const void *p) { reg_del(p); }
spx_status set_error(spx_status s, const std::string &msg) { return fail(s, msg); }
spx_status set_hip_error(hipError_t e, const char *where) { return hip_fail(e, where); }
}  // namespace spx

// ---------------------------------------------------------------- shells
namespace {

struct HostBond {
    int a, b, d[3];
    double J[9];
};

double norm3(const double v[3]) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

// Smallest spacing between lattice planes: volume / largest face area.
double plane_spacing(const double c[9]) {
    const double *a0 = c, *a1 = c + 3, *a2 = c + 6;
    auto cross = [](const double *u, const double *v, double *w) {
        w[0] = u[1] * v[2] - u[2] * v[1];
        w[1] = u[2] * v[0] - u[0] * v[2];
        w[2] = u[0] * v[1] - u[1] * v[0];
    };
    double f01[3], f12[3], f20[3];
    cross(a0, a1, f01);
    cross(a1, a2, f12);
    cross(a2, a0, f20);
    const double vol = std::fabs(a0[0] * f12[0] + a0[1] * f12[1] + a0[2] * f12[2]);
    const double area = std::max(norm3(f01), std::max(norm3(f12), norm3(f20)));
    return vol / area;
}

// Bond vector r = (delta + f_b - f_a) . cell for source b at cell offset delta.
void bond_vector(const double c[9], const double *fa, const double *fb, int dx, int dy, int dz,
                 double r[3]) {
    const double u = dx + fb[0] - fa[0], v = dy + fb[1] - fa[1], w = dz + fb[2] - fa[2];
    for (int k = 0; k < 3; ++k) r[k] = u * c[k] + v * c[3 + k] + w * c[6 + k];
}

// Directed bonds of the first n_shells distance shells.  Candidate offsets are
// gathered in a box that grows until it provably contains every vector up to
// the last shell radius (|delta_k| <= rho / spacing + 1 for |r| <= rho).
spx_status enumerate_shell_bonds(const spx_lattice_desc &lat, const spx_model_desc &m,
                                 std::vector<HostBond> &out) {
    const int ns = lat.n_sub;
    double longest = 0.0;
    for (int k = 0; k < 3; ++k) longest = std::max(longest, norm3(lat.cell + 3 * k));
    const double tol = 1e-9 * longest;
    const double h = plane_spacing(lat.cell);
    if (!(h > 0.0)) return fail(SPX_ERR_INVALID_ARG, "lattice vectors are degenerate");
    std::vector<double> shells;
    for (int M = 1; M <= 64; M *= 2) {
        std::vector<double> d;
        for (int a = 0; a < ns; ++a)
            for (int b = 0; b < ns; ++b)
                for (int dz = -M; dz <= M; ++dz)
                    for (int dy = -M; dy <= M; ++dy)
                        for (int dx = -M; dx <= M; ++dx) {
                            double r[3];
                            bond_vector(lat.cell, lat.sub_frac + 3 * a, lat.sub_frac + 3 * b, dx, dy, dz, r);
                            const double n = norm3(r);
                            if (n > tol) d.push_back(n);
                        }
        std::sort(d.begin(), d.end());
        shells.clear();
        for (double v : d) {
            if (shells.empty() || v - shells.back() > tol) shells.push_back(v);
            if ((int)shells.size() == m.n_shells) break;
        }
        if ((int)shells.size() == m.n_shells && shells.back() <= (M - 1) * h) break;
        shells.clear();
    }
    if ((int)shells.size() != m.n_shells) return fail(SPX_ERR_INVALID_ARG, "shell enumeration did not converge");
    const int R = (int)std::ceil(shells.back() / h) + 1;
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b)
            for (int dz = -R; dz <= R; ++dz)
                for (int dy = -R; dy <= R; ++dy)
                    for (int dx = -R; dx <= R; ++dx) {
                        double r[3];
                        bond_vector(lat.cell, lat.sub_frac + 3 * a, lat.sub_frac + 3 * b, dx, dy, dz, r);
                        const double n = norm3(r);
                        if (n <= tol) continue;
                        int s = -1;
                        for (int k = 0; k < m.n_shells; ++k)
                            if (std::fabs(n - shells[k]) <= tol) { s = k; break; }
                        if (s < 0) continue;
                        const double J = m.J_shell[s];
                        const double D = m.D_shell ? m.D_shell[s] : 0.0;
                        if (J == 0.0 && D == 0.0) continue;
                        // J_ij = J I + DMI matrix of D_ij = D r/|r| (Methods, bilinear tensor)
                        const double Dx = D * r[0] / n, Dy = D * r[1] / n, Dz = D * r[2] / n;
                        HostBond hb{a, b, {dx, dy, dz}, {J, Dz, -Dy, -Dz, J, Dx, Dy, -Dx, J}};
                        out.push_back(hb);
                    }
    return SPX_OK;
}

}  // namespace

// ---------------------------------------------------------------- handle
struct spx_ham {
    spx_lattice_desc lat{};
    std::vector<double> frac, mu;
    int field_prec = 0;
    int backend = 1;
    std::vector<HostBond> bonds;
    Grid grid{};
    Onsite onsite{};
    BondTable tab{};
    int radius[3] = {0, 0, 0};
    // device allocations
    int4 *d_geo = nullptr;
    float *d_Jf = nullptr;
    double *d_Jd = nullptr;
    double *d_St = nullptr;      // Heun predictor state
    double *d_Sp = nullptr;      // Heun ping-pong state
    double *d_partial = nullptr; // energy partials
    int64_t ws_bytes = 0;
    DipolarPlan *dip = nullptr;  // dipolar FFT workspace (NULL when off)
    float *d_bdip0 = nullptr, *d_bdip1 = nullptr;
    DensePlan *dense = nullptr;  // dense-window MFMA backend
    // z-march engine plan (valid when the bond table matches a shell shape)
    ZPlan zp;
    ZPlan zp64;  // FP64 plan of the same table for batched-image field passes (GNEB)
    int engine = 1;          // 1 gather, 2 z-march
    bool fusable = false;    // the fused Heun step (mode 8) applies
    int heun_field = 1;      // 1 recompute, 2 stored FP32 field, 3 stored stage (P, eta), 7 stored P only, 8 fused
    float *d_bstore = nullptr;
    void *d_ebil = nullptr;  // energy: bilinear field of the z-march pass (made at the first call)
    double *d_P = nullptr;   // heun_field 3: S^n + dt/2 f(S^n)
    double *d_eta = nullptr; // heun_field 3, 4, 5, 6: the step's thermal noise
    // Heun graph replay: 2-step graph with a device step counter
    uint64_t *d_step = nullptr;
    hipGraphExec_t heun_graph = nullptr;
    std::vector<unsigned char> graph_key;
    hipStream_t cap_stream = nullptr;  // private capture stream
    int use_graph = 1;
    MCState *mc = nullptr;              // Monte Carlo colouring and scratch
    PairList *pl = nullptr;             // pair-list Hamiltonian (backend 3)
    int64_t pl_pairs = 0;
    int tuned = 0;
    double tune_us = 0.0;
    // kernel timing: recorded (start, stop) event pairs per kind, and a pool
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed[4];
    std::vector<hipEvent_t> pool;
};

namespace {

template <typename T>
spx_status dev_alloc(spx_ham *h, T **p, size_t count, const char *what) {
    if (count == 0) { *p = nullptr; return SPX_OK; }
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(SPX_ERR_OUT_OF_MEMORY, std::string("hipMalloc failed for ") + what + " (" +
                                               std::to_string(count * sizeof(T)) + " bytes)");
    }
    h->ws_bytes += (int64_t)(count * sizeof(T));
    return SPX_OK;
}

hipEvent_t pool_event(spx_ham *h) {
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Brackets one kernel launch with events when timing is on.
struct KernelTimer {
    spx_ham *h;
    int kind;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    KernelTimer(spx_ham *h_, int k, hipStream_t s) : h(h_), kind(k), st(s) {
        if (!h->timing) return;
        a = pool_event(h);
        b = pool_event(h);
        if (a && b) (void)hipEventRecord(a, st);
    }
    ~KernelTimer() {
        if (!h->timing || !a || !b) return;
        (void)hipEventRecord(b, st);
        h->timed[kind].emplace_back(a, b);
    }
};

void free_all(spx_ham *h) {
    if (h->mc) mc_destroy(h->mc);
    h->mc = nullptr;
    if (h->pl) pl_destroy(h->pl);
    h->pl = nullptr;
    if (h->dense) dense_destroy(h->dense);
    h->dense = nullptr;
    if (h->heun_graph) (void)hipGraphExecDestroy(h->heun_graph);
    h->heun_graph = nullptr;
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    h->cap_stream = nullptr;
    if (h->d_step) (void)hipFree(h->d_step);
    h->d_step = nullptr;
    for (auto &v : h->timed)
        for (auto &pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
    for (auto &v : h->timed) v.clear();
    h->pool.clear();
    if (h->dip) destroy_dipolar(h->dip);
    h->dip = nullptr;
    for (void *p : {(void *)h->d_geo, (void *)h->d_Jf, (void *)h->d_Jd, (void *)h->d_St, (void *)h->d_Sp,
                    (void *)h->d_partial, (void *)h->d_bdip0, (void *)h->d_bdip1, (void *)h->d_bstore,
                    (void *)h->d_P, (void *)h->d_eta, h->d_ebil})
        if (p) (void)hipFree(p);
    h->d_ebil = nullptr;
    h->d_bstore = nullptr;
    h->d_P = h->d_eta = nullptr;
    h->d_geo = nullptr;
    h->d_Jf = nullptr;
    h->d_Jd = nullptr;
    h->d_St = h->d_Sp = h->d_partial = nullptr;
    h->d_bdip0 = h->d_bdip1 = nullptr;
}

spx_status check_device() {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) {
        (void)hipGetLastError();
        return fail(SPX_ERR_HIP, "no HIP device available");
    }
    return SPX_OK;
}

}  // namespace

namespace spx {
spx_status get_ham_view(spx_ham *h, HamView &v) {
    if (!reg_has(h)) return fail(SPX_ERR_BAD_HANDLE, "invalid spx_ham handle");
    v.zp64 = h->zp64.valid ? &h->zp64 : nullptr;
    v.grid = h->grid;
    v.tab = h->tab;
    v.onsite = h->onsite;
    v.field_prec = h->field_prec;
    v.mu = h->mu.data();
    v.dip = h->dip;
    v.radius[0] = h->radius[0];
    v.radius[1] = h->radius[1];
    v.radius[2] = h->radius[2];
    v.mc = &h->mc;
    v.pl = h->pl;
    return SPX_OK;
}
}  // namespace spx

static spx_status autotune_heun(spx_ham *h, const char *cache_path, bool tune_z, bool tune_field, hipStream_t st);
static spx_status heun_buffers(spx_ham *h, int hf);
// Heun modes of the z-march engine: 1 .. kMaxHeunMode (spx_options.heun_field);
// mode 8 is the temporally fused single-pass step
constexpr int kMaxHeunMode = 8;
constexpr int kHeunFused = 8;

extern "C" {

int32_t spx_abi_version(void) { return SPX_ABI_VERSION; }

const char *spx_last_error(void) { return g_last_error.c_str(); }

spx_status spx_setup_hamiltonian(const spx_lattice_desc *lat, const spx_model_desc *model,
                                 const spx_options *opts, void *stream, spx_ham **out) {
    if (!out) return fail(SPX_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!lat || !model) return fail(SPX_ERR_INVALID_ARG, "lattice or model descriptor is NULL");
    if (lat->n_sub < 1 || lat->n_sub > kMaxSub)
        return fail(SPX_ERR_INVALID_ARG, "n_sub must be in [1, " + std::to_string(kMaxSub) + "]");
    if (!lat->sub_frac || !lat->mu) return fail(SPX_ERR_INVALID_ARG, "sub_frac or mu is NULL");
    int64_t M = 1;
    for (int k = 0; k < 3; ++k) {
        if (lat->dims[k] < 1) return fail(SPX_ERR_INVALID_ARG, "dims must be >= 1");
        if (lat->periodic[k] != 0 && lat->periodic[k] != 1)
            return fail(SPX_ERR_INVALID_ARG, "periodic flags must be 0 or 1");
        M *= lat->dims[k];
    }
    if (M > (int64_t)INT32_MAX) return fail(SPX_ERR_INVALID_ARG, "more than 2^31-1 cells per sublattice");
    for (int a = 0; a < lat->n_sub; ++a)
        if (!(lat->mu[a] > 0.0)) return fail(SPX_ERR_INVALID_ARG, "moments mu must be positive");
    const int prec = opts ? opts->field_prec : SPX_FP64;
    if (prec < SPX_FP64 || prec > SPX_FP16_MFMA) return fail(SPX_ERR_INVALID_ARG, "unknown field_prec");
    const int backend_req = opts ? opts->backend : 0;
    if (backend_req < 0 || backend_req > 2) return fail(SPX_ERR_INVALID_ARG, "unknown backend");
    const int engine_req = opts ? opts->stencil_engine : 0;
    const int zchunk_req = opts ? opts->zchunk : 0;
    const int hfield_req = opts ? opts->heun_field : 0;
    if (engine_req < 0 || engine_req > 2) return fail(SPX_ERR_INVALID_ARG, "unknown stencil_engine");
    if (zchunk_req < 0 || zchunk_req > 4096) return fail(SPX_ERR_INVALID_ARG, "zchunk out of range");
    const int rows_req = opts ? opts->tile_rows : 0;
    if (rows_req != 0 && rows_req != 8 && rows_req != 16) return fail(SPX_ERR_INVALID_ARG, "tile_rows must be 0, 8 or 16");
    if (hfield_req < 0 || hfield_req > kMaxHeunMode) return fail(SPX_ERR_INVALID_ARG, "unknown heun_field");
    if ((hfield_req == 2 || hfield_req == 5 || hfield_req == 6) && prec != SPX_FP32)
        return fail(SPX_ERR_INVALID_ARG, "a stored FP32 Heun field needs field_prec SPX_FP32");
    if (model->n_shells < 0 || model->n_bonds < 0 || model->n_aniso < 0)
        return fail(SPX_ERR_INVALID_ARG, "negative counts in model descriptor");
    if (model->n_shells > 0 && !model->J_shell) return fail(SPX_ERR_INVALID_ARG, "J_shell is NULL");
    if (model->n_bonds > 0 && (!model->bond_ab || !model->bond_delta || !model->bond_J))
        return fail(SPX_ERR_INVALID_ARG, "bond arrays are NULL");
    if (model->n_aniso > kMaxAniso) return fail(SPX_ERR_INVALID_ARG, "too many anisotropy axes");
    if (model->n_aniso > 0 && (!model->K || !model->K_axis))
        return fail(SPX_ERR_INVALID_ARG, "K or K_axis is NULL");
    if (model->dipolar != 0 && model->dipolar != 1) return fail(SPX_ERR_INVALID_ARG, "dipolar must be 0 or 1");
    if (model->dipolar) {
        if (lat->n_sub != 1) return fail(SPX_ERR_UNSUPPORTED, "dipolar FFT path needs n_sub = 1");
        if (lat->periodic[0] || lat->periodic[1] || lat->periodic[2])
            return fail(SPX_ERR_UNSUPPORTED, "dipolar FFT path is open-boundary only");
    }
    if (prec >= SPX_BF16_MFMA && backend_req == 1)
        return fail(SPX_ERR_INVALID_ARG, "MFMA precisions need the dense backend");
    if (backend_req == 2 && prec != SPX_FP32 && prec < SPX_BF16_MFMA)
        return fail(SPX_ERR_INVALID_ARG,
                    "the dense backend needs field_prec SPX_FP32 (direct), SPX_BF16_MFMA or SPX_FP16_MFMA");
    // the dense window: MFMA precisions, or FP32 with the dense backend requested
    const bool want_dense = prec >= SPX_BF16_MFMA || backend_req == 2;
    if (want_dense && model->dipolar) return fail(SPX_ERR_UNSUPPORTED, "the dense backend has no dipolar term");
    spx_status s = check_device();
    if (s != SPX_OK) return s;

    spx_ham *h = new spx_ham();
    h->lat = *lat;
    h->frac.assign(lat->sub_frac, lat->sub_frac + 3 * lat->n_sub);
    h->mu.assign(lat->mu, lat->mu + lat->n_sub);
    h->lat.sub_frac = h->frac.data();
    h->lat.mu = h->mu.data();
    h->field_prec = prec;
    h->backend = 1;

    // bond table
    if (model->n_bonds > 0) {
        for (int p = 0; p < model->n_bonds; ++p) {
            HostBond hb;
            hb.a = model->bond_ab[2 * p];
            hb.b = model->bond_ab[2 * p + 1];
            if (hb.a < 0 || hb.a >= lat->n_sub || hb.b < 0 || hb.b >= lat->n_sub) {
                delete h;
                return fail(SPX_ERR_INVALID_ARG, "bond sublattice index out of range");
            }
            for (int k = 0; k < 3; ++k) hb.d[k] = model->bond_delta[3 * p + k];
            for (int k = 0; k < 9; ++k) hb.J[k] = model->bond_J[9 * p + k];
            h->bonds.push_back(hb);
        }
    } else if (model->n_shells > 0) {
        s = enumerate_shell_bonds(h->lat, *model, h->bonds);
        if (s != SPX_OK) { delete h; return s; }
    }
    std::stable_sort(h->bonds.begin(), h->bonds.end(), [](const HostBond &u, const HostBond &v) {
        if (u.a != v.a) return u.a < v.a;
        if (u.b != v.b) return u.b < v.b;
        if (u.d[2] != v.d[2]) return u.d[2] < v.d[2];
        if (u.d[1] != v.d[1]) return u.d[1] < v.d[1];
        return u.d[0] < v.d[0];
    });
    const int nb = (int)h->bonds.size();
    bool iso = true;
    for (const HostBond &hb : h->bonds) {
        const double *J = hb.J;
        if (J[1] != 0 || J[2] != 0 || J[3] != 0 || J[5] != 0 || J[6] != 0 || J[7] != 0 || J[0] != J[4] ||
            J[0] != J[8])
            iso = false;
        for (int k = 0; k < 3; ++k) h->radius[k] = std::max(h->radius[k], std::abs(hb.d[k]));
    }
    // grid
    Grid &g = h->grid;
    g.Lx = lat->dims[0];
    g.Ly = lat->dims[1];
    g.Lz = lat->dims[2];
    for (int k = 0; k < 3; ++k) g.per[k] = lat->periodic[k];
    g.n_sub = lat->n_sub;
    g.M = (int)M;
    g.N = M * lat->n_sub;
    g.wrap_general = 0;
    for (int k = 0; k < 3; ++k)
        if (h->radius[k] > lat->dims[k]) g.wrap_general = 1;
    // on-site terms
    Onsite &os = h->onsite;
    std::memset(&os, 0, sizeof(os));
    os.n_aniso = model->n_aniso;
    for (int a = 0; a < lat->n_sub; ++a) {
        for (int l = 0; l < model->n_aniso; ++l) {
            os.K[a][l] = model->K[a * model->n_aniso + l];
            for (int c = 0; c < 3; ++c) os.axis[a][l][c] = model->K_axis[3 * (a * model->n_aniso + l) + c];
        }
        for (int c = 0; c < 3; ++c) os.bz[a][c] = lat->mu[a] * kMuB * model->B_ext[c];
    }
    // device tables
    std::vector<int4> geo(nb);
    std::vector<float> Jf(iso ? nb : 9 * nb);
    std::vector<double> Jd(iso ? nb : 9 * nb);
    BondTable &tb = h->tab;
    std::memset(&tb, 0, sizeof(tb));
    tb.iso = iso ? 1 : 0;
    for (int a = 0, p = 0; a <= kMaxSub; ++a) {
        while (p < nb && h->bonds[p].a < a) ++p;
        tb.start[a] = p;
    }
    for (int p = 0; p < nb; ++p) {
        const HostBond &hb = h->bonds[p];
        geo[p] = make_int4(hb.b, hb.d[0], hb.d[1], hb.d[2]);
        if (iso) {
            Jd[p] = hb.J[0];
            Jf[p] = (float)hb.J[0];
        } else {
            for (int k = 0; k < 9; ++k) {
                Jd[9 * p + k] = hb.J[k];
                Jf[9 * p + k] = (float)hb.J[k];
            }
        }
    }
    hipStream_t st = (hipStream_t)stream;
    const size_t n3 = (size_t)3 * (size_t)g.N;
    if ((s = dev_alloc(h, &h->d_geo, std::max(nb, 1), "bond geometry")) != SPX_OK ||
        (s = dev_alloc(h, &h->d_Jf, std::max<size_t>(Jf.size(), 1), "couplings fp32")) != SPX_OK ||
        (s = dev_alloc(h, &h->d_Jd, std::max<size_t>(Jd.size(), 1), "couplings fp64")) != SPX_OK ||
        (s = dev_alloc(h, &h->d_St, n3, "Heun predictor state")) != SPX_OK ||
        (s = dev_alloc(h, &h->d_Sp, n3, "Heun ping-pong state")) != SPX_OK ||
        (s = dev_alloc(h, &h->d_partial, energy_partial_doubles(g), "energy partials")) != SPX_OK) {
        free_all(h);
        delete h;
        return s;
    }
    hipError_t e = hipSuccess;
    if (nb > 0) {
        e = hipMemcpyAsync(h->d_geo, geo.data(), nb * sizeof(int4), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->d_Jf, Jf.data(), Jf.size() * sizeof(float), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->d_Jd, Jd.data(), Jd.size() * sizeof(double), hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        free_all(h);
        delete h;
        return hip_fail(e, "spx_setup_hamiltonian: table upload");
    }
    tb.geo = h->d_geo;
    tb.Jf = h->d_Jf;
    tb.Jd = h->d_Jd;
    // z-march engine: match the bond table against the built-in shell shapes
    {
        std::vector<int> ba(nb), bb(nb), bd(3 * nb);
        std::vector<double> bJ(9 * nb);
        for (int p = 0; p < nb; ++p) {
            ba[p] = h->bonds[p].a;
            bb[p] = h->bonds[p].b;
            for (int k = 0; k < 3; ++k) bd[3 * p + k] = h->bonds[p].d[k];
            for (int k = 0; k < 9; ++k) bJ[9 * p + k] = h->bonds[p].J[k];
        }
        if (want_dense) {
            std::string why;
            if (!dense_plan(prec, lat->n_sub, ba.data(), bb.data(), bd.data(), bJ.data(), nb, &h->dense, st, why)) {
                free_all(h);
                delete h;
                return fail(SPX_ERR_UNSUPPORTED, why);
            }
            h->backend = 2;
        }
        const bool have = prec < SPX_BF16_MFMA && nb > 0 &&
                          zmarch_plan(prec, lat->n_sub, ba.data(), bb.data(), bd.data(), bJ.data(), nb, iso, h->zp);
        // an FP64 plan for the GNEB's batched field pass (FP64 arithmetic in
        // every field precision), unless the gather engine was requested
        if (nb > 0 && engine_req != 1) {
            if (!zmarch_plan(0, lat->n_sub, ba.data(), bb.data(), bd.data(), bJ.data(), nb, iso, h->zp64))
                h->zp64.valid = false;
        }
        if (engine_req == 2 && !have) {
            free_all(h);
            delete h;
            return fail(SPX_ERR_UNSUPPORTED, "the bond table matches no z-march shell shape");
        }
        h->engine = (have && engine_req != 1) ? 2 : 1;
        if (have && zchunk_req > 0) h->zp.zch = zchunk_req;
        if (have) h->zp.frows = rows_req;
        h->heun_field = 1;
        // the fused step needs a single-sublattice shape of range one cell and
        // no dipolar term (whose FFT field is taken between the two stages)
        const bool fusable = h->engine == 2 && !model->dipolar && fused_heun_supported(h->zp, h->grid);
        h->fusable = fusable;
        if (hfield_req == kHeunFused && !fusable) {
            free_all(h);
            delete h;
            return fail(SPX_ERR_UNSUPPORTED, "the fused Heun step (heun_field 8) needs the z-march engine on a "
                                             "single-sublattice shell shape of range one cell, without dipolar");
        }
        // stored stages exist in the z-march engine only; the gather engine
        // recomputes.  Default: the fused step where it applies, else mode 3
        if (h->engine == 2) {
            h->heun_field = hfield_req > 0 ? hfield_req : (fusable ? kHeunFused : 3);
            if (hfield_req == 0 && fusable && zchunk_req == 0) h->zp.zch = 64;
        }
        if ((s = heun_buffers(h, h->heun_field)) != SPX_OK) {
            free_all(h);
            delete h;
            return s;
        }
    }
    if (h->engine == 2 && opts && opts->autotune) {
        s = autotune_heun(h, opts->tune_cache_path, zchunk_req == 0, hfield_req == 0, st);
        if (s != SPX_OK) {
            free_all(h);
            delete h;
            return s;
        }
    }
    if (model->dipolar) {
        s = create_dipolar(lat->dims, lat->cell, lat->mu[0], st, &h->dip, &h->ws_bytes);
        if (s == SPX_OK) s = dev_alloc(h, &h->d_bdip0, n3, "dipolar field");
        if (s == SPX_OK) s = dev_alloc(h, &h->d_bdip1, n3, "dipolar field (predictor)");
        if (s != SPX_OK) {
            free_all(h);
            delete h;
            return s;
        }
    }
    reg_add(h);
    *out = h;
    return SPX_OK;
}

spx_status spx_setup_pairlist(const spx_pairlist_desc *d, const spx_options *opts, void *stream, spx_ham **out) {
    if (!out) return fail(SPX_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!d) return fail(SPX_ERR_INVALID_ARG, "pair-list descriptor is NULL");
    const int prec = opts ? opts->field_prec : SPX_FP64;
    if (prec != SPX_FP64 && prec != SPX_FP32)
        return fail(SPX_ERR_INVALID_ARG, "a pair list evaluates the field in SPX_FP64 or SPX_FP32");
    hipStream_t st = (hipStream_t)stream;
    PairList *pl = nullptr;
    spx_status s = pl_create(d, prec, st, &pl);
    if (s != SPX_OK) return s;
    spx_ham *h = new spx_ham();
    h->pl = pl;
    h->pl_pairs = d->n_pairs;
    h->field_prec = prec;
    h->backend = 3;
    h->engine = 1;
    Grid &g = h->grid;
    g.Lx = (int)d->n_sites;
    g.Ly = g.Lz = 1;
    g.per[0] = g.per[1] = g.per[2] = 0;
    g.n_sub = 1;
    g.M = (int)d->n_sites;
    g.N = d->n_sites;
    h->mu.assign(1, 1.0);
    reg_add(h);
    *out = h;
    return SPX_OK;
}

spx_status spx_destroy_hamiltonian(spx_ham *h) {
    if (!reg_has(h)) return fail(SPX_ERR_BAD_HANDLE, "invalid spx_ham handle");
    reg_del(h);
    (void)hipDeviceSynchronize();
    free_all(h);
    delete h;
    return SPX_OK;
}

spx_status spx_get_info(spx_ham *h, spx_ham_info *info) {
    if (!reg_has(h)) return fail(SPX_ERR_BAD_HANDLE, "invalid spx_ham handle");
    if (!info) return fail(SPX_ERR_INVALID_ARG, "info is NULL");
    info->n_sites = h->grid.N;
    info->n_bonds = h->pl ? (int32_t)std::min<int64_t>(h->pl_pairs, INT32_MAX) : (int32_t)h->bonds.size();
    info->field_prec = h->field_prec;
    info->backend = h->backend;
    for (int k = 0; k < 3; ++k) info->radius[k] = h->radius[k];
    info->dipolar = h->dip ? 1 : 0;
    info->workspace_bytes = h->ws_bytes;
    info->stencil_engine = h->engine;
    info->shape = h->engine == 2 ? h->zp.kind : -1;
    info->zchunk = h->engine == 2 ? h->zp.zch : 0;
    info->heun_field = h->heun_field;
    info->tuned = h->tuned;
    info->tuned_step_us = h->tune_us;
    info->tile_rows = (h->engine == 2 && h->heun_field == kHeunFused) ? fused_rows(h->zp) : 0;
    info->heun_graph = h->heun_graph ? 1 : 0;
    return SPX_OK;
}

spx_status spx_get_bonds(spx_ham *h, int32_t *bond_ab, int32_t *bond_delta, double *bond_J) {
    if (!reg_has(h)) return fail(SPX_ERR_BAD_HANDLE, "invalid spx_ham handle");
    if (h->pl) return fail(SPX_ERR_UNSUPPORTED, "a pair-list Hamiltonian has no lattice bond table");
    if (!bond_ab || !bond_delta || !bond_J) return fail(SPX_ERR_INVALID_ARG, "output array is NULL");
    for (size_t p = 0; p < h->bonds.size(); ++p) {
        const HostBond &hb = h->bonds[p];
        bond_ab[2 * p] = hb.a;
        bond_ab[2 * p + 1] = hb.b;
        for (int k = 0; k < 3; ++k) bond_delta[3 * p + k] = hb.d[k];
        for (int k = 0; k < 9; ++k) bond_J[9 * p + k] = hb.J[k];
    }
    return SPX_OK;
}

static spx_status dipolar_field(spx_ham *h, const double *S, float *bdip, hipStream_t st) {
    return eval_dipolar(h->dip, S, bdip, st);
}

__global__ void k_set_u64(uint64_t *p, uint64_t v) { *p = v; }
__global__ void k_add_u64(uint64_t *p, uint64_t v) { *p += v; }

// One normalised Heun step cur -> nxt (predictor into d_St, then corrector).
static spx_status enqueue_heun_step(spx_ham *h, const HeunConst &hc, uint64_t step, const double *cur, double *nxt,
                                    hipStream_t st) {
    const float *bd0 = nullptr, *bd1 = nullptr;
    if (h->dip) {
        spx_status s = dipolar_field(h, cur, h->d_bdip0, st);
        if (s != SPX_OK) return s;
        bd0 = h->d_bdip0;
    }
    hipError_t e;
    if (h->engine == 2 && h->heun_field == kHeunFused) {
        KernelTimer kt(h, 0, st);
        e = heun_fused(h->zp, h->grid, h->onsite, hc, step, cur, nxt, st);
        if (e != hipSuccess) return hip_fail(e, "spx_llg_heun_step: fused step");
        return SPX_OK;
    }
    if (h->engine == 2 && h->heun_field == 4 && hc.noise) {
        KernelTimer kt(h, 3, st);
        e = zmarch_noise(hc, step, h->grid.N, h->d_eta, st);
        if (e != hipSuccess) return hip_fail(e, "spx_llg_heun_step: noise");
    }
    if (h->engine == 2 && (h->heun_field == 5 || h->heun_field == 6)) {
        // split predictor: stencil pass for the FP32 bilinear field, then the
        // elementwise FP64 stage; corrector split (mode 5) or fused (mode 6)
        {
            KernelTimer kt(h, 0, st);
            e = zmarch_bil(h->zp, h->grid, cur, h->d_bstore, st);
            if (e == hipSuccess)
                e = heun_split_pre(h->grid, h->onsite, hc, step, cur, h->d_bstore, bd0, h->d_St, h->d_P, h->d_eta, st);
        }
        if (e != hipSuccess) return hip_fail(e, "spx_llg_heun_step: predictor");
        if (h->dip) {
            spx_status s = dipolar_field(h, h->d_St, h->d_bdip1, st);
            if (s != SPX_OK) return s;
            bd1 = h->d_bdip1;
        }
        {
            KernelTimer kt(h, 1, st);
            if (h->heun_field == 5) {
                e = zmarch_bil(h->zp, h->grid, h->d_St, h->d_bstore, st);
                if (e == hipSuccess)
                    e = heun_split_post(h->grid, h->onsite, hc, h->d_St, h->d_bstore, bd1, h->d_P, h->d_eta, nxt, st);
            } else {
                e = zmarch_correct(h->zp, h->grid, h->onsite, hc, step, cur, h->d_St, bd0, bd1, nullptr, h->d_P,
                                   hc.noise ? h->d_eta : nullptr, nxt, st);
            }
        }
        if (e != hipSuccess) return hip_fail(e, "spx_llg_heun_step: corrector");
        return SPX_OK;
    }
    {
        KernelTimer kt(h, 0, st);
        if (h->engine == 2)
        {
            const int hf = h->heun_field;
            const bool staged = hf >= 3;
            e = zmarch_predict(h->zp, h->grid, h->onsite, hc, step, cur, bd0, h->d_St,
                               hf == 2 ? h->d_bstore : nullptr, staged ? h->d_P : nullptr,
                               (hf == 3 && hc.noise) ? h->d_eta : nullptr, (hf == 4 && hc.noise) ? h->d_eta : nullptr,
                               st);
        }
        else
            e = launch_heun_predict(h->field_prec, h->tab, h->grid, h->onsite, hc, step, cur, bd0, h->d_St, st);
    }
    if (e != hipSuccess) return hip_fail(e, "spx_llg_heun_step: predictor");
    if (h->dip) {
        spx_status s = dipolar_field(h, h->d_St, h->d_bdip1, st);
        if (s != SPX_OK) return s;
        bd1 = h->d_bdip1;
    }
    {
        KernelTimer kt(h, 1, st);
        if (h->engine == 2)
            e = zmarch_correct(h->zp, h->grid, h->onsite, hc, step, cur, h->d_St, bd0, bd1,
                               h->heun_field == 2 ? h->d_bstore : nullptr, h->heun_field >= 3 ? h->d_P : nullptr,
                               (h->heun_field >= 3 && h->heun_field != 7 && hc.noise) ? h->d_eta : nullptr, nxt,
                               st);
        else
            e = launch_heun_correct(h->field_prec, h->tab, h->grid, h->onsite, hc, step, cur, h->d_St, bd0, bd1, nxt,
                                    st);
    }
    if (e != hipSuccess) return hip_fail(e, "spx_llg_heun_step: corrector");
    return SPX_OK;
}

__global__ void k_fill_up(double *S, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    S[i] = 0.0;
    S[N + i] = 0.0;
    S[2 * N + i] = 1.0;
}

// Buffers that Heun mode hf needs (allocated if missing): 2 the FP32 field
// store, 3 the stage store P and the noise store.
static spx_status heun_buffers(spx_ham *h, int hf) {
    const size_t n3 = (size_t)3 * h->grid.N;
    spx_status s = SPX_OK;
    if ((hf == 2 || hf == 5 || hf == 6) && !h->d_bstore) s = dev_alloc(h, &h->d_bstore, n3, "stored Heun field");
    const bool staged = hf >= 3 && hf <= 7;
    if (s == SPX_OK && staged && !h->d_P) s = dev_alloc(h, &h->d_P, n3, "stored Heun stage");
    if (s == SPX_OK && staged && hf != 7 && !h->d_eta) s = dev_alloc(h, &h->d_eta, n3, "stored Heun noise");
    return s;
}

// Frees the stores that the selected mode does not use.
static void heun_buffers_trim(spx_ham *h) {
    const int64_t n3 = 3 * h->grid.N;
    if (h->heun_field != 2 && h->heun_field != 5 && h->heun_field != 6 && h->d_bstore) {
        (void)hipFree(h->d_bstore);
        h->d_bstore = nullptr;
        h->ws_bytes -= (int64_t)sizeof(float) * n3;
    }
    for (double **p : {&h->d_P, &h->d_eta}) {
        const bool used = h->heun_field >= 3 && h->heun_field <= 7 && !(p == &h->d_eta && h->heun_field == 7);
        if (!used && *p) {
            (void)hipFree(*p);
            *p = nullptr;
            h->ws_bytes -= (int64_t)sizeof(double) * n3;
        }
    }
}

// Autotuner of the z-march engine: times stochastic Heun steps for every
// candidate (z planes per block, stored or recomputed corrector field, and
// for the fused step the block rows) on a scratch state and keeps the
// fastest.  Results are cached per shape key (shell shape, precision,
// sublattices, extents, boundary flags) in cache_path when it is given, one
// JSON object per line, {"key": ..., "zchunk": ..., "heun_mode": ...,
// "us": ..., "tile_rows": ...}; lines of the earlier plain form
// "key zchunk heun_mode us [tile_rows]" are read as well.
static spx_status autotune_heun(spx_ham *h, const char *cache_path, bool tune_z, bool tune_field, hipStream_t st) {
    const Grid &g = h->grid;
    char key[160];
    std::snprintf(key, sizeof(key), "shape%d_prec%d_sub%d_%dx%dx%d_per%d%d%d", h->zp.kind, h->field_prec, g.n_sub,
                  g.Lx, g.Ly, g.Lz, g.per[0], g.per[1], g.per[2]);
    // cache entries: key, z chunk, Heun mode, microseconds per step, and the
    // fused step's rows per block (0 for the other modes; plain lines
    // without it read as 0)
    const bool tune_rows = h->fusable && h->zp.kind == SHAPE_SC_NN && h->zp.prec == 1 && h->zp.frows == 0;
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "r")) {
            char line[256], k2[160];
            int z, hf, rows;
            double us;
            bool hit = false;
            int cz = 0, chf = 0, crows = 0;
            double cus = 0.0;
            while (std::fgets(line, sizeof(line), f)) {
                rows = 0;
                int n = std::sscanf(line, " {\"key\": \"%159[^\"]\", \"zchunk\": %d, \"heun_mode\": %d, \"us\": %lf, "
                                          "\"tile_rows\": %d",
                                    k2, &z, &hf, &us, &rows);
                if (n != 5) {
                    rows = 0;
                    n = line[0] == '{' ? 0 : std::sscanf(line, "%159s %d %d %lf %d", k2, &z, &hf, &us, &rows);
                }
                if (n >= 4 && std::strcmp(k2, key) == 0 && z > 0 && z <= 4096 && hf >= 1 && hf <= kMaxHeunMode &&
                    (rows == 0 || rows == 8 || rows == 16)) {
                    cz = z; chf = hf; cus = us; crows = rows; hit = true;   // the last matching line wins
                }
            }
            std::fclose(f);
            if (hit && !((chf == 2 || chf == 5 || chf == 6) && h->field_prec != SPX_FP32) &&
                !(chf == kHeunFused && !h->fusable)) {
                if (tune_z) h->zp.zch = cz;
                if (tune_field) h->heun_field = chf;
                if (tune_rows && h->heun_field == kHeunFused && chf == kHeunFused && crows != 0) h->zp.frows = crows;
                h->tune_us = cus;
                h->tuned = 1;
                spx_status s = heun_buffers(h, h->heun_field);
                heun_buffers_trim(h);
                return s;
            }
        }
    }
    // candidate z chunks: the two-sweep modes march short chunks; the fused
    // step pays a four-plane pipeline fill per chunk, so it tries longer ones
    auto zlist = [&](int hf) {
        std::vector<int> zs;
        if (!tune_z) {
            zs.push_back(h->zp.zch);
            return zs;
        }
        const std::vector<int> cand = hf == kHeunFused ? std::vector<int>{16, 32, 64, 128}
                                                       : std::vector<int>{4, 8, 16, 32};
        for (int z : cand)
            if (z <= g.Lz || zs.empty()) zs.push_back(z);
        return zs;
    };
    std::vector<int> hfs = {h->heun_field};
    if (tune_field) {
        hfs = {1, 3, 4, 7};
        if (h->field_prec == SPX_FP32) hfs = {1, 2, 3, 4, 5, 6, 7};
        if (h->fusable) hfs.push_back(kHeunFused);
    }
    for (int hf : hfs) {
        spx_status s = heun_buffers(h, hf);
        if (s != SPX_OK) return s;
    }
    double *tmp = nullptr;
    spx_status s = dev_alloc(h, &tmp, (size_t)3 * g.N, "autotune scratch state");
    if (s != SPX_OK) return s;
    h->ws_bytes -= (int64_t)(sizeof(double) * 3 * g.N);
    k_fill_up<<<(unsigned)((g.N + 255) / 256), 256, 0, st>>>(tmp, g.N);
    HeunConst hc;
    std::memset(&hc, 0, sizeof(hc));
    hc.dt = 0.1;
    hc.alpha = 0.1;
    hc.pre = -kGammaPerFs / 1.01;
    hc.seed = 1;
    hc.noise = 1;
    for (int a = 0; a < g.n_sub; ++a) {
        hc.inv_mumuB[a] = 1.0 / (h->mu[a] * kMuB);
        hc.sigma[a] = 100.0;
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best = 1e300;
    int bz = h->zp.zch, bh = h->heun_field, brows = h->zp.frows;
    const int reps = 4;
    // block shapes of the fused step: 16 or 8 rows (wavefronts) per block
    auto rowlist = [&](int hf) {
        if (hf == kHeunFused && tune_rows) return std::vector<int>{16, 8};
        return std::vector<int>{h->zp.frows};
    };
    for (int hf : hfs)
        for (int rows : rowlist(hf))
        for (int z : zlist(hf)) {
            h->zp.zch = z;
            h->zp.frows = rows;
            h->heun_field = hf;
            spx_status r = SPX_OK;
            for (int k = 0; k < 2 && r == SPX_OK; ++k) r = enqueue_heun_step(h, hc, k, tmp, h->d_Sp, st);
            (void)hipEventRecord(e0, st);
            for (int k = 0; k < reps && r == SPX_OK; ++k)
                r = enqueue_heun_step(h, hc, k, (k & 1) ? h->d_Sp : tmp, (k & 1) ? tmp : h->d_Sp, st);
            (void)hipEventRecord(e1, st);
            if (r != SPX_OK || hipEventSynchronize(e1) != hipSuccess) {
                s = r != SPX_OK ? r : hip_fail(hipGetLastError(), "autotune");
                break;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double us = 1e3 * ms / reps;
            if (us < best) { best = us; bz = z; bh = hf; brows = rows; }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(tmp);
    if (s != SPX_OK) return s;
    h->zp.zch = bz;
    h->zp.frows = brows;
    h->heun_field = bh;
    h->tuned = 1;
    h->tune_us = best;
    heun_buffers_trim(h);
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "{\"key\": \"%s\", \"zchunk\": %d, \"heun_mode\": %d, \"us\": %.3f, \"tile_rows\": %d}\n",
                         key, bz, bh, best, bh == kHeunFused ? fused_rows(h->zp) : 0);
            std::fclose(f);
        }
    }
    return SPX_OK;
}

// (Re)capture the Heun graph of gsteps (even) steps for state S, constants hc
// and stream st.  Step k of the graph draws the noise of step *d_step + k; the
// graph's last node advances d_step by gsteps.
static hipError_t heun_graph_prepare(spx_ham *h, HeunConst hc, double *S, int gsteps, hipStream_t st) {
    if (!h->d_step) {
        hipError_t e = hipMalloc((void **)&h->d_step, sizeof(uint64_t));
        if (e != hipSuccess) return e;
    }
    hc.step_dev = h->d_step;
    std::vector<unsigned char> key(sizeof(HeunConst) + sizeof(void *) + sizeof(int));
    std::memcpy(key.data(), &hc, sizeof(HeunConst));
    std::memcpy(key.data() + sizeof(HeunConst), &S, sizeof(void *));
    std::memcpy(key.data() + sizeof(HeunConst) + sizeof(void *), &gsteps, sizeof(int));
    if (h->heun_graph && key == h->graph_key) return hipSuccess;
    if (h->heun_graph) (void)hipGraphExecDestroy(h->heun_graph);
    h->heun_graph = nullptr;
    // capture on a private stream: the caller's stream may be the legacy null
    // stream, which cannot be captured; the graph is launched on st
    if (!h->cap_stream) {
        hipError_t e0 = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
        if (e0 != hipSuccess) return e0;
    }
    hipStream_t cs = h->cap_stream;
    hipGraph_t graph;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    spx_status s2 = SPX_OK;
    for (int k = 0; k < gsteps && s2 == SPX_OK; ++k)
        s2 = (k & 1) ? enqueue_heun_step(h, hc, (uint64_t)k, h->d_Sp, S, cs)
                     : enqueue_heun_step(h, hc, (uint64_t)k, S, h->d_Sp, cs);
    if (s2 == SPX_OK) k_add_u64<<<1, 1, 0, cs>>>(h->d_step, (uint64_t)gsteps);
    e = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess) return e;
    if (s2 != SPX_OK) {
        (void)hipGraphDestroy(graph);
        return hipErrorUnknown;
    }
    e = hipGraphInstantiate(&h->heun_graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        h->heun_graph = nullptr;
        return e;
    }
    h->graph_key = key;
    return hipSuccess;
}

spx_status spx_eval_field(spx_ham *h, const double *S, void *b, void *stream) {
    if (!reg_has(h)) return fail(SPX_ERR_BAD_HANDLE, "invalid spx_ham handle");
    if (!S || !b) return fail(SPX_ERR_INVALID_ARG, "S or b is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (h->pl) {
        KernelTimer kt(h, 2, st);
        hipError_t e = pl_field(h->pl, S, b, st);
        if (e != hipSuccess) return hip_fail(e, "spx_eval_field (pair list)");
        return SPX_OK;
    }
    const float *bdip = nullptr;
    if (h->dip) {
        spx_status s = dipolar_field(h, S, h->d_bdip0, st);
        if (s != SPX_OK) return s;
        bdip = h->d_bdip0;
    }
    hipError_t e;
    {
        KernelTimer kt(h, 2, st);
        if (h->dense) e = dense_field(h->dense, h->grid, h->onsite, S, (float *)b, st);
        else if (h->engine == 2) e = zmarch_field(h->zp, h->grid, h->onsite, S, bdip, b, st);
        else e = launch_field(h->field_prec, h->tab, h->grid, h->onsite, S, bdip, b, st);
    }
    if (e != hipSuccess) return hip_fail(e, "spx_eval_field");
    return SPX_OK;
}

spx_status spx_energy(spx_ham *h, const double *S, double *E, double *terms, void *stream) {
    if (!reg_has(h)) return fail(SPX_ERR_BAD_HANDLE, "invalid spx_ham handle");
    if (!S || (!E && !terms)) return fail(SPX_ERR_INVALID_ARG, "S is NULL or no output given");
    hipStream_t st = (hipStream_t)stream;
    if (h->pl) {
        hipError_t e = pl_energy(h->pl, S, E, terms, st);
        if (e != hipSuccess) return hip_fail(e, "spx_energy (pair list)");
        return SPX_OK;
    }
    const float *bdip = nullptr;
    if (h->dip) {
        spx_status s = dipolar_field(h, S, h->d_bdip0, st);
        if (s != SPX_OK) return s;
        bdip = h->d_bdip0;
    }
    // the dense MFMA backend evaluates energies with the FP32 gather kernel;
    // the z-march engine sums the energy terms in its epilogue, one quadruple
    // per tile, when they fit the partial buffer (every lattice but very thin
    // ones); otherwise its bilinear field pass feeds the gather energy kernel
    const int eprec = h->field_prec >= SPX_BF16_MFMA ? SPX_FP32 : h->field_prec;
    const void *bil = nullptr;
    hipError_t e = hipSuccess;
    if (h->engine == 2 && h->zp.valid &&
        (size_t)4 * ((size_t)zmarch_tiles(h->zp, h->grid) + kEnergyL2) <= energy_partial_doubles(h->grid)) {
        e = zmarch_energy(h->zp, h->grid, h->onsite, S, bdip, h->d_partial, st);
        if (e == hipSuccess) e = launch_energy_reduce(h->d_partial, zmarch_tiles(h->zp, h->grid), E, terms, st);
        if (e != hipSuccess) return hip_fail(e, "spx_energy (z-march)");
        return SPX_OK;
    }
    if (h->engine == 2 && h->zp.valid) {
        void *buf = (h->zp.prec == 1 && h->d_bstore) ? (void *)h->d_bstore : h->d_ebil;
        if (!buf) {
            const size_t bytes = (size_t)3 * h->grid.N * (h->zp.prec == 1 ? sizeof(float) : sizeof(double));
            spx_status s = dev_alloc(h, (unsigned char **)&h->d_ebil, bytes, "energy field buffer");
            if (s != SPX_OK) return s;
            buf = h->d_ebil;
        }
        e = h->zp.prec == 1 ? zmarch_bil(h->zp, h->grid, S, (float *)buf, st)
                            : zmarch_bil_images(h->zp, h->grid, 1, S, nullptr, nullptr, nullptr, (double *)buf, st);
        if (e != hipSuccess) return hip_fail(e, "spx_energy (field pass)");
        bil = buf;
    }
    e = launch_energy(eprec, h->tab, h->grid, h->onsite, S, bdip, bil, h->d_partial, E, terms, st);
    if (e != hipSuccess) return hip_fail(e, "spx_energy");
    return SPX_OK;
}

spx_status spx_llg_heun_step(spx_ham *h, double *S, const spx_llg_params *p, void *stream) {
    if (!reg_has(h)) return fail(SPX_ERR_BAD_HANDLE, "invalid spx_ham handle");
    if (!S || !p) return fail(SPX_ERR_INVALID_ARG, "S or params is NULL");
    if (p->n_steps < 0) return fail(SPX_ERR_INVALID_ARG, "n_steps < 0");
    if (!(p->dt_fs > 0.0)) return fail(SPX_ERR_INVALID_ARG, "dt_fs must be positive");
    if (!(p->alpha >= 0.0)) return fail(SPX_ERR_INVALID_ARG, "alpha must be >= 0");
    if (!(p->temperature_K >= 0.0)) return fail(SPX_ERR_INVALID_ARG, "temperature must be >= 0");
    if (p->temperature_K > 0.0 && p->alpha == 0.0)
        return fail(SPX_ERR_INVALID_ARG, "a thermal bath needs alpha > 0");
    if (h->dense) return fail(SPX_ERR_UNSUPPORTED, "Heun integration runs on the sparse stencil backend");
    if (p->n_steps == 0) return SPX_OK;
    hipStream_t st = (hipStream_t)stream;
    const double gamma = (p->gamma > 0.0) ? p->gamma * 1e-15 : kGammaPerFs;  // rad/(fs T)
    if (h->pl) {
        const int noise = p->temperature_K > 0.0 ? 1 : 0;
        const double sig0 = noise ? std::sqrt(2.0 * p->alpha * kKB * p->temperature_K / (gamma * kMuB * p->dt_fs)) : 0.0;
        hipError_t e = pl_heun(h->pl, S, p->alpha, p->dt_fs, -gamma / (1.0 + p->alpha * p->alpha), sig0, p->seed,
                               p->step0, p->tag, noise, p->n_steps, st);
        if (e != hipSuccess) return hip_fail(e, "spx_llg_heun_step (pair list)");
        return SPX_OK;
    }
    HeunConst hc;
    std::memset(&hc, 0, sizeof(hc));
    hc.dt = p->dt_fs;
    hc.alpha = p->alpha;
    hc.pre = -gamma / (1.0 + p->alpha * p->alpha);
    hc.seed = p->seed;
    hc.tag = p->tag;
    hc.noise = p->temperature_K > 0.0 ? 1 : 0;
    for (int a = 0; a < h->grid.n_sub; ++a) {
        hc.inv_mumuB[a] = 1.0 / (h->mu[a] * kMuB);
        hc.sigma[a] = hc.noise ? std::sqrt(2.0 * p->alpha * kKB * p->temperature_K /
                                           (gamma * h->mu[a] * kMuB * p->dt_fs))
                               : 0.0;
    }
    // Graph replay: one captured graph of gsteps steps (S -> Sp -> ... -> S)
    // whose noise steps come from a device counter that the graph itself
    // advances by gsteps; 16 steps per graph keep the counter node and the
    // graph launch off the step time of small lattices.  The remaining steps
    // are launched directly.  Not used with the dipolar FFT path or while
    // kernels are being timed.
    const int gsteps = p->n_steps >= 16 ? 16 : 2;
    int n_graphs = (h->use_graph && !h->dip && !h->timing && p->n_steps >= 4) ? p->n_steps / gsteps : 0;
    if (n_graphs > 0 && heun_graph_prepare(h, hc, S, gsteps, st) != hipSuccess) {
        (void)hipGetLastError();  // capture unsupported: direct launches from now on
        h->use_graph = 0;
        n_graphs = 0;
    }
    if (n_graphs > 0) {
        k_set_u64<<<1, 1, 0, st>>>(h->d_step, p->step0);
        hipError_t e = hipGetLastError();
        for (int k = 0; k < n_graphs && e == hipSuccess; ++k) e = hipGraphLaunch(h->heun_graph, st);
        if (e != hipSuccess) return hip_fail(e, "spx_llg_heun_step: graph replay");
    }
    double *cur = S, *nxt = h->d_Sp;
    for (int k = gsteps * n_graphs; k < p->n_steps; ++k) {
        spx_status s = enqueue_heun_step(h, hc, p->step0 + (uint64_t)k, cur, nxt, st);
        if (s != SPX_OK) return s;
        std::swap(cur, nxt);
    }
    if (cur != S) {
        hipError_t e = hipMemcpyAsync(S, cur, sizeof(double) * 3 * (size_t)h->grid.N, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "spx_llg_heun_step: copy-back");
    }
    return SPX_OK;
}

spx_status spx_set_heun_graph(spx_ham *h, int32_t enable) {
    if (!reg_has(h)) return fail(SPX_ERR_BAD_HANDLE, "invalid spx_ham handle");
    h->use_graph = enable ? 1 : 0;
    return SPX_OK;
}

spx_status spx_set_kernel_timing(spx_ham *h, int32_t enable) {
    if (!reg_has(h)) return fail(SPX_ERR_BAD_HANDLE, "invalid spx_ham handle");
    h->timing = enable != 0;
    return SPX_OK;
}

spx_status spx_get_kernel_times(spx_ham *h, int32_t kind, int64_t *count, double *total_ms) {
    if (!reg_has(h)) return fail(SPX_ERR_BAD_HANDLE, "invalid spx_ham handle");
    if (kind < 0 || kind > 3 || !count || !total_ms) return fail(SPX_ERR_INVALID_ARG, "bad kind or output");
    double tot = 0.0;
    int64_t n = 0;
    for (auto &pr : h->timed[kind]) {
        hipError_t e = hipEventSynchronize(pr.second);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
        if (e != hipSuccess) return hip_fail(e, "spx_get_kernel_times");
        tot += ms;
        ++n;
        h->pool.push_back(pr.first);
        h->pool.push_back(pr.second);
    }
    h->timed[kind].clear();
    *count = n;
    *total_ms = tot;
    return SPX_OK;
}

spx_status spx_thermal_noise(uint64_t seed, uint64_t step, uint32_t tag, int64_t N, double *eta, void *stream) {
    if (N < 0 || (N > 0 && !eta)) return fail(SPX_ERR_INVALID_ARG, "bad N or eta");
    hipError_t e = launch_thermal_noise(seed, step, tag, N, eta, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "spx_thermal_noise");
    return SPX_OK;
}

spx_status spx_stream_probe(int32_t kind, const void *src, void *dst, int64_t n_bytes, void *stream) {
    if (kind < 0 || kind > 2) return fail(SPX_ERR_INVALID_ARG, "spx_stream_probe: kind must be 0, 1 or 2");
    if (n_bytes < 0 || n_bytes % 16 != 0) return fail(SPX_ERR_INVALID_ARG, "spx_stream_probe: n_bytes must be a multiple of 16");
    if (n_bytes > 0 && ((kind != 2 && !src) || (kind != 1 && !dst)))
        return fail(SPX_ERR_INVALID_ARG, "spx_stream_probe: missing buffer");
    if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0)
        return fail(SPX_ERR_INVALID_ARG, "spx_stream_probe: buffers must be 16-byte aligned");
    hipError_t e = launch_stream(kind, src, dst, n_bytes / 16, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "spx_stream_probe");
    return SPX_OK;
}

spx_status spx_philox4x32_10(const uint32_t *ctr, const uint32_t *key, int64_t n, uint32_t *out, void *stream) {
    if (n < 0 || (n > 0 && (!ctr || !key || !out))) return fail(SPX_ERR_INVALID_ARG, "bad philox arguments");
    hipError_t e = launch_philox(ctr, key, n, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "spx_philox4x32_10");
    return SPX_OK;
}

}  // extern "C"
