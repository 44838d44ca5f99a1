/*
 * spx_oracle.c -- plain, slow FP64 CPU oracle for the spin-field / LLG-Heun /
 * energy / GNEB path of "SpinX" (arXiv 2605.26016).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * constant generator with the HIP path: every constant below is written out
 * here from its published value.
 *
 * Conventions (Methods, "Spin Hamiltonian and effective fields"):
 *   - spins are unit vectors, parameters in meV, fields b in meV,
 *     B = b / (mu * mu_B) in tesla;
 *   - site index i = x + Lx*(y + Ly*(z + Lz*a)), sublattice a outermost;
 *   - state arrays are structure-of-arrays planes S[3][N].
 * Every function is a direct transcription of the definition it cites; no
 * blocking, fusion or reordering beyond that definition.  OpenMP is used only
 * over independent sites; every reduction is a serial loop in site order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- physical constants (CODATA 2018) ---------------------------------- */
/* mu_B in meV/T; the paper quotes 5.7884e-2 (Methods, Bohr magneton eq.). */
#define OR_MU_B 5.7883818060e-2
/* k_B in meV/K (stochastic LLG: k_B T in meV). */
#define OR_K_B 8.617333262e-2
/* gyromagnetic ratio in rad / (fs T). */
#define OR_GAMMA 1.76085963023e-4
/* mu0/(4 pi) * mu_B^2 expressed in meV nm^3, from SI values. */
static double or_dip_prefactor(void) {
    const double mu0_4pi = 1.0e-7;            /* T m / A */
    const double muB_J = 9.2740100783e-24;    /* J / T   */
    const double meV_J = 1.602176634e-22;     /* J / meV */
    return mu0_4pi * muB_J * muB_J / meV_J * 1.0e27; /* m^3 -> nm^3 */
}
double or_const(int which) {
    switch (which) {
    case 0: return OR_MU_B;
    case 1: return OR_K_B;
    case 2: return OR_GAMMA;
    case 3: return or_dip_prefactor();
    default: return NAN;
    }
}

/* ---- lattice geometry -------------------------------------------------- */
typedef struct {
    int n_sub;
    int L[3];
    int periodic[3];
    double cell[3][3];   /* rows are lattice vectors (nm) */
    const double *frac;  /* [n_sub][3] */
} or_lat;

static void or_lat_fill(or_lat *lt, int n_sub, const int *L, const int *per,
                        const double *cell9, const double *frac) {
    lt->n_sub = n_sub;
    for (int k = 0; k < 3; ++k) { lt->L[k] = L[k]; lt->periodic[k] = per[k]; }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) lt->cell[r][c] = cell9[3 * r + c];
    lt->frac = frac;
}

static long or_nsites(const or_lat *lt) {
    return (long)lt->n_sub * lt->L[0] * lt->L[1] * lt->L[2];
}

/* cartesian vector of fractional coordinates f: r = sum_k f_k a_k */
static void or_frac_to_cart(const or_lat *lt, const double f[3], double r[3]) {
    for (int c = 0; c < 3; ++c)
        r[c] = f[0] * lt->cell[0][c] + f[1] * lt->cell[1][c] + f[2] * lt->cell[2][c];
}

static double or_norm3(const double v[3]) {
    return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

/* smallest distance between parallel lattice planes (used to size boxes) */
static double or_min_height(const or_lat *lt) {
    double vol, best = INFINITY;
    double c01[3], c12[3], c20[3];
    const double (*a)[3] = lt->cell;
    c01[0] = a[0][1] * a[1][2] - a[0][2] * a[1][1];
    c01[1] = a[0][2] * a[1][0] - a[0][0] * a[1][2];
    c01[2] = a[0][0] * a[1][1] - a[0][1] * a[1][0];
    c12[0] = a[1][1] * a[2][2] - a[1][2] * a[2][1];
    c12[1] = a[1][2] * a[2][0] - a[1][0] * a[2][2];
    c12[2] = a[1][0] * a[2][1] - a[1][1] * a[2][0];
    c20[0] = a[2][1] * a[0][2] - a[2][2] * a[0][1];
    c20[1] = a[2][2] * a[0][0] - a[2][0] * a[0][2];
    c20[2] = a[2][0] * a[0][1] - a[2][1] * a[0][0];
    vol = fabs(a[0][0] * c12[0] + a[0][1] * c12[1] + a[0][2] * c12[2]);
    if (or_norm3(c12) > 0) best = fmin(best, vol / or_norm3(c12));
    if (or_norm3(c20) > 0) best = fmin(best, vol / or_norm3(c20));
    if (or_norm3(c01) > 0) best = fmin(best, vol / or_norm3(c01));
    return best;
}

static double or_length_scale(const or_lat *lt) {
    double s = 0;
    for (int r = 0; r < 3; ++r) s = fmax(s, or_norm3(lt->cell[r]));
    return s;
}

static int cmp_double(const void *pa, const void *pb) {
    double a = *(const double *)pa, b = *(const double *)pb;
    return (a > b) - (a < b);
}

/*
 * Distinct neighbour distances ("shells") in ascending order, over every
 * sublattice pair (a <- b) and cell displacement.  Equal distances are merged
 * with an absolute tolerance of 1e-9 times the longest lattice vector.
 * Returns the number of shells written (<= n_max).
 */
int or_shell_distances(int n_sub, const double *cell9, const double *frac, int n_max,
                       double *out) {
    or_lat lt;
    int L1[3] = {1, 1, 1}, per[3] = {1, 1, 1};
    or_lat_fill(&lt, n_sub, L1, per, cell9, frac);
    const double tol = 1e-9 * or_length_scale(&lt);
    const double h = or_min_height(&lt);
    int M = 2;
    for (;;) {
        long cap = (long)n_sub * n_sub * (2 * M + 1) * (2 * M + 1) * (2 * M + 1);
        double *d = (double *)malloc(sizeof(double) * cap);
        long nd = 0;
        for (int a = 0; a < n_sub; ++a)
            for (int b = 0; b < n_sub; ++b)
                for (int dz = -M; dz <= M; ++dz)
                    for (int dy = -M; dy <= M; ++dy)
                        for (int dx = -M; dx <= M; ++dx) {
                            double f[3], r[3];
                            f[0] = dx + frac[3 * b + 0] - frac[3 * a + 0];
                            f[1] = dy + frac[3 * b + 1] - frac[3 * a + 1];
                            f[2] = dz + frac[3 * b + 2] - frac[3 * a + 2];
                            or_frac_to_cart(&lt, f, r);
                            double dd = or_norm3(r);
                            if (dd > tol) d[nd++] = dd;
                        }
        qsort(d, nd, sizeof(double), cmp_double);
        int ns = 0;
        for (long k = 0; k < nd && ns < n_max; ++k)
            if (ns == 0 || d[k] - out[ns - 1] > tol) out[ns++] = d[k];
        free(d);
        /* every vector of length <= the last shell lies inside a box of
           half-width last/h + 2 cells (fractional offsets are below one cell) */
        if (ns > 0 && M >= (int)ceil(out[ns - 1] / h) + 2) return ns;
        M *= 2;
        if (M > 64) return -1;
    }
}

/* Bilinear 3x3 tensor of one directed bond (Methods, bilinear tensor):
   J = J_s * I + antisymmetric DMI matrix built from D = D_s * rhat. */
static void or_bond_tensor(double Js, double Ds, const double rhat[3], double J[9]) {
    double Dx = Ds * rhat[0], Dy = Ds * rhat[1], Dz = Ds * rhat[2];
    J[0] = Js;  J[1] = Dz;  J[2] = -Dy;
    J[3] = -Dz; J[4] = Js;  J[5] = Dx;
    J[6] = Dy;  J[7] = -Dx; J[8] = Js;
}

/*
 * Directed-bond table: every (target sublattice a, source sublattice b, cell
 * offset delta) whose distance falls in one of the first n_shells shells and
 * whose coupling is non-zero.  D_shell may be NULL (no DMI).  The DMI vector
 * points along the bond from target to source (r_j - r_i), so D_ji = -D_ij.
 * Returns the number of bonds, or -1 if max_bonds is too small / shells fail.
 */
int or_build_bonds(int n_sub, const double *cell9, const double *frac, int n_shells,
                   const double *J_shell, const double *D_shell, int max_bonds,
                   int *b_a, int *b_b, int *b_delta, double *b_J, int *b_shell) {
    double *sh = (double *)malloc(sizeof(double) * (n_shells + 1));
    int ns = or_shell_distances(n_sub, cell9, frac, n_shells, sh);
    if (ns < n_shells) { free(sh); return -1; }
    or_lat lt;
    int L1[3] = {1, 1, 1}, per[3] = {1, 1, 1};
    or_lat_fill(&lt, n_sub, L1, per, cell9, frac);
    const double tol = 1e-9 * or_length_scale(&lt);
    const double h = or_min_height(&lt);
    const int M = (int)ceil(sh[n_shells - 1] / h) + 2;
    int nb = 0;
    for (int a = 0; a < n_sub; ++a)
        for (int b = 0; b < n_sub; ++b)
            for (int dz = -M; dz <= M; ++dz)
                for (int dy = -M; dy <= M; ++dy)
                    for (int dx = -M; dx <= M; ++dx) {
                        double f[3], r[3];
                        f[0] = dx + frac[3 * b + 0] - frac[3 * a + 0];
                        f[1] = dy + frac[3 * b + 1] - frac[3 * a + 1];
                        f[2] = dz + frac[3 * b + 2] - frac[3 * a + 2];
                        or_frac_to_cart(&lt, f, r);
                        double d = or_norm3(r);
                        if (d <= tol) continue;
                        int s = -1;
                        for (int k = 0; k < n_shells; ++k)
                            if (fabs(d - sh[k]) <= tol) { s = k; break; }
                        if (s < 0) continue;
                        double Js = J_shell[s];
                        double Ds = D_shell ? D_shell[s] : 0.0;
                        if (Js == 0.0 && Ds == 0.0) continue;
                        if (nb >= max_bonds) { free(sh); return -1; }
                        double rhat[3] = {r[0] / d, r[1] / d, r[2] / d};
                        b_a[nb] = a;
                        b_b[nb] = b;
                        b_delta[3 * nb + 0] = dx;
                        b_delta[3 * nb + 1] = dy;
                        b_delta[3 * nb + 2] = dz;
                        or_bond_tensor(Js, Ds, rhat, b_J + 9 * nb);
                        if (b_shell) b_shell[nb] = s;
                        ++nb;
                    }
    free(sh);
    return nb;
}

/* ---- model --------------------------------------------------------------- */
typedef struct {
    int n_bonds;
    const int *b_a, *b_b, *b_delta;
    const double *b_J;
    int n_aniso;              /* axes per sublattice */
    const double *K;          /* [n_sub][n_aniso] meV */
    const double *K_axis;     /* [n_sub][n_aniso][3] unit vectors */
    double B[3];              /* tesla */
    const double *mu;         /* [n_sub] in mu_B */
    int dipolar;              /* 1: open-boundary direct dipolar sum */
} or_model;

static void or_model_fill(or_model *m, int n_bonds, const int *b_a, const int *b_b,
                          const int *b_delta, const double *b_J, int n_aniso,
                          const double *K, const double *K_axis, const double *B3,
                          const double *mu, int dipolar) {
    m->n_bonds = n_bonds; m->b_a = b_a; m->b_b = b_b; m->b_delta = b_delta; m->b_J = b_J;
    m->n_aniso = n_aniso; m->K = K; m->K_axis = K_axis;
    m->B[0] = B3[0]; m->B[1] = B3[1]; m->B[2] = B3[2];
    m->mu = mu; m->dipolar = dipolar;
}

/* source site of a bond from cell (x,y,z), or -1 if it leaves an open face */
static long or_bond_source(const or_lat *lt, int x, int y, int z, int b, const int *delta) {
    int c[3] = {x + delta[0], y + delta[1], z + delta[2]};
    for (int k = 0; k < 3; ++k) {
        if (c[k] < 0 || c[k] >= lt->L[k]) {
            if (!lt->periodic[k]) return -1;
            c[k] %= lt->L[k];
            if (c[k] < 0) c[k] += lt->L[k];
        }
    }
    return c[0] + (long)lt->L[0] * (c[1] + (long)lt->L[1] * (c[2] + (long)lt->L[2] * b));
}

/*
 * Reduced bilinear field (Methods, sublattice convolution):
 *   b_a(R) = sum_b sum_delta K_ab(delta) S_b(R + delta),
 * periodic axes wrap, open axes drop missing neighbours (truncation).
 */
static void or_field_bil(const or_lat *lt, const or_model *m, const double *S, double *b) {
    const long N = or_nsites(lt);
    const int Lx = lt->L[0], Ly = lt->L[1], Lz = lt->L[2];
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        int x = (int)(i % Lx), y = (int)((i / Lx) % Ly), z = (int)((i / ((long)Lx * Ly)) % Lz);
        int a = (int)(i / ((long)Lx * Ly * Lz));
        double acc[3] = {0, 0, 0};
        for (int p = 0; p < m->n_bonds; ++p) {
            if (m->b_a[p] != a) continue;
            long j = or_bond_source(lt, x, y, z, m->b_b[p], m->b_delta + 3 * p);
            if (j < 0) continue;
            const double *J = m->b_J + 9 * p;
            double sj[3] = {S[j], S[N + j], S[2 * N + j]};
            for (int al = 0; al < 3; ++al)
                acc[al] += J[3 * al + 0] * sj[0] + J[3 * al + 1] * sj[1] + J[3 * al + 2] * sj[2];
        }
        b[i] = acc[0]; b[N + i] = acc[1]; b[2 * N + i] = acc[2];
    }
}

/* Zeeman field mu_a mu_B B (Methods, Zeeman term) */
static void or_field_zeeman(const or_lat *lt, const or_model *m, double *b) {
    const long N = or_nsites(lt);
    const long per_sub = N / lt->n_sub;
    for (long i = 0; i < N; ++i) {
        double s = m->mu[i / per_sub] * OR_MU_B;
        b[i] = s * m->B[0]; b[N + i] = s * m->B[1]; b[2 * N + i] = s * m->B[2];
    }
}

/* Uniaxial on-site anisotropy field 2 K (S.n) n, the negative gradient of
   -K (S.n)^2 (Methods, on-site anisotropy). */
static void or_field_aniso(const or_lat *lt, const or_model *m, const double *S, double *b) {
    const long N = or_nsites(lt);
    const long per_sub = N / lt->n_sub;
    for (long i = 0; i < N; ++i) {
        long a = i / per_sub;
        double acc[3] = {0, 0, 0};
        for (int l = 0; l < m->n_aniso; ++l) {
            double K = m->K[a * m->n_aniso + l];
            const double *n = m->K_axis + 3 * (a * m->n_aniso + l);
            double sn = S[i] * n[0] + S[N + i] * n[1] + S[2 * N + i] * n[2];
            for (int c = 0; c < 3; ++c) acc[c] += 2.0 * K * sn * n[c];
        }
        b[i] = acc[0]; b[N + i] = acc[1]; b[2 * N + i] = acc[2];
    }
}

/* cartesian position of site i (nm) */
static void or_site_pos(const or_lat *lt, long i, double r[3]) {
    const int Lx = lt->L[0], Ly = lt->L[1], Lz = lt->L[2];
    int x = (int)(i % Lx), y = (int)((i / Lx) % Ly), z = (int)((i / ((long)Lx * Ly)) % Lz);
    int a = (int)(i / ((long)Lx * Ly * Lz));
    double f[3] = {x + lt->frac[3 * a], y + lt->frac[3 * a + 1], z + lt->frac[3 * a + 2]};
    or_frac_to_cart(lt, f, r);
}

/*
 * Direct dipolar field of a finite open sample at the listed target sites:
 *   b_dip,i = (mu0/4pi) mu_B^2 mu_i sum_{j != i} mu_j [3 rhat (rhat.S_j) - S_j] / r^3,
 * the negative gradient of
 *   H_dip = -(mu0/4pi) mu_B^2 sum_{i<j} mu_i mu_j [3 (S_i.rhat)(S_j.rhat) - S_i.S_j] / r^3.
 * No periodic images, no self term.
 */
void or_dipolar_direct(int n_sub, const int *L, const double *cell9, const double *frac,
                       const double *mu, const double *S, int n_targets, const long *targets,
                       double *out /* [n_targets][3] */) {
    or_lat lt;
    int per[3] = {0, 0, 0};
    or_lat_fill(&lt, n_sub, L, per, cell9, frac);
    const long N = or_nsites(&lt);
    const long per_sub = N / n_sub;
    const double pref = or_dip_prefactor();
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < n_targets; ++t) {
        long i = targets[t];
        double ri[3];
        or_site_pos(&lt, i, ri);
        double acc[3] = {0, 0, 0};
        for (long j = 0; j < N; ++j) {
            if (j == i) continue;
            double rj[3];
            or_site_pos(&lt, j, rj);
            double d[3] = {rj[0] - ri[0], rj[1] - ri[1], rj[2] - ri[2]};
            double r = or_norm3(d);
            double u[3] = {d[0] / r, d[1] / r, d[2] / r};
            double sj[3] = {S[j], S[N + j], S[2 * N + j]};
            double us = u[0] * sj[0] + u[1] * sj[1] + u[2] * sj[2];
            double w = mu[j / per_sub] / (r * r * r);
            for (int c = 0; c < 3; ++c) acc[c] += w * (3.0 * u[c] * us - sj[c]);
        }
        double s = pref * mu[i / per_sub];
        out[3 * t + 0] = s * acc[0];
        out[3 * t + 1] = s * acc[1];
        out[3 * t + 2] = s * acc[2];
    }
}

/* per-term fields; any pointer may be NULL to skip that term */
static void or_fields(const or_lat *lt, const or_model *m, const double *S, double *b_bil,
                      double *b_z, double *b_ani, double *b_dip) {
    const long N = or_nsites(lt);
    if (b_bil) or_field_bil(lt, m, S, b_bil);
    if (b_z) or_field_zeeman(lt, m, b_z);
    if (b_ani) or_field_aniso(lt, m, S, b_ani);
    if (b_dip) {
        if (m->dipolar) {
            long *all = (long *)malloc(sizeof(long) * N);
            double *tmp = (double *)malloc(sizeof(double) * 3 * N);
            double cell9[9];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) cell9[3 * r + c] = lt->cell[r][c];
            for (long i = 0; i < N; ++i) all[i] = i;
            or_dipolar_direct(lt->n_sub, lt->L, cell9, lt->frac, m->mu, S, (int)N, all, tmp);
            for (long i = 0; i < N; ++i)
                for (int c = 0; c < 3; ++c) b_dip[c * N + i] = tmp[3 * i + c];
            free(all); free(tmp);
        } else {
            memset(b_dip, 0, sizeof(double) * 3 * N);
        }
    }
}

/* total reduced field b = b_bil + b_Z + b_ani + b_dip (meV) */
static void or_field_total(const or_lat *lt, const or_model *m, const double *S, double *b) {
    const long N = or_nsites(lt);
    double *t1 = (double *)malloc(sizeof(double) * 3 * N);
    double *t2 = (double *)malloc(sizeof(double) * 3 * N);
    double *t3 = (double *)malloc(sizeof(double) * 3 * N);
    or_fields(lt, m, S, b, t1, t2, t3);
    for (long k = 0; k < 3 * N; ++k) b[k] = b[k] + t1[k] + t2[k] + t3[k];
    free(t1); free(t2); free(t3);
}

/* exported: field with the per-term breakdown (any output may be NULL) */
void or_field(int n_sub, const int *L, const int *per, const double *cell9, const double *frac,
              int n_bonds, const int *b_a, const int *b_b, const int *b_delta, const double *b_J,
              int n_aniso, const double *K, const double *K_axis, const double *B3,
              const double *mu, int dipolar, const double *S, double *b_total, double *b_bil,
              double *b_z, double *b_ani, double *b_dip) {
    or_lat lt;
    or_model m;
    or_lat_fill(&lt, n_sub, L, per, cell9, frac);
    or_model_fill(&m, n_bonds, b_a, b_b, b_delta, b_J, n_aniso, K, K_axis, B3, mu, dipolar);
    if (b_total) or_field_total(&lt, &m, S, b_total);
    or_fields(&lt, &m, S, b_bil, b_z, b_ani, b_dip);
}

/*
 * Energy from the fields (Methods, Hamiltonian terms):
 *   E = -sum_i S_i . (b_bil/2 + b_ani/2 + b_dip/2 + b_Z).
 * terms[0..4] = bilinear, Zeeman, anisotropy, dipolar, total.  Serial sums in
 * site order.
 */
void or_energy(int n_sub, const int *L, const int *per, const double *cell9, const double *frac,
               int n_bonds, const int *b_a, const int *b_b, const int *b_delta, const double *b_J,
               int n_aniso, const double *K, const double *K_axis, const double *B3,
               const double *mu, int dipolar, const double *S, double *terms) {
    or_lat lt;
    or_model m;
    or_lat_fill(&lt, n_sub, L, per, cell9, frac);
    or_model_fill(&m, n_bonds, b_a, b_b, b_delta, b_J, n_aniso, K, K_axis, B3, mu, dipolar);
    const long N = or_nsites(&lt);
    double *f[4];
    for (int k = 0; k < 4; ++k) f[k] = (double *)malloc(sizeof(double) * 3 * N);
    or_fields(&lt, &m, S, f[0], f[1], f[2], f[3]);
    const double w[4] = {0.5, 1.0, 0.5, 0.5}; /* bil, Z, ani, dip */
    double e[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k)
        for (long i = 0; i < N; ++i)
            e[k] -= w[k] * (S[i] * f[k][i] + S[N + i] * f[k][N + i] + S[2 * N + i] * f[k][2 * N + i]);
    for (int k = 0; k < 4; ++k) { terms[k] = e[k]; free(f[k]); }
    terms[4] = e[0] + e[1] + e[2] + e[3];
}

/*
 * Brute-force bilinear field and unordered pair energy, built from positions
 * alone: every site pair and every periodic image within the cutoff of shell
 * n_shells, the coupling taken from the shell of that distance, the DMI vector
 * along the bond (Methods, pair energy -J S_i.S_j - D_ij.(S_i x S_j)).  It uses
 * no bond table.  The pair energy sums each unordered pair once, i.e.
 * pairs (i, j, image n) with i < j, plus (i, i, n) for n in one half-space.
 */
void or_bruteforce(int n_sub, const int *L, const int *per, const double *cell9, const double *frac,
                   int n_shells, const double *J_shell, const double *D_shell, const double *S,
                   double *b_out /* [3][N] */, double *E_pair /* scalar */) {
    or_lat lt;
    or_lat_fill(&lt, n_sub, L, per, cell9, frac);
    const long N = or_nsites(&lt);
    double *sh = (double *)malloc(sizeof(double) * (n_shells + 1));
    or_shell_distances(n_sub, cell9, frac, n_shells, sh);
    const double tol = 1e-9 * or_length_scale(&lt);
    const double rcut = sh[n_shells - 1] + tol;
    const double h = or_min_height(&lt);
    int M[3];
    for (int k = 0; k < 3; ++k)
        M[k] = per[k] ? (int)ceil((rcut / h + 2.0) / L[k]) + 1 : 0;
    double Epair = 0.0;
    for (long i = 0; i < N; ++i) {
        b_out[i] = b_out[N + i] = b_out[2 * N + i] = 0.0;
    }
    for (long i = 0; i < N; ++i) {
        double ri[3];
        or_site_pos(&lt, i, ri);
        double si[3] = {S[i], S[N + i], S[2 * N + i]};
        for (long j = 0; j < N; ++j) {
            double rj[3];
            or_site_pos(&lt, j, rj);
            double sj[3] = {S[j], S[N + j], S[2 * N + j]};
            for (int nz = -M[2]; nz <= M[2]; ++nz)
                for (int ny = -M[1]; ny <= M[1]; ++ny)
                    for (int nx = -M[0]; nx <= M[0]; ++nx) {
                        double shift_f[3] = {(double)nx * L[0], (double)ny * L[1], (double)nz * L[2]};
                        double shift[3];
                        or_frac_to_cart(&lt, shift_f, shift);
                        double d[3] = {rj[0] + shift[0] - ri[0], rj[1] + shift[1] - ri[1],
                                       rj[2] + shift[2] - ri[2]};
                        double r = or_norm3(d);
                        if (r <= tol || r > rcut) continue;
                        int s = -1;
                        for (int k = 0; k < n_shells; ++k)
                            if (fabs(r - sh[k]) <= tol) { s = k; break; }
                        if (s < 0) continue;
                        double Js = J_shell[s], Ds = D_shell ? D_shell[s] : 0.0;
                        double Dv[3] = {Ds * d[0] / r, Ds * d[1] / r, Ds * d[2] / r};
                        /* field on i: J S_j + S_j x D_ij */
                        double cx[3] = {sj[1] * Dv[2] - sj[2] * Dv[1], sj[2] * Dv[0] - sj[0] * Dv[2],
                                        sj[0] * Dv[1] - sj[1] * Dv[0]};
                        b_out[i] += Js * sj[0] + cx[0];
                        b_out[N + i] += Js * sj[1] + cx[1];
                        b_out[2 * N + i] += Js * sj[2] + cx[2];
                        /* unordered pair energy: count (i<j) or (i==j, n in upper half) */
                        int upper = (nz > 0) || (nz == 0 && ny > 0) || (nz == 0 && ny == 0 && nx > 0);
                        if (i < j || (i == j && upper)) {
                            double sxs[3] = {si[1] * sj[2] - si[2] * sj[1], si[2] * sj[0] - si[0] * sj[2],
                                             si[0] * sj[1] - si[1] * sj[0]};
                            Epair += -Js * (si[0] * sj[0] + si[1] * sj[1] + si[2] * sj[2])
                                     - (Dv[0] * sxs[0] + Dv[1] * sxs[1] + Dv[2] * sxs[2]);
                        }
                    }
        }
    }
    if (E_pair) *E_pair = Epair;
    free(sh);
}

/* ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ------------------ */
/* One round: two 32x32->64 products of counter words 0 and 2 with the round
   multipliers; the high halves are xored with the other counter words and the
   key, the low halves pass through; the key is bumped by the Weyl constants
   between rounds.  Ten rounds. */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter for the thermal noise of site i at step n in stream `tag`:
   ctr = (i_lo, i_hi ^ tag, n_lo, n_hi), key = (seed_lo, seed_hi). */
void or_noise_block(uint64_t seed, uint64_t step, uint32_t tag, uint64_t site, uint32_t out[4]) {
    uint32_t ctr[4] = {(uint32_t)site, (uint32_t)(site >> 32) ^ tag, (uint32_t)step,
                       (uint32_t)(step >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* uniform in (0,1): (x + 1/2) / 2^32 */
static double or_u01(uint32_t x) { return ((double)x + 0.5) * 2.3283064365386963e-10; }

/* three standard normals from one block by Box-Muller on (u0,u1) and (u2,u3) */
static void or_eta(uint64_t seed, uint64_t step, uint32_t tag, uint64_t site, double eta[3]) {
    uint32_t blk[4];
    or_noise_block(seed, step, tag, site, blk);
    const double two_pi = 6.283185307179586;
    double r0 = sqrt(-2.0 * log(or_u01(blk[0])));
    double t0 = two_pi * or_u01(blk[1]);
    double r1 = sqrt(-2.0 * log(or_u01(blk[2])));
    double t1 = two_pi * or_u01(blk[3]);
    eta[0] = r0 * cos(t0);
    eta[1] = r0 * sin(t0);
    eta[2] = r1 * cos(t1);
}

/* eta for sites site0 .. site0+N-1 (site0 > 0: a contiguous block of a
   larger lattice, whose counters are the global site indices) */
static void or_thermal_eta_at(uint64_t seed, uint64_t step, uint32_t tag, uint64_t site0, long N,
                              double *eta) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        double e[3];
        or_eta(seed, step, tag, site0 + (uint64_t)i, e);
        eta[i] = e[0]; eta[N + i] = e[1]; eta[2 * N + i] = e[2];
    }
}

void or_thermal_eta(uint64_t seed, uint64_t step, uint32_t tag, long N, double *eta /*[3][N]*/) {
    or_thermal_eta_at(seed, step, tag, 0, N, eta);
}

/* ---- Monte Carlo (Methods, Monte Carlo sampling) ------------------------ */
static void or_cross(const double a[3], const double b[3], double c[3]);
static void or_normalise(double v[3]);
/*
 * Colouring for parallel updates: site (x, y, z, a) gets the colour
 * (x + ky y + kz z + o_a) mod C.  The colouring used is the smallest C >= 2,
 * then the lexicographically smallest (ky, kz, o_1, ..., o_{n_sub-1}) with
 * o_0 = 0 and every coefficient in [0, C), for which no two sites joined by a
 * bond of the model share a colour (checked site by site on the lattice, with
 * the bonds wrapped on periodic axes and dropped at open faces).  Returns C, or
 * 0 if no colouring with C <= cmax exists; coef = (ky, kz, o_0 .. o_{n_sub-1}).
 */
static int or_colour_of(const or_lat *lt, long i, int C, const int *coef) {
    const int Lx = lt->L[0], Ly = lt->L[1], Lz = lt->L[2];
    int x = (int)(i % Lx), y = (int)((i / Lx) % Ly), z = (int)((i / ((long)Lx * Ly)) % Lz);
    int a = (int)(i / ((long)Lx * Ly * Lz));
    long v = (long)x + (long)coef[0] * y + (long)coef[1] * z + coef[2 + a];
    return (int)(((v % C) + C) % C);
}

static int or_colouring_valid(const or_lat *lt, const or_model *m, int C, const int *coef) {
    const long N = or_nsites(lt);
    const int Lx = lt->L[0], Ly = lt->L[1], Lz = lt->L[2];
    for (long i = 0; i < N; ++i) {
        int x = (int)(i % Lx), y = (int)((i / Lx) % Ly), z = (int)((i / ((long)Lx * Ly)) % Lz);
        int a = (int)(i / ((long)Lx * Ly * Lz));
        int ci = or_colour_of(lt, i, C, coef);
        for (int p = 0; p < m->n_bonds; ++p) {
            if (m->b_a[p] != a) continue;
            long j = or_bond_source(lt, x, y, z, m->b_b[p], m->b_delta + 3 * p);
            if (j < 0) continue;
            if (or_colour_of(lt, j, C, coef) == ci) return 0;
        }
    }
    return 1;
}

int or_mc_colouring(int n_sub, const int *L, const int *per, const double *cell9, const double *frac,
                    int n_bonds, const int *b_a, const int *b_b, const int *b_delta, const double *b_J,
                    int cmax, int *coef) {
    or_lat lt;
    or_model m;
    const double zero3[3] = {0, 0, 0};
    or_lat_fill(&lt, n_sub, L, per, cell9, frac);
    or_model_fill(&m, n_bonds, b_a, b_b, b_delta, b_J, 0, NULL, NULL, zero3, NULL, 0);
    const int n_free = 2 + (n_sub - 1);   /* ky, kz, o_1 .. o_{n_sub-1} */
    for (int C = 2; C <= cmax; ++C) {
        long total = 1;
        for (int k = 0; k < n_free; ++k) total *= C;
        for (long t = 0; t < total; ++t) {
            /* lexicographic order: ky most significant */
            long r = t;
            int digits[2 + 16];
            for (int k = n_free - 1; k >= 0; --k) { digits[k] = (int)(r % C); r /= C; }
            coef[0] = digits[0];
            coef[1] = digits[1];
            coef[2] = 0;
            for (int a = 1; a < n_sub; ++a) coef[2 + a] = digits[1 + a];
            if (or_colouring_valid(&lt, &m, C, coef)) return C;
        }
    }
    return 0;
}

/* counter tag of the Monte Carlo random stream */
#define OR_MC_TAG 0x4D430000u

/* local energy of spin s apart from the bilinear and Zeeman part:
   -sum_l K_l (s.n_l)^2 (Methods, on-site anisotropy) */
static double or_aniso_energy(const or_model *m, int a, const double s[3]) {
    double e = 0.0;
    for (int l = 0; l < m->n_aniso; ++l) {
        const double *n = m->K_axis + 3 * (a * m->n_aniso + l);
        double sn = s[0] * n[0] + s[1] * n[1] + s[2] * n[2];
        e -= m->K[a * m->n_aniso + l] * sn * sn;
    }
    return e;
}

/* Orthonormal frame (e1, e2) perpendicular to the unit vector e3: e1 =
   normalize(e3 x a) with a the Cartesian axis least aligned with e3 (first on
   ties), e2 = e3 x e1. */
static void or_frame(const double e3[3], double e1[3], double e2[3]) {
    int k = 0;
    double best = fabs(e3[0]);
    if (fabs(e3[1]) < best) { best = fabs(e3[1]); k = 1; }
    if (fabs(e3[2]) < best) { best = fabs(e3[2]); k = 2; }
    double ax[3] = {0, 0, 0};
    ax[k] = 1.0;
    or_cross(e3, ax, e1);
    or_normalise(e1);
    or_cross(e3, e1, e2);
}

/*
 * Heat-bath draw (Methods, Monte Carlo sampling): S ~ exp(beta b.S) on the unit
 * sphere.  With x = beta |b| the cosine to b has density proportional to
 * exp(x c) on [-1, 1], sampled by inverting its distribution function,
 * c = 1 + log1p((1 - u0) expm1(-2x)) / x (c = 2 u0 - 1 for x = 0), and the
 * azimuth is 2 pi u1 in the frame of or_frame around b (around z for b = 0).
 */
static void or_heatbath_draw(const double b[3], double beta, double u0, double u1, double s[3]) {
    double bn = or_norm3(b);
    double x = beta * bn;
    double c = (x > 0.0) ? 1.0 + log1p((1.0 - u0) * expm1(-2.0 * x)) / x : 2.0 * u0 - 1.0;
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    double e3[3] = {0.0, 0.0, 1.0};
    if (bn > 0.0) for (int k = 0; k < 3; ++k) e3[k] = b[k] / bn;
    double e1[3], e2[3];
    or_frame(e3, e1, e2);
    double st = sqrt(fmax(0.0, 1.0 - c * c));
    double phi = 6.283185307179586 * u1;
    double cp = cos(phi), sp = sin(phi);
    for (int k = 0; k < 3; ++k) s[k] = c * e3[k] + st * (cp * e1[k] + sp * e2[k]);
}

/*
 * n_sweeps Monte Carlo sweeps at temperature T_K (Methods, Monte Carlo
 * sampling).  A sweep visits the colours 0 .. C-1 (or_mc_colouring); within a
 * colour every site of that colour is updated once, in site order, against
 * the local field of the other spins, b_i = sum_j J_ij S_j + mu_i mu_B B
 * (no two sites of one colour interact, so the order inside a colour does not
 * matter).  The random numbers of site i in sweep n are one Philox block with
 * counter (i, tag, n) as for the thermal noise, tag OR_MC_TAG, uniforms
 * (x + 1/2) 2^-32.
 *   method 0, heat-bath: S_i drawn from exp(beta b_i.S) (u0, u1); the local
 *            energy must be linear in S_i (no anisotropy).
 *   method 1, Metropolis: trial S' uniform on the sphere (z = 2 u0 - 1,
 *            azimuth 2 pi u1), dH = -(S' - S_i).b_i + E_ani(S') - E_ani(S_i),
 *            accepted if u2 < exp(-beta dH).
 * beta = 1 / (k_B T).  Returns the number of accepted moves (heat-bath: every
 * draw), or -1 for an unsupported case (heat-bath with anisotropy, dipolar
 * term, T <= 0).
 */
long or_mc_sweeps(int n_sub, const int *L, const int *per, const double *cell9, const double *frac,
                  int n_bonds, const int *b_a, const int *b_b, const int *b_delta, const double *b_J,
                  int n_aniso, const double *K, const double *K_axis, const double *B3, const double *mu,
                  int dipolar, double *S, double T_K, uint64_t seed, uint64_t sweep0, int n_sweeps,
                  int method, int C, const int *coef) {
    or_lat lt;
    or_model m;
    or_lat_fill(&lt, n_sub, L, per, cell9, frac);
    or_model_fill(&m, n_bonds, b_a, b_b, b_delta, b_J, n_aniso, K, K_axis, B3, mu, dipolar);
    if (dipolar || !(T_K > 0.0) || (method == 0 && n_aniso > 0) || C < 2) return -1;
    const long N = or_nsites(&lt);
    const long per_sub = N / n_sub;
    const double beta = 1.0 / (OR_K_B * T_K);
    double *b = (double *)malloc(sizeof(double) * 3 * N);
    double *bz = (double *)malloc(sizeof(double) * 3 * N);
    or_field_zeeman(&lt, &m, bz);
    long accepted = 0;
    for (int n = 0; n < n_sweeps; ++n) {
        const uint64_t sweep = sweep0 + (uint64_t)n;
        for (int c = 0; c < C; ++c) {
            or_field_bil(&lt, &m, S, b);
            for (long i = 0; i < N; ++i) {
                if (or_colour_of(&lt, i, C, coef) != c) continue;
                double bi[3] = {b[i] + bz[i], b[N + i] + bz[N + i], b[2 * N + i] + bz[2 * N + i]};
                double si[3] = {S[i], S[N + i], S[2 * N + i]};
                uint32_t blk[4];
                or_noise_block(seed, sweep, OR_MC_TAG, (uint64_t)i, blk);
                double u0 = or_u01(blk[0]), u1 = or_u01(blk[1]), u2 = or_u01(blk[2]);
                double sn[3];
                if (method == 0) {
                    or_heatbath_draw(bi, beta, u0, u1, sn);
                    ++accepted;
                } else {
                    double z = 2.0 * u0 - 1.0, r = sqrt(fmax(0.0, 1.0 - z * z));
                    double phi = 6.283185307179586 * u1;
                    double tr[3] = {r * cos(phi), r * sin(phi), z};
                    int a = (int)(i / per_sub);
                    double dH = -((tr[0] - si[0]) * bi[0] + (tr[1] - si[1]) * bi[1] + (tr[2] - si[2]) * bi[2]) +
                                or_aniso_energy(&m, a, tr) - or_aniso_energy(&m, a, si);
                    if (u2 < exp(-beta * dH)) {
                        sn[0] = tr[0]; sn[1] = tr[1]; sn[2] = tr[2];
                        ++accepted;
                    } else {
                        sn[0] = si[0]; sn[1] = si[1]; sn[2] = si[2];
                    }
                }
                S[i] = sn[0]; S[N + i] = sn[1]; S[2 * N + i] = sn[2];
            }
        }
    }
    free(b);
    free(bz);
    return accepted;
}

/* ---- LLG + normalised Heun (Methods, atomistic spin dynamics) ----------- */
static void or_cross(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* f(S,B) = -gamma/(1+alpha^2) [S x B + alpha S x (S x B)] */
static void or_llg_rhs(const double s[3], const double B[3], double alpha, double f[3]) {
    double sxb[3], sxsxb[3];
    or_cross(s, B, sxb);
    or_cross(s, sxb, sxsxb);
    double pre = -OR_GAMMA / (1.0 + alpha * alpha);
    for (int c = 0; c < 3; ++c) f[c] = pre * (sxb[c] + alpha * sxsxb[c]);
}

static void or_normalise(double v[3]) {
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n; v[1] /= n; v[2] /= n;
}

/*
 * n_steps normalised Heun steps of the (stochastic) LLG equation, in place.
 * Predictor S~ = N[S + dt f(S)], corrector S' = N[S + dt/2 (f(S) + f(S~))].
 * For T > 0 the thermal field sigma_i eta_i^n, sigma_i =
 * sqrt(2 alpha k_B T / (gamma mu_i mu_B dt)), is added to B in both stages
 * with the same eta (Stratonovich Heun); eta for step n = step0 + k.
 * The noise counter of local site i is site0 + i (site0 = 0 for a whole
 * lattice; a z-slab of a larger single-sublattice lattice passes the global
 * index of its first site).
 */
void or_heun(int n_sub, const int *L, const int *per, const double *cell9, const double *frac,
             int n_bonds, const int *b_a, const int *b_b, const int *b_delta, const double *b_J,
             int n_aniso, const double *K, const double *K_axis, const double *B3,
             const double *mu, int dipolar, double alpha, double dt_fs, double T_K,
             uint64_t seed, uint64_t step0, uint32_t tag, uint64_t site0, int n_steps, double *S) {
    or_lat lt;
    or_model m;
    or_lat_fill(&lt, n_sub, L, per, cell9, frac);
    or_model_fill(&m, n_bonds, b_a, b_b, b_delta, b_J, n_aniso, K, K_axis, B3, mu, dipolar);
    const long N = or_nsites(&lt);
    const long per_sub = N / n_sub;
    double *b = (double *)malloc(sizeof(double) * 3 * N);
    double *f0 = (double *)malloc(sizeof(double) * 3 * N);
    double *St = (double *)malloc(sizeof(double) * 3 * N);
    double *eta = (double *)malloc(sizeof(double) * 3 * N);
    for (int k = 0; k < n_steps; ++k) {
        uint64_t step = step0 + (uint64_t)k;
        if (T_K > 0.0) or_thermal_eta_at(seed, step, tag, site0, N, eta);
        /* predictor */
        or_field_total(&lt, &m, S, b);
        for (long i = 0; i < N; ++i) {
            double mu_i = mu[i / per_sub];
            double s[3] = {S[i], S[N + i], S[2 * N + i]};
            double B[3];
            for (int c = 0; c < 3; ++c) B[c] = b[c * N + i] / (mu_i * OR_MU_B);
            if (T_K > 0.0) {
                double sig = sqrt(2.0 * alpha * OR_K_B * T_K / (OR_GAMMA * mu_i * OR_MU_B * dt_fs));
                for (int c = 0; c < 3; ++c) B[c] += sig * eta[c * N + i];
            }
            double f[3];
            or_llg_rhs(s, B, alpha, f);
            double p[3];
            for (int c = 0; c < 3; ++c) { f0[c * N + i] = f[c]; p[c] = s[c] + dt_fs * f[c]; }
            or_normalise(p);
            for (int c = 0; c < 3; ++c) St[c * N + i] = p[c];
        }
        /* corrector */
        or_field_total(&lt, &m, St, b);
        for (long i = 0; i < N; ++i) {
            double mu_i = mu[i / per_sub];
            double st[3] = {St[i], St[N + i], St[2 * N + i]};
            double B[3];
            for (int c = 0; c < 3; ++c) B[c] = b[c * N + i] / (mu_i * OR_MU_B);
            if (T_K > 0.0) {
                double sig = sqrt(2.0 * alpha * OR_K_B * T_K / (OR_GAMMA * mu_i * OR_MU_B * dt_fs));
                for (int c = 0; c < 3; ++c) B[c] += sig * eta[c * N + i];
            }
            double f[3];
            or_llg_rhs(st, B, alpha, f);
            double p[3];
            for (int c = 0; c < 3; ++c) p[c] = S[c * N + i] + 0.5 * dt_fs * (f0[c * N + i] + f[c]);
            or_normalise(p);
            for (int c = 0; c < 3; ++c) S[c * N + i] = p[c];
        }
    }
    free(b); free(f0); free(St); free(eta);
}

/* ---- spin-manifold geometry (Methods, static optimisation and MEPs) ------ */
/* geodesic angle between unit vectors: atan2(|a x b|, a.b), which equals
   arccos(a.b) but stays accurate near 0 and pi */
static double or_angle(const double a[3], const double b[3]) {
    double c[3];
    or_cross(a, b, c);
    return atan2(or_norm3(c), a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
}

/* exponential-map retraction cos|u| S + sin|u| u/|u| (u tangent at S);
   |u| = 0 returns S */
static void or_expmap(const double s[3], const double u[3], double out[3]) {
    double un = or_norm3(u);
    if (un == 0.0) { out[0] = s[0]; out[1] = s[1]; out[2] = s[2]; return; }
    double c = cos(un), sn = sin(un) / un;
    for (int k = 0; k < 3; ++k) out[k] = c * s[k] + sn * u[k];
    or_normalise(out);
}

/* image distance d(Y_n, Y_m) = [sum_i angle(S_i^n, S_i^m)^2]^(1/2) */
double or_image_distance(long N, const double *A, const double *B) {
    double acc = 0.0;
    for (long i = 0; i < N; ++i) {
        double a[3] = {A[i], A[N + i], A[2 * N + i]};
        double b[3] = {B[i], B[N + i], B[2 * N + i]};
        double t = or_angle(a, b);
        acc += t * t;
    }
    return sqrt(acc);
}

/*
 * Point at fraction t of the great-circle arc from a to b (unit vectors):
 * cos(t w) a + sin(t w) e, e = unit tangent of b at a, w = angle(a, b).  If
 * the tangent part |b - (a.b) a| is below 1e-10 the spins are parallel (the
 * point is a) or antiparallel; for antiparallel spins the arc is the rotation
 * by w = pi about the axis k = normalize(a x e_k), e_k the Cartesian axis
 * least aligned with a (first such axis on ties), so e = k x a.
 */
static void or_geodesic_point(const double a[3], const double b[3], double t, double p[3]) {
    double dot = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    double w3[3] = {b[0] - dot * a[0], b[1] - dot * a[1], b[2] - dot * a[2]};
    double wn = or_norm3(w3);
    double e[3], ang;
    if (wn < 1e-10) {
        if (dot > 0) { p[0] = a[0]; p[1] = a[1]; p[2] = a[2]; return; }
        int k = 0;
        double best = fabs(a[0]);
        if (fabs(a[1]) < best) { best = fabs(a[1]); k = 1; }
        if (fabs(a[2]) < best) { best = fabs(a[2]); k = 2; }
        double ek[3] = {0, 0, 0};
        ek[k] = 1.0;
        double ax[3];
        or_cross(a, ek, ax);
        or_normalise(ax);
        or_cross(ax, a, e); /* rotation of a about ax by +90 degrees */
        ang = M_PI;
    } else {
        for (int c = 0; c < 3; ++c) e[c] = w3[c] / wn;
        ang = atan2(wn, dot);
    }
    for (int c = 0; c < 3; ++c) p[c] = cos(t * ang) * a[c] + sin(t * ang) * e[c];
    or_normalise(p);
}

/* Geodesic initial path: image n of n_img lies at t = n/(n_img-1) on every
   spin's great circle from S_A to S_B (or_geodesic_point). */
void or_geodesic_path(long N, const double *SA, const double *SB, int n_img, double *out) {
    for (int n = 0; n < n_img; ++n) {
        double t = (n_img > 1) ? (double)n / (double)(n_img - 1) : 0.0;
        double *Y = out + (long)n * 3 * N;
        for (long i = 0; i < N; ++i) {
            double a[3] = {SA[i], SA[N + i], SA[2 * N + i]};
            double b[3] = {SB[i], SB[N + i], SB[2 * N + i]};
            double p[3];
            or_geodesic_point(a, b, t, p);
            Y[i] = p[0]; Y[N + i] = p[1]; Y[2 * N + i] = p[2];
        }
    }
}

/*
 * Reparameterisation along the geodesic reaction coordinate (Methods,
 * minimum-energy paths: the string method's second step, and image
 * redistribution).  The reaction coordinate of image n is the arc length
 * s_n = sum_{m<n} d(Y_m, Y_m+1) with the geodesic image distance.  Image n of
 * the new path sits at s*_n = alpha_n s_{n_img-1} (alpha NULL: alpha_n =
 * n/(n_img-1), equal spacing): with k the last image with s_k <= s*_n (k <=
 * n_img-2) and f = (s*_n - s_k)/(s_k+1 - s_k) (0 if that gap is 0), every spin
 * of the new image is the point at fraction f of the great-circle arc from its
 * value in Y_k to its value in Y_k+1.  The end images are kept.  in and out
 * must not overlap.
 */
void or_reparametrize(long N, int n_img, const double *in, const double *alpha, double *out) {
    const long img = 3 * N;
    double *s = (double *)malloc(sizeof(double) * n_img);
    s[0] = 0.0;
    for (int n = 0; n + 1 < n_img; ++n) s[n + 1] = s[n] + or_image_distance(N, in + n * img, in + (n + 1) * img);
    const double total = s[n_img - 1];
    for (int n = 0; n < n_img; ++n) {
        double *Y = out + (long)n * img;
        if (n == 0 || n == n_img - 1) {
            memcpy(Y, in + (long)n * img, sizeof(double) * img);
            continue;
        }
        const double a = alpha ? alpha[n] : (double)n / (double)(n_img - 1);
        const double target = a * total;
        int k = 0;
        while (k + 1 < n_img - 1 && s[k + 1] <= target) ++k;
        const double gap = s[k + 1] - s[k];
        double f = gap > 0.0 ? (target - s[k]) / gap : 0.0;
        if (f < 0.0) f = 0.0;
        if (f > 1.0) f = 1.0;
        const double *Ya = in + (long)k * img, *Yb = in + (long)(k + 1) * img;
        for (long i = 0; i < N; ++i) {
            double pa[3] = {Ya[i], Ya[N + i], Ya[2 * N + i]};
            double pb[3] = {Yb[i], Yb[N + i], Yb[2 * N + i]};
            double p[3];
            or_geodesic_point(pa, pb, f, p);
            Y[i] = p[0]; Y[N + i] = p[1]; Y[2 * N + i] = p[2];
        }
    }
    free(s);
}

/*
 * One GNEB iteration with velocity-projection (VP) optimisation and the
 * exponential-map retraction, for n_img images of one lattice; images 0 and
 * n_img-1 are pinned.  Physics (Methods, minimum-energy paths):
 *   F_i   = b_i - (b_i.S_i) S_i                  (projected -grad H, meV)
 *   tau   = upwind/energy-weighted tangent from Y_{n+1}-Y_n and Y_n-Y_{n-1}
 *           (Henkelman-Jonsson), projected per spin, normalised over the image
 *   F_gneb = F - (F.tau)tau + k (d_{n,n+1} - d_{n-1,n}) tau   (ordinary image)
 *   F_ci   = F - 2 (F.tau) tau                                  (climbing image)
 * VP over all movable images: v <- (v.F/F.F) F if v.F > 0 else 0;
 * v += (dt/m) F;  u = P_perp(dt v);  S <- exp_S(u).
 * ci_mode: 0 never, 1 switch on once max|F_gneb| < ci_on_below, 2 always,
 * 3 static minimisation of every movable image (no tangent: F_gneb = F),
 * 4 string method (Methods, minimum-energy paths): every movable image is
 * displaced by its projected physical force, u = dt F, S <- exp_S(u), with no
 * spring, no climbing image and no velocity memory, and the path is then
 * reparameterised along the geodesic reaction coordinate to the spacing alpha
 * (or_reparametrize; NULL: equal spacing); the reported force is the part of
 * F perpendicular to the improved tangent, F - (F.tau)tau.
 * *ci_on carries the switch between calls.  Outputs: energies E[n_img],
 * distances dist[n_img-1], max |F_gneb| per spin over movable images (before
 * the update), the climbing image index (-1 if none).
 */
void or_gneb_iterate(int n_sub, const int *L, const int *per, const double *cell9,
                     const double *frac, int n_bonds, const int *b_a, const int *b_b,
                     const int *b_delta, const double *b_J, int n_aniso, const double *K,
                     const double *K_axis, const double *B3, const double *mu, int n_img,
                     double *Y /* [n_img][3][N] */, double *V /* [n_img][3][N] */,
                     double k_spring, double dt, double mass, int ci_mode, double ci_on_below,
                     int *ci_on, const double *alpha, double *E, double *dist, double *max_force,
                     int *ci_index) {
    or_lat lt;
    or_model m;
    or_lat_fill(&lt, n_sub, L, per, cell9, frac);
    or_model_fill(&m, n_bonds, b_a, b_b, b_delta, b_J, n_aniso, K, K_axis, B3, mu, 0);
    const long N = or_nsites(&lt);
    const long img = 3 * N;
    double *b = (double *)malloc(sizeof(double) * img);
    double *F = (double *)malloc(sizeof(double) * img * n_img);   /* GNEB force */
    double terms[5];
    for (int n = 0; n < n_img; ++n) {
        or_energy(n_sub, L, per, cell9, frac, n_bonds, b_a, b_b, b_delta, b_J, n_aniso, K,
                  K_axis, B3, mu, 0, Y + n * img, terms);
        E[n] = terms[4];
    }
    for (int n = 0; n + 1 < n_img; ++n) dist[n] = or_image_distance(N, Y + n * img, Y + (n + 1) * img);
    int ci = -1;
    if (ci_mode == 2 || (ci_mode == 1 && *ci_on)) {
        for (int n = 1; n + 1 < n_img; ++n)
            if (ci < 0 || E[n] > E[ci]) ci = n;
    }
    double *tau = (double *)malloc(sizeof(double) * img);
    double fperp = 0.0;
    for (int n = 1; n + 1 < n_img; ++n) {
        const double *S = Y + n * img, *Sp = Y + (n + 1) * img, *Sm = Y + (n - 1) * img;
        double *Fn = F + n * img;
        or_field_total(&lt, &m, S, b);
        for (long i = 0; i < N; ++i) {
            double bs = b[i] * S[i] + b[N + i] * S[N + i] + b[2 * N + i] * S[2 * N + i];
            for (int c = 0; c < 3; ++c) Fn[c * N + i] = b[c * N + i] - bs * S[c * N + i];
        }
        /* tangent weights (Henkelman & Jonsson improved tangent) */
        double wp, wm;
        double Ep = E[n + 1], Em = E[n - 1], E0 = E[n];
        if (ci_mode == 3) { wp = 0.0; wm = 0.0; }
        else if (Ep > E0 && E0 > Em) { wp = 1.0; wm = 0.0; }
        else if (Ep < E0 && E0 < Em) { wp = 0.0; wm = 1.0; }
        else {
            double dmax = fmax(fabs(Ep - E0), fabs(Em - E0));
            double dmin = fmin(fabs(Ep - E0), fabs(Em - E0));
            if (Ep > Em) { wp = dmax; wm = dmin; } else { wp = dmin; wm = dmax; }
        }
        double tt = 0.0;
        for (long i = 0; i < N; ++i) {
            double t[3];
            for (int c = 0; c < 3; ++c)
                t[c] = wp * (Sp[c * N + i] - S[c * N + i]) + wm * (S[c * N + i] - Sm[c * N + i]);
            double ts = t[0] * S[i] + t[1] * S[N + i] + t[2] * S[2 * N + i];
            for (int c = 0; c < 3; ++c) { t[c] -= ts * S[c * N + i]; tau[c * N + i] = t[c]; }
            tt += t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
        }
        double tn = sqrt(tt);
        double ft = 0.0;
        for (long i = 0; i < N; ++i) {
            for (int c = 0; c < 3; ++c) tau[c * N + i] = (tn > 0.0) ? tau[c * N + i] / tn : 0.0;
            ft += Fn[i] * tau[i] + Fn[N + i] * tau[N + i] + Fn[2 * N + i] * tau[2 * N + i];
        }
        double coef;
        if (n == ci) coef = -2.0 * ft;
        else if (ci_mode == 4) coef = -ft;
        else coef = -ft + k_spring * (dist[n] - dist[n - 1]);
        if (ci_mode == 4) {
            /* the string step uses F itself; only its perpendicular part is reported */
            for (long i = 0; i < N; ++i) {
                double f2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                    double fp = Fn[c * N + i] + coef * tau[c * N + i];
                    f2 += fp * fp;
                }
                if (sqrt(f2) > fperp) fperp = sqrt(f2);
            }
            continue;
        }
        for (long k2 = 0; k2 < img; ++k2) Fn[k2] += coef * tau[k2];
    }
    if (ci_mode == 4) {
        for (int n = 1; n + 1 < n_img; ++n) {
            double *S = Y + n * img, *Vn = V + n * img;
            const double *Fn = F + n * img;
            for (long i = 0; i < N; ++i) {
                double s[3] = {S[i], S[N + i], S[2 * N + i]};
                double u[3], o[3];
                for (int c = 0; c < 3; ++c) {
                    u[c] = dt * Fn[c * N + i];
                    Vn[c * N + i] = 0.0;
                }
                or_expmap(s, u, o);
                S[i] = o[0]; S[N + i] = o[1]; S[2 * N + i] = o[2];
            }
        }
        double *tmp = (double *)malloc(sizeof(double) * img * n_img);
        or_reparametrize(N, n_img, Y, alpha, tmp);
        memcpy(Y, tmp, sizeof(double) * img * n_img);
        free(tmp);
        *max_force = fperp;
        *ci_index = -1;
        free(b); free(F); free(tau);
        return;
    }
    /* VP projection over all movable images */
    double vf = 0.0, ff = 0.0, fmaxv = 0.0;
    for (int n = 1; n + 1 < n_img; ++n) {
        const double *Fn = F + n * img, *Vn = V + n * img;
        for (long i = 0; i < N; ++i) {
            double f2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                vf += Vn[c * N + i] * Fn[c * N + i];
                f2 += Fn[c * N + i] * Fn[c * N + i];
            }
            ff += f2;
            if (sqrt(f2) > fmaxv) fmaxv = sqrt(f2);
        }
    }
    double proj = (vf > 0.0 && ff > 0.0) ? vf / ff : 0.0;
    for (int n = 1; n + 1 < n_img; ++n) {
        double *S = Y + n * img, *Vn = V + n * img;
        const double *Fn = F + n * img;
        for (long i = 0; i < N; ++i) {
            double s[3] = {S[i], S[N + i], S[2 * N + i]};
            double u[3];
            for (int c = 0; c < 3; ++c) {
                double v = proj * Fn[c * N + i] + (dt / mass) * Fn[c * N + i];
                Vn[c * N + i] = v;
                u[c] = dt * v;
            }
            double us = u[0] * s[0] + u[1] * s[1] + u[2] * s[2];
            for (int c = 0; c < 3; ++c) u[c] -= us * s[c];
            double o[3];
            or_expmap(s, u, o);
            S[i] = o[0]; S[N + i] = o[1]; S[2 * N + i] = o[2];
        }
    }
    *max_force = fmaxv;
    *ci_index = ci;
    if (ci_mode == 1 && !*ci_on && fmaxv < ci_on_below) *ci_on = 1;
    free(b); free(F); free(tau);
}

/* ---- pair-list Hamiltonian (Methods, pair-list backend) ---------------- */
/*
 * Explicit couplings: entry p couples target site i_p to source site j_p with
 * J_p (scalar, or 3x3 row-major if tensor).  Reduced bilinear field
 *   b_i = sum_{p: i_p = i} J_p S_{j_p}
 * (entries summed in list order), plus the site-resolved on-site terms: Zeeman
 * mu_i mu_B B and uniaxial anisotropy 2 K_i (S_i.n_i) n_i.  mu NULL: all 1;
 * K NULL: none.  Outputs b (total) and, if not NULL, b_bil.
 */
static void or_pl_fields(long N, long P, const long *ti, const long *sj, const double *J, int tensor,
                         const double *mu, const double *K, const double *axis, const double *B3,
                         const double *S, double *b, double *b_bil) {
    double *bb = (double *)calloc((size_t)3 * N, sizeof(double));
    for (long p = 0; p < P; ++p) {
        const long i = ti[p], j = sj[p];
        const double s[3] = {S[j], S[N + j], S[2 * N + j]};
        if (tensor) {
            const double *Jp = J + 9 * p;
            for (int al = 0; al < 3; ++al)
                bb[al * N + i] += Jp[3 * al] * s[0] + Jp[3 * al + 1] * s[1] + Jp[3 * al + 2] * s[2];
        } else {
            for (int al = 0; al < 3; ++al) bb[al * N + i] += J[p] * s[al];
        }
    }
    for (long i = 0; i < N; ++i) {
        const double m = mu ? mu[i] : 1.0;
        double an[3] = {0, 0, 0};
        if (K) {
            const double *n = axis + 3 * i;
            double sn = S[i] * n[0] + S[N + i] * n[1] + S[2 * N + i] * n[2];
            for (int c = 0; c < 3; ++c) an[c] = 2.0 * K[i] * sn * n[c];
        }
        for (int c = 0; c < 3; ++c) {
            b[c * N + i] = bb[c * N + i] + m * OR_MU_B * B3[c] + an[c];
            if (b_bil) b_bil[c * N + i] = bb[c * N + i];
        }
    }
    free(bb);
}

void or_pl_field(long N, long P, const long *ti, const long *sj, const double *J, int tensor, const double *mu,
                 const double *K, const double *axis, const double *B3, const double *S, double *b) {
    or_pl_fields(N, P, ti, sj, J, tensor, mu, K, axis, B3, S, b, NULL);
}

/* E terms [bilinear, Zeeman, anisotropy, dipolar (0), total]:
   -1/2 sum S.b_bil, -sum mu mu_B B.S, -sum K (S.n)^2 */
void or_pl_energy(long N, long P, const long *ti, const long *sj, const double *J, int tensor, const double *mu,
                  const double *K, const double *axis, const double *B3, const double *S, double *terms) {
    double *b = (double *)malloc(sizeof(double) * 3 * N);
    double *bb = (double *)malloc(sizeof(double) * 3 * N);
    or_pl_fields(N, P, ti, sj, J, tensor, mu, K, axis, B3, S, b, bb);
    double eb = 0.0, ez = 0.0, ea = 0.0;
    for (long i = 0; i < N; ++i) {
        const double s[3] = {S[i], S[N + i], S[2 * N + i]};
        const double m = mu ? mu[i] : 1.0;
        eb += -0.5 * (s[0] * bb[i] + s[1] * bb[N + i] + s[2] * bb[2 * N + i]);
        ez += -m * OR_MU_B * (s[0] * B3[0] + s[1] * B3[1] + s[2] * B3[2]);
        if (K) {
            const double *n = axis + 3 * i;
            double sn = s[0] * n[0] + s[1] * n[1] + s[2] * n[2];
            ea += -K[i] * sn * sn;
        }
    }
    terms[0] = eb; terms[1] = ez; terms[2] = ea; terms[3] = 0.0; terms[4] = eb + ez + ea;
    free(b);
    free(bb);
}

static void or_llg_rhs(const double s[3], const double B[3], double alpha, double f[3]);

/* n_steps normalised Heun steps with the pair-list field: the same algorithm
   as or_heun (predictor, corrector, the same eta in both stages, noise
   counter = site index), with the site's own moment mu_i. */
void or_pl_heun(long N, long P, const long *ti, const long *sj, const double *J, int tensor, const double *mu,
                const double *K, const double *axis, const double *B3, double alpha, double dt_fs, double T_K,
                uint64_t seed, uint64_t step0, uint32_t tag, int n_steps, double *S) {
    double *b = (double *)malloc(sizeof(double) * 3 * N);
    double *f0 = (double *)malloc(sizeof(double) * 3 * N);
    double *St = (double *)malloc(sizeof(double) * 3 * N);
    double *eta = (double *)malloc(sizeof(double) * 3 * N);
    for (int k = 0; k < n_steps; ++k) {
        uint64_t step = step0 + (uint64_t)k;
        if (T_K > 0.0) or_thermal_eta_at(seed, step, tag, 0, N, eta);
        for (int stage = 0; stage < 2; ++stage) {
            const double *X = stage == 0 ? S : St;
            or_pl_fields(N, P, ti, sj, J, tensor, mu, K, axis, B3, X, b, NULL);
            for (long i = 0; i < N; ++i) {
                const double mu_i = mu ? mu[i] : 1.0;
                double x[3] = {X[i], X[N + i], X[2 * N + i]};
                double B[3];
                for (int c = 0; c < 3; ++c) B[c] = b[c * N + i] / (mu_i * OR_MU_B);
                if (T_K > 0.0) {
                    double sig = sqrt(2.0 * alpha * OR_K_B * T_K / (OR_GAMMA * mu_i * OR_MU_B * dt_fs));
                    for (int c = 0; c < 3; ++c) B[c] += sig * eta[c * N + i];
                }
                double f[3], p[3];
                or_llg_rhs(x, B, alpha, f);
                if (stage == 0) {
                    for (int c = 0; c < 3; ++c) { f0[c * N + i] = f[c]; p[c] = S[c * N + i] + dt_fs * f[c]; }
                    or_normalise(p);
                    for (int c = 0; c < 3; ++c) St[c * N + i] = p[c];
                } else {
                    for (int c = 0; c < 3; ++c) p[c] = S[c * N + i] + 0.5 * dt_fs * (f0[c * N + i] + f[c]);
                    or_normalise(p);
                    for (int c = 0; c < 3; ++c) S[c * N + i] = p[c];
                }
            }
        }
    }
    free(b); free(f0); free(St); free(eta);
}

/* ---- static minimisation (Methods, static optimisation and MEPs) -------- */
/*
 * One iteration of a static minimiser on the product of unit spheres.  The
 * force F_i = b_i - (b_i.S_i) S_i is minus the tangent gradient G_i; max |F_i|
 * (before the update) is returned in *max_force.  The step u_i is
 *   method 0, velocity projection: P = sum v.F, Q = sum F.F over all spins;
 *             v <- (P/Q) F (if P > 0, else 0) + (dt/mass) F;  u = dt v;
 *   method 1, Barzilai-Borwein (BB1): alpha = sum s.s / sum s.y with
 *             s = P(u_prev) and y = G - P(G_prev) (P: projection on the current
 *             tangent planes), alpha = dt on the first iteration or when
 *             sum s.y <= 0;  u = alpha F;
 *   method 2, L-BFGS: the pair (s, y) above joins the history (at most hist
 *             pairs, oldest dropped) when s.y > 0; the two-loop recursion from
 *             q = G with the stored pairs projected on the current tangent
 *             planes, initial scale gamma = s.y / y.y of the newest pair (dt
 *             without pairs), gives r, and u = -r (u = dt F with no pairs);
 *   method 3, Adam: m <- b1 m + (1 - b1) G, w <- b2 w + (1 - b2) G*G (per
 *             Cartesian component), u = -dt m^ / (sqrt(w^) + eps) with the
 *             bias corrections m^ = m / (1 - b1^t), w^ = w / (1 - b2^t), t the
 *             iteration count from 1;
 * then u_i is projected on the tangent plane of S_i, scaled down to
 * |u_i| = max_step if longer (max_step > 0), and retracted:
 *   retraction 0, exponential map: S <- cos|u| S + sin|u| u/|u| (then normalised);
 *   retraction 1, normalised: S <- (S + u) / |S + u|.
 * State (caller-owned, zero at the start): work = [V | W | Fp | Up | s_0 ..
 * s_{hist-1} | y_0 .. y_{hist-1} | rho_0 .. rho_{hist-1}] (each block 3N
 * doubles, rho hist doubles), ist = [iteration, pairs stored, newest slot].
 */
static double or_dot3N(long n3, const double *a, const double *b) {
    double t = 0.0;
    for (long k = 0; k < n3; ++k) t += a[k] * b[k];
    return t;
}

/* x <- x - (x.S) S per spin */
static void or_tangent(long N, const double *S, double *x) {
    for (long i = 0; i < N; ++i) {
        double d = x[i] * S[i] + x[N + i] * S[N + i] + x[2 * N + i] * S[2 * N + i];
        for (int c = 0; c < 3; ++c) x[c * N + i] -= d * S[c * N + i];
    }
}

void or_min_iterate(int n_sub, const int *L, const int *per, const double *cell9, const double *frac,
                    int n_bonds, const int *b_a, const int *b_b, const int *b_delta, const double *b_J,
                    int n_aniso, const double *K, const double *K_axis, const double *B3, const double *mu,
                    int dipolar, double *S, int method, int retraction, double dt, double mass, int hist,
                    double b1, double b2, double eps, double max_step, double *work, long *ist,
                    double *max_force) {
    or_lat lt;
    or_model m;
    or_lat_fill(&lt, n_sub, L, per, cell9, frac);
    or_model_fill(&m, n_bonds, b_a, b_b, b_delta, b_J, n_aniso, K, K_axis, B3, mu, dipolar);
    const long N = or_nsites(&lt), n3 = 3 * N;
    double *V = work, *W = work + n3, *Fp = work + 2 * n3, *Up = work + 3 * n3;
    double *Sh = work + 4 * n3, *Yh = work + (4 + hist) * n3, *rho = work + (4 + 2 * hist) * n3;
    double *b = (double *)malloc(sizeof(double) * n3);
    double *F = (double *)malloc(sizeof(double) * n3);
    double *u = (double *)malloc(sizeof(double) * n3);
    or_field_total(&lt, &m, S, b);
    double fmax = 0.0;
    for (long i = 0; i < N; ++i) {
        double bs = b[i] * S[i] + b[N + i] * S[N + i] + b[2 * N + i] * S[2 * N + i];
        double f2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            F[c * N + i] = b[c * N + i] - bs * S[c * N + i];
            f2 += F[c * N + i] * F[c * N + i];
        }
        if (sqrt(f2) > fmax) fmax = sqrt(f2);
    }
    *max_force = fmax;
    const long k = ist[0];
    if (method == 0) {
        double P = or_dot3N(n3, V, F), Q = or_dot3N(n3, F, F);
        double proj = (P > 0.0 && Q > 0.0) ? P / Q : 0.0;
        for (long q = 0; q < n3; ++q) {
            V[q] = proj * F[q] + (dt / mass) * F[q];
            u[q] = dt * V[q];
        }
    } else if (method == 1 || method == 2) {
        /* s = P(u_prev), y = G - P(G_prev) = -F + P(F_prev) */
        double *sv = (double *)malloc(sizeof(double) * n3);
        double *yv = (double *)malloc(sizeof(double) * n3);
        memcpy(sv, Up, sizeof(double) * n3);
        memcpy(yv, Fp, sizeof(double) * n3);
        or_tangent(N, S, sv);
        or_tangent(N, S, yv);
        for (long q = 0; q < n3; ++q) yv[q] -= F[q];
        double ss = or_dot3N(n3, sv, sv), sy = or_dot3N(n3, sv, yv);
        if (method == 1) {
            double alpha = (k > 0 && sy > 0.0) ? ss / sy : dt;
            for (long q = 0; q < n3; ++q) u[q] = alpha * F[q];
        } else {
            if (k > 0 && sy > 0.0) {
                long slot = (ist[1] == 0) ? 0 : (ist[2] + 1) % hist;
                memcpy(Sh + slot * n3, sv, sizeof(double) * n3);
                memcpy(Yh + slot * n3, yv, sizeof(double) * n3);
                rho[slot] = 1.0 / sy;
                ist[2] = slot;
                if (ist[1] < hist) ist[1] += 1;
            }
            const long np = ist[1];
            if (np == 0) {
                for (long q = 0; q < n3; ++q) u[q] = dt * F[q];
            } else {
                double *qv = (double *)malloc(sizeof(double) * n3);
                double *py = (double *)malloc(sizeof(double) * n3);
                double *ps = (double *)malloc(sizeof(double) * n3);
                double *al = (double *)malloc(sizeof(double) * np);
                for (long q = 0; q < n3; ++q) qv[q] = -F[q];
                /* newest to oldest */
                for (long t = 0; t < np; ++t) {
                    long j = ((ist[2] - t) % hist + hist) % hist;
                    memcpy(ps, Sh + j * n3, sizeof(double) * n3);
                    memcpy(py, Yh + j * n3, sizeof(double) * n3);
                    or_tangent(N, S, ps);
                    or_tangent(N, S, py);
                    al[t] = rho[j] * or_dot3N(n3, ps, qv);
                    for (long q = 0; q < n3; ++q) qv[q] -= al[t] * py[q];
                }
                long jn = ist[2];
                memcpy(ps, Sh + jn * n3, sizeof(double) * n3);
                memcpy(py, Yh + jn * n3, sizeof(double) * n3);
                or_tangent(N, S, ps);
                or_tangent(N, S, py);
                double gamma = or_dot3N(n3, ps, py) / or_dot3N(n3, py, py);
                for (long q = 0; q < n3; ++q) qv[q] *= gamma;
                /* oldest to newest */
                for (long t = np - 1; t >= 0; --t) {
                    long j = ((ist[2] - t) % hist + hist) % hist;
                    memcpy(ps, Sh + j * n3, sizeof(double) * n3);
                    memcpy(py, Yh + j * n3, sizeof(double) * n3);
                    or_tangent(N, S, ps);
                    or_tangent(N, S, py);
                    double be = rho[j] * or_dot3N(n3, py, qv);
                    for (long q = 0; q < n3; ++q) qv[q] += (al[t] - be) * ps[q];
                }
                for (long q = 0; q < n3; ++q) u[q] = -qv[q];
                free(qv); free(py); free(ps); free(al);
            }
        }
        free(sv); free(yv);
    } else {
        const double t = (double)(k + 1);
        const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
        for (long q = 0; q < n3; ++q) {
            double g = -F[q];
            V[q] = b1 * V[q] + (1.0 - b1) * g;
            W[q] = b2 * W[q] + (1.0 - b2) * g * g;
            u[q] = -dt * (V[q] / c1) / (sqrt(W[q] / c2) + eps);
        }
    }
    or_tangent(N, S, u);
    for (long i = 0; i < N; ++i) {
        double ui[3] = {u[i], u[N + i], u[2 * N + i]};
        double un = or_norm3(ui);
        if (max_step > 0.0 && un > max_step) {
            for (int c = 0; c < 3; ++c) ui[c] *= max_step / un;
            un = max_step;
        }
        double s3[3] = {S[i], S[N + i], S[2 * N + i]}, o[3];
        if (retraction == 0) {
            or_expmap(s3, ui, o);
        } else {
            for (int c = 0; c < 3; ++c) o[c] = s3[c] + ui[c];
            or_normalise(o);
        }
        for (int c = 0; c < 3; ++c) {
            S[c * N + i] = o[c];
            Up[c * N + i] = ui[c];
            Fp[c * N + i] = F[c * N + i];
        }
    }
    ist[0] = k + 1;
    free(b); free(F); free(u);
}

/* ---- learned path corrector: 3^3 conv net (forward / backward) ---------- */
/*
 * Net: 4 layers of 3x3x3 convolutions with zero padding, channel counts
 * c[0] -> c[1] -> c[2] -> c[3] -> c[4], SiLU after layers 1..3.  Layer l may
 * be dilated by dil[l] (the dilated convolution of Yu & Koltun, ICLR 2016:
 * tap k of the 3^3 kernel reads the input at offset (k - 1) dil[l] per axis);
 * dil == NULL means 1 everywhere.
 * Activations are [C][Lz][Ly][Lx] planes.  Weights of layer l are
 * W[cout][cin][kz][ky][kx] followed by bias[cout], packed layer after layer.
 */
static int or_dil(const int *dil, int l) { return dil ? dil[l] : 1; }

/* v rounded to float, then to bfloat16 (8 significant bits), each to
   nearest even: the operands of a BF16 matrix-core convolution that reads
   FP32 data */
static double or_bf16(double v) {
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static void or_conv3(int Lx, int Ly, int Lz, int cin, int cout, int d, const double *W, const double *bias,
                     const double *in, double *out) {
    const long P = (long)Lx * Ly * Lz;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < P; ++p) {
        int x = (int)(p % Lx), y = (int)((p / Lx) % Ly), z = (int)(p / ((long)Lx * Ly));
        for (int co = 0; co < cout; ++co) {
            double acc = bias[co];
            for (int ci = 0; ci < cin; ++ci)
                for (int kz = 0; kz < 3; ++kz)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx) {
                            int xx = x + (kx - 1) * d, yy = y + (ky - 1) * d, zz = z + (kz - 1) * d;
                            if (xx < 0 || yy < 0 || zz < 0 || xx >= Lx || yy >= Ly || zz >= Lz) continue;
                            acc += W[(((long)co * cin + ci) * 3 + kz) * 9 + ky * 3 + kx] *
                                   in[ci * P + xx + (long)Lx * (yy + (long)Ly * zz)];
                        }
            out[co * P + p] = acc;
        }
    }
}

static double or_sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* number of parameters of the net for channel list c[5] */
long or_net_nparams(const int *c) {
    long n = 0;
    for (int l = 0; l < 4; ++l) n += (long)c[l + 1] * c[l] * 27 + c[l + 1];
    return n;
}

/* forward: input x [c0][P] -> raw output [c4][P]; pre-activations saved in
   `act` (layer outputs before SiLU, [c1+c2+c3+c4][P]) if non-NULL */
/* quant = 1: every layer's weights and inputs rounded by or_bf16 first (the
   emulated operands of the BF16 form); biases and sums stay FP64 */
void or_net_forward_q(int Lx, int Ly, int Lz, const int *c, const int *dil, const double *params,
                      const double *x, double *out, double *act, int quant) {
    const long P = (long)Lx * Ly * Lz;
    const double *cur = x;
    double *buf[4];
    const double *w = params;
    double *qin = NULL, *qw = NULL;
    for (int l = 0; l < 4; ++l) {
        buf[l] = (double *)malloc(sizeof(double) * c[l + 1] * P);
        const double *W = w;
        const double *bias = w + (long)c[l + 1] * c[l] * 27;
        if (quant) {
            const long nin = (long)c[l] * P, nw = (long)c[l + 1] * c[l] * 27;
            qin = (double *)realloc(qin, sizeof(double) * nin);
            qw = (double *)realloc(qw, sizeof(double) * nw);
            for (long k = 0; k < nin; ++k) qin[k] = or_bf16(cur[k]);
            for (long k = 0; k < nw; ++k) qw[k] = or_bf16(W[k]);
            or_conv3(Lx, Ly, Lz, c[l], c[l + 1], or_dil(dil, l), qw, bias, qin, buf[l]);
        } else {
            or_conv3(Lx, Ly, Lz, c[l], c[l + 1], or_dil(dil, l), W, bias, cur, buf[l]);
        }
        w = bias + c[l + 1];
        if (act) {
            long off = 0;
            for (int q = 0; q < l; ++q) off += (long)c[q + 1] * P;
            memcpy(act + off, buf[l], sizeof(double) * c[l + 1] * P);
        }
        if (l < 3)
            for (long k = 0; k < (long)c[l + 1] * P; ++k) buf[l][k] = buf[l][k] * or_sigmoid(buf[l][k]);
        cur = buf[l];
    }
    memcpy(out, buf[3], sizeof(double) * c[4] * P);
    for (int l = 0; l < 4; ++l) free(buf[l]);
    free(qin);
    free(qw);
}

void or_net_forward(int Lx, int Ly, int Lz, const int *c, const int *dil, const double *params,
                    const double *x, double *out, double *act) {
    or_net_forward_q(Lx, Ly, Lz, c, dil, params, x, out, act, 0);
}

/*
 * Predicted image: u = raw output (3 channels) projected onto the tangent plane
 * of the geodesic guess Sg, S_hat = exp_Sg(u).  Loss = mean over sites of
 * |S_hat - S_star|^2.  Returns the loss; writes S_hat if non-NULL.
 */
double or_net_predict_loss(long P, const double *raw, const double *Sg, const double *Sstar,
                           double *Shat) {
    double loss = 0.0;
    for (long p = 0; p < P; ++p) {
        double s[3] = {Sg[p], Sg[P + p], Sg[2 * P + p]};
        double u[3] = {raw[p], raw[P + p], raw[2 * P + p]};
        double us = u[0] * s[0] + u[1] * s[1] + u[2] * s[2];
        for (int c = 0; c < 3; ++c) u[c] -= us * s[c];
        double o[3];
        or_expmap(s, u, o);
        if (Shat) for (int c = 0; c < 3; ++c) Shat[c * P + p] = o[c];
        if (Sstar) {
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                double d = o[c] - Sstar[c * P + p];
                d2 += d * d;
            }
            loss += d2;
        }
    }
    return loss / (double)P;
}

/*
 * Gradient of the loss with respect to all parameters (same packing as
 * params), by the chain rule written out by hand: loss -> exp map -> tangent
 * projection -> conv layers / SiLU.  Returns the loss.
 */
double or_net_backward(int Lx, int Ly, int Lz, const int *c, const int *dil, const double *params,
                       const double *x, const double *Sg, const double *Sstar, double *grad) {
    const long P = (long)Lx * Ly * Lz;
    long tot_act = 0;
    for (int l = 0; l < 4; ++l) tot_act += (long)c[l + 1] * P;
    double *act = (double *)malloc(sizeof(double) * tot_act);
    double *raw = (double *)malloc(sizeof(double) * 3 * P);
    or_net_forward(Lx, Ly, Lz, c, dil, params, x, raw, act);
    double loss = 0.0;
    /* d loss / d raw */
    double *g = (double *)malloc(sizeof(double) * 3 * P);
    for (long p = 0; p < P; ++p) {
        double s[3] = {Sg[p], Sg[P + p], Sg[2 * P + p]};
        double r[3] = {raw[p], raw[P + p], raw[2 * P + p]};
        double rs = r[0] * s[0] + r[1] * s[1] + r[2] * s[2];
        double u[3] = {r[0] - rs * s[0], r[1] - rs * s[1], r[2] - rs * s[2]};
        double th = or_norm3(u);
        double sinc, c2;  /* sin(th)/th and (cos th - sin th/th)/th^2 */
        if (th < 1e-4) {
            double t2 = th * th;
            sinc = 1.0 - t2 / 6.0 + t2 * t2 / 120.0;
            c2 = -1.0 / 3.0 + t2 / 30.0;
        } else {
            sinc = sin(th) / th;
            c2 = (cos(th) - sinc) / (th * th);
        }
        double o[3], gs[3];
        for (int q = 0; q < 3; ++q) o[q] = cos(th) * s[q] + sinc * u[q];
        double on = or_norm3(o);
        for (int q = 0; q < 3; ++q) o[q] /= on;
        for (int q = 0; q < 3; ++q) {
            double d = o[q] - Sstar[q * P + p];
            loss += d * d;
            gs[q] = 2.0 * d / (double)P;   /* d loss / d S_hat */
        }
        /* through S_hat = cos(th) s + sinc u (the final renormalisation is a
           no-op to first order since |S_hat| = 1 exactly) */
        double ug = u[0] * gs[0] + u[1] * gs[1] + u[2] * gs[2];
        double sg = s[0] * gs[0] + s[1] * gs[1] + s[2] * gs[2];
        double gu[3];
        for (int q = 0; q < 3; ++q) gu[q] = sinc * gs[q] + c2 * ug * u[q] - sinc * sg * u[q];
        /* through the tangent projection u = r - (r.s) s */
        double gus = gu[0] * s[0] + gu[1] * s[1] + gu[2] * s[2];
        for (int q = 0; q < 3; ++q) g[q * P + p] = gu[q] - gus * s[q];
    }
    loss /= (double)P;
    /* layer offsets */
    long woff[4], aoff[4];
    long wo = 0, ao = 0;
    for (int l = 0; l < 4; ++l) {
        woff[l] = wo; wo += (long)c[l + 1] * c[l] * 27 + c[l + 1];
        aoff[l] = ao; ao += (long)c[l + 1] * P;
    }
    memset(grad, 0, sizeof(double) * wo);
    double *gout = g; /* gradient w.r.t. layer output (pre-activation for l=3) */
    for (int l = 3; l >= 0; --l) {
        const int cin = c[l], cout = c[l + 1], d = or_dil(dil, l);
        const double *W = params + woff[l];
        double *gW = grad + woff[l];
        double *gb = gW + (long)cout * cin * 27;
        /* input of layer l: x for l=0, else SiLU(pre-activation of l-1) */
        double *in = (double *)malloc(sizeof(double) * cin * P);
        if (l == 0) memcpy(in, x, sizeof(double) * cin * P);
        else {
            const double *pre = act + aoff[l - 1];
            for (long k = 0; k < (long)cin * P; ++k) in[k] = pre[k] * or_sigmoid(pre[k]);
        }
        for (int co = 0; co < cout; ++co) {
            double s = 0.0;
            for (long p = 0; p < P; ++p) s += gout[co * P + p];
            gb[co] = s;
        }
#pragma omp parallel for schedule(static)
        for (int co = 0; co < cout; ++co)
            for (int ci = 0; ci < cin; ++ci)
                for (int kz = 0; kz < 3; ++kz)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx) {
                            double s = 0.0;
                            for (long p = 0; p < P; ++p) {
                                int x0 = (int)(p % Lx), y0 = (int)((p / Lx) % Ly), z0 = (int)(p / ((long)Lx * Ly));
                                int xx = x0 + (kx - 1) * d, yy = y0 + (ky - 1) * d, zz = z0 + (kz - 1) * d;
                                if (xx < 0 || yy < 0 || zz < 0 || xx >= Lx || yy >= Ly || zz >= Lz) continue;
                                s += gout[co * P + p] * in[ci * P + xx + (long)Lx * (yy + (long)Ly * zz)];
                            }
                            gW[(((long)co * cin + ci) * 3 + kz) * 9 + ky * 3 + kx] = s;
                        }
        if (l > 0) {
            /* gradient w.r.t. the layer input, then through SiLU of layer l-1 */
            double *gin = (double *)calloc((size_t)cin * P, sizeof(double));
#pragma omp parallel for schedule(static)
            for (long p = 0; p < P; ++p) {
                int x0 = (int)(p % Lx), y0 = (int)((p / Lx) % Ly), z0 = (int)(p / ((long)Lx * Ly));
                for (int ci = 0; ci < cin; ++ci) {
                    double s = 0.0;
                    for (int co = 0; co < cout; ++co)
                        for (int kz = 0; kz < 3; ++kz)
                            for (int ky = 0; ky < 3; ++ky)
                                for (int kx = 0; kx < 3; ++kx) {
                                    /* output q = p - (k-1) d used input p through tap k */
                                    int xq = x0 - (kx - 1) * d, yq = y0 - (ky - 1) * d, zq = z0 - (kz - 1) * d;
                                    if (xq < 0 || yq < 0 || zq < 0 || xq >= Lx || yq >= Ly || zq >= Lz) continue;
                                    s += W[(((long)co * cin + ci) * 3 + kz) * 9 + ky * 3 + kx] *
                                         gout[co * P + xq + (long)Lx * (yq + (long)Ly * zq)];
                                }
                    const double pre = act[aoff[l - 1] + ci * P + p];
                    const double sg = or_sigmoid(pre);
                    gin[ci * P + p] = s * sg * (1.0 + pre * (1.0 - sg));
                }
            }
            if (gout != g) free(gout);
            gout = gin;
        }
        free(in);
    }
    if (gout != g) free(gout);
    free(g); free(raw); free(act);
    return loss;
}

/* Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
   w -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps), t >= 1 */
void or_adam(long n, double *w, const double *g, double *m, double *v, long t, double lr,
             double b1, double b2, double eps) {
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (long k = 0; k < n; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * g[k];
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
        w[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
    }
}
