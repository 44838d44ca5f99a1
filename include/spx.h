/*
 * spx.h -- C ABI of the MI355X-native spin-field / LLG-Heun / GNEB library
 * (libspx.so), implementing the hot path of the atomistic spin method of
 * arXiv 2605.26016 ("SpinX").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function is extern "C", never throws and returns an spx_status.
 *    On a non-OK status spx_last_error() returns a thread-local message.
 *  - Pointers marked [dev] are device pointers (e.g. torch.Tensor.data_ptr()
 *    of a CUDA/HIP tensor); pointers marked [host] are host memory, read only
 *    during the call.  The caller owns every [dev] buffer it passes in and
 *    keeps it alive until the stream has reached the enqueued work.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued on it; no call synchronises the device unless its
 *    comment says so.
 *  - Spin states are structure-of-arrays FP64 planes S[3][N] (x plane, then
 *    y, then z), one unit vector per site.  The site index is
 *        i = x + Lx * (y + Ly * (z + Lz * a)),
 *    a = sublattice, (x, y, z) = unit cell (Methods, sublattice channels
 *    S_a(R)).  N = n_sub * Lx * Ly * Lz; 64-bit indexing throughout.
 *  - Units: spins dimensionless, reduced fields b and energies in meV,
 *    external field in tesla, time step in fs, temperature in K, lengths in nm,
 *    moments mu in Bohr magnetons (Methods, moment and unit conventions).
 *  - Argument errors are reported synchronously.  A device fault raised by
 *    earlier work surfaces at a later call as SPX_ERR_HIP.
 *  - A handle is used from one host thread at a time.  Results are
 *    deterministic for given inputs and seed: no atomics feed any result.
 */
#ifndef SPX_H
#define SPX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPX_ABI_VERSION 1

typedef enum {
    SPX_OK = 0,
    SPX_ERR_INVALID_ARG = 1,   /* bad descriptor, size or pointer */
    SPX_ERR_UNSUPPORTED = 2,   /* valid request this build does not implement */
    SPX_ERR_OUT_OF_MEMORY = 3, /* device allocation failed */
    SPX_ERR_HIP = 4,           /* HIP runtime error (incl. faults of earlier work) */
    SPX_ERR_FFT = 5,           /* hipFFT error */
    SPX_ERR_BAD_HANDLE = 6     /* NULL, destroyed or foreign handle */
} spx_status;

/* Precision of the short-range field evaluation.  The spin state, the Heun
 * integration and every reduction stay FP64 in all modes (Methods, mixed
 * precision: fp32 field, fp64 state). */
typedef enum {
    SPX_FP64 = 0,      /* FP64 neighbours, couplings and accumulation; b is double */
    SPX_FP32 = 1,      /* neighbours rounded to FP32, FP32 couplings and accumulation; b is float */
    SPX_BF16_MFMA = 2, /* dense-window MFMA: BF16 operands, FP32 accumulation; b is float */
    SPX_FP16_MFMA = 3  /* dense-window MFMA: FP16 operands, FP32 accumulation; b is float */
} spx_precision;

typedef struct spx_ham spx_ham;   /* opaque Hamiltonian + workspace */
typedef struct spx_gneb spx_gneb; /* opaque batched GNEB object */
typedef struct spx_net spx_net;   /* opaque learned-path-corrector workspace */

/* Lattice: n_sub sublattices at fractional positions in a Bravais cell,
 * dims[k] cells along lattice vector k, periodic[k] = 1 wraps that axis,
 * 0 leaves it open (missing neighbours contribute nothing: the truncation
 * rule for finite supercells, Methods, backend representations). */
typedef struct {
    int32_t n_sub;
    int32_t dims[3];
    int32_t periodic[3];
    double cell[9];          /* [host] lattice vectors as rows, nm */
    const double *sub_frac;  /* [host] [n_sub][3] fractional positions */
    const double *mu;        /* [host] [n_sub] moment magnitudes, mu_B */
} spx_lattice_desc;

/* Hamiltonian H = H_bil + H_Z + H_ani + H_dip (Methods, total Hamiltonian).
 * Bilinear couplings come either from shells or from an explicit bond list:
 *  - shells: neighbour distances over all sublattice pairs, ascending, equal
 *    within 1e-9 of the longest lattice vector, form shells 1..n_shells;
 *    each directed bond of shell s gets J_ij = J_shell[s] I + [D]_x with
 *    D_ij = D_shell[s] * (r_j - r_i)/|r_j - r_i| (D_shell may be NULL), the
 *    antisymmetric DMI matrix of the Methods' bilinear tensor;
 *  - bonds (n_bonds > 0 overrides shells): directed bonds a <- b at cell
 *    offset delta with a full 3x3 row-major tensor J^{ab}(delta) in meV, used
 *    as b_a(R) += J S_b(R + delta).  The caller supplies both directions
 *    (J_ji = J_ij^T) if the pair energy is to be symmetric.
 * Anisotropy: n_aniso axes per sublattice, H = -sum K (S.n)^2.
 * Zeeman: H = -sum mu mu_B B.S.  Dipolar (dipolar = 1): open-boundary
 * H_dip = -(mu0/4pi) mu_B^2 sum_{i<j} mu_i mu_j [3(S_i.r)(S_j.r) - S_i.S_j]/r^3
 * evaluated by zero-padded FFT; needs n_sub = 1 and all axes open. */
typedef struct {
    int32_t n_shells;
    const double *J_shell;     /* [host] [n_shells] meV */
    const double *D_shell;     /* [host] [n_shells] meV, or NULL */
    int32_t n_bonds;
    const int32_t *bond_ab;    /* [host] [n_bonds][2] target a, source b */
    const int32_t *bond_delta; /* [host] [n_bonds][3] cell offset */
    const double *bond_J;      /* [host] [n_bonds][9] meV */
    int32_t n_aniso;
    const double *K;           /* [host] [n_sub][n_aniso] meV */
    const double *K_axis;      /* [host] [n_sub][n_aniso][3] unit vectors */
    double B_ext[3];           /* tesla */
    int32_t dipolar;           /* 0 off, 1 on */
} spx_model_desc;

/* backend: 0 auto, 1 sparse stencil, 2 dense 7^3 window (single sublattice,
 * every bond within |delta| <= 3; no dipolar term; field evaluation only):
 * field_prec SPX_BF16_MFMA / SPX_FP16_MFMA run it on the matrix cores,
 * SPX_FP32 runs the direct FP32 convolution on the vector ALUs (Methods,
 * backend representations: dense convolution).  autotune: 0 off, 1 time candidate launch shapes at setup and
 * keep the fastest (cached per shape key in tune_cache_path if non-NULL, one
 * JSON object per line: {"key": ..., "zchunk": ..., "heun_mode": ..., "us": ...,
 * "tile_rows": ...}; plain lines "key zchunk heun_mode us [tile_rows]" are
 * read as well; the last entry of a key wins).
 * stencil_engine: 0 auto, 1 gather kernel (any bond table), 2 z-marching LDS
 * engine (bond tables that match a built-in shell shape: simple cubic shells
 * 1, 1-3, 1-4; bcc shells 1-5).  zchunk: z planes per block of the z-march
 * engine (0 = default 8).  heun_field (z-march engine; the gather engine
 * always recomputes): 0 auto (3, or the autotuner's choice), 1 the
 * corrector recomputes the field of S^n, 2 the predictor stores the FP32
 * bilinear field of S^n for the corrector (FP32 field_prec only; results
 * identical to 1), 3 the predictor stores the stage P = S^n + dt/2 f(S^n)
 * and the step's noise (FP64, 48 bytes per spin of library memory), so the
 * corrector evaluates f(S~) only (results equal to 1 up to the rounding of
 * the regrouped sum S^n + dt/2 f(S^n) + dt/2 f(S~)), 4 as 3 with the noise
 * drawn by an elementwise pre-pass and read by both stages (same results
 * as 3), 5 split: each stage is a stencil pass that stores the FP32
 * bilinear field followed by an elementwise FP64 stage kernel (FP32
 * field_prec only; same results as 3), 6 split predictor with the fused
 * stored-stage corrector of mode 3 (FP32 field_prec only; same results), 7
 * as 3 without the noise store: the corrector draws the step's noise again
 * from the same Philox block (24 bytes per spin of library memory; same
 * results as 3), 8 temporally fused: predictor and corrector in one pass
 * that keeps the predicted state on chip and predicts a one-cell ring
 * around each block's tile again, each site with its own noise, so the
 * lattice is read and written once per step (single-sublattice simple cubic
 * shells 1, any tensor, or shells 1-3 isotropic; no dipolar term; results
 * equal to 3 up to the summation order of the bilinear sums).  heun_field 8
 * on any other Hamiltonian fails with SPX_ERR_UNSUPPORTED; heun_field 0
 * selects 8 where it applies (z chunk 64 unless zchunk is given), else 3. */
typedef struct {
    int32_t field_prec;        /* spx_precision */
    int32_t backend;
    int32_t autotune;
    const char *tune_cache_path;
    int32_t stencil_engine;
    int32_t zchunk;
    int32_t heun_field;
    /* rows (wavefronts) per block of the fused Heun step (heun_field 8) on
     * the FP32 nearest-neighbour shape: 16 or 8; 0 = the autotuner's choice
     * (16 without autotuning).  Other shapes use 8. */
    int32_t tile_rows;
} spx_options;

/* Build the kernel tables (directed bonds grouped per target sublattice, see
 * the Methods' sublattice convolution b_a(R) = sum_b sum_delta K_ab(delta)
 * S_b(R + delta)), allocate the library-owned workspace (Heun predictor and
 * ping-pong states, reduction scratch, dipolar FFT plans and the dipole
 * spectrum) and return a handle.  Synchronous.  Errors: INVALID_ARG for bad
 * descriptors, OUT_OF_MEMORY, UNSUPPORTED for dipolar with n_sub > 1 or a
 * periodic axis, FFT for plan failures. */
spx_status spx_setup_hamiltonian(const spx_lattice_desc *lat, const spx_model_desc *model,
                                 const spx_options *opts, void *stream, spx_ham **out);
/* Frees everything the handle owns.  Synchronises the whole device first
 * (hipDeviceSynchronize): work enqueued on any stream may still use the
 * handle's tables and scratch, and the handle does not record the streams it
 * was given. */
spx_status spx_destroy_hamiltonian(spx_ham *h);

/* Reduced effective field (Methods, reduced field b = -dH/dS in meV):
 * b_i = sum_j J_ij S_j + 2 sum_l K_l (S_i.n_l) n_l + mu_i mu_B B + b_dip,i.
 * S: [dev] double[3][N].  b: [dev] [3][N] of double (field_prec SPX_FP64) or
 * float (all other precisions). */
spx_status spx_eval_field(spx_ham *h, const double *S, void *b, void *stream);

/* Energy E = -sum_i S_i.(b_bil/2 + b_ani/2 + b_dip/2 + b_Z), which equals
 * the unordered pair form of the Methods' Hamiltonian.  E: [dev] one double.
 * terms: [dev] double[5] = bilinear, Zeeman, anisotropy, dipolar, total, or
 * NULL.  Fixed-order two-level FP64 reduction (deterministic). */
spx_status spx_energy(spx_ham *h, const double *S, double *E, double *terms, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the energy
 * and terms of spx_energy, with no allocation, synchronisation or memset in
 * the call.  The neighbours are gathered per site and the partial sums go to
 * a library-owned static device array of 4096 quadruples (128 KiB per
 * device, looked up at the first call on each device): min(ceil(N / 256),
 * 4096) blocks stride over the lattice, and one block adds their quadruples
 * in a fixed order.  Results equal spx_energy's to FP64 rounding (another
 * fixed summation order); deterministic.  Every quadruple read is written by
 * the same call, so nothing is cleared between calls, and calls that overlap
 * on one device (several streams) race on the array.  SPX_ERR_UNSUPPORTED for
 * pair-list Hamiltonians and for the dipolar term; other errors as
 * spx_energy. */
spx_status spx_energy_noalloc(spx_ham *h, const double *S, double *E, double *terms, void *stream);

/* Stochastic/deterministic LLG (Methods, atomistic spin dynamics):
 * dS/dt = -gamma/(1+alpha^2) [S x B + alpha S x (S x B)], B = b/(mu mu_B)
 * plus, for temperature_K > 0, the thermal field sigma_i eta_i^n with
 * sigma_i = sqrt(2 alpha k_B T / (gamma mu_i mu_B dt)) (stochastic LLG).
 * Each step is the normalised Heun scheme: S~ = N[S + dt f(S)],
 * S' = N[S + dt/2 (f(S) + f(S~))], the same eta in both stages.
 * eta_i^n comes from one Philox4x32-10 block with key (seed lo, seed hi) and
 * counter (i lo, i hi ^ tag, n lo, n hi), n = step0 + k for the k-th step;
 * uniforms u = (x + 1/2) 2^-32; Box-Muller on (u0,u1) gives eta_x, eta_y and
 * on (u2,u3) gives eta_z.  gamma = 0 selects 1.76085963023e11 rad/(s T).
 * S is updated in place ([dev] double[3][N]). */
typedef struct {
    double alpha;
    double dt_fs;
    double temperature_K;
    double gamma;        /* rad/(s T); 0 = CODATA electron value */
    uint64_t seed;
    uint64_t step0;
    uint32_t tag;        /* noise stream tag (ensembles); 0 by default */
    int32_t n_steps;
} spx_llg_params;

spx_status spx_llg_heun_step(spx_ham *h, double *S, const spx_llg_params *p, void *stream);

/* Graph replay of the Heun loop (default on): for n_steps >= 4 the library
 * captures g steps (g = 16 when n_steps >= 16, else 2; S -> scratch -> S ...,
 * the noise step read from a device counter that the graph's last node
 * advances by g) once per (state pointer, constants, step count g) and
 * replays it n_steps/g times on the caller's stream; the n_steps % g
 * remaining steps are launched directly.  Off while kernels are timed and
 * with the dipolar term.  Results are identical to direct launches. */
spx_status spx_set_heun_graph(spx_ham *h, int32_t enable);

/* The thermal-noise normals eta_i^n the Heun kernels use for (seed, step,
 * tag), written as [dev] double[3][N] for N sites.  Test hook of the RNG
 * stream; no handle needed. */
spx_status spx_thermal_noise(uint64_t seed, uint64_t step, uint32_t tag, int64_t N, double *eta,
                             void *stream);

/* Raw Philox4x32-10 blocks (Salmon et al., SC'11) for n counters:
 * ctr [dev] uint32[n][4], key [dev] uint32[n][2] -> out [dev] uint32[n][4]. */
spx_status spx_philox4x32_10(const uint32_t *ctr, const uint32_t *key, int64_t n, uint32_t *out,
                             void *stream);

/* ---- Pair-list Hamiltonian (Methods, pair-list backend) --------------------
 * For systems without translational symmetry (chemical disorder, defects,
 * site-resolved couplings): entry p couples target site target[p] to source
 * site source[p] with J[p] (meV; a scalar, or a row-major 3x3 block when
 * tensor = 1), and the reduced bilinear field is
 *   b_i = sum_{p: target[p] = i} J_p S_{source[p]},
 * summed in list order, plus the site-resolved Zeeman mu_i mu_B B and uniaxial
 * anisotropy 2 K_i (S_i.n_i) n_i.  The list is taken as given: reciprocal
 * entries are the caller's to supply.  All arrays are host memory, copied at
 * set-up; mu NULL means 1 everywhere, K NULL no anisotropy.  The handle works
 * with spx_eval_field, spx_energy (terms: bilinear, Zeeman, anisotropy, 0,
 * total), spx_llg_heun_step (per-site mu_i in B = b/(mu_i mu_B) and in the
 * thermal field; noise counter = site index) and the minimisers; GNEB and
 * Monte Carlo need a lattice (SPX_ERR_UNSUPPORTED).  field_prec SPX_FP64 or
 * SPX_FP32 (neighbour spins and couplings rounded to float, FP32
 * accumulation, on-site terms in FP64); other options are ignored.
 * SPX_ERR_INVALID_ARG for sites out of range or non-positive moments. */
typedef struct {
    int64_t n_sites;
    int64_t n_pairs;
    const int64_t *target;     /* [n_pairs] i_p */
    const int64_t *source;     /* [n_pairs] j_p */
    const double *J;           /* [n_pairs] or [n_pairs][9] */
    int32_t tensor;
    const double *mu;          /* [n_sites] mu_B, or NULL */
    const double *K;           /* [n_sites] meV, or NULL */
    const double *K_axis;      /* [n_sites][3] unit axes (with K) */
    double B_ext[3];           /* tesla */
} spx_pairlist_desc;
spx_status spx_setup_pairlist(const spx_pairlist_desc *d, const spx_options *opts, void *stream, spx_ham **out);

/* Introspection of a handle (host values; synchronous). */
typedef struct {
    int64_t n_sites;
    int32_t n_bonds;           /* directed bonds in the table */
    int32_t field_prec;
    int32_t backend;           /* 1 stencil, 2 dense window (MFMA or FP32 direct), 3 pair list */
    int32_t radius[3];         /* max |delta| per axis over the table */
    int32_t dipolar;
    int64_t workspace_bytes;   /* library-owned device memory */
    int32_t stencil_engine;    /* 1 gather, 2 z-march */
    int32_t shape;             /* z-march shell shape id, -1 if none */
    int32_t zchunk;
    int32_t heun_field;        /* 1 recompute, 2 stored FP32 field, 3 stored stage and noise, 4 as 3 + noise pre-pass, 5 split, 6 split predictor, 7 stored stage, noise drawn again, 8 fused single pass */
    int32_t tuned;             /* 1 if the autotuner chose zchunk / heun_field */
    double tuned_step_us;      /* its timing of one Heun step (microseconds) */
    int32_t heun_graph;        /* 1 once a captured Heun graph exists (replayed for runs of >= 4 steps) */
    int32_t tile_rows;         /* rows per block of the fused Heun step (0 when heun_field != 8) */
} spx_ham_info;
spx_status spx_get_info(spx_ham *h, spx_ham_info *info);

/* Copy the directed-bond table out (host arrays sized n_bonds): target a,
 * source b, offset delta[3], tensor J[9]. */
spx_status spx_get_bonds(spx_ham *h, int32_t *bond_ab, int32_t *bond_delta, double *bond_J);

/* ---- Monte Carlo sampling (Methods, Monte Carlo sampling) -----------------
 * Heat-bath and Metropolis sweeps of the state S ([dev] double[3][N], in
 * place) at temperature T, beta = 1/(k_B T), FP64 throughout.  The local field
 * of site i is its bilinear field plus the Zeeman field, b_i = sum_j J_ij S_j
 * + mu_i mu_B B (meV).  Sites are coloured by (x + ky y + kz z + o_a) mod C
 * with the smallest C, then the lexicographically smallest (ky, kz, o_1 ..),
 * for which no bond of the Hamiltonian joins two sites of one colour
 * (spx_mc_colouring); a sweep updates the colours 0 .. C-1 in turn, all sites
 * of a colour at once, one attempted update per spin.  Site i in sweep n draws
 * one Philox4x32-10 block, counter (i lo, i hi ^ 0x4D430000, n lo, n hi), key
 * (seed lo, seed hi), uniforms u_k = (x_k + 1/2) 2^-32.
 *   method 0, heat-bath: S_i ~ exp(beta b_i.S); the cosine to b_i is
 *     1 + log1p((1 - u0) expm1(-2x))/x, x = beta |b_i| (2 u0 - 1 for x = 0), the
 *     azimuth 2 pi u1 around b_i in the frame e1 = normalize(b^ x e_k) (e_k the
 *     Cartesian axis least aligned with b^), e2 = b^ x e1.  Needs a local energy
 *     linear in the spin: SPX_ERR_UNSUPPORTED with anisotropy.
 *   method 1, Metropolis: trial S' uniform on the sphere (z = 2 u0 - 1, azimuth
 *     2 pi u1), dH = -(S' - S_i).b_i - sum_l K_l [(S'.n_l)^2 - (S_i.n_l)^2],
 *     accepted if u2 < exp(-beta dH).
 * SPX_ERR_UNSUPPORTED with the dipolar term or when no colouring with C <= 64
 * is found (see spx_mc_find_colouring for the search's limits); SPX_ERR_INVALID_ARG for T <= 0, n_sweeps < 0, another method or layout.
 * `accepted` ([dev] uint64 or NULL) receives the number of accepted moves of
 * the call (heat-bath: every draw).  Asynchronous.  A call of two sweeps or
 * more, or of a colouring with more than two colours, copies S into a
 * colour-major layout held by the handle (allocated on the first such call,
 * about 3 N doubles plus ghost slots and rows, freed with the Hamiltonian;
 * if it cannot be allocated the sweeps run in place), runs every sweep there
 * and copies the result back; the moves and results are the same bit for
 * bit (layout = 1 keeps every call in place).  Overlapping calls on one
 * handle race. */
typedef struct {
    double temperature_K;
    uint64_t seed;
    uint64_t sweep0;     /* counter of the first sweep */
    int32_t n_sweeps;
    int32_t method;      /* 0 heat-bath, 1 Metropolis */
    int32_t layout;      /* 0: the library chooses (above); 1: in place, never the colour-major copy */
} spx_mc_params;
spx_status spx_mc_sweep(spx_ham *h, double *S, const spx_mc_params *p, unsigned long long *accepted, void *stream);
/* The colouring used by spx_mc_sweep (searched on first use, synchronous):
 * *n_colours = C, coef (host int32[2 + n_sub] or NULL) = (ky, kz, o_0 ..). */
spx_status spx_mc_colouring(spx_ham *h, int32_t *n_colours, int32_t *coef);
/* The same colouring search on the host, without a handle or a device: a
 * lattice of n_sub sublattices, dims/periodic [host] int32[3], n_bonds
 * directed bonds (bond_ab [n][2] target, source; bond_delta [n][3]), colours
 * 2 .. cmax.  SPX_ERR_UNSUPPORTED (and *n_colours = 0) when no colouring has
 * at most cmax colours, when a bond joins a site to itself (same sublattice
 * and every realised coordinate difference zero: no colouring exists), or
 * when the candidates up to cmax exceed 2^26 before one is found (the search
 * tries C^(n_sub+1) offset choices per C); the message says which. */
spx_status spx_mc_find_colouring(int32_t n_sub, const int32_t *dims, const int32_t *periodic, int32_t n_bonds,
                                 const int32_t *bond_ab, const int32_t *bond_delta, int32_t cmax, int32_t *n_colours,
                                 int32_t *coef);
/* Total moment direction sum m = sum_i S_i (Methods, thermodynamic
 * observables; reduced magnetisation m/N), m [dev] double[3], two-level
 * fixed-order reduction.  Asynchronous. */
spx_status spx_magnetization(spx_ham *h, const double *S, double *m, void *stream);

/* ---- Static minimisation (Methods, static optimisation) --------------------
 * Minimisers on the product of unit spheres for the Hamiltonian's FP64 field
 * (field_prec SPX_FP64).  The force F_i = b_i - (b_i.S_i) S_i is minus the
 * tangent gradient G_i.  Per iteration the step u_i is
 *   method 0, velocity projection: v <- (sum v.F / sum F.F) F (if sum v.F > 0,
 *             else 0) + (dt/mass) F, u = dt v;
 *   method 1, Barzilai-Borwein: u = alpha F, alpha = sum s.s / sum s.y with
 *             s = P(u_prev), y = P(F_prev) - F (P: projection on the current
 *             tangent planes); alpha = dt on the first iteration or if
 *             sum s.y <= 0;
 *   method 2, L-BFGS: (s, y) joins the history (the newest `history` pairs)
 *             when s.y > 0; the two-loop recursion from q = G with the pairs
 *             projected on the current tangent planes and the initial scale
 *             s.y/y.y of the newest pair gives r, u = -r (u = dt F without pairs);
 *   method 3, Adam: m <- beta1 m + (1-beta1) G, w <- beta2 w + (1-beta2) G*G
 *             per Cartesian component, u = -dt m^/(sqrt(w^) + eps) with the
 *             bias-corrected moments m^ = m/(1-beta1^t), w^ = w/(1-beta2^t);
 * then u_i is projected on the tangent plane of S_i, cut to |u_i| = max_step if
 * longer (max_step > 0), and retracted: retraction 0, exponential map
 * S <- cos|u| S + sin|u| u/|u|; 1, normalised S <- (S + u)/|S + u|.
 * The run stops (state frozen) after the first iteration whose max |F| (before
 * its update) is below tol_force (0: never). */
typedef struct {
    int32_t method;       /* 0 VP, 1 BB, 2 L-BFGS, 3 Adam */
    int32_t retraction;   /* 0 exponential map, 1 normalised */
    double dt;            /* VP time step; BB/L-BFGS first step; Adam step (rad) */
    double mass;          /* VP */
    int32_t history;      /* L-BFGS pairs, 1 .. 32 */
    double beta1, beta2, eps;  /* Adam */
    double max_step;      /* largest rotation per spin and iteration (rad), 0 = none */
    double tol_force;     /* meV */
} spx_min_params;
typedef struct spx_min spx_min;
/* Allocates the minimiser state (velocities or moments, previous step and
 * force, history), zeroed.  Synchronous. */
spx_status spx_min_create(spx_ham *h, const spx_min_params *p, void *stream, spx_min **out);
/* n_iter iterations of S ([dev] double[3][N], in place).  Asynchronous. */
spx_status spx_min_step(spx_min *m, double *S, int32_t n_iter, void *stream);
/* max |F| of the last iteration (meV, before its update), iterations run,
 * converged flag (host outputs, any may be NULL).  Synchronises. */
spx_status spx_min_get_stats(spx_min *m, double *max_force, int32_t *iterations, int32_t *converged, void *stream);
/* Forget the state (velocities, moments, history, counters). */
spx_status spx_min_reset(spx_min *m, void *stream);
/* Frees the minimiser's state.  Synchronises the whole device first (queued
 * iterations may still use it). */
spx_status spx_min_destroy(spx_min *m);

/* ---- Batched geodesic nudged elastic band (Methods, minimum-energy paths) --
 * One object holds n_inst independent paths ("instances"), each with its own
 * Hamiltonian (field_prec SPX_FP64, no dipolar term) and 3 <= n_img[k] <= 4096 images
 * stored in the caller's buffer images[k] ([dev] double[n_img][3][N_k]),
 * updated in place; images 0 and n_img-1 are pinned.  Every iteration runs
 * for all unconverged instances in one set of persistent launches:
 *   F_i   = b_i - (b_i.S_i) S_i        (projected -grad H, meV per spin)
 *   tau   = improved (energy-weighted upwind) tangent from Y_n+1 - Y_n and
 *           Y_n - Y_n-1, projected per spin, normalised over the image
 *   F     = F - (F.tau)tau + k (d(Y_n,Y_n+1) - d(Y_n-1,Y_n)) tau     (GNEB)
 *   F     = F - 2 (F.tau)tau on the highest-energy movable image (climbing)
 *   d     = geodesic distance [sum_i angle(S_i, S'_i)^2]^(1/2)
 * followed by velocity projection over all movable images of the instance
 * (v <- (v.F/F.F) F if v.F > 0 else 0; v += (dt/m) F) and the exponential-map
 * retraction S <- cos|u| S + sin|u| u/|u| with u = P_perp(dt v).
 * ci_mode: 0 no climbing image, 1 climbing image switched on once max |F|
 * < ci_on_below, 2 from the start, 3 static minimisation (Methods, static
 * optimisation: velocity projection with the exponential-map retraction):
 * no tangent, no springs, no climbing image, every movable image relaxes to a
 * local minimum on its own (the end images are not used); 4 string method
 * (Methods, minimum-energy paths): every movable image is displaced by its
 * projected physical force, u = vp_dt F, S <- exp_S(u), with no spring, no
 * climbing image and no velocity memory (vp_mass and spring_k unused), and the
 * path is then reparameterised along the geodesic reaction coordinate to the
 * instance's arc-length spacing (spx_gneb_redistribute); the reported max |F|
 * is that of F - (F.tau)tau.  An instance stops (and is frozen) once
 * max |F| < tol_force (and, for ci_mode 1, the climbing image is on);
 * tol_force = 0 never stops.  Deterministic, fixed-order reductions. */
typedef struct {
    double spring_k;     /* meV / rad^2 */
    double vp_dt;        /* velocity-projection time step */
    double vp_mass;
    int32_t ci_mode;
    double ci_on_below;  /* meV */
    double tol_force;    /* meV */
} spx_gneb_params;

/* Validates the instances and allocates the library-owned ping-pong images,
 * velocities, forces and reduction scratch (synchronous).  The caller's
 * images are the starting path. */
spx_status spx_gneb_create(spx_ham *const *H, int32_t n_inst, double *const *images, const int32_t *n_img,
                           const spx_gneb_params *p, void *stream, spx_gneb **out);
/* Frees the library-owned images, velocities, forces, scratch and graphs.
 * Synchronises the whole device first (queued iterations may still use
 * them). */
spx_status spx_gneb_destroy(spx_gneb *g);
/* Initial path.  method 0 (geodesic): image n at t = n/(n_img-1) on every
 * spin's great circle between the two end images; antiparallel end spins
 * rotate about normalize(S_A x e_k), e_k the Cartesian axis least aligned with
 * S_A (first on ties).  method 1 (learned): the geodesic path, then every
 * movable image corrected by the network (spx_net_forward) with parameters
 * `params` ([dev] float[spx_net_nparams()]); net and params are ignored for
 * method 0.  Lattices must be single-sublattice for method 1.  Resets
 * velocities, counters and the climbing switch. */
spx_status spx_gneb_init_path(spx_gneb *g, int32_t method, spx_net *net, const float *params, void *stream);
/* n_iter iterations for every unconverged instance (captured once as a
 * hipGraph and replayed).  On return the caller's buffers hold the state. */
spx_status spx_gneb_step(spx_gneb *g, int32_t n_iter, void *stream);
/* Per-instance statistics after the last iteration (synchronises): energies
 * E[n_img] (meV), distances dist[n_img-1], max |F| per spin over movable images
 * (meV, the force of the last iteration before its update), climbing-image
 * index (-1 if none), climbing switch, iterations run, converged flag.  Any
 * output pointer may be NULL (host memory). */
spx_status spx_gneb_get_stats(spx_gneb *g, int32_t inst, double *E, double *dist, double *max_force,
                              int32_t *ci_index, int32_t *ci_on, int32_t *iterations, int32_t *converged,
                              void *stream);
/* Target spacing of instance inst for reparameterisation (Methods,
 * minimum-energy paths: image redistribution): alpha (host double[n_img]) are
 * the images' fractions of the path's geodesic arc length, alpha[0] = 0,
 * alpha[n_img-1] = 1, nondecreasing; the default is equal spacing n/(n_img-1).
 * Synchronous.  SPX_ERR_INVALID_ARG for a bad instance or profile. */
spx_status spx_gneb_set_spacing(spx_gneb *g, int32_t inst, const double *alpha, void *stream);
/* Geodesic reparameterisation of every instance now (Methods, minimum-energy
 * paths: the string method's second step, image redistribution): with s_n the
 * cumulative geodesic distance d(Y_0,Y_1) + ... + d(Y_n-1,Y_n), movable image
 * n moves to arc length alpha_n s_last, on each spin's great-circle arc
 * between the two images that bracket it (fraction f of the arc from the last
 * image k <= n_img-2 with s_k <= alpha_n s_last; antiparallel spins as in
 * spx_gneb_init_path); end images are kept and velocities cleared.  Asynchronous;
 * on completion the caller's buffers hold the new path. */
spx_status spx_gneb_redistribute(spx_gneb *g, void *stream);
/* New parameters for every instance (same rules as spx_gneb_create), e.g.
 * from the string method to climbing-image GNEB on the relaxed path.  Clears
 * the velocities, the iteration counters, the climbing switch and the
 * converged flags (the paths are kept).  Synchronous. */
spx_status spx_gneb_set_params(spx_gneb *g, const spx_gneb_params *p, void *stream);
/* 1 (default): replay one captured hipGraph per iteration; 0: direct launches. */
spx_status spx_gneb_set_graph(spx_gneb *g, int32_t enable);

/* ---- Learned initial-path corrector (spec extension; the paper only
 * names machine-learning interfaces).  A 3^3 convolution network with
 * channels 10 -> 16 -> 16 -> 16 -> 3, zero padding and SiLU between layers,
 * FP32 parameters packed layer by layer as W[cout][cin][kz][ky][kx] then
 * bias[cout].  Input channels per image: geodesic guess S_g (3), end images
 * S_A (3), S_B (3), reaction coordinate t (1); the output u is projected on
 * the tangent plane of S_g and applied by the exponential map
 * S_hat = cos|u| S_g + sin|u| u/|u| (the Methods' retraction).
 * Arrays: S_g, S_A, S_B, S_hat, S_star [dev] double[batch][3][P] for lattices
 * dims = (Lx, Ly, Lz), P = Lx Ly Lz (single sublattice, open faces as zero
 * padding); t [dev] float[batch]. */
int64_t spx_net_nparams(void);
/* channels must be {10, 16, 16, 16, 3} (or NULL); the workspace grows with use. */
spx_status spx_net_create(const int32_t *channels, spx_net **out);
/* Frees the workspace.  Synchronises the whole device first (queued passes
 * may still use it). */
spx_status spx_net_destroy(spx_net *net);
/* Per-layer dilation dil[4] (host int32, each 1 .. 64; default 1 1 1 1):
 * tap k = (kx, ky, kz) of layer l reads the input at offset
 * ((kx-1) dil[l], (ky-1) dil[l], (kz-1) dil[l]), zero outside the lattice, so
 * the four layers see 1 + 2 (dil[0] + ... + dil[3]) cells per axis.  Applies
 * to every later forward, backward and learned initial path of the net.
 * SPX_ERR_INVALID_ARG for a value out of range. */
spx_status spx_net_set_dilation(spx_net *net, const int32_t *dil);
/* Arithmetic of the forward pass (spx_net_forward and the learned initial
 * path): SPX_FP32 (default, direct convolution on the vector ALUs) or
 * SPX_BF16_MFMA (each layer a BF16 implicit GEMM on the matrix cores:
 * activations and weights rounded to BF16 to nearest even, FP32
 * accumulation, bias and output in FP32).  spx_net_backward always runs in
 * FP32.  SPX_ERR_INVALID_ARG for another precision. */
spx_status spx_net_set_precision(spx_net *net, int32_t prec);
spx_status spx_net_forward(spx_net *net, const float *params, const int32_t *dims, int32_t batch, const double *Sg,
                           const double *SA, const double *SB, const float *t, double *Shat, void *stream);
/* Gradient of loss = mean over batch and sites of |S_hat - S_star|^2 with
 * respect to every parameter, written to grad ([dev] float, overwritten);
 * loss ([dev] double) may be NULL.  Deterministic fixed-order reductions. */
spx_status spx_net_backward(spx_net *net, const float *params, const int32_t *dims, int32_t batch, const double *Sg,
                            const double *SA, const double *SB, const float *t, const double *Sstar, float *grad,
                            double *loss, void *stream);
/* Adam (Kingma & Ba) on n FP32 parameters at step >= 1 (bias-corrected). */
spx_status spx_net_adam_step(float *params, const float *grad, float *m, float *v, int64_t n, int64_t step,
                             double lr, double b1, double b2, double eps, void *stream);

/* Streaming probe of the attainable HBM bandwidth (measurement hook): 16-byte
 * accesses over n_bytes (a multiple of 16; 16-byte aligned [dev] buffers),
 * grid-stride with four accesses in flight per thread.  kind 0 copies src to
 * dst, 1 only reads src (dst may be NULL; nothing is written unless the
 * folded word hits a sentinel, in which case dst[0] gets 4 bytes), 2 only
 * writes dst.  Asynchronous; time it with events on `stream`. */
spx_status spx_stream_probe(int32_t kind, const void *src, void *dst, int64_t n_bytes, void *stream);

/* Lane-layout check of the 32x32x16 MFMA used by the dense backend:
 * D = A B for A [32][16], B [16][32], D [32][32] ([dev] row-major float),
 * operands rounded to BF16 (prec 2) or FP16 (prec 3).  Test hook. */
spx_status spx_mfma_probe(int32_t prec, const float *A, const float *B, float *D, void *stream);
/* The same for the 16x16x32 BF16 MFMA of the network's BF16 form: D = A B for
 * A [16][32], B [32][16], D [16][16] ([dev] row-major float, operands rounded
 * to BF16).  Test hook. */
spx_status spx_mfma16_probe(const float *A, const float *B, float *D, void *stream);

/* Kernel timing instrumentation (Methods, performance measurements: device
 * time of the hot kernels).  With enable = 1 every launch of the Heun
 * predictor (kind 0), Heun corrector (kind 1), field kernel (kind 2) and
 * noise pre-pass (kind 3, Heun mode 4) on this handle is bracketed by a pair
 * of hipEvents on the launch stream.
 * spx_get_kernel_times synchronises on the recorded events and returns the
 * number of launches and their summed duration in ms since the last query
 * (then resets that kind).  enable = 0 stops recording. */
spx_status spx_set_kernel_timing(spx_ham *h, int32_t enable);
spx_status spx_get_kernel_times(spx_ham *h, int32_t kind, int64_t *count, double *total_ms);

const char *spx_last_error(void);
int32_t spx_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPX_H */
