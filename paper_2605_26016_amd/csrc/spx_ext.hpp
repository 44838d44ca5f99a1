// spx_ext.hpp -- host-side interfaces between the C-ABI front end
// (spx_api.hip) and the subsystems in their own translation units: the
// dipolar FFT pipeline, batched GNEB, the dense-window MFMA field and the
// learned path corrector.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/spx.h"
#include "spx_internal.hpp"
#include "spx_stencil.hpp"

namespace spx {

// error / handle registry shared by every entry point
spx_status set_error(spx_status s, const std::string &msg);
spx_status set_hip_error(hipError_t e, const char *where);
void register_handle(const void *p);
bool handle_alive(const void *p);
void unregister_handle(const void *p);

struct DipolarPlan;
struct MCState;
struct PairList;
// Pair-list Hamiltonian (spx_pairlist.hip).
spx_status pl_create(const spx_pairlist_desc *d, int prec, hipStream_t st, PairList **out);
void pl_destroy(PairList *p);
hipError_t pl_field(const PairList *p, const double *S, void *b, hipStream_t st);
hipError_t pl_energy(const PairList *p, const double *S, double *E, double *terms, hipStream_t st);
hipError_t pl_heun(PairList *p, double *S, double alpha, double dt, double pre, double sig0, uint64_t seed,
                   uint64_t step0, uint32_t tag, int noise, int n_steps, hipStream_t st);
// Monte Carlo state of a Hamiltonian (spx_mc.hip): colouring and scratch.
void mc_destroy(MCState *m);

// Read-only view of a Hamiltonian handle for other subsystems.
struct ZPlan;
struct HamView {
    const ZPlan *zp64;  // FP64 z-march plan of the bond table (NULL if none or engine forced to gather)
    Grid grid;
    BondTable tab;
    Onsite onsite;
    int field_prec;
    const double *mu;
    DipolarPlan *dip;
    int radius[3];
    MCState **mc;  // the handle's Monte Carlo state slot (created on first use)
    const PairList *pl;  // non-NULL for a pair-list Hamiltonian
};
spx_status get_ham_view(spx_ham *h, HamView &v);

// Open-boundary dipolar field via zero-padded FFT (spx_dipolar.hip).
// create: builds the dipole-tensor spectrum for dims/cell and moment mu.
spx_status create_dipolar(const int32_t dims[3], const double cell[9], double mu, hipStream_t st,
                          DipolarPlan **out, int64_t *ws_bytes);
void destroy_dipolar(DipolarPlan *p);
// b_dip (meV) of state S written as float[3][N].
spx_status eval_dipolar(DipolarPlan *p, const double *S, float *bdip, hipStream_t st);

// Z-march stencil engine (spx_stencil.hip): a runtime bond table matched
// against a compile-time shell shape, with the couplings packed in shape order.
struct ZPlan {
    bool valid = false;
    int kind = -1;
    int prec = 0;   // 0 FP64, 1 FP32
    int iso = 1;
    int nw = 0;
    int zch = 8;    // z planes per block
    int txw = 64;   // tile width in x (GNEB passes: 64, 32 or 16; others 64)
    int frows = 0;  // rows (wavefronts) per block of the fused Heun step, 0: 16 for FP32 NN, else 8
    double wd[9 * kMaxShapeBonds];
    float wf[9 * kMaxShapeBonds];
};
bool zmarch_plan(int prec, int n_sub, const int *bond_a, const int *bond_b, const int *bond_d,
                 const double *bond_J, int n_bonds, bool iso, ZPlan &zp);
hipError_t zmarch_field(const ZPlan &zp, const Grid &g, const Onsite &os, const double *S, const float *bdip,
                        void *b, hipStream_t st);
hipError_t zmarch_predict(const ZPlan &zp, const Grid &g, const Onsite &os, const HeunConst &hc, uint64_t step,
                          const double *S, const float *bdip, double *St, float *bstore, double *pstore,
                          double *estore, const double *eload, hipStream_t st);
hipError_t zmarch_noise(const HeunConst &hc, uint64_t step, int64_t N, double *eta, hipStream_t st);
// Energy terms of S in the z-march epilogue: one quadruple (bilinear, Zeeman,
// anisotropy, dipolar) per tile into partial[zmarch_tiles()][4], fixed order.
hipError_t zmarch_energy(const ZPlan &zp, const Grid &g, const Onsite &os, const double *S, const float *bdip,
                         double *partial, hipStream_t st);
// split Heun mode: FP32 bilinear field pass + elementwise FP64 stages
hipError_t zmarch_bil(const ZPlan &zp, const Grid &g, const double *S, float *bil, hipStream_t st);
// Bilinear field of n_img images stacked as [n_img][3][N] (FP64 plan, FP64
// output).  The source buffer is S0, or S0alt when *sel != 0 (a device flag);
// nothing is done when *skip != 0 (skip may be NULL).
// Force pass of the static minimisers fused into the FP64 z-march field
// evaluation of S (no-op when state[done_idx] != 0): writes F = b - (b.s) s
// and one set of six partials per tile (max |F|, v.F, F.F, s.s, s.y, y.y of
// the method) into partial[tile][6]; method 2 also writes the projected pair
// into history slot state[cand_idx] of Sh / Yh.
hipError_t zmarch_min_force(const ZPlan &zp, const Grid &g, const Onsite &os, const double *S, double *F,
                            const double *V, const double *Up, const double *Fp, double *Sh, double *Yh,
                            const double *state, int done_idx, int cand_idx, int method, double *partial,
                            hipStream_t st);
// Tiles of one image (x tiles x y tiles x z chunks) of the z-march engine.
int zmarch_tiles(const ZPlan &zp, const Grid &g);
// The same for the GNEB passes (256-thread blocks, tile width zp.txw), and
// the width those passes should use on a lattice.
int zmarch_gneb_tiles(const ZPlan &zp, const Grid &g);
int zmarch_gneb_width(const ZPlan &zp, const Grid &g);
// The two passes of a GNEB iteration that stores no force (see spx_stencil.hip
// ZM_GNEB_A2 / ZM_GNEB_C2), over the images of one instance.  pass 0: every
// image, eleven partials per tile into partial[(item0 + n items_per_img +
// tile) * 11 + v] (energy, squared distance to the next image, a.a, a.b, b.b,
// F.a, F.b, v.a, v.b, v.F, F.F); pass 1: interior images, the update into the
// other buffer and velocities, one max |F_gneb| per tile into
// partial[(item0 + n items_per_img + tile) * 11].  Reads the current buffer (Y0, or Y1
// when *cur != 0); no-op when *done != 0.  FP64 plans only.
struct GnebSlots {
    int n, wp, wm, tn, coef, proj;
};
struct GnebPassArgs {
    int n_img, item0, items_per_img;
    double *Y0, *Y1, *V;
    const double *cur, *done;
    const double *img, *st;
    GnebSlots slots;
    double dt, mass;
    int string;
    double *partial;
};
hipError_t zmarch_gneb_pass(int pass, const ZPlan &zp, const Grid &g, const Onsite &os, const GnebPassArgs &ga,
                            hipStream_t st);
hipError_t zmarch_bil_images(const ZPlan &zp, const Grid &g, int n_img, const double *S0, const double *S0alt,
                             const double *sel, const double *skip, double *bil, hipStream_t st);
hipError_t heun_split_pre(const Grid &g, const Onsite &os, const HeunConst &hc, uint64_t step, const double *S,
                          const float *bil, const float *bdip, double *St, double *P, double *eta, hipStream_t st);
hipError_t heun_split_post(const Grid &g, const Onsite &os, const HeunConst &hc, const double *St, const float *bil,
                           const float *bdip, const double *P, const double *eta, double *out, hipStream_t st);
// Temporally fused Heun step (spx_fused.hip): predictor and corrector in one
// z-march over the lattice, S -> out (out != S), for single-sublattice shell
// shapes of range one cell (simple cubic shells 1 and, isotropic, 1-3).
bool fused_heun_supported(const ZPlan &zp, const Grid &g);
// Rows per block the fused step launches with for this plan (16 or 8).
int fused_rows(const ZPlan &zp);
hipError_t heun_fused(const ZPlan &zp, const Grid &g, const Onsite &os, const HeunConst &hc, uint64_t step,
                      const double *S, double *out, hipStream_t st);
hipError_t zmarch_correct(const ZPlan &zp, const Grid &g, const Onsite &os, const HeunConst &hc, uint64_t step,
                          const double *S, const double *St, const float *bdipS, const float *bdipT,
                          const float *bload, const double *pload, const double *eload, double *out,
                          hipStream_t st);

// Dense-window MFMA field (spx_dense.hip).
struct DensePlan;
bool dense_plan(int prec, int n_sub, const int *bond_a, const int *bond_b, const int *bond_d, const double *bond_J,
                int n_bonds, DensePlan **out, hipStream_t st, std::string &why);
void dense_destroy(DensePlan *p);
hipError_t dense_field(const DensePlan *p, const Grid &g, const Onsite &os, const double *S, float *b, hipStream_t st);

// Learned path corrector (spx_net.hip).
spx_status net_apply(spx_net *net, const float *params, const int32_t dims[3], int32_t batch, const double *Sg,
                     const double *SA, const double *SB, int shared_ends, const float *t, double *Shat,
                     hipStream_t st);
bool net_alive(spx_net *net);

}  // namespace spx
