// spx_ext.hpp -- host-side interfaces between the C-ABI front end
// (spx_api.hip) and the subsystems in their own translation units: the
// dipolar FFT pipeline, batched GNEB, the dense-window MFMA field and the
// learned path corrector.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/spx.h"
#include "spx_internal.hpp"

namespace spx {

// error / handle registry shared by every entry point
spx_status set_error(spx_status s, const std::string &msg);
spx_status set_hip_error(hipError_t e, const char *where);
void register_handle(const void *p);
bool handle_alive(const void *p);
void unregister_handle(const void *p);

struct DipolarPlan;

// Read-only view of a Hamiltonian handle for other subsystems.
struct HamView {
    Grid grid;
    BondTable tab;
    Onsite onsite;
    int field_prec;
    const double *mu;
    DipolarPlan *dip;
    int radius[3];
};
spx_status get_ham_view(spx_ham *h, HamView &v);

// Open-boundary dipolar field via zero-padded FFT (spx_dipolar.hip).
// create: builds the dipole-tensor spectrum for dims/cell and moment mu.
spx_status create_dipolar(const int32_t dims[3], const double cell[9], double mu, hipStream_t st,
                          DipolarPlan **out, int64_t *ws_bytes);
void destroy_dipolar(DipolarPlan *p);
// b_dip (meV) of state S written as float[3][N].
spx_status eval_dipolar(DipolarPlan *p, const double *S, float *bdip, hipStream_t st);

}  // namespace spx
