// pd_plan.hpp -- host-side plan object and chain runners (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "pd_fcbm.h"
#include "pd_fcbm_testing.h"
#include "pd_passes.hpp"

// One timed kernel launch (profiling mode): events recorded on the launch
// stream right before and after the kernel, plus its algorithmic bytes.
struct ProfRec {
    char name[32];
    hipEvent_t a, b;
    double bytes;
};

struct pd_plan_s {
    // geometry
    int dim;
    int n[3], b[3];
    double dx[3];
    double delta;
    int influence;
    pd_kernel kern;
    pd_dtype dtype;
    int flags;
    hipStream_t stream0;
    int device;
    int max_lds;                 // bytes of LDS a block may use
    int lastaxis;                // PD_LASTAXIS_* (kernel choice for the last axis)
    pdk::Geo geo;
    long nb, nfft;
    // stencil and kernels
    int ns;                      // bonds per node
    int ntap;                    // taps along the last axis (max |o_last| + 1)
    int nct, ncs;                // taps components, static components
    uint32_t oddmask;            // last-axis parity of each taps component
    double alpha, m0, kappa, mu, ka, Wc, dt_max, dV;
    // spectral preconditioner of the static solve, in tap units (Ĉ/Nfft):
    // diagonal of Ĉ(0), identity shift, normalisation s0 = Ĉ(0)_xx/Nfft
    double pre_k0[3], pre_shift, pre_s0;
    int beta_comp;               // static component holding the omega_0 bond count
    // device buffers
    void* tw;                    // T twiddles: table for length N at [N, 2N)
    double* tw64;                // FP64 twiddles, same layout
    void* taps;                  // T [NP][nct][ntap], transform convention
    void* taps_d;                // T [NP][nct][ntap], direct convention
    void* taps_yz;               // T [h1][nct_yz][yz_nu]: partial x-spectra over the (y, z) quarter disc (3D)
    int yz_mt, yz_nu;            // its radius in spacings (0: no (y, z) direct pass) and tap count
    int nct_yz;                  // components in taps_yz (nct, + 3 scaled copies k_a a0_i for LPS)
    void* stat;                  // T [nb][ncs]
    void* stat_int;              // T [ncs]: the static fields at interior nodes
    double stat_int_h[10];       // the same values (rounded to T) on the host
    long n_edge;                 // body-box nodes that are not interior
    uint8_t* chiB;               // [nb] body | interior << 1 (interior: whole horizon in the body)
    uint8_t* chiO;               // [dim][nb]
    void* SA;                    // complex T workspaces (see pd_passes.hpp)
    void* SB;
    long saf_cap, sbf_cap, scf_cap;   // field capacity of each workspace
    int Pz;                      // z pitch of SB (body planes rounded up to 16)
    long sbf;                    // field stride of SB: h1*n2*Pz
    void* theta;                 // T [nb] (LPS)
    void* vtmp;                  // T [dim][nb] scratch (solver / adjoint)
    void* vtmp2;                 // T [dim][nb]
    double* partials;            // per-block reduction partials
    long partials_cap;
    double* red;                 // final reductions [8]
    double* red_host;            // pinned host copy [16]
    double* red_host_dev;        // device address of red_host (null if not mapped)
    hipEvent_t lag_ev[2];        // completion events of the solver's lagged residual reads
    int* offs_dev;               // stencil offsets [ns][3]
    void* etab;                  // T [ns][4]: xi_x, xi_y, alpha omega / |xi|^2 dV, 0 (2D bond-based energy)
    int emt;                     // largest |o_x|, |o_y| of the stencil (halo of the energy kernel)
    int energy_form;             // 0: W by direct bond sums, 1: by the convolution form (test mode)
    double* kval_dev;            // kernel values [ns][ncs]
    size_t bytes;
    std::vector<ProfRec>* prof;  // non-null while pass timing is enabled
    pd_plan_s* sub32;            // FP32 operator for the mixed solve
    pd_plan_s* parent;           // set on sub32
};

namespace pdh {

pd_status check(hipError_t e);

}  // namespace pdh
