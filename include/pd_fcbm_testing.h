/*
 * pd_fcbm_testing.h -- test-only entry point of libpdfcbm (not part of the
 * supported API; used by the FFT unit tests).
 */
#ifndef PD_FCBM_TESTING_H
#define PD_FCBM_TESTING_H

#include "pd_fcbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Correlation of a scalar body-box field x (plan dtype, DEVICE) with the
 * separable test kernel K(o) = prod_d k_d(o_d), where k_d(o) = [o = s_d] +
 * (-1)^{p_d} [o = -s_d] for s_d > 0 and [o = 0] for s_d = 0, p_d = bit d of
 * `parity`:  out(x) = sum_o K(o) x(x + o), x zero outside the body box.  It
 * runs the same FFT passes and spectral-multiply machinery as pd_force
 * (partial spectra along the last axis, i^P factor for P odd axes), so a
 * comparison with shifted copies of x checks the transforms, the
 * normalisation and the wavenumber bookkeeping.  shift: HOST int[3] with
 * s_d >= 0 and s_last <= 8; a set parity bit needs s_d > 0 (else PD_EINVAL).
 * Synchronises the stream. */
pd_status pd_test_conv(pd_plan plan, const void* x, const int* shift, int parity, void* out, void* stream);

/* Kernel selection after the x transform, for A/B tests (every later call
 * on `plan`, and on its FP32 operator for PD_PLAN_MIXED plans):
 *   PD_LASTAXIS_AUTO         3D: direct 2D correlation over (y, z) per
 *                            x-wavenumber when the horizon's (y, z) footprint
 *                            is a disc of radius 2 or 3 spacings, for the LPS
 *                            and unweighted bond-based chains; otherwise as
 *                            PD_LASTAXIS_YFFT.
 *                            2D: as PD_LASTAXIS_YFFT (default)
 *   PD_LASTAXIS_YFFT         transform along y (3D), then the direct line
 *                            correlation along the last axis when the horizon
 *                            spans at most 4 spacings there, else the
 *                            transform form
 *   PD_LASTAXIS_FFT          transforms along every axis: along the last one
 *                            transform, spectral multiply, inverse transform
 *                            (specialised kernel for 512-point lines with 4
 *                            taps, else runtime length)
 *   PD_LASTAXIS_FFT_GENERIC  transform form, runtime-length kernel only
 * All compute the same correlation; results agree to rounding.  PD_EINVAL
 * for a null plan or an unknown mode. */
enum { PD_LASTAXIS_AUTO = 0, PD_LASTAXIS_FFT = 1, PD_LASTAXIS_FFT_GENERIC = 2, PD_LASTAXIS_YFFT = 3 };
pd_status pd_test_set_lastaxis(pd_plan plan, int mode);

/* How the strain energy density W of the weighted bond-based solid is
 * evaluated (pd_force's W_out and the energy failure rule of
 * pd_verlet_step), for A/B tests:
 *   PD_ENERGY_DIRECT       direct bond sums (Eq. 42 with the weights of
 *                          Eq. 46), the default
 *   PD_ENERGY_CONVOLUTION  the convolution form (Eq. 64/102) in the force's
 *                          chain; its terms of order (chi u)^2 cancel to
 *                          (u' - u)^2, so in FP32 its error grows with the
 *                          square of the displacement
 * PD_EINVAL for a null plan or an unknown form. */
enum { PD_ENERGY_DIRECT = 0, PD_ENERGY_CONVOLUTION = 1 };
pd_status pd_test_set_energy_form(pd_plan plan, int form);

#ifdef __cplusplus
}
#endif

#endif
