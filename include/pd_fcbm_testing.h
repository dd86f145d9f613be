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

/* Kernel selection for A/B tests: generic_only != 0 makes every later call on
 * `plan` (and on its FP32 operator, for PD_PLAN_MIXED plans) use the generic
 * runtime-length last-axis kernel instead of the specialised one (512-point
 * lines, 4 taps).  Both compute the same multiplier; results agree to
 * rounding.  PD_EINVAL for a null plan. */
pd_status pd_test_set_generic(pd_plan plan, int generic_only);

#ifdef __cplusplus
}
#endif

#endif
