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

#ifdef __cplusplus
}
#endif

#endif
