/* dotpe_test.h -- hooks of libdotpe.so for checking parts of the hot path
 * on their own.  Not part of the product interface: the parity tests use
 * them to compare single steps with the oracle.  Same error convention as
 * dotpe.h. */
#ifndef DOTPE_TEST_H
#define DOTPE_TEST_H

#include "dotpe.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Evaluate the device distance-marginalisation rule (eq. lnl_dist_marginalized,
 * prior proportional to D^2 on (0, D_max]) for n (dh, hh) pairs given at
 * distance d0: out[j] = ln Lbar(dh[j], hh[j]).  d0_over_dmax = d0 / D_max.
 * dh, hh, out: host arrays of n doubles.  Synchronous.  Errors:
 * INVALID_ARG (NULL array with n > 0, n < 0), DEVICE. */
int dotpe_debug_distmarg(dotpe_ctx* ctx, int64_t n, const double* dh, const double* hh,
                         double d0_over_dmax, double* out);

/* Copy back the event's extrinsic response (eq. response_plus/cross,
 * t_at_detector): R [n_ext][n_det][n_modes][2] (interleaved complex) and
 * t [n_ext][n_det] seconds, host arrays, channels in the bank's input order.
 * Synchronous.  Errors: INVALID_ARG, DEVICE. */
int dotpe_debug_response(dotpe_ctx* ctx, const dotpe_event* ev, double* R, double* t);

/* The bound pass's certified upper bounds on each pair's largest lnL^ML over
 * the phases (eq. bestfit_lnl), from the hi parts of the split operands and
 * the Cauchy-Schwarz margin for the rest: out [2][n_sub][n_ext] host floats,
 * plane 0 with the margin from the norms of whole rows, plane 1 with the
 * margin per m group and (h|h) output; +inf where the (h|h) lower bound is
 * not positive.  Nothing is cut and the event's evidence state is
 * untouched.  Synchronous.  Errors: INVALID_ARG (FP64 bank), OOM /
 * ADMISSION, DEVICE. */
int dotpe_debug_bound(dotpe_ctx* ctx, dotpe_event* ev, float* out);

#ifdef __cplusplus
}
#endif

#endif /* DOTPE_TEST_H */
