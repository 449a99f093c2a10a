// Fixed-order dot products of Bloch vectors with expansion coefficients,
// shared by the readout entry points and the recording propagator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sun {

// out_re[i] = cre + v_i . xre, out_im[i] = cim + v_i . xim (out_im/xim may be
// NULL) for v_i = v + i*ldv, i < nvec.  With part != NULL and nb > 1 each
// vector is split over nb workgroups whose partial sums (part: 2*nb*nvec
// doubles of device scratch) are added by a second kernel; otherwise one
// workgroup per vector.  Both orders are fixed for given (M, nb).
void expect_launch(int64_t M, const double* v, int64_t nvec, int64_t ldv, const double* xre, const double* xim,
                   double cre, double cim, double* out_re, double* out_im, double* part, int nb, hipStream_t s);

}  // namespace sun
