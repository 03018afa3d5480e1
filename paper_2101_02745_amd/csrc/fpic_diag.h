// Diagnostic reductions over moment fields (fpic_diag.hip).  Not part of the
// public ABI (see include/fpic.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fpic {

// Sums over the cells of the moment magnitudes of m[72][ncell] (the layout
// fpic_moments writes): for each of n, f_x, nbar, fbar_x, the three |diagonal|
// entries and the three |off-diagonal| magnitudes, out[4][6].  nblk blocks;
// scratch holds nblk * 24 doubles of partial sums.  Fixed summation order.
hipError_t launch_domain_sums(const double *m, int64_t ncell, int nblk, double *scratch,
                              double *out24, hipStream_t s);

}  // namespace fpic
