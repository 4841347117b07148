// Closed-form grid index of a heating transition on log-uniform grids.
//
// For a transition from bin i to bin f = i + d the photon wavelength is
// lambda = hc / (E_i (r^d - 1)), so its coordinate on the wavelength grid,
// t = ln(lambda / lambda_0) / dln(lambda), splits into a column part a_i and a
// distance part b_d: t = a_i - b_d.  Both are stored split into integer and
// fractional parts, so the bracketing grid interval jlo = floor(t) and the
// weight w = t - jlo of the log-log interpolation (Sec. 2.2, eq:interpolation)
// come out of one integer add and one float subtract with no rounding of t
// itself.  The precompute and the solver both call this function, so the set
// of rows each column touches is exactly the set the solver evaluates.
#pragma once

#include <hip/hip_runtime.h>

namespace hsd {

// ia1 = floor(a_i) - 1, fa1 = a_i - floor(a_i) + 1 in [1, 2),
// nib = -floor(b_d), fb = b_d - floor(b_d) in [0, 1).
// fd = fa1 - fb lies in (0, 2), so its integer part is 0 or 1.
__device__ __forceinline__ void transition_index(int ia1, float fa1, int nib, float fb, int& jlo, float& w) {
    const float fd = fa1 - fb;
    const int fl = static_cast<int>(fd);
    jlo = ia1 + nib + fl;
    w = __builtin_amdgcn_fractf(fd);   // fd - floor(fd), exact for fd in (0, 2)
}

}  // namespace hsd
