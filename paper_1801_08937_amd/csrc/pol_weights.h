// Polarisation weights of one sample, Eq. datamodel: the pointing row of a
// sample at angle psi is (1, cos 2psi, sin 2psi).  Every kernel that forms
// the weights calls this one function, so weights computed on the fly and
// weights stored at pointing build are the same bits, and P and P^T stay
// exact transposes of each other.
#pragma once

#include <hip/hip_runtime.h>

namespace mm {

__device__ __forceinline__ void pol_weights(double psi, double &c, double &s) {
    sincos(2.0 * psi, &s, &c);
}

}  // namespace mm
