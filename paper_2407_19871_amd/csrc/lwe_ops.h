// Launchers of the streaming LWE kernels (lwe_ops.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lp {

// Preprocess (Algorithm 1): out[k] = zero[k] + (0, f(bits[k])) over cnt
// samples of n_lwe + 1 words; f(nonzero) = +1/8, f(0) = -1/8.  out may
// alias zero.
hipError_t launch_preprocess(const uint32_t* d_zero, const uint8_t* d_bits, uint32_t* d_out, size_t cnt,
                             int n_lwe, hipStream_t s);

// out[k] = (0, cst) + ex[2k] + ex[2k+1] over cnt output samples of w words
// (the MUX sum of two extracted samples); out must not alias ex.
hipError_t launch_lwe_pair_sum(const uint32_t* d_ex, uint32_t* d_out, size_t cnt, int w, uint32_t cst,
                               hipStream_t s);

}  // namespace lp
