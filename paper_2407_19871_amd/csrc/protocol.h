// Launchers of the protocol kernels (protocol.hip).
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

}  // namespace lp
