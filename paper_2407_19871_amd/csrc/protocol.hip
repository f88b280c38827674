// Cloud-side kernels of the protocol around the bootstrapping path (Sec. 3).
//
// Preprocess (Algorithm 1): the cloud encrypts its plaintext service bits
// without the secret key by adding the trivial sample (0, f(bit)) to one of
// the client's fresh samples of zero each; f(1) = +1/8 and f(0) = -1/8 on
// the torus, the encoding of Encrypt (Sec. 2.2).  It is a streaming copy
// that changes one word per sample, bound by HBM.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "protocol.h"

namespace lp {

// One row of blocks per sample (grid-strided over samples), so each block
// reads and writes consecutive words; only the body word changes.
__global__ void preprocess_kernel(const uint32_t* zero, const uint8_t* __restrict__ bits, uint32_t* out,
                                  size_t cnt, int n_lwe) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > n_lwe) return;
  for (size_t k = blockIdx.y; k < cnt; k += gridDim.y) {
    const size_t i = k * (size_t)(n_lwe + 1) + c;
    uint32_t v = zero[i];
    if (c == n_lwe) v += bits[k] ? 0x20000000u : 0xE0000000u;
    out[i] = v;
  }
}

hipError_t launch_preprocess(const uint32_t* d_zero, const uint8_t* d_bits, uint32_t* d_out, size_t cnt,
                             int n_lwe, hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  const unsigned gx = (unsigned)((n_lwe + 1 + 255) / 256);
  const unsigned gy = (unsigned)(cnt < 16384 ? cnt : 16384);
  hipLaunchKernelGGL(preprocess_kernel, dim3(gx, gy), dim3(256), 0, s, d_zero, d_bits, d_out, cnt, n_lwe);
  return hipGetLastError();
}

}  // namespace lp
