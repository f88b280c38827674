// Streaming kernels on LWE samples around the bootstrapping path, each a
// coalesced pass bound by HBM.
//
// Preprocess (Algorithm 1, Sec. 3): the cloud encrypts its plaintext service
// bits without the secret key by adding the trivial sample (0, f(bit)) to
// one of the client's fresh samples of zero each; f(1) = +1/8 and f(0) =
// -1/8 on the torus, the encoding of Encrypt (Sec. 2.2).
//
// MUX combination: a MUX bootstraps (sel AND t) and (NOT sel AND f) and
// adds the two extracted samples to (0, 1/8) before its key switch; when the
// caller asks for the samples before key switching, this pass forms that
// sum.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lwe_ops.h"

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

// out[k] = (0, cst) + ex[2k] + ex[2k+1], samples of w words; one row of
// blocks per output sample.
__global__ void lwe_pair_sum_kernel(const uint32_t* __restrict__ ex, uint32_t* __restrict__ out, size_t cnt, int w,
                                    uint32_t cst) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= w) return;
  for (size_t k = blockIdx.y; k < cnt; k += gridDim.y) {
    uint32_t v = ex[(2 * k) * (size_t)w + c] + ex[(2 * k + 1) * (size_t)w + c];
    if (c == w - 1) v += cst;
    out[k * (size_t)w + c] = v;
  }
}

hipError_t launch_lwe_pair_sum(const uint32_t* d_ex, uint32_t* d_out, size_t cnt, int w, uint32_t cst,
                               hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  const unsigned gx = (unsigned)((w + 255) / 256);
  const unsigned gy = (unsigned)(cnt < 16384 ? cnt : 16384);
  hipLaunchKernelGGL(lwe_pair_sum_kernel, dim3(gx, gy), dim3(256), 0, s, d_ex, d_out, cnt, w, cst);
  return hipGetLastError();
}

}  // namespace lp
