// Throughput of the field operations the blind rotation is built from, each
// run alone at full occupancy on every CU: the measured prices behind the
// rotation's algorithmic operation count.
//
// Every thread keeps 32 residues in registers (as a transform lane does) and
// applies one operation to them `iters` times; nothing touches memory until
// the end.  The operations are the transform code itself (ntt32.h), so the
// price of a butterfly is what the kernels execute for it:
//   FWD     pass-1 stages 4, 2, 1 and pass 2 of the forward transform
//           (48 + 80 = 128 shift-twiddle butterflies per iteration);
//   INV     the cyclic inverse pass (80 shift-twiddle butterflies);
//   DIGITS  the first two forward stages on gadget digits, exact in int64
//           (32 butterflies: 2 stages x 16), digits taken from the residues;
//   MUL     general Goldilocks products (the twists), 32 per iteration;
//   MULSUM  a b + c d with one reduction (the key products), 32;
//   ADD     additions of a reduced operand (the level sums), 32;
//   U32     32-bit integer additions, 32: the full-rate VALU reference.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "gl64.h"
#include "kernels.h"
#include "ntt32.h"

namespace lp {

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <int OP>
__global__ __launch_bounds__(256) void op_rate_kernel(uint64_t* __restrict__ out, int iters, uint64_t seed) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t a[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) a[i] = gl_canon(mix64(seed + tid * 32 + i));
  // reduced multipliers, different per thread so nothing folds
  const uint64_t w0 = gl_canon(mix64(seed ^ (tid + 1))), w1 = gl_canon(mix64(seed ^ (tid + 7)));
  const uint64_t w2 = gl_canon(mix64(seed ^ (tid + 13))), w3 = gl_canon(mix64(seed ^ (tid + 29)));
  for (int it = 0; it < iters; ++it) {
    if constexpr (OP == kOpFwd) {
      fwd1_rest(a);
      fwd2(a);
    } else if constexpr (OP == kOpInv) {
      inv_cyclic(a);
    } else if constexpr (OP == kOpDigits) {
      int32_t d[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) d[i] = (int32_t)((uint32_t)a[i] & 127u) - 64;
      fwd1_first_stages_digits(d, a);
    } else if constexpr (OP == kOpMul) {
#pragma unroll
      for (int i = 0; i < 32; ++i) a[i] = gl_mul(a[i], (i & 1) ? w1 : w0);
    } else if constexpr (OP == kOpMulSum) {
#pragma unroll
      for (int i = 0; i < 16; ++i) a[i] = gl_mul_sum(a[i], w0, a[i + 16], w1);
#pragma unroll
      for (int i = 16; i < 32; ++i) a[i] = gl_mul_sum(a[i], w2, a[i - 16], w3);
    } else if constexpr (OP == kOpAdd) {
#pragma unroll
      for (int i = 0; i < 32; ++i) a[i] = gl_add_r(a[i], (i & 1) ? w3 : w2);
    } else {
#pragma unroll
      for (int i = 0; i < 32; ++i) a[i] = (uint64_t)((uint32_t)a[i] + (uint32_t)a[(i + 1) & 31]);
    }
  }
  uint64_t x = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i) x ^= a[i];
  out[tid] = x;
}

// Launches of exactly the blocks that fit the chip at once: a short one
// sizes the iteration count to about target_ms, one launch of that size
// warms the clocks, and the next one is timed.  *elems receives the
// operations the timed launch performed.
template <int OP>
hipError_t time_op(int cus, uint64_t* buf, size_t buf_words, double target_ms, hipStream_t s, double* ms,
                   double* elems) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, op_rate_kernel<OP>, 256, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const size_t blocks = (size_t)per_cu * cus;
  if (blocks * 256 > buf_words) return hipErrorInvalidValue;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  auto timed = [&](int iters, uint64_t seed, float* out_ms) {
    hipError_t r = hipEventRecord(t0, s);
    if (r == hipSuccess) {
      hipLaunchKernelGGL(op_rate_kernel<OP>, dim3((unsigned)blocks), dim3(256), 0, s, buf, iters, seed);
      r = hipGetLastError();
    }
    if (r == hipSuccess) r = hipEventRecord(t1, s);
    if (r == hipSuccess) r = hipEventSynchronize(t1);
    if (r == hipSuccess) r = hipEventElapsedTime(out_ms, t0, t1);
    return r;
  };
  float f = 0.f;
  int iters = 16;
  if (e == hipSuccess) e = timed(iters, 1ull, &f);
  if (e == hipSuccess) {
    const double scale = f > 0.f ? target_ms / f : 1.0;
    iters = (int)std::min(1.0 * (1 << 22), std::max(16.0, 16.0 * scale));
    e = timed(iters, 2ull, &f);  // clocks settle at the new size
  }
  if (e == hipSuccess) e = timed(iters, 3ull, &f);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  *ms = f;
  *elems = (double)blocks * 256.0 * iters * (OP == kOpFwd ? 128 : OP == kOpInv ? 80 : 32);
  return e;
}

}  // namespace

hipError_t launch_op_rates(double target_ms, double* rates, double* ms_out, hipStream_t s) {
  if (!rates || !(target_ms > 0.0) || target_ms > 1000.0) return hipErrorInvalidValue;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const size_t words = (size_t)cus * 8 * 256;  // at most 8 resident blocks of 256 threads per CU
  uint64_t* buf = nullptr;
  e = hipMallocAsync((void**)&buf, words * 8, s);
  if (e != hipSuccess) return e;
  using Timer = hipError_t (*)(int, uint64_t*, size_t, double, hipStream_t, double*, double*);
  const Timer timers[kOpCount] = {time_op<kOpFwd>, time_op<kOpInv>, time_op<kOpDigits>, time_op<kOpMul>,
                                  time_op<kOpMulSum>, time_op<kOpAdd>, time_op<kOpU32>};
  for (int op = 0; op < kOpCount && e == hipSuccess; ++op) {
    double ms = 0.0, elems = 0.0;
    e = timers[op](cus, buf, words, target_ms, s, &ms, &elems);
    rates[op] = e == hipSuccess && ms > 0.0 ? elems / (ms * 1e-3) : 0.0;
    if (ms_out) ms_out[op] = ms;
  }
  const hipError_t e2 = hipFreeAsync(buf, s);
  const hipError_t e3 = hipStreamSynchronize(s);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = e3;
  return e;
}

}  // namespace lp
