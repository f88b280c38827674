// The CMux external product of one blind-rotation step (Sec. 2.2,
// Bootstrap) on the int8 matrix cores instead of the NTT: an exact
// experiment beside the NTT path.
//
// For a batch of accumulator differences D_b (TRLWE, 2 x 1024 Torus32) and
// one bootstrapping-key row set BSK_i (2l rows r = (p, j), each a TRLWE of 2
// components), the product is
//   R_b[c] = sum_r dec_r(D_b) * BSK_i[r][c]   in Z[X]/(X^1024 + 1), mod 2^32,
// with the gadget digits dec_r in [-64, 64).  As matrices: R[c] (1024 x B) =
// sum_r T(BSK_i[r][c]) (1024 x 1024) x Dig_r (1024 x B), where T(K) is the
// negacyclic Toeplitz matrix, T[i][t] = K[i - t] for i >= t and -K[i - t + N]
// otherwise.  Each key word is split into four balanced bytes, K = sum_k
// 2^(8k) K_k mod 2^32 with K_k in [-128, 128), so every product is an int8 x
// int8 MFMA (v_mfma_i32_32x32x16_i8) summed exactly in int32: a sum has 6144
// terms of magnitude at most 128 * 64, below 2^26.  The four limb sums are
// combined as sum_k 2^(8k) S_k mod 2^32.
//
// A fragment of T is eight consecutive columns of one row, i.e. eight
// consecutive bytes of the reversed, sign-extended key
//   V[y] = W[2N - 1 - y],  W[z] = K[z - N] (z >= N), -K[z] (z < N),
// at byte offset N - 1 - i + t, which is arbitrary: it is assembled from
// three aligned LDS words with two byte-aligned funnel shifts.
//
// Kernels: digits of every input ([b][r][1024] int8, padded batch), the key
// limbs of the step ([c][k][r][2N] int8), the matrix product (partial sums
// over a quarter of the 6144 products per workgroup, four waves each) and
// the sum of the quarters into [b][c][1024] u32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace lp {

namespace {

constexpr int XN = 1024;        // ring degree
constexpr int XR = 6;           // key rows (2 components x 3 gadget levels)
constexpr int XK = XR * XN;     // products summed per output coefficient
constexpr int XSPLIT = 4;       // workgroups sharing the products of one output tile
constexpr int XCOLS = 64;       // batch columns of one workgroup (two 32-wide tiles)
constexpr int XROWS = 32;       // output rows of one workgroup

typedef int v16i __attribute__((ext_vector_type(16)));

// dig[b][r][t], r = p * 3 + j: digit j of coefficient t of component p of D_b
// (signed digits, offset 0x81020400, as the blind rotation takes them);
// padded batch rows beyond cnt are zero.
__global__ void xp_digits_kernel(const uint32_t* __restrict__ d_in, int cnt, int8_t* __restrict__ dig) {
  const int b = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;  // 0 .. 2N-1 over both components
  if (t >= 2 * XN) return;
  const int p = t / XN, c = t % XN;
  const uint32_t a = b < cnt ? d_in[(size_t)b * 2 * XN + t] + 0x81020400u : 0x81020400u;
  for (int j = 0; j < 3; ++j) {
    const int d = b < cnt ? (int)((a >> (25 - 7 * j)) & 127u) - 64 : 0;
    dig[((size_t)b * XR + p * 3 + j) * XN + c] = (int8_t)d;
  }
}

// lim[c][k][r][y] = limb k of V_(r,c)[y] (see above).
__global__ void xp_key_limbs_kernel(const uint32_t* __restrict__ key, int8_t* __restrict__ lim) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;  // 0 .. 2N-1
  const int r = blockIdx.y, c = blockIdx.z;
  if (y >= 2 * XN) return;
  const int z = 2 * XN - 1 - y;
  const uint32_t k = key[((size_t)r * 2 + c) * XN + (z >= XN ? z - XN : z)];
  uint32_t w = z >= XN ? k : 0u - k;
  for (int l = 0; l < 4; ++l) {
    const int8_t v = (int8_t)(w & 0xFFu);  // balanced byte in [-128, 128)
    lim[(((size_t)c * 4 + l) * XR + r) * (2 * XN) + y] = v;
    w = (w - (uint32_t)(int32_t)v) >> 8;
  }
}

// Eight bytes at an arbitrary byte offset o of a word-aligned LDS array.
__device__ __forceinline__ long bytes8(const uint32_t* base, int o) {
  const int q = o >> 2, sh = o & 3;
  const uint32_t w0 = base[q], w1 = base[q + 1], w2 = base[q + 2];
  const uint32_t lo = __builtin_amdgcn_alignbyte(w1, w0, sh);
  const uint32_t hi = __builtin_amdgcn_alignbyte(w2, w1, sh);
  return (long)(((uint64_t)hi << 32) | lo);
}

// Workgroup (tile, split, group): output rows 32 rt .. 32 rt + 31 of
// component c, batch columns 64 g .. 64 g + 63, products of key rows/columns
// in split s's quarter; four waves each take a quarter of that.
__global__ __launch_bounds__(256, 2) void xp_mfma_kernel(const int8_t* __restrict__ dig,
                                                       const int8_t* __restrict__ lim,
                                                       int32_t* __restrict__ part, int bpad) {
  // this component's limbs, [k][r][2N] bytes; after the products, the four
  // waves' partial sums (32 KB) in the same space
  __shared__ uint32_t s_v[4 * XR * (2 * XN) / 4];
  static_assert(4 * XROWS * XCOLS <= 4 * XR * (2 * XN) / 4, "partials must fit the limb space");
  int32_t* s_red = reinterpret_cast<int32_t*>(s_v);
  const int tile = blockIdx.x, s = blockIdx.y, g = blockIdx.z;
  const int c = tile / (XN / XROWS), rt = tile % (XN / XROWS);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

  // stage the component's limbs (48 KB) in LDS
  const uint32_t* src = reinterpret_cast<const uint32_t*>(lim + (size_t)c * 4 * XR * (2 * XN));
  for (int k = threadIdx.x; k < 4 * XR * (2 * XN) / 4; k += 256) s_v[k] = src[k];
  __syncthreads();

  v16i acc[2][4];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int l = 0; l < 4; ++l) acc[ct][l] = v16i{};

  const int row = XROWS * rt + (lane & 31);  // output coefficient i of this lane's A rows
  const int kb = 8 * (lane >> 5);            // this lane's eight products within a block of 16
  const int per_wave = XK / XSPLIT / 4;      // 384 products
  const int k0 = s * (XK / XSPLIT) + wave * per_wave;
  for (int kk = k0; kk < k0 + per_wave; kk += 16) {
    const int r = kk / XN, t = kk % XN + kb;  // key row and input coefficient of byte 0
    // B fragments: digits of columns (batch) 64 g + 32 ct + lane % 32, coefficients t .. t+7
    long bf[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int b = XCOLS * g + 32 * ct + (lane & 31);
      bf[ct] = *reinterpret_cast<const long*>(dig + ((size_t)b * XR + r) * XN + t);
    }
    const int o = XN - 1 - row + t;  // V offset of A[row][t]
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const long af = bytes8(s_v + (l * XR + r) * (2 * XN) / 4, o);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) acc[ct][l] = __builtin_amdgcn_mfma_i32_32x32x16_i8(af, bf[ct], acc[ct][l], 0, 0, 0);
    }
  }
  // combine the limbs (mod 2^32) and sum the four waves' partials in LDS;
  // accumulator register q of lane holds row 8 (q / 4) + 4 (lane / 32) + q % 4,
  // column lane % 32 of its 32 x 32 tile
  __syncthreads();  // every wave is done reading the limbs
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const uint32_t v = (uint32_t)acc[ct][0][q] + ((uint32_t)acc[ct][1][q] << 8) +
                         ((uint32_t)acc[ct][2][q] << 16) + ((uint32_t)acc[ct][3][q] << 24);
      const int rr = 8 * (q / 4) + 4 * (lane >> 5) + (q % 4);
      s_red[wave * XROWS * XCOLS + rr * XCOLS + 32 * ct + (lane & 31)] = (int32_t)v;
    }
  __syncthreads();
  for (int e = threadIdx.x; e < XROWS * XCOLS; e += 256) {
    constexpr int W = XROWS * XCOLS;
    const uint32_t v = (uint32_t)s_red[e] + (uint32_t)s_red[W + e] + (uint32_t)s_red[2 * W + e] + (uint32_t)s_red[3 * W + e];
    const int rr = e / XCOLS, col = e % XCOLS;
    // part[s][b][c][i]
    part[(((size_t)s * bpad + XCOLS * g + col) * 2 + c) * XN + XROWS * rt + rr] = (int32_t)v;
  }
}

// out[b][c][i] = sum over the splits, for b < cnt.
__global__ void xp_sum_kernel(const int32_t* __restrict__ part, int cnt, int bpad, uint32_t* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)cnt * 2 * XN) return;
  uint32_t v = 0;
  for (int s = 0; s < XSPLIT; ++s) v += (uint32_t)part[(size_t)s * bpad * 2 * XN + e];
  out[e] = v;
}

}  // namespace

size_t xp_mfma_scratch_bytes(int cnt) {
  const size_t bpad = (size_t)(cnt + XCOLS - 1) / XCOLS * XCOLS;
  return bpad * XR * XN                       // digits
         + (size_t)2 * 4 * XR * 2 * XN        // key limbs
         + (size_t)XSPLIT * bpad * 2 * XN * 4 // partial sums
         + 512;
}

hipError_t launch_extprod_mfma(const uint32_t* d_key_step, const uint32_t* d_in, int cnt, uint32_t* d_out,
                               void* scratch, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  const int bpad = (cnt + XCOLS - 1) / XCOLS * XCOLS;
  char* p = static_cast<char*>(scratch);
  int8_t* dig = reinterpret_cast<int8_t*>(p);
  p += ((size_t)bpad * XR * XN + 255) & ~size_t(255);
  int8_t* lim = reinterpret_cast<int8_t*>(p);
  p += ((size_t)2 * 4 * XR * 2 * XN + 255) & ~size_t(255);
  int32_t* part = reinterpret_cast<int32_t*>(p);
  hipLaunchKernelGGL(xp_digits_kernel, dim3(2 * XN / 256, bpad), dim3(256), 0, s, d_in, cnt, dig);
  hipLaunchKernelGGL(xp_key_limbs_kernel, dim3(2 * XN / 256, XR, 2), dim3(256), 0, s, d_key_step, lim);
  hipLaunchKernelGGL(xp_mfma_kernel, dim3(2 * XN / XROWS, XSPLIT, bpad / XCOLS), dim3(256), 0, s, dig, lim, part,
                     bpad);
  const size_t outs = (size_t)cnt * 2 * XN;
  hipLaunchKernelGGL(xp_sum_kernel, dim3((unsigned)((outs + 255) / 256)), dim3(256), 0, s, part, cnt, bpad, d_out);
  return hipGetLastError();
}

}  // namespace lp
