// Register-resident 32-point transforms over the Goldilocks field: the two
// passes of a 1024-point negacyclic NTT laid out as 32 lanes x 32 registers.
//
// The 1024-point negacyclic transform evaluates a(X) at psi^(2k+1),
// k < 1024, where psi is a primitive 2048th root of unity chosen with
// psi^32 = 8.  Writing j = j1 + 32*j2 and k = ka + 32*kb:
//   pass 1 (per j1): B_j1(ka) = sum_j2 a_{j1+32 j2} rho^{j2 (2ka+1)},
//                    rho = psi^32 = 8, a negacyclic 32-point DFT;
//   twist:           C_j1(ka) = B_j1(ka) * psi^{(2ka+1) j1};
//   pass 2 (per ka): A(ka + 32 kb) = sum_j1 C_j1(ka) omega^{kb j1},
//                    omega = psi^64 = 64, a cyclic 32-point DFT.
// rho and omega are powers of two, so both passes use shift twiddles
// (gl_mul_pow2); only the twist needs general multiplications.
//
// Every butterfly is Cooley-Tukey, t = w b then (a + t, a - t), with the
// twiddle product t reduced to [0, p] so that the sum and difference need
// one correction each (gl_add_r, gl_sub_r).
//   pass 1 forward: merged negacyclic butterflies, natural order in, slot i
//     holds ka = brv5(i) out;
//   pass 2 forward: merged cyclic butterflies (root omega, twiddle 1 on the
//     first block of each stage), natural in, slot i holds kb = brv5(i) out;
//   pass 2 inverse: cyclic decimation in time with omega^-1, bit-reversed
//     in, natural out (factor 32 left over);
//   pass 1 inverse: the same cyclic inverse with rho^-2 = omega^-1, since
//     B(ka) = sum_j2 (a_j2 rho^j2) (rho^2)^(ka j2), followed by the
//     post-twist a_j2 *= rho^-j2 (factor 32 left over).
// The two factors 32 are folded into the inverse twist.
#pragma once
#include <type_traits>

#include "gl64.h"

namespace lp {

constexpr int brv5(int x) {
  return ((x & 1) << 4) | ((x & 2) << 2) | (x & 4) | ((x & 8) >> 2) | ((x & 16) >> 4);
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// ---- pass 1, forward: merged negacyclic CT, root rho = 2^3 ----------------
template <int LEN>
__device__ __forceinline__ void fwd1_stage(uint64_t (&a)[32]) {
  static_for<0, 32 / (2 * LEN)>([&](auto blk) {
    constexpr int start = decltype(blk)::value * 2 * LEN;
    constexpr int k = 32 / (2 * LEN) + start / (2 * LEN);
    constexpr int z = 3 * brv5(k);
    static_for<0, LEN>([&](auto jj) {
      constexpr int j = start + decltype(jj)::value;
      const uint64_t t = gl_mul_pow2_r<z>(a[j + LEN]);
      a[j + LEN] = gl_sub_r(a[j], t);
      a[j] = gl_add_r(a[j], t);
    });
  });
}

// The first two stages on small signed integers (gadget digits, |d| <= 64),
// exact in int64.  Stage 1 pairs j, j+16 with twiddle rho^16 = 2^48.  Stage
// 2 pairs j, j+8 with 2^24 in the first half and j+16, j+24 with 2^72 in the
// second; with 2^64 = 2^32 - 1 and 2^96 = -1 (mod p),
//   2^24 (d1 + 2^48 d3) = 2^24 d1 + (2^40 - 2^8) d3,
//   2^72 (d1 - 2^48 d3) = (2^40 - 2^8) d1 + 2^24 d3   (mod p),
// so every stage-2 output is a signed integer below 2^55 in magnitude and
// becomes a residue once.
__device__ __forceinline__ void fwd1_first_stages_digits(const int32_t (&d)[32], uint64_t (&a)[32]) {
  static_for<0, 8>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    const int64_t d0 = d[j], d1 = d[j + 8], d2 = d[j + 16], d3 = d[j + 24];
    const int64_t s0 = d0 + d2 * (1ll << 48), s1 = d0 - d2 * (1ll << 48);
    const int64_t p = d1 * (1ll << 24) + d3 * ((1ll << 40) - (1ll << 8));
    const int64_t q = d1 * ((1ll << 40) - (1ll << 8)) + d3 * (1ll << 24);
    a[j] = gl_from_i64(s0 + p);
    a[j + 8] = gl_from_i64(s0 - p);
    a[j + 16] = gl_from_i64(s1 + q);
    a[j + 24] = gl_from_i64(s1 - q);
  });
}

__device__ __forceinline__ void fwd1_rest(uint64_t (&a)[32]) {
  fwd1_stage<4>(a);
  fwd1_stage<2>(a);
  fwd1_stage<1>(a);
}

__device__ __forceinline__ void fwd1(uint64_t (&a)[32]) {
  fwd1_stage<16>(a);
  fwd1_stage<8>(a);
  fwd1_rest(a);
}

// ---- pass 2, forward: merged cyclic CT, root omega = 2^6 ------------------
// Block b of the stage with 16/LEN blocks splits X^(2 LEN) - r^2 with
// r = omega^(LEN brv(b)), brv over log2(16/LEN) bits.
template <int LEN>
__device__ __forceinline__ void fwd2_stage(uint64_t (&a)[32]) {
  constexpr int nbits = LEN == 16 ? 0 : LEN == 8 ? 1 : LEN == 4 ? 2 : LEN == 2 ? 3 : 4;
  static_for<0, 32 / (2 * LEN)>([&](auto blk) {
    constexpr int b = decltype(blk)::value;
    constexpr int start = b * 2 * LEN;
    constexpr int z = 6 * LEN * (brv5(b) >> (5 - nbits));
    static_for<0, LEN>([&](auto jj) {
      constexpr int j = start + decltype(jj)::value;
      const uint64_t t = gl_mul_pow2_r<z>(a[j + LEN]);  // z = 0: reduction only
      a[j + LEN] = gl_sub_r(a[j], t);
      a[j] = gl_add_r(a[j], t);
    });
  });
}

__device__ __forceinline__ void fwd2(uint64_t (&a)[32]) {
  fwd2_stage<16>(a);
  fwd2_stage<8>(a);
  fwd2_stage<4>(a);
  fwd2_stage<2>(a);
  fwd2_stage<1>(a);
}

// ---- cyclic inverse: CT DIT with omega^-1 (factor 32 left over) ----------
template <int LEN>
__device__ __forceinline__ void inv_cyclic_stage(uint64_t (&a)[32]) {
  static_for<0, 32 / (2 * LEN)>([&](auto blk) {
    constexpr int start = decltype(blk)::value * 2 * LEN;
    static_for<0, LEN>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      constexpr int e = (192 - 6 * (16 / LEN) * j) % 192;
      const uint64_t t = gl_mul_pow2_r<e>(a[start + j + LEN]);
      a[start + j + LEN] = gl_sub_r(a[start + j], t);
      a[start + j] = gl_add_r(a[start + j], t);
    });
  });
}

__device__ __forceinline__ void inv_cyclic(uint64_t (&a)[32]) {
  inv_cyclic_stage<1>(a);
  inv_cyclic_stage<2>(a);
  inv_cyclic_stage<4>(a);
  inv_cyclic_stage<8>(a);
  inv_cyclic_stage<16>(a);
}

__device__ __forceinline__ void inv2(uint64_t (&a)[32]) { inv_cyclic(a); }

// ---- pass 1, inverse: cyclic inverse, then a_j2 *= rho^-j2 ----------------
__device__ __forceinline__ void inv1(uint64_t (&a)[32]) {
  inv_cyclic(a);
  static_for<1, 32>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    a[j] = gl_mul_pow2<192 - 3 * j>(a[j]);
  });
}

}  // namespace lp
