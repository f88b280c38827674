// Arithmetic in the Goldilocks field Z_p, p = 2^64 - 2^32 + 1, on 64-bit
// lanes of a gfx950 wavefront.
//
// The blind rotation's external product is an exact integer negacyclic
// product of 7-bit gadget digits with 32-bit key coefficients: every output
// coefficient is a sum of 2*l*N = 6144 terms below 2^6 * 2^32, so it lies
// in (-2^50.6, 2^50.6) and is recovered exactly from its residue mod p
// (p/2 > 2^63).  The identities used for reduction are
//   2^64 = 2^32 - 1 (mod p)  and  2^96 = -1 (mod p),
// so 2 is a 192nd root of unity and every 64th root of unity is a power of
// two: the butterflies of 32-point transforms need only shifts.
//
// Representation: every value handed between these functions is canonical,
// i.e. in [0, p).  Each function documents why its result stays canonical.
#pragma once
#include <stdint.h>

#define GL_P 0xFFFFFFFF00000001ull
#define GL_EPS 0x00000000FFFFFFFFull /* 2^64 - p = 2^32 - 1 */

#ifdef __HIPCC__
#define GL_INLINE __device__ __host__ __forceinline__
#else
#define GL_INLINE inline
#endif

// a + b for a, b < p.  If the 64-bit sum carries, the true sum is s + 2^64
// = s + EPS (mod p) and s + EPS < p because s < 2p - 2^64.  Otherwise the
// sum is >= p exactly when s + EPS carries, and then s - p = s + EPS - 2^64.
GL_INLINE uint64_t gl_add(uint64_t a, uint64_t b) {
  uint64_t s = a + b;
  uint64_t t = s + GL_EPS;
  bool c1 = s < a;
  bool c2 = t < s;
  return (c1 || c2) ? t : s;
}

// a - b for a, b < p.  On borrow the wrapped difference is a - b + 2^64, and
// subtracting EPS gives a - b + p, which lies in (EPS, p) -- no second wrap.
GL_INLINE uint64_t gl_sub(uint64_t a, uint64_t b) {
  uint64_t d = a - b;
  return (a < b) ? d - GL_EPS : d;
}

GL_INLINE uint64_t gl_neg(uint64_t a) { return a == 0 ? 0 : GL_P - a; }

// x = lo + 2^64 hi (any 128-bit value) reduced to [0, p):
//   x = lo + 2^64 hl + 2^96 hh = lo - hh + (2^32 - 1) hl  (mod p).
// t0 = lo - hh: on borrow lo < hh < 2^32, so the wrapped value is >= p and
//   subtracting EPS keeps it in [0, 2^64).
// t1 = hl * (2^32 - 1) < 2^64.  r = t0 + t1: on carry the wrapped sum is
//   < 2^64 - 2^33 + 1 and adding EPS neither carries nor reaches p; without
//   carry a final conditional subtraction of p makes r canonical.
GL_INLINE uint64_t gl_reduce128(uint64_t lo, uint64_t hi) {
  uint32_t hh = (uint32_t)(hi >> 32);
  uint32_t hl = (uint32_t)hi;
  uint64_t t0 = lo - hh;
  if (lo < (uint64_t)hh) t0 -= GL_EPS;
  uint64_t t1 = ((uint64_t)hl << 32) - hl;
  uint64_t r = t0 + t1;
  bool c = r < t0;
  uint64_t u = r + GL_EPS;
  bool c2 = u < r;
  return (c || c2) ? u : r;
}

// 64 x 64 -> 128-bit product from four 32 x 32 -> 64 multiply-adds; no
// intermediate overflows because (2^32-1)^2 + 2*(2^32-1) < 2^64.
GL_INLINE void gl_mul_wide(uint64_t a, uint64_t b, uint64_t& lo, uint64_t& hi) {
  uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  uint64_t t = (uint64_t)a0 * b0;
  uint64_t m1 = (uint64_t)a0 * b1 + (t >> 32);
  uint64_t m2 = (uint64_t)a1 * b0 + (uint32_t)m1;
  uint64_t h = (uint64_t)a1 * b1 + (m1 >> 32);
  hi = h + (m2 >> 32);
  lo = (m2 << 32) | (uint32_t)t;
}

GL_INLINE uint64_t gl_mul(uint64_t a, uint64_t b) {
  uint64_t lo, hi;
  gl_mul_wide(a, b, lo, hi);
  return gl_reduce128(lo, hi);
}

// x * 2^S mod p for a compile-time S.  2^96 = -1 folds S into [0, 96);
// shifts below 64 produce a 128-bit value for gl_reduce128; shifts in
// [64, 96) are done as two smaller shifts.
template <int S>
GL_INLINE uint64_t gl_mul_pow2(uint64_t x) {
  constexpr int s = ((S % 192) + 192) % 192;
  if constexpr (s == 0) {
    return x;
  } else if constexpr (s >= 96) {
    return gl_neg(gl_mul_pow2<s - 96>(x));
  } else if constexpr (s < 64) {
    return gl_reduce128(x << s, x >> (64 - s));
  } else {
    return gl_mul_pow2<32>(gl_mul_pow2<s - 32>(x));
  }
}

// Canonical residue of a signed integer |v| < 2^63.
GL_INLINE uint64_t gl_from_i64(int64_t v) { return v < 0 ? (uint64_t)v + GL_P : (uint64_t)v; }

// Centred lift of a canonical residue to the integers, reduced mod 2^32: a
// residue r > (p-1)/2 stands for r - p, whose low word is low32(r) - 1
// because low32(p) = 1.
GL_INLINE uint32_t gl_lift_u32(uint64_t r) {
  return (uint32_t)r - (r > (GL_P >> 1) ? 1u : 0u);
}
