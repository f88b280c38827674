// Arithmetic in the Goldilocks field Z_p, p = 2^64 - 2^32 + 1, on 64-bit
// lanes of a gfx950 wavefront.
//
// The blind rotation's external product is an exact integer negacyclic
// product of 7-bit gadget digits with 32-bit key coefficients: every output
// coefficient is a sum of 2*l*N = 6144 terms below 2^6 * 2^32, so it lies
// in (-2^50.6, 2^50.6) and is recovered exactly from its residue mod p
// (p/2 > 2^63).  The identities used for reduction are
//   2^64 = 2^32 - 1 = EPS (mod p)  and  2^96 = -1 (mod p),
// so 2 is a 192nd root of unity and every 64th root of unity is a power of
// two: the butterflies of 32-point transforms need only shifts.
//
// Representation ("lazy"): a residue is held as any 64-bit value x in
// [0, 2^64) with x = residue (mod p); only gl_canon() maps to [0, p).
// Every function is exact for all 64-bit inputs.  Carries come from the
// overflow builtins, which gfx950 executes as v_add_co/v_addc_co (and the
// subtract forms) with the carry in a scalar register.
#pragma once
#include <stdint.h>

#define GL_P 0xFFFFFFFF00000001ull
#define GL_EPS 0x00000000FFFFFFFFull /* 2^64 - p = 2^32 - 1 */

#ifdef __HIPCC__
#define GL_INLINE __device__ __host__ __forceinline__
#else
#define GL_INLINE inline
#endif

// a + b.  A carry means the true sum is s + 2^64 = s + EPS (mod p).  Adding
// EPS can carry again only when s >= p; the wrapped value is then below EPS
// and a second EPS cannot carry.
GL_INLINE uint64_t gl_add(uint64_t a, uint64_t b) {
  uint64_t s;
  const bool c1 = __builtin_add_overflow(a, b, &s);
  const bool c2 = __builtin_add_overflow(s, c1 ? GL_EPS : 0ull, &s);
  return s + (c2 ? GL_EPS : 0ull);
}

// Reduces any 64-bit value to [0, p): x >= p iff x + EPS carries.
GL_INLINE uint64_t gl_canon(uint64_t a) {
  uint64_t t;
  const bool c = __builtin_add_overflow(a, GL_EPS, &t);
  return c ? t : a;
}

// x = lo + 2^64 hi (any 128-bit value) mod p:
//   x = lo + 2^64 hl + 2^96 hh = lo - hh + EPS * hl   (mod p).
// t0 = lo - hh: a borrow needs lo < hh < 2^32, so the wrapped value is at
//   least p and subtracting EPS cannot borrow again.
// t1 = hl * EPS = (hl << 32) - hl < 2^64.
// t0 + t1: a carry leaves a wrapped sum below 2^64 - 2^33 + 1, so adding EPS
//   cannot carry again.
GL_INLINE uint64_t gl_reduce128(uint64_t lo, uint64_t hi) {
  const uint32_t hh = (uint32_t)(hi >> 32);
  const uint32_t hl = (uint32_t)hi;
  uint64_t t0;
  const bool b = __builtin_sub_overflow(lo, (uint64_t)hh, &t0);
  t0 -= b ? GL_EPS : 0ull;
  const uint64_t t1 = ((uint64_t)hl << 32) - hl;
  uint64_t r;
  const bool c = __builtin_add_overflow(t0, t1, &r);
  return r + (c ? GL_EPS : 0ull);
}

// 64 x 64 -> 128-bit product from four 32 x 32 -> 64 multiply-adds; no
// intermediate overflows because (2^32-1)^2 + 2*(2^32-1) < 2^64.
GL_INLINE void gl_mul_wide(uint64_t a, uint64_t b, uint64_t& lo, uint64_t& hi) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t t = (uint64_t)a0 * b0;
  const uint64_t m1 = (uint64_t)a0 * b1 + (t >> 32);
  const uint64_t m2 = (uint64_t)a1 * b0 + (uint32_t)m1;
  const uint64_t h = (uint64_t)a1 * b1 + (m1 >> 32);
  hi = h + (m2 >> 32);
  lo = (m2 << 32) | (uint32_t)t;
}

GL_INLINE uint64_t gl_mul(uint64_t a, uint64_t b) {
  uint64_t lo, hi;
  gl_mul_wide(a, b, lo, hi);
  return gl_reduce128(lo, hi);
}

// ---- reduced operands -----------------------------------------------------
// A value in [0, p] is "reduced" (p stands for 0).  Adding or subtracting a
// reduced operand needs only one correction, which is why the transforms
// keep every twiddle product reduced.

// a + b, any a, reduced b: a carry leaves s = a + b - 2^64 < p, so adding
// EPS cannot carry again.
GL_INLINE uint64_t gl_add_r(uint64_t a, uint64_t b) {
  uint64_t s;
  const bool c = __builtin_add_overflow(a, b, &s);
  return s + (c ? GL_EPS : 0ull);
}

// a - b, any a, reduced b, as a + ~b + k (~b = 2^64 - 1 - b).  If a >= b,
// k = 1 gives a - b.  If a < b the result is a - b + p, which lies in
// [0, p) because b <= p; modulo 2^64 that is a + ~b + 1 - EPS, so
// k = 2 - 2^32.
GL_INLINE uint64_t gl_sub_r(uint64_t a, uint64_t b) {
  const uint64_t k = a < b ? 0xFFFFFFFF00000002ull : 1ull;
  return (a + ~b) + k;
}

// -y for reduced y: p - y = ~y + 2 - 2^32 (mod 2^64), again reduced.
GL_INLINE uint64_t gl_neg_r(uint64_t y) { return ~y + 0xFFFFFFFF00000002ull; }

// a b + c d mod p with one reduction, a b given as its 128-bit product
// (l1, h1).  The two 128-bit products sum to at most 2^129; the carry into
// bit 128 stands for 2^128 = 2^96 2^32 = -2^32.
GL_INLINE uint64_t gl_mul_sum_wide(uint64_t l1, uint64_t h1, uint64_t c, uint64_t d) {
  uint64_t l2, h2, lo, hi;
  gl_mul_wide(c, d, l2, h2);
  const bool c1 = __builtin_add_overflow(l1, l2, &lo);
  const bool c2 = __builtin_add_overflow(h1, h2 + (c1 ? 1ull : 0ull), &hi);  // h2 <= 2^64 - 2
  return gl_sub_r(gl_reduce128(lo, hi), c2 ? 0x100000000ull : 0ull);
}

// a b + c d mod p with one reduction.
GL_INLINE uint64_t gl_mul_sum(uint64_t a, uint64_t b, uint64_t c, uint64_t d) {
  uint64_t l1, h1;
  gl_mul_wide(a, b, l1, h1);
  return gl_mul_sum_wide(l1, h1, c, d);
}

// a b + c d + e f mod p with one reduction.  The three 128-bit products sum
// below 3 2^128: each high word is at most 2^64 - 2, so a low-word carry
// fits in it, and at most two carries leave bit 127, each standing for
// 2^128 = -2^32.
GL_INLINE uint64_t gl_mul_sum3(uint64_t a, uint64_t b, uint64_t c, uint64_t d, uint64_t e, uint64_t f) {
  uint64_t l1, h1, l2, h2, l3, h3, lo, t, hi;
  gl_mul_wide(a, b, l1, h1);
  gl_mul_wide(c, d, l2, h2);
  gl_mul_wide(e, f, l3, h3);
  const bool c1 = __builtin_add_overflow(l1, l2, &lo);
  const bool c2 = __builtin_add_overflow(lo, l3, &lo);
  const bool o1 = __builtin_add_overflow(h1, h2 + (c1 ? 1ull : 0ull), &t);
  const bool o2 = __builtin_add_overflow(t, h3 + (c2 ? 1ull : 0ull), &hi);
  const uint64_t top = (uint64_t)o1 + (uint64_t)o2;
  return gl_sub_r(gl_reduce128(lo, hi), top << 32);
}

// acc + a b mod p with one reduction: a product of two 64-bit values has
// a high word of at most 2^64 - 2, so the carry of adding acc to the low
// word fits in it.
GL_INLINE uint64_t gl_mac(uint64_t acc, uint64_t a, uint64_t b) {
  uint64_t lo, hi;
  gl_mul_wide(a, b, lo, hi);
  const bool c = __builtin_add_overflow(lo, acc, &lo);
  return gl_reduce128(lo, hi + (c ? 1ull : 0ull));
}

// x * 2^S mod p for a compile-time S; for S mod 192 = 0 the result is x
// itself, for S mod 192 in (0, 64) it is lazy, and for S mod 192 in
// [64, 192) it is reduced (see gl_mul_pow2_r).  2^96 = -1 folds S into
// [0, 96) with a negation.
//   0 < s < 32:   x 2^s = w0 + 2^32 w1 + 2^64 w2 with w2 < 2^31, i.e.
//                 (w1:w0) + EPS w2;
//   32 <= s < 64: the three high words are reduced by gl_reduce128;
//   64 <= s < 96: with k = 96 - s, x = xh 2^k + xl (xl < 2^k):
//                 x 2^s = xh 2^96 + xl 2^(s-64) 2^64 = -xh + w EPS, where
//                 w = xl 2^(s-64) < 2^32; w EPS < p and xh < 2^63, so one
//                 reduced subtraction gives a value in [0, p).
template <int S>
GL_INLINE uint64_t gl_mul_pow2_r(uint64_t x);

template <int S>
GL_INLINE uint64_t gl_mul_pow2(uint64_t x) {
  constexpr int s = ((S % 192) + 192) % 192;
  if constexpr (s == 0) {
    return x;
  } else if constexpr (s >= 96) {
    return gl_neg_r(gl_mul_pow2_r<s - 96>(x));
  } else if constexpr (s < 32) {
    const uint64_t low = x << s;
    const uint32_t w2 = (uint32_t)(x >> (64 - s));
    const uint64_t t = ((uint64_t)w2 << 32) - w2;  // EPS * w2 < 2^63
    uint64_t r;
    const bool c = __builtin_add_overflow(low, t, &r);
    return r + (c ? GL_EPS : 0ull);
  } else if constexpr (s < 64) {
    return gl_reduce128(x << s, x >> (64 - s));
  } else {
    const uint64_t xh = x >> (96 - s);
    const uint32_t w = (uint32_t)x << (s - 64);
    return gl_sub_r(((uint64_t)w << 32) - w, xh);
  }
}

// x * 2^S reduced to [0, p].
template <int S>
GL_INLINE uint64_t gl_mul_pow2_r(uint64_t x) {
  constexpr int s = ((S % 192) + 192) % 192;
  if constexpr (s < 64) {
    return gl_canon(gl_mul_pow2<s>(x));
  } else {
    return gl_mul_pow2<s>(x);  // reduced by construction
  }
}

// Residue of a signed integer |v| < 2^63.
GL_INLINE uint64_t gl_from_i64(int64_t v) { return v < 0 ? (uint64_t)v + GL_P : (uint64_t)v; }

// Centred lift of a residue to the integers, reduced mod 2^32: the canonical
// residue r > (p-1)/2 stands for r - p, whose low word is low32(r) - 1
// because low32(p) = 1.
GL_INLINE uint32_t gl_lift_u32(uint64_t x) {
  const uint64_t r = gl_canon(x);
  return (uint32_t)r - (r > (GL_P >> 1) ? 1u : 0u);
}
