// The 1024-point negacyclic Goldilocks NTT of one polynomial on a whole
// 64-lane wavefront: the same transform as ntt32.h (same evaluation points,
// same pass structure), with each 32-point column or row shared by the two
// lanes l and l + 32.
//
// Layout ("interleaved parity"): lane (h, l) = (lane >> 5, lane & 31) holds
// the 16 positions q = 2s + h (s = 0..15) of its column or row in slot s.
// Every butterfly stage pairs positions LEN apart; for LEN >= 2 both
// positions have the lane's parity, so the stage runs inside the lane, and
// its twiddle depends on the block alone -- the same shift for every lane,
// as in the 32-lane transform.  Only the LEN = 1 stage pairs the two lanes
// of a column: a half-wave swap gives both lanes both values, both form
// w * x_odd (a uniform shift per slot), and lane h keeps x_even + t (h = 0)
// or x_even - t (h = 1).
//   forward:  in  lane (h, l), slot s = coefficient l + 32 (2s + h)
//             out lane (h, l), slot s = A(k), k = brv5(l) + 32 brv5(2s + h),
//             which sits at offset 64 s + 2 l + h of the 32-lane layout
//             (ntt_pos), so NTT-domain keys are shared by both layouts;
//   inverse:  Gentleman-Sande stages undo the merged Cooley-Tukey stages in
//             reverse order, (X, Y) -> (X + Y, (X - Y) w^-1), with the same
//             per-block twiddles; each pass leaves a factor 32, and both
//             factors sit in the inverse twist table (the one of the 32-lane
//             transform), and the pass-1 stages also undo the negacyclic
//             factor, so there is no post-twist.
#pragma once
#include "ntt32.h"

namespace lp {

// Both values of a column pair in both of its lanes: v_permlane32_swap of
// a register with itself exchanges its upper half-wave with its lower one,
// returning (lower copy, upper copy) = (value at the even position, value at
// the odd position) in every lane.  A VALU operation, so no LDS round trip.
__device__ __forceinline__ void pair_values(uint64_t x, uint64_t& even, uint64_t& odd) {
  const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)x, (uint32_t)x, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(x >> 32), (uint32_t)(x >> 32), false, false);
  even = ((uint64_t)hi[0] << 32) | lo[0];
  odd = ((uint64_t)hi[1] << 32) | lo[1];
}

// hi_lane ? y : x without a branch (the lane's half is fixed, so a mask).
__device__ __forceinline__ uint64_t lane_select(uint64_t mask, uint64_t x, uint64_t y) {
  return (x & ~mask) | (y & mask);
}

// a - b for any two residues: b is canonicalised first.
GL_INLINE uint64_t gl_sub_any(uint64_t a, uint64_t b) { return gl_sub_r(a, gl_canon(b)); }

// ---- pass 1, forward -------------------------------------------------------
// Stages LEN = 16 and 8 on gadget digits, exact in int64 (see
// fwd1_first_stages_digits): the groups (j, j+8, j+16, j+24) share a parity,
// so lane h forms them for j = h, h+2, h+4, h+6 (local slots i, i+4, i+8,
// i+12).
__device__ __forceinline__ void fwd64_p1_digits(const int32_t (&d)[16], uint64_t (&a)[16]) {
  static_for<0, 4>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    const int64_t d0 = d[i], d1 = d[i + 4], d2 = d[i + 8], d3 = d[i + 12];
    const int64_t s0 = d0 + d2 * (1ll << 48), s1 = d0 - d2 * (1ll << 48);
    const int64_t p = d1 * (1ll << 24) + d3 * ((1ll << 40) - (1ll << 8));
    const int64_t q = d1 * ((1ll << 40) - (1ll << 8)) + d3 * (1ll << 24);
    a[i] = gl_from_i64(s0 + p);
    a[i + 4] = gl_from_i64(s0 - p);
    a[i + 8] = gl_from_i64(s1 + q);
    a[i + 12] = gl_from_i64(s1 - q);
  });
}

// One in-lane Cooley-Tukey stage of global distance LEN >= 2: local blocks
// of LEN slots, pairs (s, s + LEN/2); Z(blk) gives the block's shift.
template <int LEN, typename Zf>
__device__ __forceinline__ void ct64_stage(uint64_t (&a)[16], Zf zf) {
  static_for<0, 16 / LEN>([&](auto bb) {
    constexpr int blk = decltype(bb)::value;
    constexpr int z = decltype(zf(std::integral_constant<int, blk>{}))::value;
    static_for<0, LEN / 2>([&](auto jj) {
      constexpr int s0 = blk * LEN + decltype(jj)::value, s1 = s0 + LEN / 2;
      const uint64_t t = gl_mul_pow2_r<z>(a[s1]);
      a[s1] = gl_sub_r(a[s0], t);
      a[s0] = gl_add_r(a[s0], t);
    });
  });
}

// The LEN = 1 stage across the two lanes of a column; Z(s) per slot.
template <typename Zf>
__device__ __forceinline__ void ct64_cross(uint64_t (&a)[16], Zf zf, int lane) {
  const uint64_t odd = lane >= 32 ? ~0ull : 0ull;
  static_for<0, 16>([&](auto ss) {
    constexpr int s = decltype(ss)::value;
    constexpr int z = decltype(zf(std::integral_constant<int, s>{}))::value;
    uint64_t xe, xo;
    pair_values(a[s], xe, xo);
    const uint64_t t = gl_mul_pow2_r<z>(xo);
    a[s] = lane_select(odd, gl_add_r(xe, t), gl_sub_r(xe, t));
  });
}

template <int K>
struct IC {
  static constexpr int value = K;
};

// pass 1 (negacyclic, root rho = 2^3): block k of the stage of distance LEN
// is k = 32/(2 LEN) + blk, shift 3 brv5(k)
template <int LEN>
struct Z1 {
  template <typename B>
  constexpr auto operator()(B) const {
    return IC<3 * brv5(32 / (2 * LEN) + B::value)>{};
  }
};
// pass 2 (cyclic, root omega = 2^6): 6 LEN (brv5(b) >> (5 - log2(32/(2 LEN))))
template <int LEN>
struct Z2 {
  static constexpr int nbits = LEN == 16 ? 0 : LEN == 8 ? 1 : LEN == 4 ? 2 : LEN == 2 ? 3 : 4;
  template <typename B>
  constexpr auto operator()(B) const {
    return IC<6 * LEN * (brv5(B::value) >> (5 - nbits))>{};
  }
};

__device__ __forceinline__ void fwd64_p1_rest(uint64_t (&a)[16], int lane) {
  ct64_stage<4>(a, Z1<4>{});
  ct64_stage<2>(a, Z1<2>{});
  ct64_cross(a, Z1<1>{}, lane);
}

__device__ __forceinline__ void fwd64_p2(uint64_t (&a)[16], int lane) {
  ct64_stage<16>(a, Z2<16>{});
  ct64_stage<8>(a, Z2<8>{});
  ct64_stage<4>(a, Z2<4>{});
  ct64_stage<2>(a, Z2<2>{});
  ct64_cross(a, Z2<1>{}, lane);
}

// ---- inverse: Gentleman-Sande ---------------------------------------------
// Stages after the first take reduced inputs (every stage leaves its
// outputs reduced: sums canonicalised, products by gl_mul_pow2_r), so the
// sum and the difference need one correction each.
template <int LEN, typename Zf>
__device__ __forceinline__ void gs64_stage(uint64_t (&a)[16], Zf zf) {
  static_for<0, 16 / LEN>([&](auto bb) {
    constexpr int blk = decltype(bb)::value;
    constexpr int z = decltype(zf(std::integral_constant<int, blk>{}))::value;
    static_for<0, LEN / 2>([&](auto jj) {
      constexpr int s0 = blk * LEN + decltype(jj)::value, s1 = s0 + LEN / 2;
      const uint64_t x = a[s0], y = a[s1];
      a[s0] = gl_canon(gl_add_r(x, y));
      a[s1] = gl_mul_pow2_r<192 - z>(gl_sub_r(x, y));
    });
  });
}

// The first stage of a pass, across the two lanes of a column; its inputs
// may be lazy, its outputs are reduced.
template <typename Zf>
__device__ __forceinline__ void gs64_cross(uint64_t (&a)[16], Zf zf, int lane) {
  const uint64_t odd = lane >= 32 ? ~0ull : 0ull;
  static_for<0, 16>([&](auto ss) {
    constexpr int s = decltype(ss)::value;
    constexpr int z = decltype(zf(std::integral_constant<int, s>{}))::value;
    uint64_t x, y;
    pair_values(a[s], x, y);
    const uint64_t yr = gl_canon(y);
    const uint64_t dif = gl_mul_pow2_r<192 - z>(gl_sub_r(x, yr));
    a[s] = lane_select(odd, gl_canon(gl_add_r(x, yr)), dif);
  });
}

__device__ __forceinline__ void inv64_p2(uint64_t (&a)[16], int lane) {
  gs64_cross(a, Z2<1>{}, lane);
  gs64_stage<2>(a, Z2<2>{});
  gs64_stage<4>(a, Z2<4>{});
  gs64_stage<8>(a, Z2<8>{});
  gs64_stage<16>(a, Z2<16>{});
}

__device__ __forceinline__ void inv64_p1(uint64_t (&a)[16], int lane) {
  gs64_cross(a, Z1<1>{}, lane);
  gs64_stage<2>(a, Z1<2>{});
  gs64_stage<4>(a, Z1<4>{});
  gs64_stage<8>(a, Z1<8>{});
  gs64_stage<16>(a, Z1<16>{});
}

}  // namespace lp
