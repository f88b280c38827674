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
//             (ntt_pos), so NTT-domain keys are shared by both layouts.
// The inverses below (on one, two or four waves) are Gentleman-Sande
// stages that undo the merged Cooley-Tukey stages in reverse order,
// (X, Y) -> (X + Y, (X - Y) w^-1), with the same per-block twiddles; each
// pass leaves a factor 32, both factors sit in the inverse twist table (the
// one of the 32-lane transform), and the pass-1 stages also undo the
// negacyclic factor, so there is no post-twist.
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

// hi_lane ? -y : y for reduced y, again reduced: -y = ~y + (2 - 2^32)
// (gl_neg_r), so the upper lanes flip y and add the constant.
__device__ __forceinline__ uint64_t lane_negate(uint64_t mask, uint64_t y) {
  return (y ^ mask) + (mask & 0xFFFFFFFF00000002ull);
}

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

// The LEN = 1 stage across the two lanes of a column; Z(s) per slot.  The
// lower lane keeps x_even + t, the upper one x_even - t, each with one
// addition (of t or of -t).
template <typename Zf>
__device__ __forceinline__ void ct64_cross(uint64_t (&a)[16], Zf zf, int lane) {
  const uint64_t odd = lane >= 32 ? ~0ull : 0ull;
  static_for<0, 16>([&](auto ss) {
    constexpr int s = decltype(ss)::value;
    constexpr int z = decltype(zf(std::integral_constant<int, s>{}))::value;
    uint64_t xe, xo;
    pair_values(a[s], xe, xo);
    a[s] = gl_add_r(xe, lane_negate(odd, gl_mul_pow2_r<z>(xo)));
  });
}

// ---- the distance-1 stage on slot pairs --------------------------------------
// v_permlane32_swap of two different registers trades the upper half-wave of
// `a` for the lower half-wave of `b`.  For the slots (s, s + 8) that leaves
// every lane with both values of one column pair: the lower lane gets
// (position 2s, position 2s + 1) of its column, the upper lane (2s + 16,
// 2s + 17).  Applied again, it restores the interleaved layout.
__device__ __forceinline__ void swap_halves(uint64_t& a, uint64_t& b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)b, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
  a = ((uint64_t)hi[0] << 32) | lo[0];
  b = ((uint64_t)hi[1] << 32) | lo[1];
}

// x * 2^S mod p, reduced to [0, p], for a shift S held per lane and known to
// lie in [LO, HI] (the two lanes of a slot pair shift by z and z + 6).  The
// forms are those of gl_mul_pow2 with the shift counts in registers; a
// 64-bit shift uses its count modulo 64, so no count may reach 64:
//   HI < 32:        x 2^S = low + 2^64 w2, w2 = x >> (64 - S) < 2^31 (for
//                   LO = 0, w2 = (x >> 1) >> (63 - S), which is 0 at S = 0);
//   1 <= LO, HI < 64: the 128-bit product (x << S, x >> (64 - S)) reduced;
//   64 < LO:        -xh + w EPS with c = 96 - S in [1, 31], xh = x >> c,
//                   w = low32(x) << (S - 64), as in gl_mul_pow2;
//   LO < 64 <= HI:  y = x 2^(S - 32) as (lo, hi), then x 2^S = lo 2^32 +
//                   hi 2^96 = lo 2^32 - hi with hi < 2^63.
template <int LO, int HI>
GL_INLINE uint64_t gl_mul_pow2_lane(uint64_t x, uint32_t S) {
  static_assert(0 <= LO && LO <= HI && HI < 96, "shift range");
  if constexpr (HI < 32) {
    const uint64_t low = x << S;
    const uint64_t w2 = LO == 0 ? (x >> 1) >> (63 - S) : x >> (64 - S);
    const uint64_t t = (w2 << 32) - w2;  // EPS w2 < 2^63
    uint64_t r;
    const bool c = __builtin_add_overflow(low, t, &r);
    return gl_canon(r + (c ? GL_EPS : 0ull));
  } else if constexpr (HI < 64) {
    static_assert(LO >= 1, "shift range");
    return gl_canon(gl_reduce128(x << S, x >> (64 - S)));
  } else if constexpr (LO > 64) {
    const uint64_t xh = x >> (96 - S);
    const uint32_t w = (uint32_t)x << (S - 64);
    return gl_sub_r(((uint64_t)w << 32) - w, xh);
  } else {
    static_assert(LO > 32, "shift range");
    const uint64_t lo = x << (S - 32), hi = x >> (96 - S);
    return gl_canon(gl_sub_r(gl_reduce128(lo << 32, lo >> 32), hi));
  }
}

// Position within its column (pass 1) or row (pass 2) of register r of a
// lane in half h after a paired distance-1 stage ("pair layout").
__device__ __host__ constexpr int pair_pos(int r, int h) { return 16 * h + 2 * (r & 7) + (r >> 3); }

// The forward LEN = 1 stage on the slot pairs (s, s + 8).  After
// swap_halves, every lane runs one whole butterfly: the lower lane that of
// slot s, the upper lane that of slot s + 8, whose twiddle is 2^6 times slot
// s's (the block's brv5 grows by 2 in both passes), so the lane shifts by
// z(s) + 6h.  Output in the pair layout (pair_pos).  Against ct64_cross,
// each lane forms half the twiddle products and needs no register copies.
template <typename Zf>
__device__ __forceinline__ void ct64_cross_pairs(uint64_t (&a)[16], Zf zf, uint32_t h6) {
  static_for<0, 8>([&](auto ss) {
    constexpr int s = decltype(ss)::value;
    constexpr int z = decltype(zf(std::integral_constant<int, s>{}))::value;
    static_assert(decltype(zf(std::integral_constant<int, s + 8>{}))::value == z + 6, "pair twiddles");
    swap_halves(a[s], a[s + 8]);
    const uint64_t t = gl_mul_pow2_lane<z, z + 6>(a[s + 8], (uint32_t)z + h6);
    a[s + 8] = gl_sub_r(a[s], t);
    a[s] = gl_add_r(a[s], t);
  });
}

// Back from the pair layout to the interleaved one.
__device__ __forceinline__ void pairs_to_interleaved(uint64_t (&a)[16]) {
  static_for<0, 8>([&](auto ss) {
    constexpr int s = decltype(ss)::value;
    swap_halves(a[s], a[s + 8]);
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

// The same passes ending in the paired distance-1 stage: output in the pair
// layout, h6 = 6 (lane >> 5).
__device__ __forceinline__ void fwd64_p1_rest_pairs(uint64_t (&a)[16], uint32_t h6) {
  ct64_stage<4>(a, Z1<4>{});
  ct64_stage<2>(a, Z1<2>{});
  ct64_cross_pairs(a, Z1<1>{}, h6);
}

__device__ __forceinline__ void fwd64_p2_pairs(uint64_t (&a)[16], uint32_t h6) {
  ct64_stage<16>(a, Z2<16>{});
  ct64_stage<8>(a, Z2<8>{});
  ct64_stage<4>(a, Z2<4>{});
  ct64_stage<2>(a, Z2<2>{});
  ct64_cross_pairs(a, Z2<1>{}, h6);
}

// ---- inverse on one wave: Gentleman-Sande ---------------------------------
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
// may be lazy, its outputs are reduced.  The lower lane keeps X + Y, the
// upper one (X - Y) w^-1, both from one addition (of Y or of -Y).
template <typename Zf>
__device__ __forceinline__ void gs64_cross(uint64_t (&a)[16], Zf zf, int lane) {
  const uint64_t odd = lane >= 32 ? ~0ull : 0ull;
  static_for<0, 16>([&](auto ss) {
    constexpr int s = decltype(ss)::value;
    constexpr int z = decltype(zf(std::integral_constant<int, s>{}))::value;
    uint64_t x, y;
    pair_values(a[s], x, y);
    const uint64_t v = gl_add_r(x, lane_negate(odd, gl_canon(y)));
    a[s] = lane_select(odd, gl_canon(v), gl_mul_pow2_r<192 - z>(v));
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

// ---- inverse on two waves (four lanes per row) -------------------------------
// The inverse transform of one polynomial spread over 128 lanes: wave w
// (0, 1) holds rows 16 w .. 16 w + 15, lane 4 r + h of the wave holds the
// eight positions q = 4 s + h (s = 0..7) of row 16 w + r.  Stages of
// distance LEN >= 4 stay inside a lane, with per-block twiddles as above;
// the distance-2 and distance-1 stages pair lanes h ^ 2 and h ^ 1 of a
// row's quad (DPP quad permutations).  The distance-2 stage's block
// (q / 4 = s) is uniform; the distance-1 stage's block (q / 2 = 2 s +
// (h >> 1)) takes two values per slot, so both shifts are formed and each
// lane keeps its own.  Between the passes the rows are transposed through
// LDS across both waves; the output is, in lane 4 r + h of wave w, slot s,
// coefficient j1 + 32 q with j1 = 16 w + r, q = 4 s + h.

// The value held by lane ^ D of the quad (D = 1 or 2).
template <int D>
__device__ __forceinline__ uint64_t quad_xor(uint64_t v) {
  constexpr int ctrl = D == 1 ? 0xB1 : 0x4E;  // quad_perm [1,0,3,2] / [2,3,0,1]
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, ctrl, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), ctrl, 0xF, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}

// Gentleman-Sande stage of distance D in {1, 2} across the quad; FIRST:
// the inputs may be lazy.  Masks: upper = ~0 in the upper lane of each
// pair (h & D), second = ~0 in lanes h >= 2 (the second pair of the row).
// Each lane forms only its own output from one addition: the partner's
// value plus this lane's own, negated in the upper lane, i.e. X + Y in the
// lower lane and X - Y in the upper one, which then takes the twiddle.
template <int D, bool FIRST, typename Zf>
__device__ __forceinline__ void gs128_cross(uint64_t (&a)[8], Zf zf, uint64_t upper, uint64_t second) {
  static_for<0, 8>([&](auto ss) {
    constexpr int s = decltype(ss)::value;
    const uint64_t other = quad_xor<D>(a[s]);
    const uint64_t self = FIRST ? gl_canon(a[s]) : a[s];
    const uint64_t v = gl_add_r(other, lane_negate(upper, self));
    uint64_t up;
    if constexpr (D == 1) {
      constexpr int za = decltype(zf(std::integral_constant<int, 2 * s>{}))::value;
      constexpr int zb = decltype(zf(std::integral_constant<int, 2 * s + 1>{}))::value;
      up = lane_select(second, gl_mul_pow2_r<192 - za>(v), gl_mul_pow2_r<192 - zb>(v));
    } else {
      constexpr int z = decltype(zf(std::integral_constant<int, s>{}))::value;
      up = gl_mul_pow2_r<192 - z>(v);
    }
    a[s] = lane_select(upper, gl_canon(v), up);
  });
}

// In-lane Gentleman-Sande stage of distance LEN in {4, 8, 16}: slots s and
// s + LEN / 4 within blocks of LEN / 2 slots; reduced inputs and outputs.
template <int LEN, typename Zf>
__device__ __forceinline__ void gs128_stage(uint64_t (&a)[8], Zf zf) {
  static_for<0, 16 / LEN>([&](auto bb) {
    constexpr int blk = decltype(bb)::value;
    constexpr int z = decltype(zf(std::integral_constant<int, blk>{}))::value;
    static_for<0, LEN / 4>([&](auto jj) {
      constexpr int s0 = blk * (LEN / 2) + decltype(jj)::value, s1 = s0 + LEN / 4;
      const uint64_t x = a[s0], y = a[s1];
      a[s0] = gl_canon(gl_add_r(x, y));
      a[s1] = gl_mul_pow2_r<192 - z>(gl_sub_r(x, y));
    });
  });
}

__device__ __forceinline__ void inv128_p2(uint64_t (&a)[8], uint64_t upper1, uint64_t upper2, uint64_t second) {
  gs128_cross<1, true>(a, Z2<1>{}, upper1, second);
  gs128_cross<2, false>(a, Z2<2>{}, upper2, second);
  gs128_stage<4>(a, Z2<4>{});
  gs128_stage<8>(a, Z2<8>{});
  gs128_stage<16>(a, Z2<16>{});
}

__device__ __forceinline__ void inv128_p1(uint64_t (&a)[8], uint64_t upper1, uint64_t upper2, uint64_t second) {
  gs128_cross<1, true>(a, Z1<1>{}, upper1, second);
  gs128_cross<2, false>(a, Z1<2>{}, upper2, second);
  gs128_stage<4>(a, Z1<4>{});
  gs128_stage<8>(a, Z1<8>{});
  gs128_stage<16>(a, Z1<16>{});
}

// ---- inverse on four waves (eight lanes per row) -----------------------------
// The same inverse over 256 lanes: wave w (0..3) holds rows 8 w .. 8 w + 7,
// lane 8 r + h of the wave holds the four positions q = 8 s + h (s = 0..3)
// of row 8 w + r.  Stages of distance 16 and 8 stay in the lane; distance
// 4 pairs lanes h ^ 4 with a uniform block (q / 8 = s); distance 2 pairs
// h ^ 2 with two blocks per slot (q / 4 = 2 s + (h >> 2)), both shifts
// formed; distance 1 pairs h ^ 1 with four blocks per slot (q / 2 = 4 s +
// (h >> 1)), so each lane multiplies by its own twiddle, computed once per
// launch (gl_pow2).  Output, in lane 8 r + h of wave w, slot s: coefficient
// j1 + 32 q with j1 = 8 w + r, q = 8 s + h.

// The value held by lane ^ 4 of each group of eight: lanes h < 4 read
// lane + 4 (DPP row_shl:4), lanes h >= 4 lane - 4 (row_shr:4); hi4 = ~0 in
// lanes h >= 4.
__device__ __forceinline__ uint32_t oct_xor4_u32(uint32_t x, bool hi4) {
  const uint32_t up = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x104, 0xF, 0xF, false);
  const uint32_t dn = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);
  return hi4 ? dn : up;
}
__device__ __forceinline__ uint64_t oct_xor4(uint64_t v, bool hi4) {
  return ((uint64_t)oct_xor4_u32((uint32_t)(v >> 32), hi4) << 32) | oct_xor4_u32((uint32_t)v, hi4);
}

// 2^e mod p, reduced, for a runtime e in [0, 192).
__device__ __forceinline__ uint64_t gl_pow2(int e) {
  uint64_t w = 1;
  for (int k = 0; k < e; ++k) w = gl_add(w, w);
  return gl_canon(w);
}

// Gentleman-Sande stage of distance D in {1, 2, 4} across the eight lanes
// of a row; FIRST: the inputs may be lazy.  upper: ~0 in the upper lane of
// each pair (h & D); hi4: ~0 in lanes h >= 4; w1: the lane's twiddles of
// the distance-1 stage (one per slot, 1 in the lower lanes).  As in
// gs128_cross, each lane forms only its own output: the partner's value
// plus its own, negated in the upper lane, then the upper lane's twiddle.
template <int D, bool FIRST, typename Zf>
__device__ __forceinline__ void gs256_cross(uint64_t (&a)[4], Zf zf, uint64_t upper, uint64_t hi4,
                                            const uint64_t (&w1)[4]) {
  static_for<0, 4>([&](auto ss) {
    constexpr int s = decltype(ss)::value;
    uint64_t other;
    if constexpr (D == 4) other = oct_xor4(a[s], hi4 != 0);
    else other = quad_xor<D>(a[s]);
    const uint64_t self = FIRST ? gl_canon(a[s]) : a[s];
    const uint64_t v = gl_add_r(other, lane_negate(upper, self));
    if constexpr (D == 4) {
      constexpr int z = decltype(zf(std::integral_constant<int, s>{}))::value;
      a[s] = lane_select(upper, gl_canon(v), gl_mul_pow2_r<192 - z>(v));
    } else if constexpr (D == 2) {
      constexpr int za = decltype(zf(std::integral_constant<int, 2 * s>{}))::value;
      constexpr int zb = decltype(zf(std::integral_constant<int, 2 * s + 1>{}))::value;
      a[s] = lane_select(upper, gl_canon(v), lane_select(hi4, gl_mul_pow2_r<192 - za>(v), gl_mul_pow2_r<192 - zb>(v)));
    } else {
      a[s] = gl_canon(gl_mul(v, w1[s]));
    }
  });
}

// In-lane stage of distance LEN in {8, 16}: slots s and s + LEN / 16 within
// blocks of LEN / 4 slots.
template <int LEN, typename Zf>
__device__ __forceinline__ void gs256_stage(uint64_t (&a)[4], Zf zf) {
  constexpr int span = LEN / 4;
  static_for<0, 4 / span>([&](auto bb) {
    constexpr int blk = decltype(bb)::value;
    constexpr int z = decltype(zf(std::integral_constant<int, blk>{}))::value;
    static_for<0, span / 2>([&](auto jj) {
      constexpr int s0 = blk * span + decltype(jj)::value, s1 = s0 + span / 2;
      const uint64_t x = a[s0], y = a[s1];
      a[s0] = gl_canon(gl_add_r(x, y));
      a[s1] = gl_mul_pow2_r<192 - z>(gl_sub_r(x, y));
    });
  });
}

// The lane's distance-1 twiddles of each pass: in the upper lane of a pair
// (h odd) 2^(192 - z) for the block 4 s + (h >> 1) of slot s (pass 2: z =
// 6 (brv5(b) >> 1); pass 1: z = 3 brv5(16 + b)); 1 in the lower lane, which
// keeps the sum.
__device__ __forceinline__ void inv256_twiddles(int h, uint64_t (&w2)[4], uint64_t (&w1)[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int b = 4 * s + (h >> 1);
    w2[s] = (h & 1) ? gl_pow2((192 - 6 * (brv5(b) >> 1)) % 192) : 1ull;
    w1[s] = (h & 1) ? gl_pow2((192 - 3 * brv5(16 + b)) % 192) : 1ull;
  }
}

__device__ __forceinline__ void inv256_p2(uint64_t (&a)[4], uint64_t upper1, uint64_t upper2, uint64_t upper4,
                                          const uint64_t (&w2)[4]) {
  gs256_cross<1, true>(a, Z2<1>{}, upper1, upper4, w2);
  gs256_cross<2, false>(a, Z2<2>{}, upper2, upper4, w2);
  gs256_cross<4, false>(a, Z2<4>{}, upper4, upper4, w2);
  gs256_stage<8>(a, Z2<8>{});
  gs256_stage<16>(a, Z2<16>{});
}

__device__ __forceinline__ void inv256_p1(uint64_t (&a)[4], uint64_t upper1, uint64_t upper2, uint64_t upper4,
                                          const uint64_t (&w1)[4]) {
  gs256_cross<1, true>(a, Z1<1>{}, upper1, upper4, w1);
  gs256_cross<2, false>(a, Z1<2>{}, upper2, upper4, w1);
  gs256_cross<4, false>(a, Z1<4>{}, upper4, upper4, w1);
  gs256_stage<8>(a, Z1<8>{});
  gs256_stage<16>(a, Z1<16>{});
}

}  // namespace lp
