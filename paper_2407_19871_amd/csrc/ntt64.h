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
// of a column.  It runs on slot pairs (s, s + 8): one half-wave swap of the
// two registers gives the lower lane both values of slot s and the upper
// lane both values of slot s + 8, and each lane forms a whole butterfly.
// That leaves the "pair layout": register r of lane (h, l) holds position
// pair_pos(r, h) = 16h + 2(r & 7) + (r >> 3).
//   forward:  in  lane (h, l), slot s = coefficient l + 32 (2s + h)
//             out lane (h, l), register r = A(k), k = brv5(l) + 32 brv5(q),
//             q = pair_pos(r, h), which sits at offset 64 (q >> 1) + 2 l +
//             (q & 1) of the 32-lane layout (ntt_pos), so NTT-domain keys
//             are shared by both layouts.
// The inverses below (on one, two or four waves) are Gentleman-Sande
// stages that undo the merged Cooley-Tukey stages in reverse order,
// (X, Y) -> (X + Y, (X - Y) w^-1), with the same per-block twiddles; each
// pass leaves a factor 32, both factors sit in the inverse twist table (the
// one of the 32-lane transform), and the pass-1 stages also undo the
// negacyclic factor, so there is no post-twist.
#pragma once
#include "ntt32.h"

namespace lp {

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
//   64 < LO:        -xh + w EPS with c = 96 - S in [0, 31], xh = x >> c,
//                   w = low32(x) << (S - 64), as in gl_mul_pow2 (w formed as
//                   low32(x) 2^32 >> c, which is 0 at S = 96; there xh = x,
//                   so HI = 96 needs a reduced x);
//   LO < 64 <= HI:  y = x 2^(S - 32) as (lo, hi), then x 2^S = lo 2^32 +
//                   hi 2^96 = lo 2^32 - hi with hi < 2^63.
template <int LO, int HI>
GL_INLINE uint64_t gl_mul_pow2_lane(uint64_t x, uint32_t S) {
  static_assert(0 <= LO && LO <= HI && (HI < 96 || (HI == 96 && LO > 64)), "shift range");
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
    const uint32_t c = 96 - S;
    const uint64_t xh = x >> c;
    const uint32_t w = (uint32_t)(((uint64_t)(uint32_t)x << 32) >> c);
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

// Pass 1 after its digit stages, and pass 2, each ending in the paired
// distance-1 stage: output in the pair layout, h6 = 6 (lane >> 5).
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

// The first stage of a pass with its input in the pair layout (X in register
// s, Y in s + 8: positions 2t and 2t + 1 of its row, t = s + 8h), lazy: an
// in-lane butterfly (X, Y) -> (X + Y, (X - Y) 2^(192 - z(t))), then the swap
// back to the interleaved layout.  With -1 = 2^96, (X - Y) 2^(192 - z) =
// (Y - X) 2^(96 - z), and z(t) = z(s) + 6h, so the lane shifts Y - X by
// 96 - z(s) - 6h, in [0, 96] (96 only at z = 0, on a reduced Y - X).
template <typename Zf>
__device__ __forceinline__ void gs64_cross_pairs(uint64_t (&a)[16], Zf zf, uint32_t h6) {
  static_for<0, 8>([&](auto ss) {
    constexpr int s = decltype(ss)::value;
    constexpr int z = decltype(zf(std::integral_constant<int, s>{}))::value;
    static_assert(decltype(zf(std::integral_constant<int, s + 8>{}))::value == z + 6, "pair twiddles");
    const uint64_t x = gl_canon(a[s]), y = gl_canon(a[s + 8]);
    a[s] = gl_canon(gl_add_r(x, y));
    a[s + 8] = gl_mul_pow2_lane<90 - z, 96 - z>(gl_sub_r(y, x), (uint32_t)(96 - z) - h6);
    swap_halves(a[s], a[s + 8]);
  });
}

// The one-wave inverse passes, input in the pair layout, output interleaved.
__device__ __forceinline__ void inv64_p2_pairs(uint64_t (&a)[16], uint32_t h6) {
  gs64_cross_pairs(a, Z2<1>{}, h6);
  gs64_stage<2>(a, Z2<2>{});
  gs64_stage<4>(a, Z2<4>{});
  gs64_stage<8>(a, Z2<8>{});
  gs64_stage<16>(a, Z2<16>{});
}

__device__ __forceinline__ void inv64_p1_pairs(uint64_t (&a)[16], uint32_t h6) {
  gs64_cross_pairs(a, Z1<1>{}, h6);
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
// The inverse over 256 lanes: wave w (0..3) holds rows 8 w .. 8 w + 7, and
// lane 8 r + h of the wave holds four positions of row 8 w + r.  The input
// layout puts the two low position bits in registers: register s holds
// q = 4 h + s.  The distance-1 and -2 stages then run inside the lane.
// Each of the distance-4, -8 and -16 stages first trades one register of
// each pair with the partner lane h ^ 1, h ^ 2, h ^ 4, which moves the
// stage's position bit (a lane bit until then) into a register and sends a
// position bit that is already done (bits 0, 1, 2) out to the lane; every
// lane then runs whole butterflies.  The upper lane of a traded pair holds
// Y - X where the butterfly needs X - Y, so its twiddle carries a minus
// sign.  Output: register s holds q = h + 8 (s >> 1) + 16 (s & 1).

// Exponent z of the forward stage of distance LEN at block b (as Z1 and Z2,
// for a block known at run time); the inverse multiplies by 2^(192 - z).
__device__ __host__ constexpr int z_fwd(int pass, int len, int b) {
  return pass == 1 ? 3 * brv5(32 / (2 * len) + b)
                   : 6 * len * (brv5(b) >> (len == 16 ? 5 : len == 8 ? 4 : len == 4 ? 3 : len == 2 ? 2 : 1));
}

// 2^e mod p, reduced, for a runtime e in [0, 192).
__device__ __host__ inline uint64_t gl_pow2(int e) {
  uint64_t w = 1;
  for (int k = 0; k < e; ++k) w = gl_add(w, w);
  return gl_canon(w);
}

// The lane's twiddles for one pass (1 or 2) of the four-wave inverse, h =
// lane & 7: w[0], w[1] distance 1 (blocks 2h, 2h + 1), w[2] distance 2
// (block h), w[3] distance 4 (block h >> 1, negated in lanes with h & 1),
// w[4] distance 8 (block h >> 2, negated in lanes with h & 2).  Distance 16
// has block 0 in both passes.
__device__ __host__ inline void inv256_twiddles(int pass, int h, uint64_t (&w)[5]) {
  auto tw = [&](int len, int b) { return gl_pow2((192 - z_fwd(pass, len, b)) % 192); };
  w[0] = tw(1, 2 * h);
  w[1] = tw(1, 2 * h + 1);
  w[2] = tw(2, h);
  w[3] = (h & 1) ? gl_neg_r(tw(4, h >> 1)) : tw(4, h >> 1);
  w[4] = (h & 2) ? gl_neg_r(tw(8, h >> 2)) : tw(8, h >> 2);
}

// In-lane Gentleman-Sande butterfly, reduced inputs and outputs:
// (x, y) -> (x + y, (x - y) w).
__device__ __forceinline__ void gs_bf(uint64_t& x, uint64_t& y, uint64_t w) {
  const uint64_t d = gl_sub_r(x, y);
  x = gl_canon(gl_add_r(x, y));
  y = gl_canon(gl_mul(d, w));
}

// Trade within the pair (a, b) with the partner lane, `upper` = ~0 in the
// lane whose traded bit is set: the lower lane keeps a and receives the
// partner's a, the upper lane receives the partner's b and keeps b.  Returns
// k (kept) and r (received); the butterfly's X, Y are (k, r) in the lower
// lane and (r, k) in the upper one, so X + Y = k + r and X - Y = +-(k - r).
template <int D>
__device__ __forceinline__ void quad_trade(uint64_t a, uint64_t b, uint64_t upper, uint64_t& k, uint64_t& r) {
  r = quad_xor<D>(lane_select(upper, b, a));
  k = lane_select(upper, a, b);
}

// The same with the lane h ^ 4 of the group of eight: lanes h < 4 (DPP banks
// 0 and 2 of a row) read lane + 4's a, lanes h >= 4 (banks 1 and 3) lane -
// 4's b, each DPP writing only its own banks.
__device__ __forceinline__ uint32_t oct_trade_u32(uint32_t a, uint32_t b) {
  const int from_lower = __builtin_amdgcn_update_dpp(0, (int)b, 0x114, 0xF, 0xA, false);  // row_shr:4
  return (uint32_t)__builtin_amdgcn_update_dpp(from_lower, (int)a, 0x104, 0xF, 0x5, false);  // row_shl:4
}
__device__ __forceinline__ void oct_trade(uint64_t a, uint64_t b, uint64_t upper, uint64_t& k, uint64_t& r) {
  r = ((uint64_t)oct_trade_u32((uint32_t)(a >> 32), (uint32_t)(b >> 32)) << 32) |
      oct_trade_u32((uint32_t)a, (uint32_t)b);
  k = lane_select(upper, a, b);
}

// One pass; FIRST inputs may be lazy (the distance-1 stage reduces them).
// u4 = ~0 in lanes h >= 4; w from inv256_twiddles of this pass.
template <int PASS>
__device__ __forceinline__ void inv256_pass(uint64_t (&a)[4], uint64_t u1, uint64_t u2, uint64_t u4,
                                            const uint64_t (&w)[5]) {
  // distance 1: (q, q + 1) = registers (2j, 2j + 1), lazy inputs
  static_for<0, 2>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    const uint64_t x = a[2 * j], y = gl_canon(a[2 * j + 1]);
    a[2 * j] = gl_canon(gl_add_r(x, y));
    a[2 * j + 1] = gl_canon(gl_mul(gl_sub_r(x, y), w[j]));
  });
  // distance 2: registers (j, j + 2)
  gs_bf(a[0], a[2], w[2]);
  gs_bf(a[1], a[3], w[2]);
  // distance 4: trade with h ^ 1 on the pairs (0, 1), (2, 3); bit 2 then
  // sits in register bit 0
  static_for<0, 2>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    uint64_t k, r;
    quad_trade<1>(a[2 * j], a[2 * j + 1], u1, k, r);
    a[2 * j] = k;
    a[2 * j + 1] = r;
    gs_bf(a[2 * j], a[2 * j + 1], w[3]);
  });
  // distance 8: trade with h ^ 2 on the pairs (0, 2), (1, 3); bit 3 then
  // sits in register bit 1
  static_for<0, 2>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    uint64_t k, r;
    quad_trade<2>(a[j], a[j + 2], u2, k, r);
    a[j] = k;
    a[j + 2] = r;
    gs_bf(a[j], a[j + 2], w[4]);
  });
  // distance 16: trade with h ^ 4 on the pairs (0, 1), (2, 3); block 0:
  // twiddle 1 in pass 2, 2^(192 - 48) = -2^48 in pass 1, times the trade's
  // sign (-1 in the upper lanes)
  static_for<0, 2>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    uint64_t k, r;
    oct_trade(a[2 * j], a[2 * j + 1], u4, k, r);
    const uint64_t d = gl_sub_r(k, r);
    a[2 * j] = gl_canon(gl_add_r(k, r));
    if constexpr (PASS == 2) {
      a[2 * j + 1] = lane_negate(u4, d);
    } else {
      static_assert(z_fwd(1, 16, 0) == 48, "pass-1 distance-16 twiddle");
      a[2 * j + 1] = lane_negate(~u4, gl_mul_pow2_r<48>(d));
    }
  });
}

}  // namespace lp
