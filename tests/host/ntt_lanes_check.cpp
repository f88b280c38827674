// Host model of the cross-lane transforms of the GPU path
// (paper_2407_19871_amd/csrc/ntt64.h, compiled here with the host compiler):
// every lane of one 64-lane wave runs the header's own code in a host
// thread, and the lane-exchange builtins it uses are emulated with the
// semantics the header relies on (a barrier before and after each
// exchange):
//   update_dpp quad_perm [1,0,3,2] / [2,3,0,1]: lane L reads lane
//     (L & ~3) + perm[L & 3]; row_shl:4 / row_shr:4: lane L reads L + 4 /
//     L - 4 within its row of 16 lanes, else keeps `old`; a lane whose bank
//     (four lanes of a row, (L & 15) >> 2) is clear in bank_mask keeps `old`;
//   permlane32_swap(a, b): the upper half-wave of a trades places with the
//     lower half-wave of b, so lane L < 32 gets (a of L, a of L + 32) and
//     lane L >= 32 gets (b of L - 32, b of L); with a = b every lane gets
//     (x of lane L & 31, x of lane (L & 31) + 32).
// Each pass (the forward passes on the 64-lane layout, the inverse passes
// on all three) is compared with its definition over Z_p, p = 2^64 -
// 2^32 + 1, for every lane layout the kernels use (64 lanes: lane (h, l) holds row l,
// positions 2s + h; 128: lane 4r + h holds row r, positions 4s + h; 256:
// lane 8r + h holds row r, positions 4h + s on entry and h + 8 (s >> 1) +
// 16 (s & 1) on exit), on random and lazy inputs
// (values at or above p, 2^64 - 1) and on digits at their extremes:
//   forward pass 1: out[P] = sum_j a[j] rho^(j (2 brv5(P) + 1)), rho = 2^3
//   forward pass 2: out[P] = sum_j c[j] omega^(brv5(P) j),       omega = 2^6
//   inverse pass 2: out[j] = sum_P x[P] omega^(-brv5(P) j)
//   inverse pass 1: out[j] = sum_P x[P] rho^(-j (2 brv5(P) + 1))
// Prints "ok <checks>" and exits 0, or the first mismatch and exits 1.
#include <barrier>
#include <array>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <thread>
#include <vector>

#define __device__
#define __host__
#define __forceinline__ inline

namespace emu {
struct Wave {
  std::barrier<> bar{64};
  uint32_t buf[64], buf2[64];
};
thread_local int lane = 0;
thread_local Wave* wave = nullptr;

inline uint32_t exchange(uint32_t v, int src_lane, bool valid, uint32_t old) {
  wave->buf[lane] = v;
  wave->bar.arrive_and_wait();
  const uint32_t r = valid ? wave->buf[src_lane] : old;
  wave->bar.arrive_and_wait();
  return r;
}
inline int update_dpp(int old, int src, int ctrl, int bank_mask) {
  const int L = lane;
  const bool on = (bank_mask >> ((L & 15) >> 2)) & 1;
  if (ctrl == 0xB1 || ctrl == 0x4E) {
    const int perm[4] = {ctrl == 0xB1 ? 1 : 2, ctrl == 0xB1 ? 0 : 3, ctrl == 0xB1 ? 3 : 0, ctrl == 0xB1 ? 2 : 1};
    return (int)exchange((uint32_t)src, (L & ~3) + perm[L & 3], on, (uint32_t)old);
  }
  if (ctrl == 0x104) return (int)exchange((uint32_t)src, L + 4, on && (L & 15) + 4 < 16, (uint32_t)old);
  if (ctrl == 0x114) return (int)exchange((uint32_t)src, L - 4, on && (L & 15) >= 4, (uint32_t)old);
  std::printf("unmodelled DPP control 0x%x\n", ctrl);
  std::exit(2);
}
inline std::array<uint32_t, 2> permlane32_swap(uint32_t a, uint32_t b) {
  wave->buf[lane] = a;
  wave->buf2[lane] = b;
  wave->bar.arrive_and_wait();
  const std::array<uint32_t, 2> r = lane < 32 ? std::array<uint32_t, 2>{wave->buf[lane], wave->buf[lane + 32]}
                                              : std::array<uint32_t, 2>{wave->buf2[lane - 32], wave->buf2[lane]};
  wave->bar.arrive_and_wait();
  return r;
}
}  // namespace emu

#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) emu::update_dpp((old), (src), (ctrl), (bm))
#define __builtin_amdgcn_permlane32_swap(a, b, fi, bc) emu::permlane32_swap((a), (b))

#include "ntt64.h"

typedef unsigned __int128 u128;
static const uint64_t P = GL_P;
static uint64_t checks = 0;
static uint64_t mulp(uint64_t a, uint64_t b) { return (uint64_t)((u128)(a % P) * (b % P) % P); }
static uint64_t addp(uint64_t a, uint64_t b) { return (uint64_t)(((u128)(a % P) + (b % P)) % P); }
static uint64_t powp(uint64_t b, long e) {
  e %= 192;  // 2 has order 192
  if (e < 0) e += 192;
  uint64_t r = 1;
  for (long i = 0; i < e; ++i) r = mulp(r, b);
  return r;
}

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t rnd() {
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// One wave: fn(lane) runs on 64 host threads.
static void run_wave(const std::function<void(int)>& fn) {
  emu::Wave w;
  std::vector<std::thread> th;
  for (int L = 0; L < 64; ++L)
    th.emplace_back([&, L] {
      emu::lane = L;
      emu::wave = &w;
      fn(L);
    });
  for (auto& t : th) t.join();
}

// A layout: lanes per row G (2, 4, 8) and slots per lane S = 32 / G.  Lane
// L holds row r(L) and positions q = G s + h(L).
struct Layout {
  int G;
  int row(int L) const { return G == 2 ? (L & 31) : L / G; }
  int h(int L) const { return G == 2 ? (L >> 5) : L % G; }
  int rows() const { return 64 / G; }
};

[[noreturn]] static void fail(const char* what, int G, int row, int pos, uint64_t got, uint64_t want) {
  std::printf("MISMATCH %s layout %d lanes/row, row %d, position %d: got %016llx want %016llx\n", what, G, row, pos,
              (unsigned long long)got, (unsigned long long)want);
  std::exit(1);
}

// in[row][pos] -> lanes, run, lanes -> out[row][pos] (canonical)
template <int S, typename F>
static void run_layout(const Layout& Lo, const std::vector<std::array<uint64_t, 32>>& in,
                       std::vector<std::array<uint64_t, 32>>& out, F body) {
  out.assign(Lo.rows(), {});
  run_wave([&](int L) {
    uint64_t a[S];
    const int r = Lo.row(L), h = Lo.h(L);
    for (int s = 0; s < S; ++s) a[s] = in[r][Lo.G * s + h];
    body(a, L);
    for (int s = 0; s < S; ++s) out[r][Lo.G * s + h] = gl_canon(a[s]);
  });
}

static std::vector<std::array<uint64_t, 32>> inputs(int rows, int kind) {
  std::vector<std::array<uint64_t, 32>> v(rows);
  for (auto& r : v)
    for (int j = 0; j < 32; ++j) {
      const uint64_t x = rnd();
      switch (kind) {
        case 0: r[j] = x % P; break;                                  // canonical
        case 1: r[j] = (x & 1) ? P + x % (0xFFFFFFFFull) : x;         // lazy: at or above p, or any
        case 2: r[j] = (j & 1) ? 0xFFFFFFFFFFFFFFFFull : P; break;    // extremes
        default: r[j] = (x & 3) == 0 ? P - 1 : (x & 3) == 1 ? P : (x & 3) == 2 ? P + 1 : x; break;
      }
    }
  return v;
}

static void check(const char* what, const Layout& Lo, const std::vector<std::array<uint64_t, 32>>& in,
                  const std::vector<std::array<uint64_t, 32>>& out,
                  const std::function<uint64_t(const std::array<uint64_t, 32>&, int)>& ref) {
  for (int r = 0; r < Lo.rows(); ++r)
    for (int q = 0; q < 32; ++q) {
      ++checks;
      const uint64_t want = ref(in[r], q);
      if (out[r][q] % P != want) fail(what, Lo.G, r, q, out[r][q], want);
    }
}

static uint64_t ref_fwd1(const std::array<uint64_t, 32>& a, int q) {
  uint64_t s = 0;
  for (int j = 0; j < 32; ++j) s = addp(s, mulp(a[j], powp(8, (long)j * (2 * lp::brv5(q) + 1))));
  return s;
}
static uint64_t ref_fwd2(const std::array<uint64_t, 32>& c, int q) {
  uint64_t s = 0;
  for (int j = 0; j < 32; ++j) s = addp(s, mulp(c[j], powp(64, (long)lp::brv5(q) * j)));
  return s;
}
static uint64_t ref_inv2(const std::array<uint64_t, 32>& x, int j) {
  uint64_t s = 0;
  for (int q = 0; q < 32; ++q) s = addp(s, mulp(x[q], powp(64, -(long)lp::brv5(q) * j)));
  return s;
}
static uint64_t ref_inv1(const std::array<uint64_t, 32>& x, int j) {
  uint64_t s = 0;
  for (int q = 0; q < 32; ++q) s = addp(s, mulp(x[q], powp(8, -(long)j * (2 * lp::brv5(q) + 1))));
  return s;
}

// gl_mul_pow2_lane<LO, HI> at both of its shifts, on edge and random
// operands: congruent to x 2^S and reduced (at most p), which the paired
// butterflies' one-correction sum and difference rely on.
template <int LO, int HI>
static void check_lane_shift() {
  const uint64_t edge[] = {0, 1, 2, 0xFFFFFFFFull, 0x100000000ull, P - 1, P, P + 1, 0x7FFFFFFFFFFFFFFFull,
                           0x8000000000000000ull, 0xFFFFFFFEFFFFFFFFull, 0xFFFFFFFFFFFFFFFEull, 0xFFFFFFFFFFFFFFFFull};
  for (int S : {LO, HI}) {
    for (int i = 0; i < 13 + 4000; ++i) {
      const uint64_t x = i < 13 ? edge[i] : rnd();
      const uint64_t got = lp::gl_mul_pow2_lane<LO, HI>(x, (uint32_t)S);
      ++checks;
      if (HI == 96 && x > P) continue;  // the S = 96 form takes reduced operands
      if (got > P || got % P != mulp(x, powp(2, S))) {
        std::printf("MISMATCH gl_mul_pow2_lane<%d, %d> S %d x %016llx: got %016llx\n", LO, HI, S,
                    (unsigned long long)x, (unsigned long long)got);
        std::exit(1);
      }
    }
  }
}

int main() {
  using namespace lp;
  // the slot pairs' shifts: pass 1 z = 3 brv5(16 + s), pass 2 z = 6 (brv5(s) >> 1), s < 8
  static_for<0, 8>([&](auto ss) {
    constexpr int s = decltype(ss)::value;
    constexpr int z1 = 3 * brv5(16 + s), z2 = 6 * (brv5(s) >> 1);
    check_lane_shift<z1, z1 + 6>();
    check_lane_shift<z2, z2 + 6>();
    check_lane_shift<90 - z1, 96 - z1>();  // the inverse's first stage
    check_lane_shift<90 - z2, 96 - z2>();
  });
  const Layout L64{2}, L128{4}, L256{8};
  for (int kind = 0; kind < 4; ++kind) {
    // ---- 64 lanes: forward passes (pass 1 from gadget digits) and inverses
    {
      std::vector<std::array<uint64_t, 32>> dig(32), out;
      for (auto& r : dig)
        for (int j = 0; j < 32; ++j) {
          const int d = kind == 2 ? ((j & 1) ? 64 : -64) : kind == 3 ? -64 : (int)(rnd() % 129) - 64;
          r[j] = (uint64_t)(int64_t)d;
        }
      std::vector<std::array<uint64_t, 32>> dres(32);
      for (int r = 0; r < 32; ++r)
        for (int j = 0; j < 32; ++j) dres[r][j] = gl_from_i64((int64_t)dig[r][j]);
      // output in the pair layout
      out.assign(32, {});
      run_wave([&](int Ln) {
        const int h = Ln >> 5, l = Ln & 31;
        int32_t d[16];
        uint64_t a[16];
        for (int s = 0; s < 16; ++s) d[s] = (int32_t)(int64_t)dig[l][2 * s + h];
        fwd64_p1_digits(d, a);
        fwd64_p1_rest_pairs(a, 6u * (uint32_t)h);
        for (int r = 0; r < 16; ++r) out[l][pair_pos(r, h)] = gl_canon(a[r]);
      });
      check("fwd64 pass 1 (digits)", L64, dres, out, ref_fwd1);
    }
    auto in = inputs(32, kind);
    std::vector<std::array<uint64_t, 32>> out;
    out.assign(32, {});
    run_wave([&](int Ln) {
      const int h = Ln >> 5, l = Ln & 31;
      uint64_t a[16];
      for (int s = 0; s < 16; ++s) a[s] = in[l][2 * s + h];
      fwd64_p2_pairs(a, 6u * (uint32_t)h);
      for (int r = 0; r < 16; ++r) out[l][pair_pos(r, h)] = gl_canon(a[r]);
    });
    check("fwd64 pass 2 (pair layout)", L64, in, out, ref_fwd2);
    // the inverses from the pair layout (interleaved output)
    for (int pass = 1; pass <= 2; ++pass) {
      out.assign(32, {});
      run_wave([&](int Ln) {
        const int h = Ln >> 5, l = Ln & 31;
        uint64_t a[16];
        for (int r = 0; r < 16; ++r) a[r] = in[l][pair_pos(r, h)];
        if (pass == 2) inv64_p2_pairs(a, 6u * (uint32_t)h);
        else inv64_p1_pairs(a, 6u * (uint32_t)h);
        for (int s = 0; s < 16; ++s) out[l][2 * s + h] = gl_canon(a[s]);
      });
      check(pass == 2 ? "inv64 pass 2 (pair layout)" : "inv64 pass 1 (pair layout)", L64, in, out,
            pass == 2 ? ref_inv2 : ref_inv1);
    }
    // ---- 128 lanes (one of the two waves: 16 rows at four lanes per row)
    auto in128 = inputs(16, kind);
    auto b128 = [](int Ln, uint64_t& u1, uint64_t& u2) {
      const int hq = Ln & 3;
      u1 = (hq & 1) ? ~0ull : 0ull;
      u2 = (hq & 2) ? ~0ull : 0ull;
    };
    run_layout<8>(L128, in128, out, [&](uint64_t(&a)[8], int Ln) {
      uint64_t u1, u2;
      b128(Ln, u1, u2);
      inv128_p2(a, u1, u2, u2);
    });
    check("inv128 pass 2", L128, in128, out, ref_inv2);
    run_layout<8>(L128, in128, out, [&](uint64_t(&a)[8], int Ln) {
      uint64_t u1, u2;
      b128(Ln, u1, u2);
      inv128_p1(a, u1, u2, u2);
    });
    check("inv128 pass 1", L128, in128, out, ref_inv1);
    // ---- 256 lanes (one of the four waves: 8 rows at eight lanes per row);
    // in: lane 8r + h, register s holds q = 4h + s; out: q = h + 8 (s >> 1)
    // + 16 (s & 1)
    auto in256 = inputs(8, kind);
    for (int pass = 1; pass <= 2; ++pass) {
      out.assign(8, {});
      run_wave([&](int Ln) {
        const int r = Ln >> 3, h = Ln & 7;
        const uint64_t u1 = (h & 1) ? ~0ull : 0ull, u2 = (h & 2) ? ~0ull : 0ull, u4 = (h & 4) ? ~0ull : 0ull;
        uint64_t a[4], w[5];
        inv256_twiddles(pass, h, w);
        for (int s = 0; s < 4; ++s) a[s] = in256[r][4 * h + s];
        if (pass == 2) inv256_pass<2>(a, u1, u2, u4, w);
        else inv256_pass<1>(a, u1, u2, u4, w);
        for (int s = 0; s < 4; ++s) {
          if (a[s] > P) fail("inv256 output not reduced", 8, r, h + 8 * (s >> 1) + 16 * (s & 1), a[s], 0);
          out[r][h + 8 * (s >> 1) + 16 * (s & 1)] = a[s];
        }
      });
      check(pass == 2 ? "inv256 pass 2" : "inv256 pass 1", L256, in256, out, pass == 2 ? ref_inv2 : ref_inv1);
    }
  }
  std::printf("ok %llu\n", (unsigned long long)checks);
  return 0;
}
