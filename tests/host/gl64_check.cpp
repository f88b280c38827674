// Host check of the Goldilocks field operations of the GPU path
// (paper_2407_19871_amd/csrc/gl64.h, compiled here with the host compiler)
// against exact 128-bit arithmetic: every function, every shift amount of
// gl_mul_pow2 / gl_mul_pow2_r (all 192 residues of the exponent, plus
// negative and >= 192 exponents), on edge operands (0, 1, EPS, p - 1, p,
// p + 1, 2^63, 2^64 - 1, ...) crossed with each other and with random
// 64-bit values, including lazy operands at or above p.
// Prints "ok <checks>" and exits 0, or prints the first mismatch and exits 1.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <utility>
#include <vector>

#include "gl64.h"

typedef unsigned __int128 u128;
static const uint64_t P = GL_P;
static uint64_t checks = 0;

static uint64_t modp(u128 x) { return (uint64_t)(x % P); }
static uint64_t pow2mod(long e) {  // 2^e mod p, e may be negative (2^192 = 1)
  e %= 192;
  if (e < 0) e += 192;
  u128 r = 1;
  for (long i = 0; i < e; ++i) r = (r * 2) % P;
  return (uint64_t)r;
}

[[noreturn]] static void fail(const char* what, uint64_t a, uint64_t b, uint64_t got, uint64_t want) {
  std::printf("MISMATCH %s a=%016llx b=%016llx got=%016llx want=%016llx\n", what, (unsigned long long)a,
              (unsigned long long)b, (unsigned long long)got, (unsigned long long)want);
  std::exit(1);
}
static void expect_mod(const char* what, uint64_t a, uint64_t b, uint64_t got, uint64_t want_mod) {
  ++checks;
  if (modp(got) != want_mod) fail(what, a, b, got, want_mod);
}
static void expect_reduced(const char* what, uint64_t a, uint64_t b, uint64_t got) {
  ++checks;
  if (got > P) fail(what, a, b, got, P);
}

static uint64_t rng_state = 0x243F6A8885A308D3ull;
static uint64_t rnd() {  // SplitMix64 step (a test-input source only)
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <int S>
static void check_shift(const std::vector<uint64_t>& xs) {
  const uint64_t m = pow2mod(S);
  constexpr int s = ((S % 192) + 192) % 192;
  for (uint64_t x : xs) {
    const uint64_t want = modp((u128)modp(x) * m);
    const uint64_t lazy = gl_mul_pow2<S>(x);
    expect_mod("gl_mul_pow2", x, (uint64_t)S, lazy, want);
    if (s >= 64) expect_reduced("gl_mul_pow2 (reduced range)", x, (uint64_t)S, lazy);
    const uint64_t red = gl_mul_pow2_r<S>(x);
    expect_mod("gl_mul_pow2_r", x, (uint64_t)S, red, want);
    expect_reduced("gl_mul_pow2_r", x, (uint64_t)S, red);
  }
}
template <int... S>
static void check_shifts(const std::vector<uint64_t>& xs, std::integer_sequence<int, S...>) {
  (check_shift<S>(xs), ...);
}

int main() {
  std::vector<uint64_t> edge = {0, 1, 2, 3, GL_EPS - 1, GL_EPS, GL_EPS + 1, 1ull << 32, (1ull << 32) + 1,
                                P - 2, P - 1, P, P + 1, P + 2, 1ull << 63, (1ull << 63) - 1, (1ull << 63) + 1,
                                0xFFFFFFFFFFFFFFFEull, 0xFFFFFFFFFFFFFFFFull, 0xFFFFFFFF00000000ull,
                                0x00000000FFFFFFFEull, 0x7FFFFFFF80000000ull, P >> 1, (P >> 1) + 1};
  std::vector<uint64_t> red;  // reduced operands [0, p]
  for (uint64_t v : edge)
    if (v <= P) red.push_back(v);
  std::vector<uint64_t> xs = edge;
  for (int i = 0; i < 2000; ++i) xs.push_back(rnd());
  for (int i = 0; i < 200; ++i) xs.push_back(P + (rnd() % GL_EPS));  // lazy values in [p, 2^64)
  for (int i = 0; i < 2000; ++i) red.push_back(rnd() % (P + 1));

  for (uint64_t a : xs) {
    expect_mod("gl_canon", a, 0, gl_canon(a), modp(a));
    ++checks;
    if (gl_canon(a) >= P) fail("gl_canon range", a, 0, gl_canon(a), P);
    const uint32_t lift = gl_lift_u32(a);
    const uint64_t r = modp(a);
    const uint32_t want_lift = r > (P - 1) / 2 ? (uint32_t)(uint64_t)((int64_t)0 - (int64_t)(P - r)) : (uint32_t)r;
    ++checks;
    if (lift != want_lift) fail("gl_lift_u32", a, 0, lift, want_lift);
  }
  for (size_t i = 0; i < xs.size(); ++i)
    for (size_t j = 0; j < xs.size(); j += (i < edge.size() ? 1 : 37)) {
      const uint64_t a = xs[i], b = xs[j];
      expect_mod("gl_add", a, b, gl_add(a, b), modp((u128)modp(a) + modp(b)));
      uint64_t lo, hi;
      gl_mul_wide(a, b, lo, hi);
      ++checks;
      const u128 prod = (u128)a * b;
      if (lo != (uint64_t)prod || hi != (uint64_t)(prod >> 64)) fail("gl_mul_wide", a, b, hi, (uint64_t)(prod >> 64));
      expect_mod("gl_reduce128", a, b, gl_reduce128(a, b), modp(((u128)b << 64) | a));
      expect_mod("gl_mul", a, b, gl_mul(a, b), modp((u128)modp(a) * modp(b)));
      const uint64_t c = xs[(i * 7 + j * 13 + 5) % xs.size()], d = xs[(i * 11 + j * 3 + 1) % xs.size()];
      const uint64_t want_ms = modp((u128)modp((u128)modp(a) * modp(b)) + modp((u128)modp(c) * modp(d)));
      expect_mod("gl_mul_sum", a, b, gl_mul_sum(a, b, c, d), want_ms);
      expect_mod("gl_mul_sum_wide", a, b, gl_mul_sum_wide(lo, hi, c, d), want_ms);
      expect_mod("gl_mac", a, b, gl_mac(c, a, b), modp((u128)modp(c) + modp((u128)modp(a) * modp(b))));
      const uint64_t e = xs[(i * 5 + j * 17 + 3) % xs.size()], f = xs[(i * 13 + j * 7 + 2) % xs.size()];
      expect_mod("gl_mul_sum3", a, b, gl_mul_sum3(a, b, c, d, e, f),
                 modp((u128)want_ms + modp((u128)modp(e) * modp(f))));
    }
  // three maximal products carry twice out of bit 127
  for (uint64_t a : std::vector<uint64_t>{0xFFFFFFFFFFFFFFFFull, 0xFFFFFFFFFFFFFFFEull, P, P - 1})
    for (uint64_t b : std::vector<uint64_t>{0xFFFFFFFFFFFFFFFFull, 0xFFFFFFFFFFFFFFFEull, P + 1}) {
      const uint64_t want = modp((u128)modp((u128)modp(a) * modp(b)) * 3);
      expect_mod("gl_mul_sum3 (carries)", a, b, gl_mul_sum3(a, b, a, b, a, b), want);
    }
  for (uint64_t a : xs)
    for (size_t j = 0; j < red.size(); j += (j < edge.size() ? 1 : 7)) {
      const uint64_t b = red[j];
      expect_mod("gl_add_r", a, b, gl_add_r(a, b), modp((u128)modp(a) + modp(b)));
      expect_mod("gl_sub_r", a, b, gl_sub_r(a, b), modp((u128)modp(a) + P - modp(b)));
    }
  for (uint64_t y : red) {
    expect_mod("gl_neg_r", y, 0, gl_neg_r(y), modp(P - modp(y)));
    expect_reduced("gl_neg_r", y, 0, gl_neg_r(y));
    // reduced operands keep the sum/difference of reduced values reduced-or-lazy but exact
    for (uint64_t z : edge)
      if (z <= P) expect_mod("gl_sub_r(reduced)", y, z, gl_sub_r(y, z), modp((u128)modp(y) + P - modp(z)));
  }
  for (int64_t v : {0ll, 1ll, -1ll, (1ll << 62), -(1ll << 62), (1ll << 50) + 12345, -(1ll << 50) - 777,
                    0x7FFFFFFFFFFFFFFFll, -0x7FFFFFFFFFFFFFFFll}) {
    const uint64_t want = v < 0 ? P - (uint64_t)(-v) % P : (uint64_t)v % P;
    expect_mod("gl_from_i64", (uint64_t)v, 0, gl_from_i64(v), want % P);
  }
  check_shifts(xs, std::make_integer_sequence<int, 192>{});
  check_shift<-1>(xs);
  check_shift<-96>(xs);
  check_shift<200>(xs);
  check_shift<383>(xs);
  std::printf("ok %llu\n", (unsigned long long)checks);
  return 0;
}
