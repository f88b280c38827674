// Host side of liblocpir: the C ABI declared in include/locpir.h.
//
//   * client operations (KeyGen, Encrypt, Decrypt of Sec. 2.2) on the host;
//   * device keys: upload and NTT-domain conversion of the bootstrapping key;
//   * gate batches and key-switch batches on the GPU;
//   * the bounding-box circuit of Algorithms 2-5 compiled to a level plan
//     (a DAG cut into depth levels; each level = one blind-rotation launch
//     plus one key-switch launch over every gate of that level).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/locpir.h"
#include "internal.h"
#include "jobs.h"
#include "kernels.h"
#include "lwe_ops.h"

using lp::BrJob;
using lp::KsJob;

// ---------------------------------------------------------------- errors
namespace {
thread_local std::string g_err;
}  // namespace

lp_status lp::fail(lp_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

namespace {
using lp::fail;

bool params_ok(const lp_params* P, std::string* why) {
  if (!P) { *why = "null params"; return false; }
  if (P->n == 0 || P->n > 4096) { *why = "n out of range"; return false; }
  if (P->N < 2 || P->N > 4096 || (P->N & (P->N - 1))) { *why = "N must be a power of two"; return false; }
  if (P->k != 1) { *why = "only k = 1 is supported"; return false; }
  if (P->bg_bit == 0 || P->l == 0 || P->bg_bit * P->l > 31) { *why = "bad gadget"; return false; }
  if (P->ks_base_bit == 0 || P->ks_base_bit > 8 || P->ks_t == 0 || P->ks_base_bit * P->ks_t > 31) {
    *why = "bad key-switching base/digits";
    return false;
  }
  if (!(P->lwe_sigma >= 0) || !(P->bk_sigma >= 0)) { *why = "bad sigma"; return false; }
  return true;
}

bool gpu_params_ok(const lp_params& P, std::string* why) {
  if (P.N != 1024 || P.k != 1 || P.bg_bit != 7 || P.l != 3) {
    *why = "GPU kernels need N = 1024, k = 1, bg_bit = 7, l = 3";
    return false;
  }
  if (P.n > 1024) { *why = "GPU kernels need n <= 1024"; return false; }
  if (P.ks_base_bit > 4) { *why = "GPU key switching needs ks_base_bit <= 4"; return false; }
  return true;
}

// ---------------------------------------------------------------- random
// SplitMix64 (Steele, Lea, Flood 2014).  The k-th output (k from 0) of a
// generator started at state x is finalize(x + (k+1) * 0x9E3779B97F4A7C15).
// A draw is addressed by (seed, stream, index): the stream's key is output
// `stream` of SplitMix64(seed), the draw is output `index` of
// SplitMix64(key).  Counter addressing lets rows be generated in parallel.
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

inline uint64_t finalize64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return x;
}

struct Stream {
  uint64_t key;
  Stream(uint64_t seed, uint64_t id) : key(finalize64(seed + (id + 1) * kGolden)) {}
  uint64_t u64(uint64_t idx) const { return finalize64(key + (idx + 1) * kGolden); }
  uint32_t u32(uint64_t idx) const { return (uint32_t)(u64(idx) >> 32); }
  uint8_t bit(uint64_t idx) const { return (uint8_t)(u64(idx) >> 63); }
  // centred Gaussian in Torus32 units, std sigma (torus): Box-Muller, cosine
  // branch, from draws 2 idx and 2 idx + 1; rounded half away from zero
  uint32_t gauss(uint64_t idx, double sigma) const {
    const double u1 = (double)((u64(2 * idx) >> 11) + 1) * 0x1p-53;
    const double u2 = (double)(u64(2 * idx + 1) >> 11) * 0x1p-53;
    const double radius = std::sqrt(-2.0 * std::log(u1));
    const double z = radius * std::cos(6.283185307179586 * u2);
    const double scaled = z * (sigma * 4294967296.0);
    return (uint32_t)(uint64_t)std::llround(scaled);
  }
};

enum : uint64_t { kStLweKey = 0, kStRingKey = 1, kStBskMask = 2, kStBskNoise = 3, kStKskMask = 4,
                  kStKskNoise = 5, kStEncMask = 6, kStEncNoise = 7, kStZeroMask = 8, kStZeroNoise = 9 };

void parallel_rows(size_t rows, const std::function<void(size_t)>& fn) {
  unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (rows < 64 || hw == 1) {
    for (size_t r = 0; r < rows; ++r) fn(r);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned t = 0; t < hw; ++t)
    th.emplace_back([&, t] {
      for (size_t r = t; r < rows; r += hw) fn(r);
    });
  for (auto& x : th) x.join();
}
}  // namespace

extern "C" size_t lp_bsk_words(const lp_params* P) {
  return P ? (size_t)P->n * 2 * P->l * 2 * P->N : 0;
}
extern "C" size_t lp_ksk_words(const lp_params* P) {
  return P ? (size_t)P->N * P->ks_t * ((1u << P->ks_base_bit) - 1) * (P->n + 1) : 0;
}

extern "C" const char* lp_last_error(void) { return g_err.c_str(); }
extern "C" const char* lp_version(void) { return "locpir-mi355x 0.1"; }

extern "C" lp_status lp_params_default(lp_params* out) {
  if (!out) return fail(LP_EINVAL, "null output");
  *out = lp_params{630, 1024, 1, 7, 3, 2, 8, std::ldexp(1.0, -15), std::ldexp(1.0, -25)};
  return LP_OK;
}

extern "C" lp_status lp_params_lambda80(lp_params* out) {
  if (!out) return fail(LP_EINVAL, "null output");
  *out = lp_params{540, 1024, 1, 7, 3, 2, 8, std::exp2(-20.2), std::ldexp(1.0, -25)};
  return LP_OK;
}

// ---------------------------------------------------------------- KeyGen
// B = A * S in Z_{2^32}[X]/(X^N + 1) for a binary S: B[j] = sum over set
// bits t of S of (X^t A)[j].  With the sign-extended table
// W[y] = -A[y] (y < N), A[y - N] (y >= N), (X^t A)[j] = W[N + j - t].
static void ring_times_binary(uint32_t N, const uint32_t* A, const uint8_t* S, uint32_t* B) {
  std::vector<uint32_t> W(2 * N);
  for (uint32_t y = 0; y < N; ++y) {
    W[y] = 0u - A[y];
    W[N + y] = A[y];
  }
  std::fill(B, B + N, 0u);
  for (uint32_t t = 0; t < N; ++t) {
    if (!S[t]) continue;
    const uint32_t* w = W.data() + (N - t);
    for (uint32_t j = 0; j < N; ++j) B[j] += w[j];
  }
}

// LWE sample of torus value mu under binary key s (dimension n)
static void lwe_sample(uint32_t n, const uint8_t* s, uint32_t mu, const Stream& mask, const Stream& noise,
                       uint64_t idx, double sigma, uint32_t* out) {
  uint32_t dot = 0;
  for (uint32_t c = 0; c < n; ++c) {
    out[c] = mask.u32(idx * n + c);
    if (s[c]) dot += out[c];
  }
  out[n] = dot + mu + noise.gauss(idx, sigma);
}

extern "C" lp_status lp_keygen(const lp_params* P, uint64_t seed, lp_secret_key** sk, lp_cloud_key** ck) {
  std::string why;
  if (!params_ok(P, &why)) return fail(LP_EINVAL, "lp_keygen: %s", why.c_str());
  if (!sk || !ck) return fail(LP_EINVAL, "lp_keygen: null output");
  try {
    auto s = std::make_unique<lp_secret_key>();
    auto c = std::make_unique<lp_cloud_key>();
    s->P = c->P = *P;
    const uint32_t n = P->n, N = P->N, l = P->l, rows = 2 * l;
    const Stream st_s(seed, kStLweKey), st_S(seed, kStRingKey);
    s->s.resize(n);
    s->S.resize(N);
    for (uint32_t i = 0; i < n; ++i) s->s[i] = st_s.bit(i);
    for (uint32_t i = 0; i < N; ++i) s->S[i] = st_S.bit(i);

    // bootstrapping key: BSK_i = TGSW_S(s_i), row r = (p, j) with p = r / l
    c->bsk.resize(lp_bsk_words(P));
    const Stream st_a(seed, kStBskMask), st_e(seed, kStBskNoise);
    parallel_rows((size_t)n * rows, [&](size_t row) {
      const uint32_t i = (uint32_t)(row / rows), r = (uint32_t)(row % rows);
      uint32_t* A = c->bsk.data() + row * 2 * N;
      uint32_t* B = A + N;
      for (uint32_t k = 0; k < N; ++k) A[k] = st_a.u32(row * N + k);
      ring_times_binary(N, A, s->S.data(), B);
      for (uint32_t k = 0; k < N; ++k) B[k] += st_e.gauss(row * N + k, P->bk_sigma);
      if (s->s[i]) {
        const uint32_t p = r / l, j = r % l;
        const uint32_t g = 1u << (32 - P->bg_bit * (j + 1));  // 1/Bg^(j+1)
        (p == 0 ? A : B)[0] += g;
      }
    });

    // key-switching key: KSK[i][j][v-1] = LWE_s(v S_i / base^(j+1))
    const uint32_t nv = (1u << P->ks_base_bit) - 1;
    c->ksk.resize(lp_ksk_words(P));
    const Stream st_ka(seed, kStKskMask), st_ke(seed, kStKskNoise);
    parallel_rows((size_t)N * P->ks_t, [&](size_t ij) {
      const uint32_t i = (uint32_t)(ij / P->ks_t), j = (uint32_t)(ij % P->ks_t);
      for (uint32_t v = 1; v <= nv; ++v) {
        const uint64_t row = ij * nv + (v - 1);
        const uint32_t msg = s->S[i] ? v << (32 - P->ks_base_bit * (j + 1)) : 0u;
        lwe_sample(n, s->s.data(), msg, st_ka, st_ke, row, P->lwe_sigma, c->ksk.data() + row * (n + 1));
      }
    });
    *sk = s.release();
    *ck = c.release();
    return LP_OK;
  } catch (const std::bad_alloc&) {
    return fail(LP_ENOMEM, "lp_keygen: out of host memory");
  }
}

extern "C" lp_status lp_secret_key_import(const lp_params* P, const uint8_t* s, const uint8_t* S,
                                          lp_secret_key** sk) {
  std::string why;
  if (!params_ok(P, &why)) return fail(LP_EINVAL, "lp_secret_key_import: %s", why.c_str());
  if (!s || !S || !sk) return fail(LP_EINVAL, "lp_secret_key_import: null argument");
  auto k = std::make_unique<lp_secret_key>();
  k->P = *P;
  k->s.assign(s, s + P->n);
  k->S.assign(S, S + P->N);
  for (auto& b : k->s) if (b > 1) return fail(LP_EINVAL, "lp_secret_key_import: key bits must be 0/1");
  for (auto& b : k->S) if (b > 1) return fail(LP_EINVAL, "lp_secret_key_import: key bits must be 0/1");
  *sk = k.release();
  return LP_OK;
}

extern "C" lp_status lp_secret_key_export(const lp_secret_key* sk, uint8_t* s, uint8_t* S) {
  if (!sk) return fail(LP_EINVAL, "lp_secret_key_export: null key");
  if (s) std::memcpy(s, sk->s.data(), sk->s.size());
  if (S) std::memcpy(S, sk->S.data(), sk->S.size());
  return LP_OK;
}

extern "C" lp_status lp_cloud_key_import(const lp_params* P, const uint32_t* bsk, const uint32_t* ksk,
                                         lp_cloud_key** ck) {
  std::string why;
  if (!params_ok(P, &why)) return fail(LP_EINVAL, "lp_cloud_key_import: %s", why.c_str());
  if (!bsk || !ksk || !ck) return fail(LP_EINVAL, "lp_cloud_key_import: null argument");
  try {
    auto k = std::make_unique<lp_cloud_key>();
    k->P = *P;
    k->bsk.assign(bsk, bsk + lp_bsk_words(P));
    k->ksk.assign(ksk, ksk + lp_ksk_words(P));
    *ck = k.release();
    return LP_OK;
  } catch (const std::bad_alloc&) {
    return fail(LP_ENOMEM, "lp_cloud_key_import: out of host memory");
  }
}

extern "C" lp_status lp_cloud_key_export(const lp_cloud_key* ck, uint32_t* bsk, uint32_t* ksk) {
  if (!ck) return fail(LP_EINVAL, "lp_cloud_key_export: null key");
  if (bsk) std::memcpy(bsk, ck->bsk.data(), ck->bsk.size() * 4);
  if (ksk) std::memcpy(ksk, ck->ksk.data(), ck->ksk.size() * 4);
  return LP_OK;
}

// ---------------------------------------------------------------- PK wire format
// 64-byte header, then the key words (the host is little-endian):
//   0  "LPCK"   4  format version (1)   8  n, N, k, bg_bit, l, ks_base_bit,
//   ks_t (u32 each)   36  lwe_sigma, bk_sigma (f64)   52  zero padding
//   64  bsk words   then  ksk words   (all u32)
namespace {
constexpr size_t kPkHeader = 64;
constexpr uint32_t kPkVersion = 1;
}  // namespace

extern "C" lp_status lp_cloud_key_serialize(const lp_cloud_key* ck, void* buf, size_t* len) {
  if (!ck || !len) return fail(LP_EINVAL, "lp_cloud_key_serialize: null argument");
  const size_t need = kPkHeader + (ck->bsk.size() + ck->ksk.size()) * 4;
  if (!buf) {
    *len = need;
    return LP_OK;
  }
  if (*len < need) return fail(LP_EINVAL, "lp_cloud_key_serialize: buffer of %zu bytes, need %zu", *len, need);
  unsigned char* b = static_cast<unsigned char*>(buf);
  std::memset(b, 0, kPkHeader);
  std::memcpy(b, "LPCK", 4);
  std::memcpy(b + 4, &kPkVersion, 4);
  const uint32_t f[7] = {ck->P.n, ck->P.N, ck->P.k, ck->P.bg_bit, ck->P.l, ck->P.ks_base_bit, ck->P.ks_t};
  std::memcpy(b + 8, f, sizeof f);
  std::memcpy(b + 36, &ck->P.lwe_sigma, 8);
  std::memcpy(b + 44, &ck->P.bk_sigma, 8);
  std::memcpy(b + kPkHeader, ck->bsk.data(), ck->bsk.size() * 4);
  std::memcpy(b + kPkHeader + ck->bsk.size() * 4, ck->ksk.data(), ck->ksk.size() * 4);
  *len = need;
  return LP_OK;
}

extern "C" lp_status lp_cloud_key_deserialize(const void* buf, size_t len, lp_cloud_key** ck) {
  if (!buf || !ck) return fail(LP_EINVAL, "lp_cloud_key_deserialize: null argument");
  const unsigned char* b = static_cast<const unsigned char*>(buf);
  uint32_t version = 0;
  if (len < kPkHeader || std::memcmp(b, "LPCK", 4) != 0)
    return fail(LP_EINVAL, "lp_cloud_key_deserialize: not a serialized cloud key");
  std::memcpy(&version, b + 4, 4);
  if (version != kPkVersion) return fail(LP_EINVAL, "lp_cloud_key_deserialize: format version %u", version);
  uint32_t f[7];
  std::memcpy(f, b + 8, sizeof f);
  lp_params P{f[0], f[1], f[2], f[3], f[4], f[5], f[6], 0.0, 0.0};
  std::memcpy(&P.lwe_sigma, b + 36, 8);
  std::memcpy(&P.bk_sigma, b + 44, 8);
  std::string why;
  if (!params_ok(&P, &why)) return fail(LP_EINVAL, "lp_cloud_key_deserialize: %s", why.c_str());
  const size_t nb = lp_bsk_words(&P), nk = lp_ksk_words(&P);
  if (len != kPkHeader + (nb + nk) * 4)
    return fail(LP_EINVAL, "lp_cloud_key_deserialize: %zu bytes, the parameters need %zu", len,
                kPkHeader + (nb + nk) * 4);
  const uint32_t* w = reinterpret_cast<const uint32_t*>(b + kPkHeader);
  if (reinterpret_cast<uintptr_t>(w) % alignof(uint32_t) == 0) return lp_cloud_key_import(&P, w, w + nb, ck);
  // unaligned blob: copy the words out first
  try {
    std::vector<uint32_t> words(nb + nk);
    std::memcpy(words.data(), b + kPkHeader, (nb + nk) * 4);
    return lp_cloud_key_import(&P, words.data(), words.data() + nb, ck);
  } catch (const std::bad_alloc&) {
    return fail(LP_ENOMEM, "lp_cloud_key_deserialize: out of host memory");
  }
}

extern "C" lp_status lp_cloud_key_params(const lp_cloud_key* ck, lp_params* out) {
  if (!ck || !out) return fail(LP_EINVAL, "lp_cloud_key_params: null argument");
  *out = ck->P;
  return LP_OK;
}

// ---------------------------------------------------------------- Encrypt / Decrypt
extern "C" lp_status lp_encrypt_bits(const lp_secret_key* sk, const uint8_t* bits, size_t cnt, uint64_t seed,
                                     uint64_t first_index, uint32_t* ct) {
  if (!sk || (cnt && (!bits || !ct))) return fail(LP_EINVAL, "lp_encrypt_bits: null argument");
  const uint32_t n = sk->P.n;
  const Stream mask(seed, kStEncMask), noise(seed, kStEncNoise);
  for (size_t k = 0; k < cnt; ++k) {
    if (bits[k] > 1) return fail(LP_EINVAL, "lp_encrypt_bits: bits must be 0/1");
    const uint32_t mu = bits[k] ? 0x20000000u : 0xE0000000u;  // f(m) = m/4 - 1/8
    lwe_sample(n, sk->s.data(), mu, mask, noise, first_index + k, sk->P.lwe_sigma, ct + k * (n + 1));
  }
  return LP_OK;
}

extern "C" lp_status lp_encrypt_zeros(const lp_secret_key* sk, size_t cnt, uint64_t seed, uint64_t first_index,
                                      uint32_t* ct) {
  if (!sk || (cnt && !ct)) return fail(LP_EINVAL, "lp_encrypt_zeros: null argument");
  const uint32_t n = sk->P.n;
  const Stream mask(seed, kStZeroMask), noise(seed, kStZeroNoise);
  for (size_t k = 0; k < cnt; ++k)
    lwe_sample(n, sk->s.data(), 0u, mask, noise, first_index + k, sk->P.lwe_sigma, ct + k * (n + 1));
  return LP_OK;
}

extern "C" lp_status lp_bbox_wire_bytes(const lp_params* P, uint32_t l, uint32_t n_boxes, uint32_t m,
                                        lp_wire_bytes* out) {
  std::string why;
  if (!params_ok(P, &why)) return fail(LP_EINVAL, "lp_bbox_wire_bytes: %s", why.c_str());
  if (!out) return fail(LP_EINVAL, "lp_bbox_wire_bytes: null output");
  if (l == 0 || l > 64 || n_boxes == 0 || m == 0) return fail(LP_EINVAL, "lp_bbox_wire_bytes: empty shape");
  const size_t s = ((size_t)P->n + 1) * 4;
  out->lwe_sample = s;
  out->public_key = (lp_bsk_words(P) + lp_ksk_words(P)) * 4;
  out->service_samples = (size_t)n_boxes * m * s;
  out->coordinate = (size_t)l * s;
  out->query = 2 * (size_t)l * s;
  out->result = (size_t)m * s;
  return LP_OK;
}

extern "C" lp_status lp_decrypt_bits(const lp_secret_key* sk, const uint32_t* ct, size_t cnt, uint8_t* bits,
                                     int32_t* phase) {
  if (!sk || (cnt && (!ct || !bits))) return fail(LP_EINVAL, "lp_decrypt_bits: null argument");
  const uint32_t n = sk->P.n;
  for (size_t k = 0; k < cnt; ++k) {
    const uint32_t* c = ct + k * (n + 1);
    uint32_t dot = 0;
    for (uint32_t i = 0; i < n; ++i)
      if (sk->s[i]) dot += c[i];
    const int32_t ph = (int32_t)(c[n] - dot);
    bits[k] = ph > 0 ? 1 : 0;
    if (phase) phase[k] = ph;
  }
  return LP_OK;
}

// ---------------------------------------------------------------- twiddles
namespace {
constexpr uint64_t kP = 0xFFFFFFFF00000001ull;

uint64_t mulmod_p(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) % kP); }
uint64_t powmod_p(uint64_t b, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = mulmod_p(r, b);
    b = mulmod_p(b, b);
    e >>= 1;
  }
  return r;
}
int bit_reverse5(int x) {
  int r = 0;
  for (int b = 0; b < 5; ++b) r |= ((x >> b) & 1) << (4 - b);
  return r;
}

// psi: a primitive 2048th root of unity with psi^32 = 8.  7 generates Z_p^*
// (checked against every prime factor of p - 1 = 2^32 3 5 17 257 65537).
// g = 7^((p-1)/2048) is a primitive 2048th root; g^32 is a primitive 64th
// root, i.e. 8^c for some odd c, and psi = g^e with (g^32)^e = 8.
bool make_twiddles(std::vector<uint64_t>& fwd, std::vector<uint64_t>& inv) {
  for (uint64_t f : {2ull, 3ull, 5ull, 17ull, 257ull, 65537ull})
    if (powmod_p(7, (kP - 1) / f) == 1) return false;
  const uint64_t g = powmod_p(7, (kP - 1) / 2048);
  const uint64_t g32 = powmod_p(g, 32);
  uint64_t e = 0;
  for (uint64_t c = 1; c < 64; c += 2)
    if (powmod_p(g32, c) == 8) { e = c; break; }
  if (!e) return false;
  const uint64_t psi = powmod_p(g, e);
  if (powmod_p(psi, 32) != 8 || powmod_p(psi, 1024) != kP - 1) return false;
  const uint64_t psi_inv = powmod_p(psi, 2047);
  const uint64_t n_inv = powmod_p(1024, kP - 2);
  fwd.assign(1024, 0);
  inv.assign(1024, 0);
  for (int i = 0; i < 32; ++i)
    for (int l = 0; l < 32; ++l) {
      const uint64_t ex = (uint64_t)(2 * bit_reverse5(i) + 1) * l;
      fwd[i * 32 + l] = powmod_p(psi, ex % 2048);
    }
  for (int m = 0; m < 32; ++m)
    for (int l = 0; l < 32; ++l) {
      const uint64_t ex = (uint64_t)(2 * bit_reverse5(l) + 1) * m;
      inv[m * 32 + l] = mulmod_p(powmod_p(psi_inv, ex % 2048), n_inv);
    }
  return true;
}

struct DeviceTables {
  uint64_t* fwd = nullptr;
  uint64_t* inv = nullptr;
};
std::mutex g_tw_mu;
std::map<int, DeviceTables> g_tw;

}  // namespace

// Twiddle tables of the current device, uploaded once and kept for the
// process lifetime.
lp_status lp::device_twiddles(lp::Twiddles* out) {
  int dev = 0;
  LP_HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_tw_mu);
  auto it = g_tw.find(dev);
  if (it == g_tw.end()) {
    std::vector<uint64_t> f, i;
    if (!make_twiddles(f, i)) return fail(LP_EDEVICE, "twiddle construction failed");
    DeviceTables t;
    LP_HIP_TRY(hipMalloc(&t.fwd, 1024 * 8));
    LP_HIP_TRY(hipMalloc(&t.inv, 1024 * 8));
    LP_HIP_TRY(hipMemcpy(t.fwd, f.data(), 1024 * 8, hipMemcpyHostToDevice));
    LP_HIP_TRY(hipMemcpy(t.inv, i.data(), 1024 * 8, hipMemcpyHostToDevice));
    it = g_tw.emplace(dev, t).first;
  }
  out->fwd = it->second.fwd;
  out->inv = it->second.inv;
  return LP_OK;
}

using lp::as_stream;
using lp::device_twiddles;
using lp::pick_br_wpb;
using lp::pick_ks_split;
using lp::pick_ks_tile;
using lp::ProfScope;
using lp::ScopedDevice;
using lp::kProfBR;
using lp::kProfKS;

// ---------------------------------------------------------------- profiling
namespace lp {
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof;
}  // namespace lp
using lp::g_prof;
using lp::g_prof_mu;
using lp::g_prof_on;
using lp::ProfRecord;
using lp::kProfKinds;
namespace {
const char* kProfNames[lp::kProfKinds] = {"blind_rotate", "keyswitch"};
}

lp_status lp::split_stall_error(const char* who, uint32_t stalls) {
  return fail(LP_EDEVICE,
              "%s: %u split-rotation wait(s) ran out of polls (a partner workgroup did not arrive in time); "
              "the affected outputs are undefined", who, stalls);
}

extern "C" lp_status lp_split_stall_count(uint32_t* count) {
  if (!count) return fail(LP_EINVAL, "lp_split_stall_count: null argument");
  LP_HIP_TRY(hipDeviceSynchronize());
  LP_HIP_TRY(lp::split_stall_count(count));
  return LP_OK;
}

extern "C" lp_status lp_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return LP_OK;
}

namespace {
// Takes the recorded launches and their event-measured durations (ms),
// oldest first, and clears the record.
lp_status drain_profile(const char* who, std::vector<ProfRecord>* recs, std::vector<float>* ms) {
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recs->swap(g_prof);
  }
  lp_status st = LP_OK;
  ms->assign(recs->size(), 0.f);
  for (size_t i = 0; i < recs->size(); ++i) {
    ProfRecord& r = (*recs)[i];
    hipError_t e = hipEventSynchronize(r.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&(*ms)[i], r.start, r.stop);
    if (e != hipSuccess) st = fail(LP_EDEVICE, "%s: %s", who, hipGetErrorString(e));
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  return st;
}
}  // namespace

extern "C" lp_status lp_profile_collect(lp_kernel_stat* stats, int* count) {
  if (!count) return fail(LP_EINVAL, "lp_profile_collect: null count");
  std::vector<ProfRecord> recs;
  std::vector<float> ms;
  const lp_status st = drain_profile("lp_profile_collect", &recs, &ms);
  lp_kernel_stat agg[kProfKinds];
  for (int k = 0; k < kProfKinds; ++k) agg[k] = lp_kernel_stat{kProfNames[k], 0, 0, 0.0};
  for (size_t i = 0; i < recs.size(); ++i) {
    agg[recs[i].kind].launches += 1;
    agg[recs[i].kind].jobs += recs[i].jobs;
    agg[recs[i].kind].total_ms += ms[i];
  }
  const int n = std::min(*count, (int)kProfKinds);
  if (stats)
    for (int k = 0; k < n; ++k) stats[k] = agg[k];
  *count = stats ? n : 0;
  return st;
}

extern "C" lp_status lp_profile_collect_launches(lp_launch_record* recs, int* count) {
  if (!count || (*count > 0 && !recs)) return fail(LP_EINVAL, "lp_profile_collect_launches: null argument");
  std::vector<ProfRecord> all;
  std::vector<float> ms;
  const lp_status st = drain_profile("lp_profile_collect_launches", &all, &ms);
  const int n = (int)std::min<size_t>(std::max(*count, 0), all.size());
  for (int i = 0; i < n; ++i)
    recs[i] = lp_launch_record{kProfNames[all[i].kind], all[i].jobs, all[i].shape, (double)ms[i]};
  *count = n;
  return st;
}

// ---------------------------------------------------------------- device keys
extern "C" void lp_device_key_free(lp_device_key* dk);

extern "C" lp_status lp_device_key_create(const lp_cloud_key* ck, void* stream, lp_device_key** dk) {
  if (!ck || !dk) return fail(LP_EINVAL, "lp_device_key_create: null argument");
  std::string why;
  if (!gpu_params_ok(ck->P, &why)) return fail(LP_EUNSUPPORTED, "lp_device_key_create: %s", why.c_str());
  hipStream_t s = as_stream(stream);
  auto k = std::make_unique<lp_device_key>();
  k->P = ck->P;
  LP_HIP_TRY(hipGetDevice(&k->device));
  lp_status st = device_twiddles(&k->tw);
  if (st != LP_OK) return st;
  const size_t bw = ck->bsk.size(), kw = ck->ksk.size();
  uint32_t* tmp = nullptr;
  hipError_t e = hipMalloc(&k->bsk_ntt, bw * 8);
  if (e == hipSuccess) e = hipMalloc(&k->ksk, kw * 4);
  if (e == hipSuccess) e = hipMalloc(&tmp, bw * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&k->bsk_tab, sizeof(void*));
  if (e == hipSuccess) e = hipMalloc((void**)&k->ksk_tab, sizeof(void*));
  if (e != hipSuccess) {
    if (tmp) (void)hipFree(tmp);
    lp_device_key_free(k.release());
    return fail(LP_ENOMEM, "lp_device_key_create: device allocation failed (%s)", hipGetErrorString(e));
  }
  e = hipMemcpyAsync(tmp, ck->bsk.data(), bw * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(k->ksk, ck->ksk.data(), kw * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(k->bsk_tab, &k->bsk_ntt, sizeof(void*), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(k->ksk_tab, &k->ksk, sizeof(void*), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = lp::launch_bsk_to_ntt(tmp, k->bsk_ntt, (int)(bw / 1024), k->tw, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(tmp);
  if (e != hipSuccess) {
    lp_device_key_free(k.release());
    return fail(LP_EDEVICE, "lp_device_key_create: %s", hipGetErrorString(e));
  }
  k->bytes = bw * 8 + kw * 4;
  *dk = k.release();
  return LP_OK;
}

extern "C" lp_status lp_device_key_bytes(const lp_device_key* dk, size_t* bytes) {
  if (!dk || !bytes) return fail(LP_EINVAL, "lp_device_key_bytes: null argument");
  *bytes = dk->bytes;
  return LP_OK;
}

// ---------------------------------------------------------------- gate batches
namespace {
struct GateCombo {
  int nbr;  // 0 = linear only, 1 = one blind rotation, 2 = MUX
  uint32_t cst;
  int32_t c0, c1;
};

// Linear pre-combination whose phase sign is the gate's value; HomAND =
// Bootstrap((0, -1/8) + c1 + c2) (Sec. 2.2), the rest alike.
bool gate_combo(lp_gate g, GateCombo* c) {
  const uint32_t E = 0x20000000u, Qr = 0x40000000u;  // 1/8, 1/4
  switch (g) {
    case LP_GATE_NAND: *c = {1, E, -1, -1}; return true;
    case LP_GATE_AND: *c = {1, 0u - E, 1, 1}; return true;
    case LP_GATE_OR: *c = {1, E, 1, 1}; return true;
    case LP_GATE_NOR: *c = {1, 0u - E, -1, -1}; return true;
    case LP_GATE_XOR: *c = {1, Qr, 2, 2}; return true;
    case LP_GATE_XNOR: *c = {1, 0u - Qr, -2, -2}; return true;
    case LP_GATE_MUX: *c = {2, 0, 0, 0}; return true;
    case LP_GATE_NOT: *c = {0, 0, -1, 0}; return true;
    case LP_GATE_COPY: *c = {0, 0, 1, 0}; return true;
  }
  return false;
}

}  // namespace

namespace {
// Gate bootstrapping of a batch: blind rotations (sample extraction
// included) and, with_ks, the key switch into d_out (cnt * (n+1) words);
// without it d_out receives the samples the key switch would take
// (cnt * (N+1) words).  Working memory (job lists, extract slots, the split
// area) comes from the stream-ordered allocator, or from `pre` when given
// (the static scratch: then nothing is allocated).
lp_status bootstrap_batch(const char* who, const lp_device_key* dk, lp_gate gate, const uint32_t* d_in0,
                          const uint32_t* d_in1, const uint32_t* d_in2, size_t cnt, uint32_t* d_out, bool with_ks,
                          void* stream, const lp::NoAllocScratch* pre = nullptr) {
  if (!dk) return fail(LP_EINVAL, "%s: null key", who);
  GateCombo gc;
  if (!gate_combo(gate, &gc)) return fail(LP_EINVAL, "%s: unknown gate %d", who, (int)gate);
  if (!with_ks && gc.nbr == 0) return fail(LP_EINVAL, "%s: NOT and COPY do not bootstrap", who);
  if (cnt == 0) return LP_OK;
  if (!d_in0 || !d_out) return fail(LP_EINVAL, "%s: null buffer", who);
  if (gc.nbr >= 1 && gate != LP_GATE_MUX && !d_in1) return fail(LP_EINVAL, "%s: gate needs d_in1", who);
  if (gate == LP_GATE_MUX && (!d_in1 || !d_in2)) return fail(LP_EINVAL, "%s: MUX needs three inputs", who);
  if (cnt > (size_t)(lp::REF_INDEX_MASK / 2)) return fail(LP_EINVAL, "%s: batch too large", who);
  if (pre && cnt > (size_t)lp::kNoAllocMaxGates)
    return fail(LP_EINVAL, "%s: %zu gates exceed the static scratch's maximum of %d per call", who, cnt,
                lp::kNoAllocMaxGates);
  ScopedDevice sd(dk->device);
  hipStream_t s = as_stream(stream);
  const uint32_t n = dk->P.n, N = dk->P.N;
  if (gc.nbr == 0) {
    LP_HIP_TRY(lp::launch_lwe_scale(d_in0, d_out, cnt * (n + 1), gc.c0, s));
    return LP_OK;
  }
  const size_t nbr = cnt * gc.nbr;
  // single-rotation gates without a key switch extract straight into d_out
  const bool direct = !with_ks && gc.nbr == 1;
  const size_t ex_bytes = direct ? 0 : nbr * (N + 1) * 4, br_bytes = nbr * sizeof(BrJob),
               ks_bytes = cnt * sizeof(KsJob);
  int waves = pick_br_wpb(nbr);
  // the static scratch's split area holds kNoAllocSplitJobs jobs; a wider
  // split launch there takes four waves two per CU instead
  if (pre && lp::is_split(waves) && nbr > (size_t)pre->split.max_jobs) waves = 5;
  char* scratch = nullptr;
  uint32_t* ex = d_out;
  BrJob* br = nullptr;
  KsJob* ks = nullptr;
  lp::SplitArea split;
  if (pre) {
    if (!direct) ex = pre->ex;
    br = pre->br;
    ks = pre->ks;
    if (lp::is_split(waves)) {
      split = pre->split;
      // the control words start at zero whatever an earlier call left
      LP_HIP_TRY(lp::launch_clear_words(split.sync, lp::split_sync_bytes(split.max_jobs) / 4, s));
    }
  } else {
    LP_HIP_TRY(hipMallocAsync((void**)&scratch, ex_bytes + br_bytes + ks_bytes + 512, s));
    if (!direct) ex = reinterpret_cast<uint32_t*>(scratch);
    br = reinterpret_cast<BrJob*>(scratch + ((ex_bytes + 255) & ~size_t(255)));
    ks = reinterpret_cast<KsJob*>(reinterpret_cast<char*>(br) + ((br_bytes + 255) & ~size_t(255)));
  }
  hipError_t e = lp::launch_make_batch_jobs(gc.nbr, gc.cst, gc.c0, gc.c1, d_in1 != nullptr, cnt, br, ks, s);
  lp::SrcBases src{};
  src.p[0] = d_in0;
  src.p[1] = d_in1;
  src.p[2] = d_in2;
  lp::DstBases dst{};
  dst.p[0] = d_out;
  // stream-ordered, freed below (the static scratch's area is kept)
  if (e == hipSuccess && lp::is_split(waves) && !pre) e = lp::split_area_alloc_async(&split, (int)nbr, s);
  if (e == hipSuccess) {
    ProfScope ps(kProfBR, nbr, waves, s);
    e = lp::launch_blind_rotate(br, (int)nbr, src, ex, dk->bsk_tab, nullptr, (int)n, (int)n, 0, dk->tw, waves, s,
                                &split);
  }
  if (e == hipSuccess && with_ks) {
    const int tile = pick_ks_tile(cnt);
    ProfScope ps(kProfKS, cnt, tile, s);
    e = lp::launch_keyswitch(ks, (int)cnt, ex, dst, dk->ksk_tab, nullptr, (int)n, (int)N, (int)dk->P.ks_t,
                             (int)dk->P.ks_base_bit, tile, pick_ks_split(cnt, tile, n), s);
  } else if (e == hipSuccess && !direct) {
    // MUX: (0, 1/8) + u1 + u2, the sample its key switch would take
    e = lp::launch_lwe_pair_sum(ex, d_out, cnt, (int)N + 1, 0x20000000u, s);
  }
  // split rotations: wait for the batch and read the area's give-up record
  uint32_t stalls = 0;
  if (e == hipSuccess && lp::is_split(waves)) e = lp::split_area_take_stalls(&split, s, &stalls, nullptr);
  hipError_t e2 = hipSuccess;
  if (!pre) {
    e2 = hipFreeAsync(scratch, s);
    const hipError_t e3 = lp::split_area_free_async(&split, s);
    if (e2 == hipSuccess) e2 = e3;
  }
  if (e != hipSuccess) return fail(LP_EDEVICE, "%s: %s", who, hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(LP_EDEVICE, "%s: %s", who, hipGetErrorString(e2));
  if (stalls) return lp::split_stall_error(who, stalls);
  return LP_OK;
}
}  // namespace

extern "C" lp_status lp_bootstrap_batch(const lp_device_key* dk, lp_gate gate, const uint32_t* d_in0,
                                        const uint32_t* d_in1, const uint32_t* d_in2, size_t cnt, uint32_t* d_out,
                                        void* stream) {
  return bootstrap_batch("lp_bootstrap_batch", dk, gate, d_in0, d_in1, d_in2, cnt, d_out, true, stream);
}

extern "C" lp_status lp_bootstrap_batch_noks(const lp_device_key* dk, lp_gate gate, const uint32_t* d_in0,
                                             const uint32_t* d_in1, const uint32_t* d_in2, size_t cnt,
                                             uint32_t* d_out_big, void* stream) {
  return bootstrap_batch("lp_bootstrap_batch_noks", dk, gate, d_in0, d_in1, d_in2, cnt, d_out_big, false, stream);
}

extern "C" lp_status lp_bootstrap_batch_noalloc(const lp_device_key* dk, lp_gate gate, const uint32_t* d_in0,
                                                const uint32_t* d_in1, const uint32_t* d_in2, size_t cnt,
                                                uint32_t* d_out, void* stream) {
  if (!dk) return fail(LP_EINVAL, "lp_bootstrap_batch_noalloc: null key");
  if (cnt > (size_t)lp::kNoAllocMaxGates)
    return fail(LP_EINVAL, "lp_bootstrap_batch_noalloc: %zu gates exceed the static scratch's maximum of %d per call",
                cnt, lp::kNoAllocMaxGates);
  ScopedDevice sd(dk->device);
  lp::NoAllocScratch pre;
  const hipError_t e = lp::noalloc_scratch(&pre);
  if (e != hipSuccess)
    return fail(LP_EDEVICE, "lp_bootstrap_batch_noalloc: static scratch lookup failed (%s)", hipGetErrorString(e));
  return bootstrap_batch("lp_bootstrap_batch_noalloc", dk, gate, d_in0, d_in1, d_in2, cnt, d_out, true, stream, &pre);
}

extern "C" lp_status lp_preprocess(const lp_device_key* dk, const uint32_t* d_zero, const uint8_t* d_bits, size_t cnt,
                                   uint32_t* d_out, void* stream) {
  if (!dk) return fail(LP_EINVAL, "lp_preprocess: null key");
  if (cnt == 0) return LP_OK;
  if (!d_zero || !d_bits || !d_out) return fail(LP_EINVAL, "lp_preprocess: null buffer");
  ScopedDevice sd(dk->device);
  LP_HIP_TRY(lp::launch_preprocess(d_zero, d_bits, d_out, cnt, (int)dk->P.n, as_stream(stream)));
  return LP_OK;
}

extern "C" lp_status lp_keyswitch_batch(const lp_device_key* dk, const uint32_t* d_in, size_t cnt, uint32_t* d_out,
                                        void* stream) {
  if (!dk) return fail(LP_EINVAL, "lp_keyswitch_batch: null key");
  if (cnt == 0) return LP_OK;
  if (!d_in || !d_out) return fail(LP_EINVAL, "lp_keyswitch_batch: null buffer");
  if (cnt > (size_t)lp::REF_INDEX_MASK) return fail(LP_EINVAL, "lp_keyswitch_batch: batch too large");
  ScopedDevice sd(dk->device);
  hipStream_t s = as_stream(stream);
  std::vector<KsJob> jobs(cnt);
  for (size_t k = 0; k < cnt; ++k) jobs[k] = KsJob{(uint32_t)k, lp::REF_NONE, 0u, lp::make_ref(0, (uint32_t)k), 0u, {0, 0, 0}};
  KsJob* dj = nullptr;
  LP_HIP_TRY(hipMallocAsync((void**)&dj, cnt * sizeof(KsJob), s));
  hipError_t e = hipMemcpyAsync(dj, jobs.data(), cnt * sizeof(KsJob), hipMemcpyHostToDevice, s);
  lp::DstBases dst{};
  dst.p[0] = d_out;
  if (e == hipSuccess) {
    const int tile = pick_ks_tile(cnt);
    e = lp::launch_keyswitch(dj, (int)cnt, d_in, dst, dk->ksk_tab, nullptr, (int)dk->P.n, (int)dk->P.N, (int)dk->P.ks_t,
                             (int)dk->P.ks_base_bit, tile, pick_ks_split(cnt, tile, dk->P.n), s);
  }
  // the host staging vector must outlive the copy
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipError_t e2 = hipFreeAsync(dj, s);
  if (e != hipSuccess) return fail(LP_EDEVICE, "lp_keyswitch_batch: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(LP_EDEVICE, "lp_keyswitch_batch: %s", hipGetErrorString(e2));
  return LP_OK;
}

// ---------------------------------------------------------------- diagnostics
extern "C" lp_status lp_debug_negacyclic_mul(const int32_t* d_digits, const uint32_t* d_poly, size_t cnt,
                                             uint32_t* d_out, void* stream) {
  if (cnt == 0) return LP_OK;
  if (!d_digits || !d_poly || !d_out) return fail(LP_EINVAL, "lp_debug_negacyclic_mul: null buffer");
  if (cnt > (1u << 20)) return fail(LP_EINVAL, "lp_debug_negacyclic_mul: too many products");
  hipStream_t s = as_stream(stream);
  lp::Twiddles tw;
  lp_status st = device_twiddles(&tw);
  if (st != LP_OK) return st;
  uint64_t* tmp = nullptr;
  LP_HIP_TRY(hipMallocAsync((void**)&tmp, cnt * 1024 * 8, s));
  hipError_t e = lp::launch_bsk_to_ntt(d_poly, tmp, (int)cnt, tw, s);
  if (e == hipSuccess) e = lp::launch_debug_polymul(d_digits, tmp, d_out, (int)cnt, tw, s);
  hipError_t e2 = hipFreeAsync(tmp, s);
  if (e != hipSuccess || e2 != hipSuccess) return fail(LP_EDEVICE, "lp_debug_negacyclic_mul: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  return LP_OK;
}

extern "C" lp_status lp_debug_external_product_mfma(const uint32_t* d_key_step, const uint32_t* d_in, size_t cnt,
                                                    uint32_t* d_out, void* stream) {
  if (cnt == 0) return LP_OK;
  if (!d_key_step || !d_in || !d_out) return fail(LP_EINVAL, "lp_debug_external_product_mfma: null buffer");
  if (cnt > 65536) return fail(LP_EINVAL, "lp_debug_external_product_mfma: at most 65536 inputs");
  hipStream_t s = as_stream(stream);
  void* scratch = nullptr;
  LP_HIP_TRY(hipMallocAsync(&scratch, lp::xp_mfma_scratch_bytes((int)cnt), s));
  hipError_t e = lp::launch_extprod_mfma(d_key_step, d_in, (int)cnt, d_out, scratch, s);
  const hipError_t e2 = hipFreeAsync(scratch, s);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return fail(LP_EDEVICE, "lp_debug_external_product_mfma: %s", hipGetErrorString(e));
  return LP_OK;
}

extern "C" lp_status lp_debug_field_op_rates(double target_ms, double* rates, double* ms, void* stream) {
  if (!rates) return fail(LP_EINVAL, "lp_debug_field_op_rates: null rates");
  if (!(target_ms > 0.0) || target_ms > 1000.0) return fail(LP_EINVAL, "lp_debug_field_op_rates: target_ms outside (0, 1000]");
  const hipError_t e = lp::launch_op_rates(target_ms, rates, ms, as_stream(stream));
  if (e != hipSuccess) return fail(LP_EDEVICE, "lp_debug_field_op_rates: %s", hipGetErrorString(e));
  return LP_OK;
}

extern "C" lp_status lp_debug_split_profile(const lp_device_key* dk, const uint32_t* d_in, size_t cnt, int waves,
                                           double* cycles, double* ms, void* stream) {
  if (!dk || !d_in || !cycles) return fail(LP_EINVAL, "lp_debug_split_profile: null argument");
  if (!lp::is_split(waves)) return fail(LP_EINVAL, "lp_debug_split_profile: waves must be 6 or 7");
  if (cnt == 0 || cnt > (size_t)lp::split_max_jobs(waves))
    return fail(LP_EINVAL, "lp_debug_split_profile: 1..%d rotations", lp::split_max_jobs(waves));
  ScopedDevice sd(dk->device);
  hipStream_t s = as_stream(stream);
  const int N = (int)dk->P.N, wpw = 4;
  const int grid = 16 * (((int)cnt + 7) / 8);
  const size_t pwords = (size_t)grid * wpw * lp::kSplitPhaseWords;
  std::vector<BrJob> jobs(cnt);
  for (size_t k = 0; k < cnt; ++k)
    jobs[k] = BrJob{lp::make_ref(0, (uint32_t)k), lp::REF_NONE, 1, 0, 0u, (uint32_t)k, 0u, 0u};
  BrJob* dj = nullptr;
  uint32_t* dacc = nullptr;
  uint64_t* dprof = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  LP_HIP_TRY(hipMallocAsync((void**)&dj, cnt * sizeof(BrJob), s));
  hipError_t e = hipMallocAsync((void**)&dacc, cnt * 2 * N * 4, s);
  if (e == hipSuccess) e = hipMallocAsync((void**)&dprof, pwords * 8, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dj, jobs.data(), cnt * sizeof(BrJob), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = lp::launch_clear_words(reinterpret_cast<uint32_t*>(dprof), pwords * 2, s);
  lp::SplitArea split;
  if (e == hipSuccess) e = lp::split_area_alloc_async(&split, (int)cnt, s);
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  lp::SrcBases src{};
  src.p[0] = d_in;
  if (e == hipSuccess) e = hipEventRecord(t0, s);
  if (e == hipSuccess)
    e = lp::launch_split_profiled(dj, (int)cnt, src, dacc, dk->bsk_tab, (int)dk->P.n, (int)dk->P.n, dk->tw, waves,
                                  &split, dprof, s);
  if (e == hipSuccess) e = hipEventRecord(t1, s);
  std::vector<uint64_t> prof(pwords);
  if (e == hipSuccess) e = hipMemcpyAsync(prof.data(), dprof, pwords * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  float f = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, t0, t1);
  uint32_t stalls = 0;
  if (e == hipSuccess) e = lp::split_area_take_stalls(&split, s, &stalls, nullptr);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  (void)lp::split_area_free_async(&split, s);
  (void)hipFreeAsync(dprof, s);
  (void)hipFreeAsync(dacc, s);
  (void)hipFreeAsync(dj, s);
  if (e != hipSuccess) return fail(LP_EDEVICE, "lp_debug_split_profile: %s", hipGetErrorString(e));
  if (stalls) return lp::split_stall_error("lp_debug_split_profile", stalls);
  constexpr int P = lp::kSplitPhaseWords - 1;
  for (int w = 0; w < wpw; ++w) {
    double steps = 0.0, sum[P] = {};
    for (int b = 0; b < grid; ++b) {
      const uint64_t* r = prof.data() + ((size_t)b * wpw + w) * lp::kSplitPhaseWords;
      steps += (double)r[P];
      for (int k = 0; k < P; ++k) sum[k] += (double)r[k];
    }
    for (int k = 0; k < P; ++k) cycles[w * P + k] = steps > 0 ? sum[k] / steps : 0.0;
  }
  if (ms) *ms = f;
  return LP_OK;
}

extern "C" lp_status lp_debug_blind_rotate(const lp_device_key* dk, const uint32_t* d_in, size_t cnt, uint32_t steps,
                                           uint32_t* d_acc, void* stream) {
  if (!dk) return fail(LP_EINVAL, "lp_debug_blind_rotate: null key");
  if (cnt == 0) return LP_OK;
  if (!d_in || !d_acc) return fail(LP_EINVAL, "lp_debug_blind_rotate: null buffer");
  if (cnt > (size_t)lp::REF_INDEX_MASK) return fail(LP_EINVAL, "lp_debug_blind_rotate: batch too large");
  ScopedDevice sd(dk->device);
  hipStream_t s = as_stream(stream);
  std::vector<BrJob> jobs(cnt);
  for (size_t k = 0; k < cnt; ++k)
    jobs[k] = BrJob{lp::make_ref(0, (uint32_t)k), lp::REF_NONE, 1, 0, 0u, (uint32_t)k, 0u, 0u};
  BrJob* dj = nullptr;
  LP_HIP_TRY(hipMallocAsync((void**)&dj, cnt * sizeof(BrJob), s));
  hipError_t e = hipMemcpyAsync(dj, jobs.data(), cnt * sizeof(BrJob), hipMemcpyHostToDevice, s);
  lp::SrcBases src{};
  src.p[0] = d_in;
  const int st = (int)std::min<uint32_t>(steps, dk->P.n);
  const int waves = pick_br_wpb(cnt);
  lp::SplitArea split;
  if (e == hipSuccess && lp::is_split(waves)) e = lp::split_area_alloc_async(&split, (int)cnt, s);
  if (e == hipSuccess)
    e = lp::launch_blind_rotate(dj, (int)cnt, src, d_acc, dk->bsk_tab, nullptr, (int)dk->P.n, st, 1, dk->tw, waves, s,
                                &split);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  uint32_t stalls = 0;
  if (e == hipSuccess && lp::is_split(waves)) e = lp::split_area_take_stalls(&split, s, &stalls, nullptr);
  hipError_t e2 = hipFreeAsync(dj, s);
  const hipError_t e3 = lp::split_area_free_async(&split, s);
  if (e2 == hipSuccess) e2 = e3;
  if (e != hipSuccess || e2 != hipSuccess) return fail(LP_EDEVICE, "lp_debug_blind_rotate: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  if (stalls) return lp::split_stall_error("lp_debug_blind_rotate", stalls);
  return LP_OK;
}

// ---------------------------------------------------------------- free
extern "C" void lp_secret_key_free(lp_secret_key* sk) { delete sk; }
extern "C" void lp_cloud_key_free(lp_cloud_key* ck) { delete ck; }
extern "C" void lp_device_key_free(lp_device_key* dk) {
  if (!dk) return;
  ScopedDevice sd(dk->device);
  lp::sched_forget_key(dk);
  if (dk->bsk_ntt) (void)hipFree(dk->bsk_ntt);
  if (dk->ksk) (void)hipFree(dk->ksk);
  if (dk->bsk_tab) (void)hipFree(dk->bsk_tab);
  if (dk->ksk_tab) (void)hipFree(dk->ksk_tab);
  delete dk;
}
