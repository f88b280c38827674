/*
 * CPU oracle for the LocPIR gate-bootstrapping path -- TEST INFRASTRUCTURE.
 * See locpir_oracle.h for scope.  Plain C, written for readability: every
 * function follows one passage of the paper or one step of the TFHE gate
 * bootstrap in the order the construction defines it.
 */
#include "locpir_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ======================================================================
 * Counter-based random numbers.
 * SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): a generator with state s
 * returns, for its k-th output (k = 0, 1, ...), mix(s + (k+1)*GAMMA).
 * Stream key:  key(seed, stream) = output number `stream` of SplitMix64(seed)
 * Draw:        u64(seed, stream, idx) = output number `idx` of SplitMix64(key)
 * ==================================================================== */
static const uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ull;

static uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t orc_rand_u64(uint64_t seed, uint64_t stream, uint64_t idx) {
  uint64_t key = sm_mix(seed + (stream + 1) * SM_GAMMA);
  return sm_mix(key + (idx + 1) * SM_GAMMA);
}

/* Gaussian noise in Torus32 units: Box-Muller (cosine branch) from two
 * uniform draws, scaled by sigma*2^32 and rounded half away from zero. */
int32_t orc_gauss_torus(uint64_t seed, uint64_t stream, uint64_t idx, double sigma) {
  uint64_t x1 = orc_rand_u64(seed, stream, 2 * idx);
  uint64_t x2 = orc_rand_u64(seed, stream, 2 * idx + 1);
  double u1 = (double)((x1 >> 11) + 1) * 0x1p-53; /* (0, 1] */
  double u2 = (double)(x2 >> 11) * 0x1p-53;       /* [0, 1) */
  double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  double e = z * (sigma * 4294967296.0);
  return (int32_t)(uint32_t)(uint64_t)llround(e);
}

/* stream numbers */
enum { ST_SK_LWE = 0, ST_SK_RING = 1, ST_BSK_A = 2, ST_BSK_E = 3, ST_KSK_A = 4,
       ST_KSK_E = 5, ST_ENC_A = 6, ST_ENC_E = 7, ST_ZERO_A = 8, ST_ZERO_E = 9 };

static uint32_t rand_u32(uint64_t seed, uint64_t stream, uint64_t idx) {
  return (uint32_t)(orc_rand_u64(seed, stream, idx) >> 32);
}

/* ======================================================================
 * The oracle's NTT: a prime q = 1 (mod 4096) just below 2^62, found at start
 * by Miller-Rabin; negacyclic product by the convolution theorem with the
 * twist a_j -> psi^j a_j (psi a primitive 2N-th root of unity), a textbook
 * iterative radix-2 cyclic transform with omega = psi^2, and the untwist.
 * Multiplication mod q uses Montgomery's REDC with R = 2^64.
 * ==================================================================== */
static uint64_t Q, QNEG_INV, R2_MOD_Q;

static uint64_t mulmod_slow(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)(((u128)a * b) % m); }

static uint64_t powmod_slow(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = mulmod_slow(r, b, m);
    b = mulmod_slow(b, b, m);
    e >>= 1;
  }
  return r;
}

/* deterministic Miller-Rabin for n < 3.3e24 with the first 12 primes */
static int is_prime_u64(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; i++) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; s++; }
  for (int i = 0; i < 12; i++) {
    uint64_t x = powmod_slow(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int comp = 1;
    for (int r = 1; r < s; r++) {
      x = mulmod_slow(x, x, n);
      if (x == n - 1) { comp = 0; break; }
    }
    if (comp) return 0;
  }
  return 1;
}

static inline uint64_t redc(u128 t) {
  uint64_t m = (uint64_t)t * QNEG_INV;
  u128 u = (t + (u128)m * Q) >> 64; /* t < q^2 < 2^124, m*q < 2^126 */
  uint64_t r = (uint64_t)u;
  return r >= Q ? r - Q : r;
}
static inline uint64_t mont_mul(uint64_t a, uint64_t b) { return redc((u128)a * b); }
static inline uint64_t to_mont(uint64_t a) { return mont_mul(a % Q, R2_MOD_Q); }
static inline uint64_t addq(uint64_t a, uint64_t b) { uint64_t s = a + b; return s >= Q ? s - Q : s; }
static inline uint64_t subq(uint64_t a, uint64_t b) { return a >= b ? a - b : a + Q - b; }

#define MAX_LOGN 11 /* N up to 2048 */
typedef struct {
  uint64_t psi_pow[2048];     /* psi^j * R        (twist)                 */
  uint64_t psi_inv_pow[2048]; /* psi^-j * N^-1 * R (untwist and scaling)   */
  uint64_t w_pow[1024];       /* omega^k * R, k < N/2                     */
  uint64_t w_inv_pow[1024];   /* omega^-k * R                             */
} ntt_tables;
static ntt_tables* TABLES[MAX_LOGN + 1];
static pthread_once_t INIT_ONCE = PTHREAD_ONCE_INIT;

static void init_field(void) {
  /* largest q < 2^62 with q = 1 mod 4096 */
  uint64_t q = ((1ull << 62) / 4096) * 4096 + 1;
  while (q >= (1ull << 62)) q -= 4096;
  while (!is_prime_u64(q)) q -= 4096;
  Q = q;
  uint64_t inv = q; /* Newton iteration for q^-1 mod 2^64 */
  for (int i = 0; i < 6; i++) inv *= 2 - q * inv;
  QNEG_INV = (uint64_t)0 - inv;
  uint64_t r1 = (uint64_t)(((u128)1 << 64) % q);
  R2_MOD_Q = mulmod_slow(r1, r1, q);
  for (int logn = 1; logn <= MAX_LOGN; logn++) {
    uint32_t N = 1u << logn;
    ntt_tables* T = (ntt_tables*)calloc(1, sizeof(ntt_tables));
    /* primitive 2N-th root of unity: psi = g^((q-1)/2N) with psi^N = -1 */
    uint64_t psi = 0;
    for (uint64_t g = 2; g < 1000; g++) {
      uint64_t c = powmod_slow(g, (q - 1) / (2 * N), q);
      if (powmod_slow(c, N, q) == q - 1) { psi = c; break; }
    }
    uint64_t psi_inv = powmod_slow(psi, 2 * N - 1, q);
    uint64_t n_inv = powmod_slow(N, q - 2, q);
    uint64_t omega = mulmod_slow(psi, psi, q), omega_inv = mulmod_slow(psi_inv, psi_inv, q);
    uint64_t a = 1, b = n_inv;
    for (uint32_t j = 0; j < N; j++) {
      T->psi_pow[j] = to_mont(a);
      T->psi_inv_pow[j] = to_mont(b);
      a = mulmod_slow(a, psi, q);
      b = mulmod_slow(b, psi_inv, q);
    }
    a = 1; b = 1;
    for (uint32_t k = 0; k < N / 2; k++) {
      T->w_pow[k] = to_mont(a);
      T->w_inv_pow[k] = to_mont(b);
      a = mulmod_slow(a, omega, q);
      b = mulmod_slow(b, omega_inv, q);
    }
    TABLES[logn] = T;
  }
}
static void ensure_init(void) { pthread_once(&INIT_ONCE, init_field); }

static int log2_u32(uint32_t N) {
  int k = 0;
  while ((1u << k) < N) k++;
  return ((1u << k) == N) ? k : -1;
}

uint64_t orc_ntt_prime(void) { ensure_init(); return Q; }
uint64_t orc_mulmod(uint64_t a, uint64_t b) {
  ensure_init();
  return mont_mul(mont_mul(a % Q, b % Q), R2_MOD_Q);
}

/* cyclic radix-2 decimation-in-time transform, twiddles w[k] (Montgomery) */
static void ntt_cyclic(uint64_t* a, uint32_t N, const uint64_t* w) {
  for (uint32_t i = 1, j = 0; i < N; i++) { /* bit-reversal permutation */
    uint32_t bit = N >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; }
  }
  for (uint32_t len = 2; len <= N; len <<= 1) {
    uint32_t half = len >> 1, step = N / len;
    for (uint32_t i = 0; i < N; i += len)
      for (uint32_t j = 0; j < half; j++) {
        uint64_t u = a[i + j];
        uint64_t v = mont_mul(a[i + j + half], w[j * step]);
        a[i + j] = addq(u, v);
        a[i + j + half] = subq(u, v);
      }
  }
}

/* forward negacyclic transform of an integer polynomial (values reduced mod q) */
static void ntt_neg_forward(uint32_t N, const ntt_tables* T, const int64_t* in, uint64_t* out) {
  for (uint32_t j = 0; j < N; j++) {
    int64_t v = in[j] % (int64_t)Q;
    uint64_t r = v < 0 ? (uint64_t)(v + (int64_t)Q) : (uint64_t)v;
    out[j] = mont_mul(r, T->psi_pow[j]);
  }
  ntt_cyclic(out, N, T->w_pow);
}

/* inverse transform and centred lift to the exact integers (|x| < q/2) */
static void ntt_neg_inverse(uint32_t N, const ntt_tables* T, uint64_t* a, int64_t* out) {
  ntt_cyclic(a, N, T->w_inv_pow);
  for (uint32_t j = 0; j < N; j++) {
    uint64_t r = mont_mul(a[j], T->psi_inv_pow[j]);
    out[j] = r > Q / 2 ? (int64_t)r - (int64_t)Q : (int64_t)r;
  }
}

int orc_negacyclic_mul_ntt(uint32_t N, const int64_t* a, const int64_t* b, int64_t* out) {
  ensure_init();
  int logn = log2_u32(N);
  if (logn < 1 || logn > MAX_LOGN) return -1;
  const ntt_tables* T = TABLES[logn];
  uint64_t* A = (uint64_t*)malloc(sizeof(uint64_t) * N);
  uint64_t* B = (uint64_t*)malloc(sizeof(uint64_t) * N);
  ntt_neg_forward(N, T, a, A);
  ntt_neg_forward(N, T, b, B);
  for (uint32_t j = 0; j < N; j++) A[j] = mont_mul(mont_mul(A[j], B[j]), R2_MOD_Q);
  ntt_neg_inverse(N, T, A, out);
  free(A);
  free(B);
  return 0;
}

void orc_negacyclic_mul_schoolbook(uint32_t N, const int64_t* a, const int64_t* b, int64_t* out) {
  /* c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j   (X^N = -1) */
  for (uint32_t k = 0; k < N; k++) out[k] = 0;
  for (uint32_t i = 0; i < N; i++)
    for (uint32_t j = 0; j < N; j++) {
      int64_t p = a[i] * b[j];
      if (i + j < N) out[i + j] += p;
      else out[i + j - N] -= p;
    }
}

/* ======================================================================
 * Torus32 polynomials.
 * ==================================================================== */
/* out = X^k * in in T[X]/(X^N+1), 0 <= k < 2N */
void orc_poly_rotate(uint32_t N, const uint32_t* in, uint32_t k, uint32_t* out) {
  k %= 2 * N;
  for (uint32_t j = 0; j < N; j++) {
    /* coefficient j of X^k * in comes from index j-k, with a sign flip for
     * every wrap past X^N */
    int64_t src = (int64_t)j - (int64_t)k;
    int neg = 0;
    while (src < 0) { src += N; neg ^= 1; }
    out[j] = neg ? (uint32_t)0 - in[src] : in[src];
  }
}

/* B = A * S with S binary, negacyclic, mod 2^32 (schoolbook over the set bits) */
static void poly_mul_binary(uint32_t N, const uint32_t* A, const uint8_t* S, uint32_t* B) {
  for (uint32_t j = 0; j < N; j++) B[j] = 0;
  for (uint32_t t = 0; t < N; t++) {
    if (!S[t]) continue;
    for (uint32_t j = 0; j < N; j++) {
      if (j >= t) B[j] += A[j - t];
      else B[j] -= A[j + N - t];
    }
  }
}

/* ======================================================================
 * KeyGen, Encrypt, Decrypt (Sec. 2.2).
 * ==================================================================== */
size_t orc_bsk_words(const orc_params* P) { return (size_t)P->n * (2 * P->l) * 2 * P->N; }
size_t orc_ksk_words(const orc_params* P) {
  return (size_t)P->N * P->ks_t * ((1u << P->ks_base_bit) - 1) * (P->n + 1);
}

/* phase of an LWE sample: b - <a, key> */
uint32_t orc_phase(uint32_t dim, const uint8_t* key, const uint32_t* ct) {
  uint32_t dot = 0;
  for (uint32_t i = 0; i < dim; i++) dot += ct[i] * (uint32_t)key[i];
  return ct[dim] - dot;
}

/* LWE encryption of torus value mu: a uniform, b = <a,s> + mu + e */
static void lwe_encrypt(uint32_t n, const uint8_t* s, uint32_t mu, uint64_t seed,
                        uint64_t st_a, uint64_t st_e, uint64_t idx, double sigma, uint32_t* out) {
  uint32_t dot = 0;
  for (uint32_t c = 0; c < n; c++) {
    out[c] = rand_u32(seed, st_a, idx * n + c);
    dot += out[c] * (uint32_t)s[c];
  }
  out[n] = dot + mu + (uint32_t)orc_gauss_torus(seed, st_e, idx, sigma);
}

void orc_keygen(const orc_params* P, uint64_t seed, uint8_t* s_lwe, uint8_t* s_ring,
                uint32_t* bsk, uint32_t* ksk) {
  const uint32_t n = P->n, N = P->N, l = P->l, R = 2 * l;
  for (uint32_t i = 0; i < n; i++) s_lwe[i] = (uint8_t)(orc_rand_u64(seed, ST_SK_LWE, i) >> 63);
  for (uint32_t i = 0; i < N; i++) s_ring[i] = (uint8_t)(orc_rand_u64(seed, ST_SK_RING, i) >> 63);

  /* BSK_i: TGSW encryption of s_i = 2l TRLWE rows; row r = (p, j) is a fresh
   * TRLWE_S(0) plus s_i / Bg^(j+1) on the constant coefficient of component
   * p (p = 0 mask polynomial, p = 1 body polynomial). */
  for (uint32_t i = 0; i < n; i++)
    for (uint32_t r = 0; r < R; r++) {
      uint64_t row = (uint64_t)i * R + r;
      uint32_t* A = bsk + (row * 2 + 0) * N;
      uint32_t* B = bsk + (row * 2 + 1) * N;
      for (uint32_t c = 0; c < N; c++) A[c] = rand_u32(seed, ST_BSK_A, row * N + c);
      poly_mul_binary(N, A, s_ring, B);
      for (uint32_t c = 0; c < N; c++)
        B[c] += (uint32_t)orc_gauss_torus(seed, ST_BSK_E, row * N + c, P->bk_sigma);
      uint32_t p = r / l, j = r % l;
      if (s_lwe[i]) (p == 0 ? A : B)[0] += 1u << (32 - P->bg_bit * (j + 1));
    }

  /* KSK[i][j][v]: LWE_s encryption of v * S_i / base^(j+1), v = 1..base-1 */
  const uint32_t base = 1u << P->ks_base_bit;
  for (uint32_t i = 0; i < N; i++)
    for (uint32_t j = 0; j < P->ks_t; j++)
      for (uint32_t v = 1; v < base; v++) {
        uint64_t row = ((uint64_t)i * P->ks_t + j) * (base - 1) + (v - 1);
        uint32_t msg = v * (uint32_t)s_ring[i] * (1u << (32 - P->ks_base_bit * (j + 1)));
        lwe_encrypt(n, s_lwe, msg, seed, ST_KSK_A, ST_KSK_E, row, P->lwe_sigma,
                    ksk + row * (n + 1));
      }
}

/* Encrypt(m): mu = f(m) = m/4 - 1/8, i.e. +2^29 for 1 and -2^29 for 0 */
void orc_encrypt_bits(const orc_params* P, const uint8_t* s_lwe, const uint8_t* bits,
                      size_t cnt, uint64_t seed, uint64_t first_index, uint32_t* ct) {
  for (size_t k = 0; k < cnt; k++) {
    uint32_t mu = bits[k] ? 0x20000000u : 0xE0000000u;
    lwe_encrypt(P->n, s_lwe, mu, seed, ST_ENC_A, ST_ENC_E, first_index + k, P->lwe_sigma,
                ct + k * (P->n + 1));
  }
}

/* The client's fresh samples of Sec. 3: LWE encryptions of the torus value
 * 0, which the cloud later turns into payload ciphertexts (Algorithm 1). */
void orc_encrypt_zeros(const orc_params* P, const uint8_t* s_lwe, size_t cnt, uint64_t seed,
                       uint64_t first_index, uint32_t* ct) {
  for (size_t k = 0; k < cnt; k++)
    lwe_encrypt(P->n, s_lwe, 0u, seed, ST_ZERO_A, ST_ZERO_E, first_index + k, P->lwe_sigma,
                ct + k * (P->n + 1));
}

/* Decrypt: the phase rounded to the nearer of -1/8, +1/8, i.e. its sign */
void orc_decrypt_bits(const orc_params* P, const uint8_t* s_lwe, const uint32_t* ct,
                      size_t cnt, uint8_t* bits, int32_t* phase) {
  for (size_t k = 0; k < cnt; k++) {
    uint32_t ph = orc_phase(P->n, s_lwe, ct + k * (P->n + 1));
    bits[k] = (int32_t)ph > 0 ? 1 : 0;
    if (phase) phase[k] = (int32_t)ph;
  }
}

/* ======================================================================
 * Gate bootstrapping.
 * ==================================================================== */
/* round(x * 2N / 2^32) mod 2N */
uint32_t orc_modswitch(uint32_t x, uint32_t N) {
  int shift = 32 - (log2_u32(N) + 1);
  return ((x + (1u << (shift - 1))) >> shift) & (2 * N - 1);
}

/* signed gadget digits d_1..d_l in [-Bg/2, Bg/2): a ~ sum_j d_j * 2^(32 - bg_bit*j) */
void orc_decompose(const orc_params* P, uint32_t a, int32_t* digits) {
  const uint32_t Bg = 1u << P->bg_bit, half = Bg / 2;
  uint32_t offset = 1u << (32 - P->bg_bit * P->l - 1); /* rounding of the dropped bits */
  for (uint32_t j = 1; j <= P->l; j++) offset += half * (1u << (32 - P->bg_bit * j));
  uint32_t t = a + offset;
  for (uint32_t j = 1; j <= P->l; j++)
    digits[j - 1] = (int32_t)((t >> (32 - P->bg_bit * j)) & (Bg - 1)) - (int32_t)half;
}

struct orc_ctx {
  orc_params P;
  const uint32_t* bsk;
  const uint32_t* ksk;
  const ntt_tables* T;
  uint64_t* bsk_hat; /* [n][2l][2][N], transform domain, Montgomery form */
};

orc_ctx* orc_ctx_create(const orc_params* P, const uint32_t* bsk, const uint32_t* ksk) {
  ensure_init();
  int logn = log2_u32(P->N);
  if (logn < 1 || logn > MAX_LOGN) return NULL;
  orc_ctx* C = (orc_ctx*)calloc(1, sizeof(orc_ctx));
  C->P = *P;
  C->bsk = bsk;
  C->ksk = ksk;
  C->T = TABLES[logn];
  const size_t polys = (size_t)P->n * 2 * P->l * 2;
  C->bsk_hat = (uint64_t*)malloc(sizeof(uint64_t) * polys * P->N);
  #pragma omp parallel
  {
    int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * P->N);
    #pragma omp for schedule(static)
    for (long long k = 0; k < (long long)polys; k++) {
      for (uint32_t c = 0; c < P->N; c++) tmp[c] = (int64_t)bsk[k * P->N + c]; /* 0..2^32-1 */
      uint64_t* dst = C->bsk_hat + k * P->N;
      ntt_neg_forward(P->N, C->T, tmp, dst);
      for (uint32_t c = 0; c < P->N; c++) dst[c] = mont_mul(dst[c], R2_MOD_Q); /* -> Montgomery */
    }
    free(tmp);
  }
  return C;
}

void orc_ctx_free(orc_ctx* C) {
  if (!C) return;
  free(C->bsk_hat);
  free(C);
}

/* ExtProd(BSK_i, D) = sum_{p,j} dec_j(D_p) (*) BSK_i[p,j] as exact integer
 * polynomials, reduced mod 2^32 at the end.  The sum is formed in the
 * transform domain: with |digit| <= Bg/2 and coefficients < 2^32 every
 * output coefficient is below 2l*N*(Bg/2)*2^32 (2^50.6 here) < q/2, so the
 * centred lift is the exact integer. */
void orc_external_product(const orc_ctx* C, uint32_t i, const uint32_t* d_in, uint32_t* acc_out) {
  const orc_params* P = &C->P;
  const uint32_t N = P->N, l = P->l;
  int64_t* dig = (int64_t*)malloc(sizeof(int64_t) * N * l);
  uint64_t* dhat = (uint64_t*)malloc(sizeof(uint64_t) * N);
  uint64_t* sum = (uint64_t*)calloc(2 * N, sizeof(uint64_t));
  int64_t* res = (int64_t*)malloc(sizeof(int64_t) * N);
  int32_t dg[16];
  for (uint32_t p = 0; p < 2; p++) {
    for (uint32_t c = 0; c < N; c++) {
      orc_decompose(P, d_in[p * N + c], dg);
      for (uint32_t j = 0; j < l; j++) dig[j * N + c] = dg[j];
    }
    for (uint32_t j = 0; j < l; j++) {
      ntt_neg_forward(N, C->T, dig + j * N, dhat);
      uint32_t r = p * l + j;
      for (uint32_t q = 0; q < 2; q++) {
        const uint64_t* bh = C->bsk_hat + ((((size_t)i * 2 * l + r) * 2 + q) * N);
        for (uint32_t c = 0; c < N; c++) sum[q * N + c] = addq(sum[q * N + c], mont_mul(dhat[c], bh[c]));
      }
    }
  }
  for (uint32_t q = 0; q < 2; q++) {
    ntt_neg_inverse(N, C->T, sum + q * N, res);
    for (uint32_t c = 0; c < N; c++) acc_out[q * N + c] = (uint32_t)(uint64_t)res[c];
  }
  free(dig); free(dhat); free(sum); free(res);
}

/* BlindRotate: ACC = (0, X^{-b~} v) with test vector v = sum_j (1/8) X^j;
 * then for each i: ACC <- ACC + ExtProd(BSK_i, X^{a~_i} ACC - ACC) (CMux). */
void orc_blind_rotate(const orc_ctx* C, const uint32_t* ct, uint32_t steps, uint32_t* acc) {
  const orc_params* P = &C->P;
  const uint32_t N = P->N, n = P->n;
  uint32_t* v = (uint32_t*)malloc(sizeof(uint32_t) * N);
  uint32_t* rot = (uint32_t*)malloc(sizeof(uint32_t) * 2 * N);
  uint32_t* ext = (uint32_t*)malloc(sizeof(uint32_t) * 2 * N);
  for (uint32_t j = 0; j < N; j++) v[j] = 0x20000000u;
  uint32_t bbar = orc_modswitch(ct[n], N);
  for (uint32_t j = 0; j < N; j++) acc[j] = 0;
  orc_poly_rotate(N, v, (2 * N - bbar) % (2 * N), acc + N);
  if (steps > n) steps = n;
  for (uint32_t i = 0; i < steps; i++) {
    uint32_t abar = orc_modswitch(ct[i], N);
    for (uint32_t p = 0; p < 2; p++) {
      orc_poly_rotate(N, acc + p * N, abar, rot + p * N);
      for (uint32_t j = 0; j < N; j++) rot[p * N + j] -= acc[p * N + j];
    }
    orc_external_product(C, i, rot, ext);
    for (uint32_t j = 0; j < 2 * N; j++) acc[j] += ext[j];
  }
  free(v); free(rot); free(ext);
}

/* SampleExtract at coefficient 0: a'_0 = A_0, a'_j = -A_{N-j}, b' = B_0 */
void orc_sample_extract(uint32_t N, const uint32_t* acc, uint32_t* lwe_big) {
  lwe_big[0] = acc[0];
  for (uint32_t j = 1; j < N; j++) lwe_big[j] = (uint32_t)0 - acc[N - j];
  lwe_big[N] = acc[N];
}

/* KeySwitch from the ring key (dimension N) to s (dimension n): each a'_i is
 * rounded to t base-2^b digits; out = (0, b') - sum_{i,j} KSK[i][j][digit] */
void orc_keyswitch(const orc_ctx* C, const uint32_t* lwe_big, uint32_t* out) {
  const orc_params* P = &C->P;
  const uint32_t n = P->n, N = P->N, bb = P->ks_base_bit, t = P->ks_t;
  const uint32_t base = 1u << bb;
  const uint32_t prec_offset = 1u << (32 - 1 - bb * t);
  for (uint32_t c = 0; c < n; c++) out[c] = 0;
  out[n] = lwe_big[N];
  for (uint32_t i = 0; i < N; i++) {
    uint32_t abar = lwe_big[i] + prec_offset;
    for (uint32_t j = 0; j < t; j++) {
      uint32_t d = (abar >> (32 - (j + 1) * bb)) & (base - 1);
      if (d == 0) continue;
      const uint32_t* row = C->ksk + (((size_t)i * t + j) * (base - 1) + (d - 1)) * (n + 1);
      for (uint32_t c = 0; c <= n; c++) out[c] -= row[c];
    }
  }
}

void orc_bootstrap_raw(const orc_ctx* C, const uint32_t* ct, uint32_t* out_big, uint32_t* out) {
  const uint32_t N = C->P.N;
  uint32_t* acc = (uint32_t*)malloc(sizeof(uint32_t) * 2 * N);
  uint32_t* big = (uint32_t*)malloc(sizeof(uint32_t) * (N + 1));
  orc_blind_rotate(C, ct, C->P.n, acc);
  orc_sample_extract(N, acc, big);
  if (out_big) memcpy(out_big, big, sizeof(uint32_t) * (N + 1));
  if (out) orc_keyswitch(C, big, out);
  free(acc);
  free(big);
}

/* out = (0, cst) + k1*c1 + k2*c2 over LWE samples of dimension dim */
static void lwe_lincomb(uint32_t dim, uint32_t* out, uint32_t cst, const uint32_t* c1, int32_t k1,
                        const uint32_t* c2, int32_t k2) {
  for (uint32_t c = 0; c <= dim; c++) {
    uint32_t v = (c == dim) ? cst : 0;
    if (c1) v += (uint32_t)k1 * c1[c];
    if (c2) v += (uint32_t)k2 * c2[c];
    out[c] = v;
  }
}

#define EIGHTH 0x20000000u /* 1/8 */
#define QUARTER 0x40000000u /* 1/4 */

/* Gates: a linear pre-combination whose phase sign is the gate's truth value,
 * then a gate bootstrap.  HomAND = Bootstrap((0,-1/8) + c1 + c2) as printed
 * in Sec. 2.2; the others are the same construction with other constants. */
int orc_gate_big(const orc_ctx* C, int gate, const uint32_t* c1, const uint32_t* c2,
                 const uint32_t* c3, uint32_t* big) {
  const uint32_t n = C->P.n, N = C->P.N;
  uint32_t* tmp = (uint32_t*)malloc(sizeof(uint32_t) * (n + 1));
  int ok = 1;
  switch (gate) {
    case ORC_NAND: lwe_lincomb(n, tmp, EIGHTH, c1, -1, c2, -1); break;
    case ORC_AND: lwe_lincomb(n, tmp, 0u - EIGHTH, c1, 1, c2, 1); break;
    case ORC_OR: lwe_lincomb(n, tmp, EIGHTH, c1, 1, c2, 1); break;
    case ORC_NOR: lwe_lincomb(n, tmp, 0u - EIGHTH, c1, -1, c2, -1); break;
    case ORC_XOR: lwe_lincomb(n, tmp, QUARTER, c1, 2, c2, 2); break;
    case ORC_XNOR: lwe_lincomb(n, tmp, 0u - QUARTER, c1, -2, c2, -2); break;
    case ORC_MUX: {
      /* u1 = sel AND t, u2 = (NOT sel) AND f, each bootstrapped without key
       * switching; big = (0, 1/8) + u1 + u2 */
      uint32_t* u1 = (uint32_t*)malloc(sizeof(uint32_t) * (N + 1));
      uint32_t* u2 = (uint32_t*)malloc(sizeof(uint32_t) * (N + 1));
      lwe_lincomb(n, tmp, 0u - EIGHTH, c1, 1, c2, 1);
      orc_bootstrap_raw(C, tmp, u1, NULL);
      lwe_lincomb(n, tmp, 0u - EIGHTH, c1, -1, c3, 1);
      orc_bootstrap_raw(C, tmp, u2, NULL);
      lwe_lincomb(N, big, EIGHTH, u1, 1, u2, 1);
      free(u1); free(u2);
      free(tmp);
      return 1;
    }
    default: ok = 0;
  }
  if (ok) orc_bootstrap_raw(C, tmp, big, NULL);
  free(tmp);
  return ok;
}

void orc_gate(const orc_ctx* C, int gate, const uint32_t* c1, const uint32_t* c2,
              const uint32_t* c3, uint32_t* out) {
  const uint32_t n = C->P.n, N = C->P.N;
  if (gate == ORC_NOT) { lwe_lincomb(n, out, 0, c1, -1, NULL, 0); return; }
  if (gate == ORC_COPY) { lwe_lincomb(n, out, 0, c1, 1, NULL, 0); return; }
  uint32_t* big = (uint32_t*)malloc(sizeof(uint32_t) * (N + 1));
  if (orc_gate_big(C, gate, c1, c2, c3, big)) orc_keyswitch(C, big, out);
  else memset(out, 0, sizeof(uint32_t) * (n + 1));
  free(big);
}

int orc_gate_batch(const orc_ctx* C, int gate, size_t cnt, const uint32_t* c1,
                   const uint32_t* c2, const uint32_t* c3, uint32_t* out) {
  const size_t w = C->P.n + 1;
  int threads = 1;
  #pragma omp parallel
  {
    #ifdef _OPENMP
    #pragma omp single
    threads = omp_get_num_threads();
    #endif
    #pragma omp for schedule(dynamic, 1)
    for (long long k = 0; k < (long long)cnt; k++)
      orc_gate(C, gate, c1 + k * w, c2 ? c2 + k * w : NULL, c3 ? c3 + k * w : NULL, out + k * w);
  }
  return threads;
}

int orc_gate_big_batch(const orc_ctx* C, int gate, size_t cnt, const uint32_t* c1,
                       const uint32_t* c2, const uint32_t* c3, uint32_t* big) {
  const size_t w = C->P.n + 1, wb = C->P.N + 1;
  int ok = 1;
  #pragma omp parallel for schedule(dynamic, 1) reduction(&& : ok)
  for (long long k = 0; k < (long long)cnt; k++)
    ok = ok && orc_gate_big(C, gate, c1 + k * w, c2 ? c2 + k * w : NULL, c3 ? c3 + k * w : NULL, big + k * wb);
  return ok;
}

/* ======================================================================
 * The bounding-box circuit, Algorithms 2-5.  A walker either evaluates
 * gates (ctx != NULL) or only counts them and tracks their depth.
 * ==================================================================== */
typedef struct {
  const orc_ctx* C;
  uint32_t w;          /* words per ciphertext */
  uint64_t n_br, n_ks; /* counting mode tallies */
} walker;

typedef struct {
  uint32_t* ct; /* NULL in counting mode */
  uint32_t level;
} wct;

static uint32_t maxu(uint32_t a, uint32_t b) { return a > b ? a : b; }

static void wgate(walker* W, int gate, const wct* a, const wct* b, const wct* c, wct* out) {
  uint32_t lv = a->level;
  if (b) lv = maxu(lv, b->level);
  if (c) lv = maxu(lv, c->level);
  if (gate == ORC_NOT || gate == ORC_COPY) out->level = lv;
  else out->level = lv + 1;
  if (W->C) {
    orc_gate(W->C, gate, a->ct, b ? b->ct : NULL, c ? c->ct : NULL, out->ct);
  } else {
    if (gate == ORC_MUX) { W->n_br += 2; W->n_ks += 1; }
    else if (gate != ORC_NOT && gate != ORC_COPY) { W->n_br += 1; W->n_ks += 1; }
  }
}

static wct wnew(walker* W) {
  wct r;
  r.ct = W->C ? (uint32_t*)calloc(W->w, sizeof(uint32_t)) : NULL;
  r.level = 0;
  return r;
}
static void wfree(wct* r) { free(r->ct); r->ct = NULL; }

/* Algorithm 2, HomCompS: Enc(1) iff c1 < c2.  Bits LSB first.  t0 starts as
 * the noiseless trivial sample of 0, i.e. (0, -1/8).  The MSB flip (its
 * lines 2-3) turns the unsigned ripple comparison into a two's-complement one
 * and is applied only to signed inputs. */
static wct hom_comp_s(walker* W, uint32_t l, int is_signed, const wct* c1, const wct* c2) {
  wct* a = (wct*)malloc(sizeof(wct) * l);
  wct* b = (wct*)malloc(sizeof(wct) * l);
  for (uint32_t i = 0; i < l; i++) {
    a[i] = c1[i];
    b[i] = c2[i];
  }
  wct na = {0}, nb = {0};
  if (is_signed) {
    na = wnew(W); nb = wnew(W);
    wgate(W, ORC_NOT, &c1[l - 1], NULL, NULL, &na);
    wgate(W, ORC_NOT, &c2[l - 1], NULL, NULL, &nb);
    a[l - 1] = na;
    b[l - 1] = nb;
  }
  wct t0 = wnew(W);
  if (t0.ct) t0.ct[W->w - 1] = 0u - EIGHTH;
  wct t1 = wnew(W), nt0 = wnew(W);
  for (uint32_t i = 0; i < l; i++) {
    wgate(W, ORC_XNOR, &a[i], &b[i], NULL, &t1);
    /* t0 <- MUX(t1, t0, c2[i]): keep t0 when the bits agree */
    wgate(W, ORC_MUX, &t1, &t0, &b[i], &nt0);
    wct sw = t0; t0 = nt0; nt0 = sw;
  }
  wfree(&t1); wfree(&nt0);
  if (is_signed) { wfree(&na); wfree(&nb); }
  free(a);
  free(b);
  return t0;
}

static void bbox_walk(walker* W, uint32_t l, uint32_t N, uint32_t m, int is_signed,
                      const uint32_t* x, const uint32_t* y, const uint32_t* bounds,
                      const uint32_t* payload, uint32_t* out, uint32_t* depth) {
  const uint32_t w = W->w;
  wct* X = (wct*)calloc(l, sizeof(wct));
  wct* Y = (wct*)calloc(l, sizeof(wct));
  for (uint32_t i = 0; i < l; i++) {
    X[i].ct = W->C ? (uint32_t*)(x + (size_t)i * w) : NULL;
    Y[i].ct = W->C ? (uint32_t*)(y + (size_t)i * w) : NULL;
  }
  wct* T = (wct*)calloc((size_t)N * m, sizeof(wct)); /* masked services S_i */

  /* Algorithm 3, comparisons: per box x_l = HomCompLE(x1, x) =
   * NOT HomCompS(x, x1), x_r = HomCompS(x, x2), and the same for y.  The 4N
   * comparisons are independent and run in parallel. */
  wct* cmp = (wct*)calloc((size_t)4 * N, sizeof(wct));
  uint64_t br0 = 0, ks0 = 0;
  #pragma omp parallel for schedule(dynamic, 1) if (W->C) reduction(+ : br0, ks0)
  for (long long ci = 0; ci < (long long)4 * N; ci++) {
    walker Wl = {W->C, W->w, 0, 0};
    const long long bi = ci / 4, k = ci % 4;
    wct* Bk = (wct*)calloc(l, sizeof(wct));
    for (uint32_t i = 0; i < l; i++)
      Bk[i].ct = W->C ? (uint32_t*)(bounds + (((size_t)bi * 4 + k) * l + i) * w) : NULL;
    const wct* V = (k < 2) ? X : Y;
    cmp[ci] = hom_comp_s(&Wl, l, is_signed, V, Bk);
    free(Bk);
    br0 += Wl.n_br;
    ks0 += Wl.n_ks;
  }
  W->n_br += br0;
  W->n_ks += ks0;

  /* validation ANDs and bitwiseAND (Algorithm 4) of each box's service bits */
  uint64_t br1 = 0, ks1 = 0;
  #pragma omp parallel for schedule(dynamic, 1) if (W->C) reduction(+ : br1, ks1)
  for (long long bi = 0; bi < (long long)N; bi++) {
    walker Wl = {W->C, W->w, 0, 0};
    wct* c = cmp + bi * 4;
    wct xl = wnew(&Wl), yl = wnew(&Wl);
    wgate(&Wl, ORC_NOT, &c[0], NULL, NULL, &xl);
    wgate(&Wl, ORC_NOT, &c[2], NULL, NULL, &yl);
    wct v1 = wnew(&Wl), v2 = wnew(&Wl), f = wnew(&Wl);
    wgate(&Wl, ORC_AND, &xl, &c[1], NULL, &v1);
    wgate(&Wl, ORC_AND, &yl, &c[3], NULL, &v2);
    wgate(&Wl, ORC_AND, &v1, &v2, NULL, &f);
    for (uint32_t j = 0; j < m; j++) {
      wct s = {W->C ? (uint32_t*)(payload + ((size_t)bi * m + j) * w) : NULL, 0};
      T[bi * m + j] = wnew(&Wl);
      wgate(&Wl, ORC_AND, &f, &s, NULL, &T[bi * m + j]);
    }
    for (int k = 0; k < 4; k++) wfree(&c[k]);
    wfree(&xl); wfree(&yl); wfree(&v1); wfree(&v2); wfree(&f);
    br1 += Wl.n_br;
    ks1 += Wl.n_ks;
  }
  W->n_br += br1;
  W->n_ks += ks1;
  free(cmp);

  /* Algorithm 5, HomAddXOR, as a balanced tree: pairs taken left to right,
   * an odd last element carried to the next round. */
  uint32_t maxlevel = 0;
  for (uint32_t j = 0; j < m; j++) {
    uint32_t cnt = N;
    wct* cur = (wct*)malloc(sizeof(wct) * N);
    for (uint32_t i = 0; i < N; i++) cur[i] = T[(size_t)i * m + j];
    while (cnt > 1) {
      uint32_t half = cnt / 2;
      wct* nxt = (wct*)malloc(sizeof(wct) * (half + (cnt & 1)));
      uint64_t br = 0, ks = 0;
      #pragma omp parallel for schedule(dynamic, 1) if (W->C) reduction(+ : br, ks)
      for (long long k = 0; k < (long long)half; k++) {
        walker Wl = {W->C, W->w, 0, 0};
        nxt[k] = wnew(&Wl);
        wgate(&Wl, ORC_XOR, &cur[2 * k], &cur[2 * k + 1], NULL, &nxt[k]);
        br += Wl.n_br;
        ks += Wl.n_ks;
      }
      W->n_br += br;
      W->n_ks += ks;
      for (uint32_t k = 0; k < 2 * half; k++) wfree(&cur[k]);
      if (cnt & 1) nxt[half] = cur[cnt - 1];
      free(cur);
      cur = nxt;
      cnt = half + (cnt & 1);
    }
    if (cur[0].level > maxlevel) maxlevel = cur[0].level;
    if (W->C) memcpy(out + (size_t)j * w, cur[0].ct, sizeof(uint32_t) * w);
    wfree(&cur[0]);
    free(cur);
  }
  if (depth) *depth = maxlevel;
  free(X);
  free(Y);
  free(T);
}

void orc_bbox_query(const orc_ctx* C, uint32_t l, uint32_t n_boxes, uint32_t m, int is_signed,
                    const uint32_t* x, const uint32_t* y, const uint32_t* bounds,
                    const uint32_t* payload, uint32_t* out) {
  walker W = {C, C->P.n + 1, 0, 0};
  bbox_walk(&W, l, n_boxes, m, is_signed, x, y, bounds, payload, out, NULL);
}

void orc_bbox_counts(uint32_t l, uint32_t n_boxes, uint32_t m, uint64_t* n_br,
                     uint64_t* n_ks, uint32_t* depth) {
  walker W = {NULL, 1, 0, 0};
  bbox_walk(&W, l, n_boxes, m, 1, NULL, NULL, NULL, NULL, NULL, depth);
  *n_br = W.n_br;
  *n_ks = W.n_ks;
}
