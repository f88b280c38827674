/*
 * CPU oracle for the LocPIR gate-bootstrapping path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table
 * or constant generator with the GPU path.
 *
 * What it computes (paper: "Fast Private Location-based Information
 * Retrieval over the Torus", LocPIR):
 *   - TFHE KeyGen / Encrypt / Decrypt of single bits (Sec. 2.2), with the
 *     encoding f(m) = m/4 - 1/8 and the phase b - a.K;
 *   - gate bootstrapping (Sec. 2.2, EvalGate and the HomAND identity; the
 *     other basic gates follow the cited TFHE construction): modulus
 *     switch, blind rotation by CMux external products, sample extraction
 *     and LWE key switching;
 *   - the bounding-box circuit of Algorithms 2-5 (HomCompS, LocPIR,
 *     bitwiseAND, HomAddXOR).
 *
 * Torus32 convention: a torus value t is the uint32 round(t * 2^32) mod 2^32.
 * All additions and subtractions of torus values wrap mod 2^32.
 *
 * Parity status: each function is pinned by the CPU test-suite (schoolbook
 * products, closed forms, truth tables, brute force, the paper's worked
 * examples, the noise model).  The exact ciphertext bits of a bootstrap
 * depend on conventions that the paper leaves to the TFHE library (rounding
 * offsets, digit ranges, row order); those conventions are fixed here and are
 * "parity unpinned" against any external TFHE implementation: only the
 * decrypted semantics and the noise statistics tie them to TFHE as published.
 */
#ifndef LOCPIR_ORACLE_H
#define LOCPIR_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  uint32_t n;           /* LWE dimension of gate ciphertexts                */
  uint32_t N;           /* ring degree of the accumulator (power of two)    */
  uint32_t bg_bit;      /* log2 of the gadget base Bg                        */
  uint32_t l;           /* gadget levels                                     */
  uint32_t ks_base_bit; /* log2 of the key-switching base                    */
  uint32_t ks_t;        /* key-switching digits                              */
  double lwe_sigma;     /* noise std (torus units) of fresh LWE and the KSK  */
  double bk_sigma;      /* noise std (torus units) of the bootstrapping key  */
} orc_params;

enum { ORC_NAND = 0, ORC_AND = 1, ORC_OR = 2, ORC_XOR = 3, ORC_XNOR = 4,
       ORC_NOR = 5, ORC_MUX = 6, ORC_NOT = 7, ORC_COPY = 8 };

/* ---- arithmetic ---- */
uint64_t orc_ntt_prime(void);
uint64_t orc_mulmod(uint64_t a, uint64_t b);
/* exact negacyclic product in Z[X]/(X^N+1) via the oracle's NTT; returns 0,
 * or -1 if N is unsupported.  Requires |result coefficient| < q/2. */
int orc_negacyclic_mul_ntt(uint32_t N, const int64_t* a, const int64_t* b, int64_t* out);
/* the same product by its definition (used to pin the NTT) */
void orc_negacyclic_mul_schoolbook(uint32_t N, const int64_t* a, const int64_t* b, int64_t* out);

/* ---- counter-based random numbers (SplitMix64 outputs) ---- */
uint64_t orc_rand_u64(uint64_t seed, uint64_t stream, uint64_t idx);
int32_t orc_gauss_torus(uint64_t seed, uint64_t stream, uint64_t idx, double sigma);

/* ---- keys (KeyGen, Sec. 2.2) ---- */
size_t orc_bsk_words(const orc_params* P); /* n * 2l * 2 * N                */
size_t orc_ksk_words(const orc_params* P); /* N * t * (base-1) * (n+1)      */
void orc_keygen(const orc_params* P, uint64_t seed, uint8_t* s_lwe, uint8_t* s_ring,
                uint32_t* bsk, uint32_t* ksk);

/* ---- Encrypt / Decrypt (Sec. 2.2) ---- */
void orc_encrypt_bits(const orc_params* P, const uint8_t* s_lwe, const uint8_t* bits,
                      size_t cnt, uint64_t seed, uint64_t first_index, uint32_t* ct);
void orc_encrypt_zeros(const orc_params* P, const uint8_t* s_lwe, size_t cnt, uint64_t seed,
                       uint64_t first_index, uint32_t* ct);
void orc_decrypt_bits(const orc_params* P, const uint8_t* s_lwe, const uint32_t* ct,
                      size_t cnt, uint8_t* bits, int32_t* phase);
uint32_t orc_phase(uint32_t dim, const uint8_t* key, const uint32_t* ct);

/* ---- bootstrapping steps ---- */
uint32_t orc_modswitch(uint32_t x, uint32_t N);
void orc_decompose(const orc_params* P, uint32_t a, int32_t* digits);
void orc_poly_rotate(uint32_t N, const uint32_t* in, uint32_t k, uint32_t* out);
void orc_sample_extract(uint32_t N, const uint32_t* acc, uint32_t* lwe_big);

/* Evaluation context: parameters, the keys (borrowed, caller keeps them
 * alive) and the bootstrapping key in the oracle's transform domain. */
typedef struct orc_ctx orc_ctx;
orc_ctx* orc_ctx_create(const orc_params* P, const uint32_t* bsk, const uint32_t* ksk);
void orc_ctx_free(orc_ctx* C);

/* one external product of step i: acc_out = ExtProd(BSK_i, d_in) (both [2][N]) */
void orc_external_product(const orc_ctx* C, uint32_t i, const uint32_t* d_in, uint32_t* acc_out);
/* blind rotation of an LWE_n sample over its first `steps` key bits; acc is
 * [2][N]: mask polynomial then body polynomial */
void orc_blind_rotate(const orc_ctx* C, const uint32_t* ct, uint32_t steps, uint32_t* acc);
void orc_keyswitch(const orc_ctx* C, const uint32_t* lwe_big, uint32_t* out);
/* bootstrap of an already combined LWE_n sample: blind rotation and sample
 * extraction into out_big (N+1 words, may be NULL), then key switching into
 * out (n+1 words, may be NULL) */
void orc_bootstrap_raw(const orc_ctx* C, const uint32_t* ct, uint32_t* out_big, uint32_t* out);
/* one bootstrapped gate up to its key switch: big (N+1 words) is the sample
 * the key switch takes; returns 0 (big untouched) for NOT, COPY and unknown
 * gates, which do not bootstrap */
int orc_gate_big(const orc_ctx* C, int gate, const uint32_t* c1, const uint32_t* c2,
                 const uint32_t* c3, uint32_t* big);
/* cnt of them over the host's threads; big: cnt x (N+1); 0 if the gate
 * does not bootstrap */
int orc_gate_big_batch(const orc_ctx* C, int gate, size_t cnt, const uint32_t* c1,
                       const uint32_t* c2, const uint32_t* c3, uint32_t* big);
/* one gate; MUX(c1 = select, c2 = if one, c3 = if zero) */
void orc_gate(const orc_ctx* C, int gate, const uint32_t* c1, const uint32_t* c2,
              const uint32_t* c3, uint32_t* out);
/* cnt independent gates, spread over the host's threads (OpenMP);
 * returns the number of threads used */
int orc_gate_batch(const orc_ctx* C, int gate, size_t cnt, const uint32_t* c1,
                   const uint32_t* c2, const uint32_t* c3, uint32_t* out);

/* ---- the bounding-box circuit (Algorithms 2-5) ----
 * x, y: l ciphertexts each, bit 0 = LSB.  bounds: n_boxes x {x1,x2,y1,y2} x l.
 * payload: n_boxes x m.  out: m ciphertexts.  is_signed keeps the MSB flip of
 * Algorithm 2 (two's-complement order); unsigned inputs omit it. */
void orc_bbox_query(const orc_ctx* C, uint32_t l, uint32_t n_boxes, uint32_t m, int is_signed,
                    const uint32_t* x, const uint32_t* y, const uint32_t* bounds,
                    const uint32_t* payload, uint32_t* out);
/* blind rotations and key switches the same circuit performs (counted by
 * walking it, not by formula) and its depth in bootstrapped-gate levels */
void orc_bbox_counts(uint32_t l, uint32_t n_boxes, uint32_t m, uint64_t* n_br,
                     uint64_t* n_ks, uint32_t* depth);

#ifdef __cplusplus
}
#endif
#endif
