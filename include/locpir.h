/*
 * locpir.h -- C ABI of the MI355X gate-bootstrapping library for LocPIR
 * ("Fast Private Location-based Information Retrieval over the Torus").
 *
 * Scope: TFHE gate bootstrapping (blind rotation by CMux external products,
 * sample extraction, LWE key switching) for every gate of the paper's
 * bounding-box circuit (Algorithms 2-5), on one GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Torus32: a torus value t is the uint32 round(t * 2^32) mod 2^32; sums wrap.
 * LWE ciphertext ("TLWE sample" in the paper, Sec. 2.2): n+1 little-endian
 *   uint32 words, mask a[0..n) then body b.  Arrays of ciphertexts are
 *   [count][n+1], densely packed.  Bit encoding f(m) = m/4 - 1/8, i.e. the
 *   plaintext of bit 1 is +2^29 and of bit 0 is -2^29.
 * Extracted ("big") LWE sample: N+1 words under the ring key.
 * Pointers named d_* are device pointers (HIP global memory of the device the
 *   key lives on); all others are host pointers.  The caller owns every
 *   buffer it passes in; the library owns the opaque handles and frees them
 *   with the matching *_free call.
 * stream: a hipStream_t passed as void* (NULL = the null stream).  Device
 *   calls are asynchronous on that stream unless stated otherwise; they may
 *   allocate device memory with the stream-ordered allocator.
 * Errors: every call returns lp_status (0 on success, negative on error) and
 *   never throws; lp_last_error() gives a thread-local message for the last
 *   failing call of the calling thread.
 * Thread safety: handles are immutable after creation.  The library's own
 *   caches (compiled query programs, launch-shape tables, twiddle tables)
 *   are internally locked.  Calls that share an lp_device_key on different
 *   streams may run concurrently; calls that share a stream and a compiled
 *   program are serialised.
 */
#ifndef LOCPIR_H
#define LOCPIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lp_status;
#define LP_OK 0
#define LP_EINVAL (-1)       /* bad argument, size or parameter set      */
#define LP_ENOMEM (-2)       /* host or device allocation failed          */
#define LP_EDEVICE (-3)      /* a HIP call failed                         */
#define LP_EUNSUPPORTED (-4) /* parameters the GPU kernels do not handle  */
#define LP_EBUDGET (-5)      /* server admission beyond the memory budget */
#define LP_EAGAIN (-6)       /* server request not finished yet           */
#define LP_ECANCELED (-7)    /* server request cancelled                  */

/* TFHE parameters.  n, lwe_sigma: LWE dimension and noise of gate
 * ciphertexts (KeyGen outputs n and sigma, Sec. 2.2).  N, k: ring degree and
 * TRLWE dimension of the accumulator; bg_bit, l: gadget base 2^bg_bit and
 * levels; bk_sigma: noise of the bootstrapping key; ks_base_bit, ks_t:
 * key-switching base 2^ks_base_bit and digit count.  The GPU kernels support
 * N = 1024, k = 1, bg_bit = 7, l = 3, n <= 1024 and ks_base_bit <= 4. */
typedef struct {
  uint32_t n, N, k, bg_bit, l, ks_base_bit, ks_t;
  double lwe_sigma, bk_sigma;
} lp_params;

typedef struct lp_secret_key lp_secret_key; /* client: LWE key s, ring key S     */
typedef struct lp_cloud_key lp_cloud_key;   /* PK = {bootstrapping key, KS key}  */
typedef struct lp_device_key lp_device_key; /* PK resident on one GPU            */

/* Gates (Sec. 2.2 EvalGate; the paper's HomAND, HomXNOR, HomMUX, HomXOR,
 * HomNOT, plus the other two-input gates of the same construction).
 * MUX(in0 = select, in1 = if one, in2 = if zero).  NOT and COPY do not
 * bootstrap. */
typedef enum {
  LP_GATE_NAND = 0, LP_GATE_AND = 1, LP_GATE_OR = 2, LP_GATE_XOR = 3,
  LP_GATE_XNOR = 4, LP_GATE_NOR = 5, LP_GATE_MUX = 6, LP_GATE_NOT = 7,
  LP_GATE_COPY = 8
} lp_gate;

const char* lp_last_error(void);
const char* lp_version(void);

/* Default parameters: n = 630, lwe_sigma = 2^-15, N = 1024, k = 1,
 * bg_bit = 7, l = 3, bk_sigma = 2^-25, ks_base_bit = 2, ks_t = 8.  This is
 * the paper's lambda 128 set (Sec. 5: TLWE dimension n = 630); the paper
 * fixes no other parameter of it, so the noise widths, the ring, the gadget
 * and the key-switching base are those of the standard TFHE gate
 * bootstrapping set that Sec. 2.2 builds on (TFHE library 1.1, which the
 * experiments of Sec. 5 use). */
lp_status lp_params_default(lp_params* out);
/* The paper's lambda 80 set (Sec. 5): n = 540, lwe_sigma = 2^-20.2; the
 * paper gives nothing else for it, so the ring, gadget and key-switching
 * parameters are the default ones. */
lp_status lp_params_lambda80(lp_params* out);

/* ---- client side (host) -------------------------------------------------- */

/* KeyGen(lambda) of Sec. 2.2 with the parameters given: a binary LWE key s,
 * a binary ring key S, PK = {BSK, KSK}.  Deterministic in seed (SplitMix64
 * counter-based draws).  BSK_i is a TGSW encryption of s_i: 2l TRLWE rows,
 * row (p, j) = TRLWE_S(0) + s_i/Bg^(j+1) on component p.  KSK[i][j][v-1]
 * (v = 1..base-1) is LWE_s(v * S_i / base^(j+1)).  Host only; no GPU needed. */
lp_status lp_keygen(const lp_params* P, uint64_t seed, lp_secret_key** sk, lp_cloud_key** ck);

/* Raw key material.  s: n bytes in {0,1}; S: N bytes in {0,1}.
 * bsk: [n][2l][2][N] uint32 (row r = p*l + j; component 0 = mask polynomial,
 *   1 = body polynomial).  ksk: [N][ks_t][base-1][n+1] uint32.
 * Import copies the arrays; export writes into caller arrays of these sizes. */
lp_status lp_secret_key_import(const lp_params* P, const uint8_t* s, const uint8_t* S, lp_secret_key** sk);
lp_status lp_secret_key_export(const lp_secret_key* sk, uint8_t* s, uint8_t* S);
lp_status lp_cloud_key_import(const lp_params* P, const uint32_t* bsk, const uint32_t* ksk, lp_cloud_key** ck);
lp_status lp_cloud_key_export(const lp_cloud_key* ck, uint32_t* bsk, uint32_t* ksk);
lp_status lp_cloud_key_params(const lp_cloud_key* ck, lp_params* out);
/* PK as one byte blob for the client's upload (Sec. 3): a 64-byte header
 * ("LPCK", format version 1, the parameters as u32 n, N, k, bg_bit, l,
 * ks_base_bit, ks_t and f64 lwe_sigma, bk_sigma, little-endian, zero padded)
 * followed by the bsk and ksk words in the layouts above.  serialize: with
 * buf == NULL, *len receives the size; otherwise *len must hold at least
 * that many bytes and receives the size written.  deserialize: a new key
 * owned by the caller; LP_EINVAL for a foreign, truncated or inconsistent
 * blob. */
lp_status lp_cloud_key_serialize(const lp_cloud_key* ck, void* buf, size_t* len);
lp_status lp_cloud_key_deserialize(const void* buf, size_t len, lp_cloud_key** ck);
size_t lp_bsk_words(const lp_params* P);
size_t lp_ksk_words(const lp_params* P);

/* Encrypt(m, K, n, sigma) of Sec. 2.2, bit by bit (Sec. 4.1): ct[k] =
 * (a, <a,s> + f(bits[k]) + e), a uniform, e ~ N(0, lwe_sigma), drawn from
 * (seed, first_index + k).  ct: cnt*(n+1) uint32, host. */
lp_status lp_encrypt_bits(const lp_secret_key* sk, const uint8_t* bits, size_t cnt, uint64_t seed,
                          uint64_t first_index, uint32_t* ct);
/* The client's fresh samples of Sec. 3, sent once with PK: LWE encryptions
 * of the torus value 0, ct[k] = (a, <a,s> + e) drawn from (seed,
 * first_index + k) on streams of their own.  The cloud turns them into
 * encrypted services with lp_preprocess.  ct: cnt*(n+1) uint32, host. */
lp_status lp_encrypt_zeros(const lp_secret_key* sk, size_t cnt, uint64_t seed, uint64_t first_index, uint32_t* ct);

/* Decrypt(ct, K) of Sec. 2.2: bit = sign of the phase b - <a,s>.  phase may
 * be NULL; otherwise it receives the signed phase (int32 Torus32). */
lp_status lp_decrypt_bits(const lp_secret_key* sk, const uint32_t* ct, size_t cnt, uint8_t* bits,
                          int32_t* phase);

/* ---- cloud side (device) ------------------------------------------------- */

/* The cloud's copy of PK (KeyGen's bootstrapping key and key-switching key,
 * Sec. 2.2), resident on the current HIP device: uploads both and transforms
 * the bootstrapping key to the NTT domain there (about 62 MB of BSK plus
 * 62 MB of KSK per key; lp_device_key_bytes gives the total).  ck stays
 * owned by the caller and may be freed afterwards; *dk is owned by the
 * caller and freed with lp_device_key_free.  Synchronous on stream.
 * LP_EUNSUPPORTED for parameters the GPU kernels do not handle, LP_ENOMEM
 * when the device allocation fails, LP_EDEVICE for other HIP failures. */
lp_status lp_device_key_create(const lp_cloud_key* ck, void* stream, lp_device_key** dk);
lp_status lp_device_key_bytes(const lp_device_key* dk, size_t* bytes);

/* EvalGate(ct1, ct2, PK) of Sec. 2.2 over a batch: the gate's linear
 * pre-combination (HomAND = Bootstrap((0, -1/8) + ct1 + ct2), the other
 * gates alike), then Bootstrap (blind rotation, sample extraction, key
 * switching).  cnt gates of one kind on device ciphertexts:
 * d_out[k] = gate(d_in0[k], d_in1[k], d_in2[k]).  d_in1 is ignored for NOT/COPY; d_in2 is used by MUX
 * only.  All arrays are cnt*(n+1) uint32 on the key's device.  Every
 * bootstrapped gate runs the blind rotation, sample extraction and key
 * switching (MUX: two blind rotations, one key switch).  d_out may be one of
 * the inputs (it is written by the key switch, after every input was read).
 * cnt = 0 is a no-op.  A batch of at most 256 blind rotations runs them
 * split over two workgroups each (lp_split_stall_count); the call then waits
 * for the stream and returns LP_EDEVICE if one of their bounded waits ran
 * out (the outputs are then undefined). */
lp_status lp_bootstrap_batch(const lp_device_key* dk, lp_gate gate, const uint32_t* d_in0,
                             const uint32_t* d_in1, const uint32_t* d_in2, size_t cnt,
                             uint32_t* d_out, void* stream);

/* lp_bootstrap_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same gates, kernels and outputs, but every working buffer
 * (job lists, the extracted samples, the split-rotation area) lives in the
 * library's static device scratch, a fixed array of 13 MiB that each GPU the
 * library runs on holds until the process ends.  The call allocates no
 * device memory and calls no allocating library routine.  cnt is at most
 * 1024 gates per call (LP_EINVAL above, nothing launched).  Every call on
 * one GPU shares that GPU's scratch: calls that overlap in time on one GPU
 * (different streams or threads) race and must be serialised by the caller;
 * calls in order on one stream are safe.  The split area's control words are
 * cleared (by a fill kernel) at the start of each call that uses them.  Other
 * arguments, errors and waiting behave as in lp_bootstrap_batch. */
lp_status lp_bootstrap_batch_noalloc(const lp_device_key* dk, lp_gate gate, const uint32_t* d_in0,
                                     const uint32_t* d_in1, const uint32_t* d_in2, size_t cnt,
                                     uint32_t* d_out, void* stream);

/* EvalGate of Sec. 2.2 stopped before Bootstrap's final key switch:
 * d_out_big[k] (N+1 words, LWE of dimension N under the ring key S) is the
 * sample that gate's key switch takes: the sample extracted from the blind rotation of the gate's input
 * combination, or for MUX (0, 1/8) + u1 + u2 of its two rotations.
 * lp_keyswitch_batch of d_out_big equals lp_bootstrap_batch bit for bit.
 * d_out_big (cnt*(N+1) uint32) must not overlap the inputs: the rotations
 * write it while others still read theirs.  NOT and COPY do not bootstrap:
 * LP_EINVAL.  cnt = 0 is a no-op.  Split rotations are waited for and
 * checked as in lp_bootstrap_batch. */
lp_status lp_bootstrap_batch_noks(const lp_device_key* dk, lp_gate gate, const uint32_t* d_in0,
                                  const uint32_t* d_in1, const uint32_t* d_in2, size_t cnt,
                                  uint32_t* d_out_big, void* stream);

/* Key switching alone, the last step of Bootstrap (Sec. 2.2: PK's key
 * switching key brings the bootstrapped sample back under the TLWE key):
 * d_in holds cnt extracted samples of N+1 words under the ring key; d_out
 * receives cnt samples of n+1 words under s.  Both on the key's device, owned
 * by the caller.  d_out must not overlap d_in.  Waits for the stream before
 * returning (its job list is staged in host memory).  cnt = 0 is a no-op;
 * LP_EINVAL for a null buffer or a batch above 2^28. */
lp_status lp_keyswitch_batch(const lp_device_key* dk, const uint32_t* d_in, size_t cnt,
                             uint32_t* d_out, void* stream);

/* The bounding-box query of Algorithm 3 (LocPIR): four ripple comparators
 * per box (Algorithm 2, HomCompS and HomCompLE = NOT HomCompS with swapped
 * arguments), the validation ANDs, bitwiseAND with the box's service bits
 * (Algorithm 4) and the XOR sum over boxes (Algorithm 5, as a balanced tree).
 * Bits are LSB first.  is_signed = 1 applies the MSB flip of Algorithm 2
 * (two's-complement coordinates); 0 compares unsigned codes.  Boxes are
 * half-open: x1 <= x < x2 and y1 <= y < y2.
 *   d_x, d_y:    l ciphertexts each
 *   d_bounds:    n_boxes x {x1, x2, y1, y2} x l ciphertexts
 *   d_payload:   n_boxes x m ciphertexts
 * d_out receives m ciphertexts.  The circuit is cut into depth levels; each
 * level is one batched bootstrap launch plus one key-switch launch.
 * LP_EINVAL for l outside 1..64, n_boxes outside 1..65536, m outside
 * 1..4096 or a null input.  When some level runs split rotations (see
 * lp_split_stall_count) the call waits for the stream at its end and
 * returns LP_EDEVICE if one of their bounded waits ran out; d_out is then
 * undefined.  Otherwise it returns without waiting. */
typedef struct {
  uint32_t l, n_boxes, m;
  int32_t is_signed;
  const uint32_t* d_x;
  const uint32_t* d_y;
  const uint32_t* d_bounds;
  const uint32_t* d_payload;
} lp_bbox_query;
lp_status lp_eval_bbox_query(const lp_device_key* dk, const lp_bbox_query* q, uint32_t* d_out,
                             void* stream);
/* Several queries, each under its own device key (keys[k], queries[k],
 * d_outs[k] for k < nq), evaluated together: depth level L of every query
 * runs in one fused blind-rotation launch and one fused key-switch launch,
 * each job selecting its query's key.  All keys must live on one device with
 * equal n, ks_base_bit and ks_t.  The compiled program (job lists, ciphertext
 * pool, one graph per level for the blind rotations and one for the key
 * switches) is cached per (stream, keys, query shapes) and replayed; calls
 * that share a stream and a program are serialised by the library.  Set the
 * environment variable LOCPIR_GRAPHS=0 to launch the kernels directly.
 * Split rotations are waited for and checked as in lp_eval_bbox_query (a
 * give-up fails the whole call). */
lp_status lp_eval_bbox_batch(const lp_device_key* const* keys, const lp_bbox_query* queries, size_t nq,
                             uint32_t* const* d_outs, void* stream);
/* The one-time part of lp_eval_bbox_batch for the same keys, query shapes
 * and stream, done ahead: compiles the circuit of Algorithms 2-5 for every
 * query into depth levels, uploads the job lists, allocates the ciphertext
 * pool and captures the per-level graphs, launching nothing.  The following
 * lp_eval_bbox_batch with the same keys, shapes and stream finds the program
 * cached (the cache keeps the 16 most recent programs).  Only the shapes and
 * keys are read (input pointers must be non-null but are not dereferenced).
 * Errors as lp_eval_bbox_batch. */
lp_status lp_eval_bbox_prepare(const lp_device_key* const* keys, const lp_bbox_query* queries, size_t nq,
                               void* stream);

/* Preprocess (Algorithm 1), cloud side: the cloud encrypts its plaintext
 * service bits S_i[j] without the secret key by adding the trivial sample
 * (0, f(bit)) to one of the client's fresh samples of zero each:
 * d_out[k] = d_zero[k] + (0, f(d_bits[k])), f(nonzero) = +1/8 and
 * f(0) = -1/8, the encoding of Encrypt.  d_zero, d_out: cnt*(n+1) uint32;
 * d_bits: cnt bytes; all on the key's device.  d_out may equal d_zero.  An
 * all-zero d_zero gives noiseless trivial samples, which is how the cloud
 * enters its own plaintext box bounds.  cnt = 0 is a no-op. */
lp_status lp_preprocess(const lp_device_key* dk, const uint32_t* d_zero, const uint8_t* d_bits, size_t cnt,
                        uint32_t* d_out, void* stream);

/* Bytes the protocol of Sec. 3 moves for one query shape, ciphertexts as
 * cnt*(n+1) little-endian uint32 words with no header (the sizes Sec. 6.1
 * reports): one LWE sample; PK (bootstrapping and key-switching keys in
 * Torus32 form; lp_cloud_key_serialize adds its 64-byte header); the
 * n_boxes*m fresh samples for the services; one encrypted
 * coordinate (l samples); the query (x and y); the result (m samples). */
typedef struct {
  size_t lwe_sample, public_key, service_samples, coordinate, query, result;
} lp_wire_bytes;
lp_status lp_bbox_wire_bytes(const lp_params* P, uint32_t l, uint32_t n_boxes, uint32_t m, lp_wire_bytes* out);

/* Bootstraps, key switches and depth levels of that circuit. */
lp_status lp_bbox_counts(uint32_t l, uint32_t n_boxes, uint32_t m, uint64_t* n_br, uint64_t* n_ks,
                         uint32_t* n_levels);
/* Blind rotations per depth level of that circuit as the library schedules
 * a lone query of the shape on the calling thread's current device (signed
 * shape).  Only the comparators' XNORs have slack; they go either early
 * (all at the first level, then l levels of MUXes alone) or late (each next
 * to the MUX that uses it, as late as its consumers allow).  With a timed
 * shape table (lp_autotune) a program, one query or many fused by
 * lp_eval_bbox_batch, takes early when the summed launch times the table
 * predicts are at least 2 % lower; without one, a lone query takes early
 * exactly when that lets its MUX levels run as split rotations one
 * workgroup per CU (br_waves 6, see lp_tune_entry) and a level holding
 * MUXes and XNORs together could not, and fused queries take late.  The server always takes late.  The
 * environment variable LOCPIR_XNOR_EARLY = 0 or 1 overrides the choice.
 * The depth is the same either way.  widths: host array of *n_levels
 * entries on input; *n_levels receives the depth (entries beyond the array
 * are not written). */
lp_status lp_bbox_level_widths(uint32_t l, uint32_t n_boxes, uint32_t m, uint32_t* widths, uint32_t* n_levels);

/* ---- query server (continuous batching) ------------------------------------
 * Serves bounding-box queries from many clients, each request bringing its
 * own cloud key (PK).  A scheduler thread admits queued requests in arrival
 * order while the device bytes they need (keys, ciphertext pool, extract and
 * job buffers; see lp_server_request_bytes) fit hbm_budget and fewer than
 * max_inflight are admitted.  Each scheduler tick runs the next depth level
 * of every admitted request in one fused blind-rotation launch and one fused
 * key-switch launch per parameter shape (requests fuse with those of equal
 * n, ks_base_bit and ks_t; keys of the lambda 128 and lambda 80 sets are
 * served side by side in separate launches); requests that arrive meanwhile
 * join at the next tick.  stats.ticks counts fused launch pairs.
 * max_tick_rotations > 0 caps the blind rotations of one tick: requests
 * with less of their level left than an equal share run all of it, the
 * others split the rest (at least one gate each), and a level that does not
 * fit runs over several ticks; results are unchanged, and a wide request no
 * longer stretches the ticks of every narrow one beside it.
 * LP_TICK_CAP_AUTO takes, at every tick, the narrowest launch width of the
 * device's timed launch-shape table (lp_autotune) whose rotation time per
 * job is within 15 % of the table's best, or 2048 without a timed table.
 * stats.widest_tick is the most rotations one fused launch has held.
 * A finished request's result is kept on the host until polled; its device
 * memory is released at once.  A failing request (allocation, upload, or a
 * split rotation of its gates whose bounded wait ran out: LP_EDEVICE) ends
 * alone; the others continue.  Latency is measured from submit to the end of
 * the result copy.  The server runs on the HIP device current at creation. */
typedef struct lp_server lp_server;
typedef struct {
  size_t hbm_budget;     /* device bytes the admitted requests may hold together     */
  uint32_t max_inflight; /* admitted requests at once; 0 = bounded by the budget only */
  int32_t simulate;      /* 1: schedule without a GPU (results are zero); for tests   */
  uint64_t fail_ticket;  /* fault injection: this ticket's set-up fails (0 = none)    */
  uint32_t max_tick_rotations; /* blind rotations per tick at most; 0 = a whole level */
} lp_server_config;
#define LP_TICK_CAP_AUTO 0xFFFFFFFFu /* max_tick_rotations from the timed shape table */
/* A query whose ciphertexts are in host memory (same layout as lp_bbox_query). */
typedef struct {
  uint32_t l, n_boxes, m;
  int32_t is_signed;
  const uint32_t* x;
  const uint32_t* y;
  const uint32_t* bounds;
  const uint32_t* payload;
} lp_bbox_query_host;
typedef struct {
  uint64_t submitted, admitted, completed, failed, cancelled, ticks, fused_bootstraps;
  uint32_t pending, active;
  size_t bytes_in_use, peak_bytes;
  uint64_t widest_tick;
} lp_server_stats;
lp_status lp_server_create(const lp_server_config* cfg, lp_server** out);
/* Device bytes a request of this key and shape holds while admitted. */
lp_status lp_server_request_bytes(const lp_cloud_key* ck, const lp_bbox_query_host* q, size_t* bytes);
/* Copies the query's ciphertexts and queues it; ck must stay alive until the
 * request ends.  LP_EBUDGET if it can never fit the budget, LP_EINVAL for a
 * malformed shape.  *ticket identifies the request. */
lp_status lp_server_submit(lp_server* s, const lp_cloud_key* ck, const lp_bbox_query_host* q, uint64_t* ticket);
/* The same request as the client sends it (Sec. 3: PK uploaded with the
 * query): key_blob is PK as lp_cloud_key_serialize writes it, key_len its
 * length in bytes.  The server deserializes it into a key of its own, which
 * the request holds until it ends; the caller's blob may be freed when the
 * call returns.  Latency is measured from the call's entry, so it includes
 * the deserialization.  LP_EINVAL for a foreign, truncated or inconsistent
 * blob (nothing is queued), otherwise as lp_server_submit. */
lp_status lp_server_submit_blob(lp_server* s, const void* key_blob, size_t key_len, const lp_bbox_query_host* q,
                                uint64_t* ticket);
/* LP_EAGAIN while the request runs (wait = 0), or blocks until it ends
 * (wait != 0).  On LP_OK copies the m result ciphertexts to out (host,
 * may be NULL) and the latency in seconds; other statuses report how the
 * request ended.  A ticket can be polled to completion once. */
lp_status lp_server_poll(lp_server* s, uint64_t ticket, int wait, uint32_t* out, double* latency_s);
/* Ends a queued or running request at the next tick with LP_ECANCELED. */
lp_status lp_server_cancel(lp_server* s, uint64_t ticket);
lp_status lp_server_stats_get(lp_server* s, lp_server_stats* out);
/* Finishes every queued and running request, then frees the server. */
void lp_server_free(lp_server* s);

/* ---- diagnostics (device) ------------------------------------------------ */

/* Exact negacyclic products mod 2^32 of cnt pairs (digit polynomial,
 * Torus32 polynomial) of degree < 1024, by the library's NTT.  d_digits:
 * cnt*1024 int32 with |d| <= 64; d_poly, d_out: cnt*1024 uint32. */
lp_status lp_debug_negacyclic_mul(const int32_t* d_digits, const uint32_t* d_poly, size_t cnt,
                                  uint32_t* d_out, void* stream);
/* Blind rotation of cnt LWE_n samples over their first `steps` key bits
 * (steps >= n: all); d_acc receives cnt accumulators of [2][N] uint32.
 * Synchronous; split rotations are checked as in lp_bootstrap_batch. */
lp_status lp_debug_blind_rotate(const lp_device_key* dk, const uint32_t* d_in, size_t cnt,
                                uint32_t steps, uint32_t* d_acc, void* stream);

/* The CMux external product of one blind-rotation step (Sec. 2.2, Bootstrap:
 * ACC + ExtProd(BSK_i, X^a ACC - ACC)) computed on the int8 matrix cores, an
 * exact alternative to the NTT: d_out[b] = sum over the 2l key rows r of
 * dec_r(d_in[b]) * d_key_step[r] in Z[X]/(X^N + 1) mod 2^32, where dec_r is
 * gadget digit j of component p (r = p l + j, signed digits in [-64, 64)).
 * The key words are split into four balanced bytes and every negacyclic
 * product is an int8 Toeplitz matrix product summed exactly in int32.
 * d_key_step: [2l][2][N] uint32 (one step's rows in lp_cloud_key_export's
 * bsk layout); d_in, d_out: cnt x [2][N] uint32 (TRLWE samples, mask then
 * body); all on the current device, owned by the caller.  N = 1024, l = 3
 * only; cnt <= 65536 (LP_EINVAL above).  Allocates stream-ordered scratch. */
lp_status lp_debug_external_product_mfma(const uint32_t* d_key_step, const uint32_t* d_in, size_t cnt,
                                         uint32_t* d_out, void* stream);

/* Throughput of the field operations the blind rotation's external product
 * (Sec. 2.2, Bootstrap) is built from, measured on the current device: each
 * runs alone at full occupancy on every compute unit, on residues held in
 * registers, in launches sized to about target_ms (0 < target_ms <= 1000).
 * rates[LP_OPRATE_COUNT] receives operations per second on the whole device,
 * ms (may be NULL) the timed launch of each.  The operations, in order:
 *   0 forward-transform butterflies (the 1024-point transform's shift-twiddle
 *     stages as the kernels run them: pass-1 stages 4, 2, 1 and pass 2);
 *   1 inverse-transform butterflies (the cyclic inverse pass);
 *   2 digit butterflies (the first two forward stages on gadget digits, int64);
 *   3 general products mod p (the twists);
 *   4 a*b + c*d mod p with one reduction (the key products);
 *   5 additions of a reduced operand mod p (the sums over gadget levels);
 *   6 32-bit integer additions (the full-rate reference).
 * These price the rotation's operation count in the benchmark's roofline.
 * Synchronous on stream; allocates a small device buffer. */
#define LP_OPRATE_COUNT 7
lp_status lp_debug_field_op_rates(double target_ms, double* rates, double* ms, void* stream);

/* Where a split blind rotation's time goes (br_waves 6 or 7): the blind
 * rotation of cnt (1..128 for 6, 1..256 for 7) LWE_n samples d_in (device,
 * cnt*(n+1) words) in the shape's profiling build, which reads the shader
 * clock at the phase boundaries of every step.  waves must be 6 or 7.  cycles (host, 4 x 12
 * doubles) receives, per wave index of a workgroup and phase, the clock
 * cycles per executed step averaged over the launch's workgroups: [0]
 * digits and key requests, [1] the barrier after them, [2] the forward
 * transform and its copy to LDS, [3] the barrier after it, [4] the
 * partner component's key products and their stores, [5] the wait for
 * those stores and the flag, [6] the wait for the partner's flag, [7]
 * loading the partner's products, this half's own and the sum, [8] the inverse's first pass
 * and twist, [9] the barrier inside the inverse, [10] its second pass and
 * the accumulator update, [11] the closing barrier.  ms (may be NULL)
 * receives the launch's duration.  Synchronous; allocates its working
 * memory. */
lp_status lp_debug_split_profile(const lp_device_key* dk, const uint32_t* d_in, size_t cnt, int waves,
                                 double* cycles, double* ms, void* stream);

/* ---- profiling ----------------------------------------------------------- */

/* Per-kernel statistics: when enabled, the library records a HIP event pair
 * around every blind-rotation and key-switch launch on the launch stream.
 * lp_profile_collect waits for the recorded events, writes one entry per
 * kernel kind (at most *count entries; *count receives the number written)
 * and clears the record.  name: static string ("blind_rotate",
 * "keyswitch"); jobs: bootstraps or key switches launched; total_ms: sum of
 * event-measured kernel durations. */
typedef struct {
  const char* name;
  uint64_t launches;
  uint64_t jobs;
  double total_ms;
} lp_kernel_stat;
lp_status lp_profile_enable(int on);
lp_status lp_profile_collect(lp_kernel_stat* stats, int* count);
/* The same record one launch at a time, oldest first: name as above; jobs;
 * shape: waves per bootstrap (blind rotation) or key switches per tile (key
 * switching); ms: event-measured duration.  Writes min(*count, recorded)
 * entries, sets *count to the number written and clears the whole record.
 * A query launches one blind rotation and one key switch per depth level,
 * in level order. */
typedef struct {
  const char* name;
  uint64_t jobs;
  int32_t shape;
  double ms;
} lp_launch_record;
lp_status lp_profile_collect_launches(lp_launch_record* recs, int* count);
/* Split blind rotations (br_waves 6 and 7) pair two workgroups that wait for each
 * other's transforms every step; each wait is bounded (about a second of
 * polling), so a partner that never arrives cannot hang the device.  Such a
 * wait ends the job's exchange, its output is then undefined, and the
 * current device's count of these events, since the library was loaded,
 * goes up by one per wave.  The call that launched the rotation learns of it
 * too: lp_bootstrap_batch, lp_bootstrap_batch_noks, lp_debug_blind_rotate,
 * lp_eval_bbox_query and lp_eval_bbox_batch return LP_EDEVICE, and the server
 * fails the requests whose gates were affected.  Writes that count to *count (synchronous: waits
 * for the device).  Pairing draws tickets on arrival, so the count stays 0
 * unless other work holds every CU for the whole bound.  The environment
 * variable LOCPIR_SPLIT_SPIN, when set to a smaller positive number of
 * polls, lowers the bound for the launches made while it is set (a test of
 * the give-up path; captured query graphs keep the bound they were captured
 * with). */
lp_status lp_split_stall_count(uint32_t* count);

/* ---- launch-shape autotuning --------------------------------------------- */

/* One row of a device's launch-shape table.  A launch of `count` jobs uses
 * the first row (rows sorted by `jobs`, ascending) with count <= jobs, or
 * the last row when count exceeds every bound.
 *   br_waves: waves cooperating on one blind rotation, 1 (throughput), 2
 *             (one accumulator component per wave, the two trading their
 *             cross terms in the NTT domain; two waves per SIMD at four
 *             rotations per CU), 3 (one gadget level per wave, latency), 4
 *             (three level waves,
 *             then the levels summed in the NTT domain and each component
 *             inverted once on two waves; one rotation per CU), 5 (the
 *             same, sized for two rotations per CU), 6 (the rotation split
 *             over two workgroups, normally two CUs, each owning one
 *             accumulator component and trading its key products for the
 *             other component with the other every step; lower latency
 *             again, for launches of at most 128 rotations) or 7 (the same
 *             split sized for two workgroups per CU, for launches of at
 *             most 256) -- a wider launch that looks up a split shape runs
 *             7 when it fits, else 5;
 *   ks_tile:  key switches per wave tile, 1, 4, 8 or 16;
 *   ks_split: ranges the ring index of a key switch is split into (partial
 *             sums added atomically), 1, 2, 4, 8 or 16;
 *   br_us, ks_us: measured microseconds per job of the chosen shapes at
 *             `jobs` (0 when the row was installed with lp_tune_set).
 * The environment variables LOCPIR_BR_WAVES, LOCPIR_KS_TILE and
 * LOCPIR_KS_SPLIT, when set to a valid value, override the table. */
typedef struct {
  uint32_t jobs;
  int32_t br_waves, ks_tile, ks_split;
  float br_us, ks_us;
} lp_tune_entry;
#define LP_TUNE_MAX_ROWS 32

/* Times every blind-rotation and key-switch launch shape at each batch size
 * in bucket_jobs (nbuckets <= LP_TUNE_MAX_ROWS, each 1..65536, distinct) on
 * the calling thread's current device, with dk's key, random inputs and the
 * blind rotation cut to br_steps (1..n) key bits (the per-step cost does not
 * depend on the bit); installs the fastest shapes as the device's table and
 * writes the rows, sorted by jobs, to out (nbuckets entries, may be NULL).
 * A key-switch shape is scored together with the blind rotation launched
 * after it: in a circuit every key switch is followed by one, and the shape
 * can change that rotation's time through the cache state it leaves.
 * Synchronous on `stream`.  Cached query programs are dropped so that later
 * queries launch with the new shapes. */
lp_status lp_autotune(const lp_device_key* dk, const uint32_t* bucket_jobs, int nbuckets, uint32_t br_steps,
                      void* stream, lp_tune_entry* out);
/* Installs rows (validated: jobs 1..2^22 and distinct, shapes from the sets
 * above; n <= LP_TUNE_MAX_ROWS; sorted by the library)
 * as the current device's table; n = 0 clears it (built-in defaults). */
lp_status lp_tune_set(const lp_tune_entry* rows, int n);
/* Copies the current device's table: at most *n rows; *n receives the count. */
lp_status lp_tune_get(lp_tune_entry* rows, int* n);
/* The shapes a launch of `jobs` jobs gets now on the current device
 * (environment, then table, then built-in defaults); n_lwe sizes the
 * default key-switch split.  br_us and ks_us are returned as 0. */
lp_status lp_tune_pick(uint32_t jobs, uint32_t n_lwe, lp_tune_entry* out);

void lp_secret_key_free(lp_secret_key* sk);
void lp_cloud_key_free(lp_cloud_key* ck);
void lp_device_key_free(lp_device_key* dk);

#ifdef __cplusplus
}
#endif
#endif
