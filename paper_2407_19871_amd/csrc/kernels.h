// Launchers of the gfx950 kernels (C++ linkage, internal to liblocpir).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "jobs.h"

namespace lp {

// Twiddle tables of the 32 x 32 NTT (each 1024 u64, see ntt32.h):
//   tw_f[i*32 + l] = psi^((2 brv5(i) + 1) l)
//   tw_i[m*32 + l] = psi^(-(2 brv5(l) + 1) m) / 1024
struct Twiddles {
  const uint64_t* fwd;
  const uint64_t* inv;
};

// Torus32 polynomials [npoly][1024] -> NTT domain [npoly][16 slot pairs][32 lanes][2].
hipError_t launch_bsk_to_ntt(const uint32_t* d_src, uint64_t* d_dst, int npoly, Twiddles tw,
                             hipStream_t s);

// Split shapes: one bootstrap on two workgroups of four waves; 6 sized for
// one workgroup per CU (launches of up to kSplitMaxJobs jobs), 7 for two
// (up to kSplitDualMaxJobs).
inline bool is_split(int waves_per_job) { return waves_per_job == 6 || waves_per_job == 7; }

// Exchange area of split blind rotations (waves_per_job = 6: one bootstrap
// on two workgroups, one per accumulator component, that trade their key
// products for the other component every step).  The owner allocates it
// for at most max_jobs jobs per launch; the sync words are zero before the
// first launch, and every launch leaves its counters and XCD-id words zero
// (the step flags are cleared by the launch that uses them, at its start).
// One launch at a time may use an area.
constexpr int kSplitMaxJobs = 128;
constexpr int kSplitDualMaxJobs = 256;
// The widest launch of a split shape (0 for any other).
inline int split_max_jobs(int waves_per_job) {
  return waves_per_job == 7 ? kSplitDualMaxJobs : waves_per_job == 6 ? kSplitMaxJobs : 0;
}
struct SplitArea {
  uint64_t* xbuf = nullptr;  // [job][role 2][step parity 2][1024] u64
  uint32_t* sync = nullptr;  // 8 ticket counters, finish count, status; 16 flag words per job; give-up marks
  int max_jobs = 0;
};
size_t split_xbuf_bytes(int max_jobs);
size_t split_sync_bytes(int max_jobs);
// Synchronous allocation (hipMalloc, zeroed), for 1..kSplitDualMaxJobs
// jobs; split_area_free releases it.
hipError_t split_area_alloc(SplitArea* a, int max_jobs);
void split_area_free(SplitArea* a);
// Stream-ordered allocation (hipMallocAsync, cleared by a kernel) and release.
hipError_t split_area_alloc_async(SplitArea* a, int max_jobs, hipStream_t s);
hipError_t split_area_free_async(SplitArea* a, hipStream_t s);
// Clears `words` 32-bit words with a fill kernel on stream s.
hipError_t launch_clear_words(uint32_t* d, size_t words, hipStream_t s);

// Static scratch of the gate-batch entry point that allocates nothing: a
// fixed device array per GPU (csrc/scratch.hip) carved into a split area for
// kNoAllocSplitJobs jobs, job descriptors and extract slots for at most
// kNoAllocMaxGates gates (2 blind rotations each for MUX).
constexpr int kNoAllocMaxGates = 1024;
constexpr int kNoAllocSplitJobs = kSplitMaxJobs;
constexpr int RING_N_MAX = 1024;
constexpr size_t kNoAllocScratchBytes = size_t(13) << 20;
struct NoAllocScratch {
  SplitArea split;
  BrJob* br = nullptr;
  KsJob* ks = nullptr;
  uint32_t* ex = nullptr;
};
// The current device's copy of the array, its address looked up on the
// first call on that device and kept.
hipError_t noalloc_scratch(NoAllocScratch* out);

// Waits of split launches that ran out of polls on this device since the
// process started (0 unless a partner workgroup never arrived).
hipError_t split_stall_count(uint32_t* out);
// After every launch on the area that s has queued: waits (synchronously
// for s) and reads the area's give-up record, the number of waits that ran
// out since it was last taken and (jobs, may be null) the launch-relative
// indices of the jobs they belong to, whose outputs are undefined; then
// clears the record.  With jobs null it allocates nothing.
hipError_t split_area_take_stalls(const SplitArea* a, hipStream_t s, uint32_t* count, std::vector<int>* jobs);

// Blind rotation + sample extraction (or raw accumulator output) of njobs
// jobs.  ex: extract buffer, N+1 words per slot (2N per slot when raw_acc).
// waves_per_job: 1 (one wave per bootstrap), 2 (one wave per accumulator
// component, two bootstraps per SIMD), 3 (one wave per gadget level),
// 4 (three level waves, the levels' NTT-domain sum inverted once per
// component on two waves each; one bootstrap per CU), 5 (the same, two
// bootstraps per CU), 6 (split over two workgroups of four waves; needs
// `split` with room for njobs) or 7 (the same, two workgroups per CU).
// d_pool_tab (may be null) resolves operands with base KEY_POOL_BASE to the
// pool of the job's key.
hipError_t launch_blind_rotate(const BrJob* d_jobs, int njobs, const SrcBases& src, uint32_t* d_ex,
                               const uint64_t* const* d_bsk_tab, uint32_t* const* d_pool_tab, int n_lwe,
                               int steps, int raw_acc, Twiddles tw, int waves_per_job, hipStream_t s,
                               const SplitArea* split = nullptr);

// The split rotation's launch (waves_per_job 6 or 7), in split.hip; `split`
// must have room for njobs, and njobs is at most split_max_jobs(waves).
hipError_t launch_split(const BrJob* d_jobs, int njobs, const SrcBases& src, uint32_t* d_ex,
                        const uint64_t* const* d_bsk_tab, uint32_t* const* d_pool_tab, int n_lwe, int steps,
                        int raw_acc, Twiddles tw, int waves_per_job, const SplitArea* split, hipStream_t s);

// The split rotation's profiling instantiation (waves_per_job 6, raw
// accumulators into d_ex): every wave of every workgroup writes, at
// d_prof + (block * 4 + wave) * kSplitPhaseWords, its shader cycles in each
// of the kSplitPhaseWords - 1 phases of a step summed over its executed
// steps, then that step count.  The phases: [0] digits and key requests;
// [1] the barrier after them; [2] the forward transform and its copy to
// LDS; [3] the barrier after it; [4] the partner component's key products
// and their stores; [5] the wait for those stores and the flag; [6] the
// wait for the partner's flag; [7] loading the partner's products, this
// half's own and the sum; [8] the inverse's first pass and twist; [9] the barrier inside
// the inverse; [10] its second pass and the accumulator update; [11] the
// closing barrier.
constexpr int kSplitPhaseWords = 13;
hipError_t launch_split_profiled(const BrJob* d_jobs, int njobs, const SrcBases& src, uint32_t* d_ex,
                                 const uint64_t* const* d_bsk_tab, int n_lwe, int steps, Twiddles tw,
                                 int waves_per_job, const SplitArea* split, uint64_t* d_prof, hipStream_t s);

// Key switching of njobs jobs (tiles of `tile` consecutive jobs share one
// key; jobs with ex0 == REF_NONE are padding and skipped); the ring index is
// split into `isplit` ranges (N divisible by 64 isplit).
hipError_t launch_keyswitch(const KsJob* d_jobs, int njobs, const uint32_t* d_ex, const DstBases& dst,
                            const uint32_t* const* d_ksk_tab, uint32_t* const* d_pool_tab, int n_lwe, int N,
                            int ks_t, int ks_base_bit, int tile, int isplit, hipStream_t s);

// Descriptors of cnt equal gates on arrays in0/in1/in2 (bases 0, 1, 2).
// nbr = 1: one blind rotation per gate with (cst, c0*in0 + c1*in1);
// nbr = 2 (MUX): rotations (sel AND t) and (NOT sel AND f), one key switch
// of their sum plus 1/8.
hipError_t launch_make_batch_jobs(int nbr, uint32_t cst, int32_t c0, int32_t c1, int has_in1,
                                  size_t cnt, BrJob* d_br, KsJob* d_ks, hipStream_t s);

// out[k] = sign * in[k] over cnt samples of `words` words (NOT, COPY).
hipError_t launch_lwe_scale(const uint32_t* d_in, uint32_t* d_out, size_t words, int32_t sign,
                            hipStream_t s);

// out[j] = src[ref[j] + index_offset] for cnt LWE_n samples.
hipError_t launch_gather(const uint32_t* d_refs, int cnt, const SrcBases& src, uint32_t index_offset,
                         uint32_t* d_out, int n_lwe, hipStream_t s);

// Field-operation throughput (csrc/oprate.hip): each operation alone at full
// occupancy in a launch sized to about target_ms; rates[op] receives
// operations per second on the whole device, ms[op] (may be null) the timed
// launch.  Synchronous.
enum { kOpFwd = 0, kOpInv = 1, kOpDigits = 2, kOpMul = 3, kOpMulSum = 4, kOpAdd = 5, kOpU32 = 6, kOpCount = 7 };
hipError_t launch_op_rates(double target_ms, double* rates, double* ms, hipStream_t s);

// The external product of one blind-rotation step on the int8 matrix cores
// (csrc/extprod_mfma.hip): d_out[b] = sum_r dec_r(d_in[b]) * key[r] for cnt
// TRLWE inputs [cnt][2][1024]; key: the step's 2l = 6 key rows [6][2][1024]
// in Torus32 form.  scratch: xp_mfma_scratch_bytes(cnt) device bytes.
size_t xp_mfma_scratch_bytes(int cnt);
hipError_t launch_extprod_mfma(const uint32_t* d_key_step, const uint32_t* d_in, int cnt, uint32_t* d_out,
                               void* scratch, hipStream_t s);

// cnt exact negacyclic products (digits x NTT-domain polynomial) mod 2^32.
hipError_t launch_debug_polymul(const int32_t* d_digits, const uint64_t* d_poly_ntt, uint32_t* d_out,
                                int cnt, Twiddles tw, hipStream_t s);

}  // namespace lp
