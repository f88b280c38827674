// The split blind rotation: one gate bootstrap on two workgroups, normally
// on two CUs of one XCD, for circuit levels too narrow to fill the GPU; its
// exchange area and launches.  A translation unit of its own, so that it
// can be compiled with the scheduler that favours instruction-level
// parallelism: one wave per SIMD gains from it, the kernels at two waves
// per SIMD lose registers to it (kernels.hip).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdlib>
#include <vector>

#include "gl64.h"
#include "jobs.h"
#include "kernel_util.h"
#include "kernels.h"
#include "ntt64.h"

namespace lp {

// ---------------------------------------------------------------------------
// Split blind rotation: one bootstrap on two workgroups of four waves,
// normally on two CUs of one XCD, for levels too narrow to fill the GPU.
// Workgroup role c owns accumulator component c (0 = mask A, 1 = body B);
// its wave j < 3 runs the forward transform of gadget level j (whole-wave
// transforms, ntt64.h).  Output component c needs the digits of both
// components,
//   S_c = sum_j NTT(d_(c,j)) BSK[(c,j)][c] + sum_j NTT(d_(1-c,j)) BSK[(1-c,j)][c],
// so every step each role forms its own half of S_c and the half of
// S_(1-c) its digits contribute, and trades the latter with its partner:
//   1. D_c = X^a ACC_c - ACC_c, digits of level j -> forward NTT F_(c,j)
//      on wave j, copied to LDS;
//   2. all four waves, each at the 256 NTT-domain positions its part of
//      the inverse reads (eight lanes per row, ntt64.h): the two sums over
//      the levels, sum_j F_(c,j) BSK[(c,j)][c] and sum_j F_(c,j)
//      BSK[(c,j)][1-c], one reduction each;
//   3. wave w stores the second sum in its slot of this role's exchange
//      area, raises its flag to the step count, waits for the partner
//      wave w's flag and loads the partner's sum for these positions;
//   4. the four waves invert S_c together and add its centred lift to ACC_c.
// When both halves run on one XCD, exchange data and flags go through that
// XCD's L2 (plain stores, device-scope loads); otherwise they are
// agent-scope relaxed atomics.  Either way a full vector memory wait orders
// the data before the flag, and the data loads follow the observed flag.
// Slots alternate by the parity of the executed-step
// count: a role rewrites a slot only after the partner has raised its flag
// for the following step, which it does after its loads of that slot.
//
// Pairing: a workgroup draws a ticket on arrival from the counter of its
// class x = blockIdx % 8 (the XCD that round-robin dispatch gives it);
// tickets 2k and 2k + 1 of a class form a pair (job 8 k + x, role t & 1).
// Arrival order is not launch order, so pairing by class rather than by
// arrival keeps both halves on one XCD.  The grid is a multiple of 16, so
// every class holds an even count and every ticket finds its partner; at
// most one workgroup per class waits for a partner, so no co-residency is
// assumed.  Every wait is bounded:
// a partner missing for SPLIT_SPIN_LIMIT polls ends the wait, counts in
// g_split_stalls and in the area's own status word, marks the job, and the
// job's output is then undefined; the kernel still exits.  Each half
// clears its step flags when it starts, and the last workgroup to finish
// clears the tickets and the XCD-id words; the status word and the
// job marks stay until the host has read them (split_area_take_stalls), so
// every call that launched the kernel can report a give-up as an error.
constexpr int SPLIT_SPIN_LIMIT = 1 << 22;
constexpr int SPLIT_DONE = 8;    // finish counter (words 0-7: ticket counters per class)
constexpr int SPLIT_STATUS = 9;  // waits of this area that ran out, until the host clears it
constexpr int SPLIT_FLAGS = 64;  // first flag word of the sync area
constexpr int SPLIT_FLAGS_PER_JOB = 16;  // [role 2][8]: the four waves' step flags, then the XCD id in word 7

__device__ uint32_t g_split_stalls;

// Accesses of an exchange between two workgroups on one XCD, through that
// XCD's L2 (the coherence point of its CUs): plain stores, which write
// through the CU's L1 into the L2; loads with sc1 (device scope), which miss
// the reading CU's L1 and are served by the L2.  Agent-scope stores would
// write through to memory and reach the partner several times later.
// Buffer resources (raw, no stride) over the exchange slots and the sync
// words.  No access is volatile: the compiler would complete each volatile
// access before the next one (and widen it to system scope).  Order comes
// from an explicit wait for the data stores before the flag store, a
// compiler memory barrier in every poll iteration (so the flag is read
// anew) and one after the poll.
//
// Such plain stores may leave the lines dirty in that L2 until the kernel
// ends, when every L2 writes its dirty bytes back.  So no word an exchange
// writes this way may be written from another XCD during the same launch:
// each workgroup clears its own step flags at its start (before it announces
// itself to its partner) rather than the last workgroup clearing all of
// them at the end.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t l2_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
constexpr int kL2Load = 0x10;  // sc1
__device__ __forceinline__ void st_l2(__amdgpu_buffer_rsrc_t r, uint32_t off, uint64_t v) {
  const u32x2 x = {(uint32_t)v, (uint32_t)(v >> 32)};
  __builtin_amdgcn_raw_buffer_store_b64(x, r, off, 0, 0);
}
__device__ __forceinline__ uint64_t ld_l2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kL2Load);
  return ((uint64_t)x.y << 32) | x.x;
}
__device__ __forceinline__ void st_l2_u32(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, 0);
}
__device__ __forceinline__ uint32_t ld_l2_u32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  asm volatile("" ::: "memory");
  return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kL2Load);
}
// The XCD this wave runs on.
__device__ __forceinline__ uint32_t xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20); }

// Rows of NTT-domain values in LDS with eight spare words after every 64:
// offset o sits at o + 8 (o >> 6).  The split rotation reads them at the
// inverse's positions (lane 8 r + h of wave w: 64 (h >> 1) + 16 w + 2 r +
// (h & 1) + 256 s), where plain rows put four lanes of each half-wave on
// one bank pair; the padding moves (h >> 1) onto banks 8 apart.
constexpr int KROW = RING_N + RING_N / 8;
__device__ __forceinline__ int kpad(int o) { return o + 8 * (o >> 6); }

// Per-wave cycle counts of the phases of a split step (the profiling
// instantiation only; the production one compiles none of it).  mark<K>()
// adds the shader cycles since the previous mark to phase K; store() writes
// phases 0..kPhases-1 and the executed-step count for this wave.
// Scheduling barriers around each clock read keep the compiler from moving
// work across a phase boundary (the profiling build schedules a little
// differently for it).
constexpr int kSplitPhases = 12;
template <bool PROF>
struct PhaseClock {
  uint64_t t = 0;
  uint64_t acc[kSplitPhases] = {};
  __device__ __forceinline__ void start() {
    if constexpr (PROF) {
      __builtin_amdgcn_sched_barrier(0);
      t = __builtin_amdgcn_s_memtime();
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  template <int K>
  __device__ __forceinline__ void mark() {
    if constexpr (PROF) {
      __builtin_amdgcn_sched_barrier(0);
      const uint64_t n = __builtin_amdgcn_s_memtime();
      __builtin_amdgcn_sched_barrier(0);
      acc[K] += n - t;
      t = n;
    }
  }
  __device__ __forceinline__ void store(uint64_t* out, int lane, uint32_t done) {
    if constexpr (PROF) {
      if (out && lane == 0) {
#pragma unroll
        for (int k = 0; k < kSplitPhases; ++k) out[k] = acc[k];
        out[kSplitPhases] = done;
      }
    }
  }
};

// DUAL: the same rotation sized for two workgroups per CU (launches of up to
// kSplitDualMaxJobs jobs), in at most half the CU's LDS: the fourth wave
// stages only the partner's three key rows and each wave loads its own-sum
// rows from global memory while it waits for the partner; the inverse
// twist comes from global memory; the forward transposes use the wave's
// partial-sum row, and D uses the inverse's transpose block (each read
// before the next write of the aliased space, at the step's barriers).
template <bool PROF, bool DUAL>
__global__ __launch_bounds__(256, DUAL ? 2 : 1) void blind_rotate_split_kernel(
    const BrJob* __restrict__ jobs, int njobs, SrcBases src, uint32_t* __restrict__ ex_out,
    const uint64_t* const* __restrict__ bsk_tab, uint32_t* const* __restrict__ pool_tab, int n_lwe, int steps,
    int raw_acc, const uint64_t* __restrict__ tw_f, const uint64_t* __restrict__ tw_i, uint64_t* __restrict__ xbuf,
    uint32_t* __restrict__ sync, uint32_t* __restrict__ marks, int spin_limit, int allow_l2,
    uint64_t* __restrict__ prof) {
  __shared__ uint32_t s_acc[RING_N];
  __shared__ __align__(16) uint32_t s_tr[DUAL ? 1 : 3][DUAL ? 1 : LDS_HALF];
  // the levels' forward transforms and the step's key rows (c, j), both
  // output components (DUAL: the partner's only), NTT domain, rows padded
  // (kpad) for conflict-free reads at the inverse's positions
  __shared__ __align__(16) uint64_t s_part[3][KROW];
  __shared__ __align__(16) uint64_t s_key[DUAL ? 3 : 6][KROW];
  __shared__ uint32_t s_Dn[DUAL ? 1 : RING_N];
  __shared__ __align__(16) uint64_t s_t128[32 * T128_ROW];  // two-wave transpose
  // the twist tables, read every step at LDS latency instead of L2's (DUAL:
  // the forward one)
  __shared__ __align__(16) uint64_t s_twf[RING_N], s_twi[DUAL ? 1 : RING_N];
  __shared__ uint16_t s_abar[MAX_LWE + 4];
  __shared__ uint32_t s_ticket, s_last, s_local;
  // X^a ACC_c - ACC_c
  uint32_t* const s_D = DUAL ? reinterpret_cast<uint32_t*>(s_t128) : s_Dn;

  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, h = lane >> 5, l = lane & 31;
  const uint32_t h6 = 6u * (uint32_t)h;  // the lane's extra shift in a paired distance-1 stage
  const bool lvl = wave < 3;  // waves 0-2 run the gadget levels; all four invert
  // four-wave inverse: row (or column) 8 wave + r8, lane h8 of the row's eight
  const int r8 = lane >> 3, h8 = lane & 7, row = 8 * wave + r8;
  const uint64_t upper1 = (h8 & 1) ? ~0ull : 0ull, upper2 = (h8 & 2) ? ~0ull : 0ull,
                 upper4 = (h8 & 4) ? ~0ull : 0ull;
  uint64_t tw2[5], tw1[5];  // the lane's inverse twiddles of passes 2 and 1
  inv256_twiddles(2, h8, tw2);
  inv256_twiddles(1, h8, tw1);
  for (int k = threadIdx.x; k < RING_N; k += 256) {
    // forward entry 64 r + lane: the factor of register r of that lane in
    // the pair layout that the forward's first pass leaves
    s_twf[k] = tw_f[pair_pos(k >> 6, (k >> 5) & 1) * 32 + (k & 31)];
    if constexpr (!DUAL) s_twi[k] = tw_i[k];
  }
  const int cls = (int)(blockIdx.x & 7u);
  if (threadIdx.x == 0) s_ticket = atomicAdd(sync + cls, 1u);
  __syncthreads();
  const uint32_t t = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_ticket);
  const int job = (int)(t >> 1) * 8 + cls;
  const int c = (int)(t & 1u);

  if (job < njobs) {
    const BrJob J = jobs[job];
    uint32_t* buf = DUAL ? reinterpret_cast<uint32_t*>(s_part[lvl ? wave : 0]) : s_tr[lvl ? wave : 0];
    {
      auto operand = [&](uint32_t r) -> const uint32_t* {
        if (r == REF_NONE) return nullptr;
        const uint32_t base = r >> REF_SHIFT;
        const uint32_t* b = base == KEY_POOL_BASE ? pool_tab[J.key] : src.p[base];
        return b + (size_t)(r & REF_INDEX_MASK) * (n_lwe + 1);
      };
      const uint32_t* in0 = operand(J.in0);
      const uint32_t* in1 = operand(J.in1);
      for (int k = threadIdx.x; k <= n_lwe; k += 256) {
        uint32_t v = (k == n_lwe) ? J.cst : 0u;
        if (in0) v += (uint32_t)J.c0 * in0[k];
        if (in1) v += (uint32_t)J.c1 * in1[k];
        s_abar[k] = (uint16_t)(((v + (1u << 20)) >> 21) & 2047u);
      }
    }
    __syncthreads();
    // ACC_0 = 0, ACC_1 = X^{-b} v (coefficient j: +1/8 if (j + b) mod 2N < N)
    const uint32_t bbar = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_abar[n_lwe]);
    for (int j = threadIdx.x; j < RING_N; j += 256)
      s_acc[j] = c == 0 ? 0u : ((((uint32_t)j + bbar) & 2047u) < 1024u ? 0x20000000u : 0xE0000000u);
    __syncthreads();

    const gmem_u64* bsk = as_global(bsk_tab[J.key]);
    const int nsteps = steps < n_lwe ? steps : n_lwe;
    // wave w trades with the partner's wave w: the partner's component of the
    // key products at the NTT-domain offsets both waves' inverses read
    uint64_t* my_x = xbuf + (size_t)(job * 2 + c) * 2 * RING_N;
    const uint64_t* peer_x = xbuf + (size_t)(job * 2 + (1 - c)) * 2 * RING_N;
    uint32_t* my_flag = sync + SPLIT_FLAGS + job * SPLIT_FLAGS_PER_JOB + c * 8 + wave;
    const uint32_t* peer_flag = sync + SPLIT_FLAGS + job * SPLIT_FLAGS_PER_JOB + (1 - c) * 8 + wave;
    const int sh = 25 - 7 * wave;
    uint32_t done = 0;  // executed steps, the same count in both roles
    bool stalled = false;
    PhaseClock<PROF> pc;
    // Both halves on one XCD (the normal placement of the class pairing)
    // trade through that XCD's L2, unless the launch forbids it (allow_l2 =
    // 0); otherwise past it, as agent-scope accesses.  Each half clears its own step flags, then publishes its XCD
    // id in its spare flag word 7; the partner reads its flags only after
    // that word (bounded wait as for the products).  Word 7 is only ever
    // accessed at agent scope, and the last workgroup clears it.
    const uint32_t my_xcc = xcc_id();
    if (threadIdx.x == 0) {
      uint32_t* mine = sync + SPLIT_FLAGS + job * SPLIT_FLAGS_PER_JOB + c * 8;
      for (int w = 0; w < 4; ++w) store_agent(mine + w, 0u);
      vm_wait_all();
      store_agent(mine + 7, my_xcc + 1);
      const uint32_t* px = sync + SPLIT_FLAGS + job * SPLIT_FLAGS_PER_JOB + (1 - c) * 8 + 7;
      uint32_t v = 0;
      for (int it = 0; it < spin_limit && (v = load_agent(px)) == 0; ++it) __builtin_amdgcn_s_sleep(1);
      s_local = allow_l2 && v == my_xcc + 1 ? 1u : 0u;
    }
    __syncthreads();
    const bool local = __builtin_amdgcn_readfirstlane((int)s_local) != 0;
    const __amdgpu_buffer_rsrc_t xr = l2_rsrc(xbuf, (gridDim.x / 2) * 4u * RING_N * 8u);
    const __amdgpu_buffer_rsrc_t fr = l2_rsrc(sync, (SPLIT_FLAGS + (gridDim.x / 2) * SPLIT_FLAGS_PER_JOB) * 4u);
    const uint32_t my_xo = (uint32_t)(my_x - xbuf) * 8u, peer_xo = (uint32_t)(peer_x - xbuf) * 8u;
    const uint32_t my_fo = (uint32_t)(my_flag - sync) * 4u, peer_fo = (uint32_t)(peer_flag - sync) * 4u;
    // this lane's four inverse positions (row `row`, q = 4 h8 + s): their
    // NTT-domain offsets 64 (q >> 1) + 2 row + (q & 1) in the padded rows
    int po[4], og[4];  // og: the same offsets in an unpadded key row (DUAL's own rows)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      og[s] = 128 * h8 + 64 * (s >> 1) + 2 * row + (s & 1);
      po[s] = kpad(og[s]);
    }

    for (int i = 0; i < nsteps; ++i) {
      const uint32_t a = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_abar[i]);
      if (a == 0) continue;  // X^0 ACC - ACC = 0: no digits, no exchange
      pc.start();

      // D = X^a ACC_c - ACC_c (coefficient k: ACC_c[(k - a) mod 2N] with the
      // negacyclic sign, minus ACC_c[k]), four coefficients per thread
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t k = threadIdx.x + 256u * q;
        const uint32_t e = (k - a) & 2047u;
        const uint32_t v = s_acc[e & 1023u];
        s_D[k] = ((e & 1024u) ? (0u - v) : v) - s_acc[k];
      }
      pc.template mark<0>();
      __syncthreads();  // D is complete, and every wave has read ACC_c before any adds to it
      pc.template mark<1>();
      const gmem_u64* step_key = bsk + (size_t)i * 6 * 2 * RING_N;
      if (lvl) {
        int32_t dg[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          const uint32_t D = s_D[l + 32 * (2 * s + h)];
          dg[s] = (int32_t)(((D + 0x81020400u) >> sh) & 127u) - 64;
        }
        // forward transform, both passes ending in the paired distance-1
        // stage; register r then holds row l, position q = pair_pos(r, h),
        // whose NTT-domain offset is 64 (q >> 1) + 2 l + (q & 1)
        uint64_t f[16];
        fwd64_p1_digits(dg, f);
        fwd64_p1_rest_pairs(f, h6);
#pragma unroll
        for (int s = 0; s < 16; ++s) f[s] = gl_mul(f[s], s_twf[64 * s + lane]);
        transpose64_pairs(f, buf, h, l);
        fwd64_p2_pairs(f, h6);
#pragma unroll
        for (int r = 0; r < 16; ++r) s_part[wave][kpad(512 * h + 64 * (r & 7) + 2 * l + (r >> 3))] = f[r];
      } else {
        // meanwhile the fourth wave stages the step's key rows (c, j) in
        // LDS: row 2 j + 0 for output component c, 2 j + 1 for 1 - c (DUAL:
        // row j for 1 - c only)
#pragma unroll 1
        for (int r = 0; r < (DUAL ? 3 : 6); ++r) {
          const int j = DUAL ? r : r >> 1, comp = (DUAL || (r & 1)) ? 1 - c : c;
          const gmem_u64* src_row = step_key + (size_t)((c * 3 + j) * 2 + comp) * RING_N;
          uint64_t t[16];
#pragma unroll
          for (int k = 0; k < 16; ++k) t[k] = src_row[lane + 64 * k];
#pragma unroll
          for (int k = 0; k < 16; ++k) s_key[r][kpad(lane + 64 * k)] = t[k];
        }
      }
      pc.template mark<2>();
      __syncthreads();
      pc.template mark<3>();

      // the partner's component of the products, summed over the levels
      // with one reduction, goes out first; this half's own follows while
      // the partner's is on its way
      uint64_t F[3][4], oth[4];
      // DUAL: this half's own key rows at the same positions, from global
      // memory, requested first: they arrive while the partner's sums are
      // formed, so the wait that orders the exchange stores does not also
      // wait for them
      uint64_t kown[3][4];
      if constexpr (DUAL) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const gmem_u64* kr = step_key + (size_t)((c * 3 + j) * 2 + c) * RING_N;
#pragma unroll
          for (int s = 0; s < 4; ++s) kown[j][s] = kr[og[s]];
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int j = 0; j < 3; ++j) F[j][s] = s_part[j][po[s]];
        oth[s] = gl_mul_sum3(F[0][s], s_key[DUAL ? 0 : 1][po[s]], F[1][s], s_key[DUAL ? 1 : 3][po[s]], F[2][s],
                             s_key[DUAL ? 2 : 5][po[s]]);
      }

      const uint32_t par = (done & 1u) * RING_N;
      const uint32_t slot = par + 64 * wave + lane;  // + 256 s
      if (local) {
#pragma unroll
        for (int s = 0; s < 4; ++s) st_l2(xr, my_xo + (slot + 256 * s) * 8u, oth[s]);
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) store_agent(my_x + slot + 256 * s, oth[s]);
      }
      pc.template mark<4>();
      vm_wait_all();
      if (lane == 0) {
        if (local) st_l2_u32(fr, my_fo, done + 1);
        else store_agent(my_flag, done + 1);
      }
      pc.template mark<5>();
      if (!stalled) {
        int it = 0;
        while ((local ? ld_l2_u32(fr, peer_fo) : load_agent(peer_flag)) < done + 1) {
          if (++it >= spin_limit) break;
          __builtin_amdgcn_s_sleep(1);
        }
        if (it >= spin_limit) {
          stalled = true;
          if (lane == 0) {
            atomicAdd(&g_split_stalls, 1u);
            atomicAdd(sync + SPLIT_STATUS, 1u);
            store_agent(marks + job, 1u);
          }
        }
      }
      asm volatile("" ::: "memory");  // the partner's products are read after its flag
      pc.template mark<6>();
      uint64_t v[4];
      if (local) {
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = ld_l2(xr, peer_xo + (slot + 256 * s) * 8u);
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = load_agent(peer_x + slot + 256 * s);
      }
      uint64_t own[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if constexpr (DUAL) own[s] = gl_mul_sum3(F[0][s], kown[0][s], F[1][s], kown[1][s], F[2][s], kown[2][s]);
        else own[s] = gl_mul_sum3(F[0][s], s_key[0][po[s]], F[1][s], s_key[2][po[s]], F[2][s], s_key[4][po[s]]);
      }
      // every own product before the first wait for the partner's (ordered
      // empty asm statements that the sums depend on)
#pragma unroll
      for (int s = 0; s < 4; ++s) asm volatile("" : "+v"(own[s]));
#pragma unroll
      for (int s = 0; s < 4; ++s) v[s] = gl_add(own[s], v[s]);
      pc.template mark<7>();

      // one inverse of the sum on all four waves: each holds eight rows at
      // eight lanes per row; each pass leaves register s at position
      // h8 + 8 (s >> 1) + 16 (s & 1)
      {
        uint64_t twv[4];  // DUAL: the inverse twist factors, requested ahead of the pass
        if constexpr (DUAL) {
#pragma unroll
          for (int s = 0; s < 4; ++s) twv[s] = as_global(tw_i)[(h8 + 8 * (s >> 1) + 16 * (s & 1)) * 32 + row];
        }
        inv256_pass<2>(v, upper1, upper2, upper4, tw2);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int j = h8 + 8 * (s >> 1) + 16 * (s & 1);
          s_t128[row * T128_ROW + j] = gl_mul(v[s], DUAL ? twv[s] : s_twi[j * 32 + row]);
        }
        pc.template mark<8>();
        __syncthreads();
        pc.template mark<9>();
        // column j1 = row of this lane, positions q = 4 h8 + s
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = s_t128[(4 * h8 + s) * T128_ROW + row];
        inv256_pass<1>(v, upper1, upper2, upper4, tw1);
        // the sum is an exact integer polynomial (|coefficient| < 2^50.6),
        // so its centred lift reduced mod 2^32 is exact
#pragma unroll
        for (int s = 0; s < 4; ++s) s_acc[row + 32 * (h8 + 8 * (s >> 1) + 16 * (s & 1))] += gl_lift_u32(v[s]);
      }
      pc.template mark<10>();
      ++done;
      __syncthreads();
      pc.template mark<11>();
    }
    pc.store(prof ? prof + ((size_t)blockIdx.x * 4 + wave) * kSplitPhaseWords : nullptr, lane, done);

    if (raw_acc) {
      uint32_t* o = ex_out + (size_t)J.out * (2 * RING_N) + c * RING_N;
      for (int j = threadIdx.x; j < RING_N; j += 256) o[j] = s_acc[j];
    } else {
      // sample extraction at coefficient 0: a'_0 = A_0, a'_j = -A_{N-j}, b' = B_0
      uint32_t* o = ex_out + (size_t)J.out * (RING_N + 1);
      if (c == 0) {
        for (int j = threadIdx.x; j < RING_N; j += 256) {
          if (j == 0) o[0] = s_acc[0];
          else o[RING_N - j] = 0u - s_acc[j];
        }
      } else if (threadIdx.x == 0) {
        o[RING_N] = s_acc[0];
      }
    }
  }

  // the last workgroup to finish clears the tickets and the XCD-id words
  // for the next launch on this area (every other one has finished using
  // them); the step flags are their owners' to clear
  vm_wait_all();
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(sync + SPLIT_DONE, 1u) == gridDim.x - 1 ? 1u : 0u;
  __syncthreads();
  if (s_last) {
    const int nroles = (int)gridDim.x;  // two roles per job slot
    for (int k = threadIdx.x; k < nroles; k += 256) store_agent(sync + SPLIT_FLAGS + k * 8 + 7, 0u);
    if (threadIdx.x <= SPLIT_DONE) store_agent(sync + threadIdx.x, 0u);  // the 8 class counters and the finish count
  }
}

__global__ void split_area_clear_kernel(uint32_t* sync, int words) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < words) sync[k] = 0u;
}

// ---------------------------------------------------------------------------
// Host side: launches, the exchange area and its give-up record.
int split_spin_limit();
static int split_allow_l2();
static int split_jobs_padded(int max_jobs) { return (max_jobs + 7) / 8 * 8; }
// sync area: 64 control words, 16 flag words per job, then one give-up mark per job
static size_t split_marks_offset(int max_jobs) {
  return (size_t)SPLIT_FLAGS + (size_t)split_jobs_padded(max_jobs) * SPLIT_FLAGS_PER_JOB;
}

hipError_t launch_split(const BrJob* d_jobs, int njobs, const SrcBases& src, uint32_t* d_ex,
                        const uint64_t* const* d_bsk_tab, uint32_t* const* d_pool_tab, int n_lwe, int steps,
                        int raw_acc, Twiddles tw, int waves_per_job, const SplitArea* split, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  if (!is_split(waves_per_job) || njobs > split_max_jobs(waves_per_job) || !split || !split->xbuf ||
      !split->sync || njobs > split->max_jobs)
    return hipErrorInvalidValue;
  const int grid = 16 * ((njobs + 7) / 8);
  auto kernel = waves_per_job == 7 ? blind_rotate_split_kernel<false, true> : blind_rotate_split_kernel<false, false>;
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(256), 0, s, d_jobs, njobs, src, d_ex, d_bsk_tab, d_pool_tab, n_lwe,
                     steps, raw_acc, tw.fwd, tw.inv, split->xbuf, split->sync,
                     split->sync + split_marks_offset(split->max_jobs), split_spin_limit(), split_allow_l2(),
                     nullptr);
  return hipGetLastError();
}

hipError_t launch_split_profiled(const BrJob* d_jobs, int njobs, const SrcBases& src, uint32_t* d_ex,
                                 const uint64_t* const* d_bsk_tab, int n_lwe, int steps, Twiddles tw,
                                 int waves_per_job, const SplitArea* split, uint64_t* d_prof, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  if (!is_split(waves_per_job) || njobs > split_max_jobs(waves_per_job) || !split || !split->xbuf ||
      !split->sync || njobs > split->max_jobs || !d_prof)
    return hipErrorInvalidValue;
  const int grid = 16 * ((njobs + 7) / 8);
  auto kernel = waves_per_job == 7 ? blind_rotate_split_kernel<true, true> : blind_rotate_split_kernel<true, false>;
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(256), 0, s, d_jobs, njobs, src, d_ex, d_bsk_tab, nullptr, n_lwe,
                     steps, 1, tw.fwd, tw.inv, split->xbuf, split->sync,
                     split->sync + split_marks_offset(split->max_jobs), split_spin_limit(), split_allow_l2(),
                     d_prof);
  return hipGetLastError();
}

// Polls of a split wait before it gives up: SPLIT_SPIN_LIMIT, or a smaller
// positive LOCPIR_SPLIT_SPIN (tests force the give-up path with it; every
// wave still runs to the end).
// Whether pairs on one XCD may trade through its L2: 1, or 0 when
// LOCPIR_SPLIT_AGENT=1 makes every pair trade at agent scope, as pairs on
// two XCDs do (tests cover that path with it).
static int split_allow_l2() {
  const char* v = std::getenv("LOCPIR_SPLIT_AGENT");
  return (v && v[0] == '1') ? 0 : 1;
}

int split_spin_limit() {
  const char* v = std::getenv("LOCPIR_SPLIT_SPIN");
  const long x = (v && *v) ? std::atol(v) : 0;
  return x > 0 && x < SPLIT_SPIN_LIMIT ? (int)x : SPLIT_SPIN_LIMIT;
}
size_t split_xbuf_bytes(int max_jobs) { return (size_t)split_jobs_padded(max_jobs) * 4 * RING_N * 8; }
size_t split_sync_bytes(int max_jobs) {
  return (split_marks_offset(max_jobs) + split_jobs_padded(max_jobs)) * 4;
}

hipError_t split_area_take_stalls(const SplitArea* a, hipStream_t s, uint32_t* count, std::vector<int>* jobs) {
  if (!a || !count) return hipErrorInvalidValue;
  *count = 0;
  if (jobs) jobs->clear();
  if (!a->sync) return hipSuccess;
  uint32_t st = 0;
  hipError_t e = hipMemcpyAsync(&st, a->sync + SPLIT_STATUS, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess || st == 0) return e;
  const int padded = split_jobs_padded(a->max_jobs);
  uint32_t* dm = a->sync + split_marks_offset(a->max_jobs);
  if (jobs) {
    std::vector<uint32_t> marks(padded);
    e = hipMemcpyAsync(marks.data(), dm, (size_t)padded * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (int j = 0; j < padded; ++j)
      if (marks[j]) jobs->push_back(j);
  }
  // clear the status word and the marks for the next launch on this area
  hipLaunchKernelGGL(split_area_clear_kernel, dim3(1), dim3(256), 0, s, a->sync + SPLIT_STATUS, 1);
  hipLaunchKernelGGL(split_area_clear_kernel, dim3((padded + 255) / 256), dim3(256), 0, s, dm, padded);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  *count = st;
  return e;
}

hipError_t launch_clear_words(uint32_t* d, size_t words, hipStream_t s) {
  if (words == 0) return hipSuccess;
  if (!d || words > (size_t)INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(split_area_clear_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, d, (int)words);
  return hipGetLastError();
}

hipError_t split_area_alloc(SplitArea* a, int max_jobs) {
  if (!a || max_jobs < 1 || max_jobs > kSplitDualMaxJobs) return hipErrorInvalidValue;
  *a = SplitArea{};
  hipError_t e = hipMalloc((void**)&a->xbuf, split_xbuf_bytes(max_jobs));
  if (e == hipSuccess) e = hipMalloc((void**)&a->sync, split_sync_bytes(max_jobs));
  if (e == hipSuccess) e = hipMemset(a->sync, 0, split_sync_bytes(max_jobs));
  if (e != hipSuccess) {
    split_area_free(a);
    return e;
  }
  a->max_jobs = max_jobs;
  return hipSuccess;
}

void split_area_free(SplitArea* a) {
  if (!a) return;
  if (a->xbuf) (void)hipFree(a->xbuf);
  if (a->sync) (void)hipFree(a->sync);
  *a = SplitArea{};
}

hipError_t split_area_alloc_async(SplitArea* a, int max_jobs, hipStream_t s) {
  if (!a || max_jobs < 1 || max_jobs > kSplitDualMaxJobs) return hipErrorInvalidValue;
  *a = SplitArea{};
  hipError_t e = hipMallocAsync((void**)&a->xbuf, split_xbuf_bytes(max_jobs), s);
  if (e == hipSuccess) e = hipMallocAsync((void**)&a->sync, split_sync_bytes(max_jobs), s);
  if (e == hipSuccess) {
    const int words = (int)(split_sync_bytes(max_jobs) / 4);
    hipLaunchKernelGGL(split_area_clear_kernel, dim3((words + 255) / 256), dim3(256), 0, s, a->sync, words);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    (void)split_area_free_async(a, s);
    return e;
  }
  a->max_jobs = max_jobs;
  return hipSuccess;
}

hipError_t split_area_free_async(SplitArea* a, hipStream_t s) {
  if (!a) return hipSuccess;
  hipError_t e = hipSuccess;
  if (a->xbuf) e = hipFreeAsync(a->xbuf, s);
  if (a->sync) {
    const hipError_t e2 = hipFreeAsync(a->sync, s);
    if (e == hipSuccess) e = e2;
  }
  *a = SplitArea{};
  return e;
}

hipError_t split_stall_count(uint32_t* out) {
  if (!out) return hipErrorInvalidValue;
  return hipMemcpyFromSymbol(out, HIP_SYMBOL(g_split_stalls), sizeof(uint32_t), 0, hipMemcpyDeviceToHost);
}

}  // namespace lp
