// gfx950 kernels of the gate bootstrap: NTT-domain key conversion, the
// blind rotation (CMux external products) with sample extraction, key
// switching, and small helpers.
//
// Blind rotation layout (one 64-lane wave per bootstrap):
//   half-wave h = lane / 32 owns accumulator component h (0 = mask A,
//   1 = body B); lane l = lane % 32 holds coefficients l + 32 m, m < 32, of
//   that component in registers.  Each step i:
//     1. D_h = X^{a_i} ACC_h - ACC_h via this half's LDS block;
//     2. for each gadget level j: digits of D_h -> forward NTT (first two
//        stages fused with the digit extraction); the transform crosses to
//        the other half (lane ^ 32), and half h accumulates output component h
//        = NTT(d_(h,j)) BSK_i[(h,j)][h] + NTT(d_(1-h,j)) BSK_i[(1-h,j)][h]
//        with one modular reduction per coefficient;
//     3. inverse NTT of the accumulated component, centred lift mod 2^32,
//        ACC_h += result.
//   The bootstrapping key is streamed from global memory in the NTT
//   domain, laid out [i][row][q][slot pair][lane][2] so that each half-wave
//   reads 512 contiguous bytes per 16-byte load.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdlib>

#include "gl64.h"
#include "jobs.h"
#include "kernel_util.h"
#include "kernels.h"
#include "ntt32.h"
#include "ntt64.h"

namespace lp {

// 32 x 32 transpose through a half-wave LDS block of 32 x 33 words, in two
// 32-bit passes (low words, then high words): on entry lane l holds row l
// (a[i] = (l, i)); on exit lane l holds column l (a[m] = (m, l)).  Rows are
// padded to 33 words so both phases are bank-conflict free.
__device__ __forceinline__ void transpose32(uint64_t (&a)[32], uint32_t* buf, int l) {
  uint32_t lo[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) buf[l * ROW + i] = (uint32_t)a[i];
  wave_fence();
#pragma unroll
  for (int m = 0; m < 32; ++m) lo[m] = buf[m * ROW + l];
  wave_fence();
#pragma unroll
  for (int i = 0; i < 32; ++i) buf[l * ROW + i] = (uint32_t)(a[i] >> 32);
  wave_fence();
#pragma unroll
  for (int m = 0; m < 32; ++m) a[m] = ((uint64_t)buf[m * ROW + l] << 32) | lo[m];
  wave_fence();
}

// Twist between the passes: slot i of lane l times tw[i * 32 + l].  All 32
// table loads are issued before the first product (global address space,
// so they wait on the vector-memory counter alone) and the latency is paid
// once per twist.
__device__ __forceinline__ void twist(uint64_t (&f)[32], const uint64_t* __restrict__ tw, int l) {
  const gmem_u64* t = as_global(tw) + l;
  uint64_t w[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) w[i] = t[i * 32];
#pragma unroll
  for (int i = 0; i < 32; ++i) f[i] = gl_mul(f[i], w[i]);
}

// Forward negacyclic NTT of one polynomial per half-wave.  In: lane l,
// slot m = coefficient l + 32 m.  Out: lane l -> ka = brv5(l), slot i ->
// kb = brv5(i).
__device__ __forceinline__ void ntt_fwd(uint64_t (&f)[32], uint32_t* buf, const uint64_t* __restrict__ tw_f,
                                        int l) {
  fwd1(f);
  twist(f, tw_f, l);
  transpose32(f, buf, l);
  fwd2(f);
}

// The same for small signed digits, first two butterfly stages fused.
__device__ __forceinline__ void ntt_fwd_digits(const int32_t (&d)[32], uint64_t (&f)[32], uint32_t* buf,
                                               const uint64_t* __restrict__ tw_f, int l) {
  fwd1_first_stages_digits(d, f);
  fwd1_rest(f);
  twist(f, tw_f, l);
  transpose32(f, buf, l);
  fwd2(f);
}

// Inverse of ntt_fwd including the 1/1024 scaling.
__device__ __forceinline__ void ntt_inv(uint64_t (&f)[32], uint32_t* buf, const uint64_t* __restrict__ tw_i,
                                        int l) {
  inv2(f);
  twist(f, tw_i, l);
  transpose32(f, buf, l);
  inv1(f);
}

// Offset of (slot s, lane l) inside one NTT-domain polynomial.
__device__ __forceinline__ int ntt_pos(int s, int l) { return (s >> 1) * 64 + l * 2 + (s & 1); }

// ---------------------------------------------------------------------------
// Bootstrapping key -> NTT domain.  One polynomial per half-wave.
__global__ __launch_bounds__(64) void bsk_to_ntt_kernel(const uint32_t* __restrict__ src,
                                                        uint64_t* __restrict__ dst, int npoly,
                                                        const uint64_t* __restrict__ tw_f) {
  __shared__ uint32_t s_buf[2][LDS_HALF];
  const int lane = threadIdx.x, h = lane >> 5, l = lane & 31;
  const int poly = blockIdx.x * 2 + h;
  const bool live = poly < npoly;
  uint64_t f[32];
#pragma unroll
  for (int m = 0; m < 32; ++m) f[m] = live ? (uint64_t)src[(size_t)poly * RING_N + l + 32 * m] : 0ull;
  ntt_fwd(f, s_buf[h], tw_f, l);
  if (live) {
    uint64_t* d = dst + (size_t)poly * RING_N;
#pragma unroll
    for (int s = 0; s < 32; ++s) d[ntt_pos(s, l)] = f[s];
  }
}

// ---------------------------------------------------------------------------
// Blind rotation.  W waves cooperate on one bootstrap:
//   W = 1: the wave runs the three gadget levels in turn (throughput mode:
//          independent bootstraps fill the GPU);
//   W = 3: wave w runs gadget level w and the inverse NTT of that level's
//          partial product, and adds its lifted partial into the LDS
//          accumulator with LDS atomics (latency mode for narrow circuit
//          levels; 35 KB of LDS, so four bootstraps fit one CU);
//   W = 4: waves 0-2 run the gadget levels as in W = 3 but leave their
//          partial products in LDS; the levels' sum of each component is
//          inverted once, by two waves at four lanes per row (ntt64.h),
//          waves 0-1 for the mask and 2-3 for the body (latency mode, one
//          bootstrap per CU: 102 KB of LDS);
//   W = 5: the same four waves sized for two bootstraps per CU: key rows
//          loaded where they are used (at most 256 registers), and the
//          forward transposes placed in the partials' space behind one
//          more barrier per step (76 KB of LDS).
// The accumulator lives in LDS ([component][coefficient] u32); each level
// re-reads it to form X^a ACC - ACC.
template <int W>
__global__ __launch_bounds__(64 * (W == 5 ? 4 : W), (W == 1 || W == 5) ? 2 : 1) void blind_rotate_kernel(
    const BrJob* __restrict__ jobs, int njobs, SrcBases src, uint32_t* __restrict__ ex_out,
    const uint64_t* const* __restrict__ bsk_tab, uint32_t* const* __restrict__ pool_tab, int n_lwe, int steps,
    int raw_acc, const uint64_t* __restrict__ tw_f, const uint64_t* __restrict__ tw_i) {
  constexpr int NW = W == 5 ? 4 : W;   // waves per bootstrap
  constexpr int NL = W >= 4 ? 3 : W;   // waves that run gadget levels
  constexpr bool SUM = W >= 4;         // levels summed in the NTT domain
  constexpr bool DUAL = W == 5;        // two bootstraps per CU
  __shared__ uint32_t s_acc[2][RING_N];
  __shared__ __align__(16) uint32_t s_tr[DUAL ? 1 : NL][2][DUAL ? 4 : LDS_HALF];
  __shared__ __align__(16) uint64_t s_part[SUM ? 3 : 1][2][SUM ? RING_N : 2];
  __shared__ __align__(16) uint64_t s_t128[2][SUM ? 32 * T128_ROW : 1];
  __shared__ uint16_t s_abar[MAX_LWE + 4];

  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, h = lane >> 5, l = lane & 31;
  const int job = blockIdx.x;
  if (job >= njobs) return;  // uniform over the block

  const BrJob J = jobs[job];
  const int lw = wave < NL ? wave : 0;  // level of this wave (any, for a wave without one)
  uint32_t* buf = DUAL ? reinterpret_cast<uint32_t*>(&s_part[0][0][0]) + (lw * 2 + h) * LDS_HALF : s_tr[lw][h];
  uint32_t* acc = s_acc[h];

  // modulus switch of the combined input (0, cst) + c0 in0 + c1 in1
  {
    auto operand = [&](uint32_t r) -> const uint32_t* {
      if (r == REF_NONE) return nullptr;
      const uint32_t base = r >> REF_SHIFT;
      const uint32_t* b = base == KEY_POOL_BASE ? pool_tab[J.key] : src.p[base];
      return b + (size_t)(r & REF_INDEX_MASK) * (n_lwe + 1);
    };
    const uint32_t* in0 = operand(J.in0);
    const uint32_t* in1 = operand(J.in1);
    for (int c = threadIdx.x; c <= n_lwe; c += 64 * NW) {
      uint32_t v = (c == n_lwe) ? J.cst : 0u;
      if (in0) v += (uint32_t)J.c0 * in0[c];
      if (in1) v += (uint32_t)J.c1 * in1[c];
      s_abar[c] = (uint16_t)(((v + (1u << 20)) >> 21) & 2047u);
    }
  }
  __syncthreads();

  // ACC = (0, X^{-b} v), v = sum_j (1/8) X^j: coefficient j of X^{-b} v is
  // +1/8 when (j + b) mod 2N < N, else -1/8
  const uint32_t bbar = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_abar[n_lwe]);
  for (int c = threadIdx.x; c < 2 * RING_N; c += 64 * NW) {
    const uint32_t j = (uint32_t)c & 1023u;
    s_acc[c >> 10][j] = c < RING_N ? 0u : ((((j + bbar) & 2047u) < 1024u) ? 0x20000000u : 0xE0000000u);
  }
  __syncthreads();

  const gmem_u64* bsk = as_global(bsk_tab[J.key]);
  const int nsteps = steps < n_lwe ? steps : n_lwe;

  for (int i = 0; i < nsteps; ++i) {
    const uint32_t a = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_abar[i]);
    if (a == 0) continue;  // X^0 ACC - ACC = 0 decomposes to zero digits

    if constexpr (SUM) {
      const gmem_u64* step_key = bsk + (size_t)i * 6 * 2 * RING_N;
      const bool lvl = wave < NL;
      // rows (h, j) and (1-h, j), component h, of level j = wave
      const gmem_u64* ko = step_key + (size_t)((h * 3 + lw) * 2 + h) * RING_N + l * 2;
      const gmem_u64* kt = step_key + (size_t)(((1 - h) * 3 + lw) * 2 + h) * RING_N + l * 2;
      uint64_t kpre[DUAL ? 1 : 64];
      int32_t dg[32];
      if (lvl) {
        if constexpr (!DUAL) {
#pragma unroll
          for (int sp = 0; sp < 16; ++sp) {
            kpre[4 * sp + 0] = ko[sp * 64];
            kpre[4 * sp + 1] = ko[sp * 64 + 1];
            kpre[4 * sp + 2] = kt[sp * 64];
            kpre[4 * sp + 3] = kt[sp * 64 + 1];
          }
        }
        const int sh = 25 - 7 * wave;
#pragma unroll
        for (int m = 0; m < 32; ++m) {
          const uint32_t j = (uint32_t)(l + 32 * m);
          const uint32_t e = (j - a) & 2047u;
          const uint32_t v = acc[e & 1023u];
          const uint32_t D = ((e & 1024u) ? (0u - v) : v) - acc[j];
          dg[m] = (int32_t)(((D + 0x81020400u) >> sh) & 127u) - 64;
        }
      }
      __syncthreads();  // every wave has read ACC before any adds to it
      uint64_t f[32];
      if (lvl) ntt_fwd_digits(dg, f, buf, opaque(tw_f), l);
      // DUAL: the key rows of a slot pair are requested KD pairs ahead of
      // their products (the first KD before the barrier), in a ring of KD
      constexpr int KD = 4;
      uint64_t kr[DUAL ? KD : 1][4];
      auto request = [&](int sp, uint64_t(&k)[4]) {
        k[0] = ko[sp * 64];
        k[1] = ko[sp * 64 + 1];
        k[2] = kt[sp * 64];
        k[3] = kt[sp * 64 + 1];
      };
      if constexpr (DUAL) {
        if (lvl) {
#pragma unroll
          for (int sp = 0; sp < KD; ++sp) request(sp, kr[sp]);
        }
        __syncthreads();  // the transposes are done before the partials take their space
      }
      if (lvl) {
        uint64_t* part = s_part[wave][h];
#pragma unroll
        for (int sp = 0; sp < 16; ++sp) {
          uint64_t k0, k1, k2, k3;
          if constexpr (DUAL) {
            k0 = kr[sp % KD][0];
            k1 = kr[sp % KD][1];
            k2 = kr[sp % KD][2];
            k3 = kr[sp % KD][3];
            if (sp + KD < 16) request(sp + KD, kr[sp % KD]);
          } else {
            k0 = kpre[4 * sp];
            k1 = kpre[4 * sp + 1];
            k2 = kpre[4 * sp + 2];
            k3 = kpre[4 * sp + 3];
          }
          const uint64_t g0 = from_other_half(f[2 * sp], lane), g1 = from_other_half(f[2 * sp + 1], lane);
          part[sp * 64 + 2 * l] = gl_mul_sum(f[2 * sp], k0, g0, k2);
          part[sp * 64 + 2 * l + 1] = gl_mul_sum(f[2 * sp + 1], k1, g1, k3);
        }
      }
      __syncthreads();
      // component c = wave >> 1 on waves 2c and 2c + 1, rows 16 (wave & 1) + r
      {
        const int c = wave >> 1, r4 = lane >> 2, hq = lane & 3, row = 16 * (wave & 1) + r4;
        const uint64_t upper1 = (hq & 1) ? ~0ull : 0ull, upper2 = (hq & 2) ? ~0ull : 0ull;
        uint64_t v[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int off = 128 * s + 64 * (hq >> 1) + 2 * row + (hq & 1);
          v[s] = gl_add(gl_add(s_part[0][c][off], s_part[1][c][off]), s_part[2][c][off]);
        }
        inv128_p2(v, upper1, upper2, upper2);
        {
          const gmem_u64* t = as_global(opaque(tw_i)) + hq * 32 + row;
          uint64_t w[8];
#pragma unroll
          for (int s = 0; s < 8; ++s) w[s] = t[s * 128];
#pragma unroll
          for (int s = 0; s < 8; ++s) v[s] = gl_mul(v[s], w[s]);
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) s_t128[c][row * T128_ROW + 4 * s + hq] = v[s];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = s_t128[c][(4 * s + hq) * T128_ROW + row];
        inv128_p1(v, upper1, upper2, upper2);
        // the levels' sum is an exact integer polynomial (|coefficient| <
        // 2^50.6), so its centred lift reduced mod 2^32 is exact
#pragma unroll
        for (int s = 0; s < 8; ++s) s_acc[c][row + 32 * (4 * s + hq)] += gl_lift_u32(v[s]);
      }
      __syncthreads();
      continue;
    }

    // BSK_i in the NTT domain: rows (p, j) = 3p + j, each with components q
    // = 0, 1.  Output component h of level j is
    //   NTT(d_(h,j)) BSK[(h,j)][h] + NTT(d_(1-h,j)) BSK[(1-h,j)][h],
    // so this half-wave reads component h of rows (h, j) and (1-h, j).
    const gmem_u64* step_key = bsk + (size_t)i * 6 * 2 * RING_N;
    // W > 1: the wave's gadget level is fixed, so both rows are loaded now
    // and arrive while the digits are transformed.
    uint64_t kpre[W > 1 ? 64 : 1];
    if constexpr (W > 1) {
      const gmem_u64* ko = step_key + (size_t)((h * 3 + wave) * 2 + h) * RING_N + l * 2;
      const gmem_u64* kt = step_key + (size_t)(((1 - h) * 3 + wave) * 2 + h) * RING_N + l * 2;
#pragma unroll
      for (int sp = 0; sp < 16; ++sp) {
        kpre[4 * sp + 0] = ko[sp * 64];
        kpre[4 * sp + 1] = ko[sp * 64 + 1];
        kpre[4 * sp + 2] = kt[sp * 64];
        kpre[4 * sp + 3] = kt[sp * 64 + 1];
      }
    }
    uint64_t outv[32];
#pragma nounroll
    for (int jj = (W == 1 ? 0 : wave); jj < (W == 1 ? 3 : wave + 1); ++jj) {
      // signed digit of level jj+1 of D = X^a ACC_h - ACC_h:
      // ((D + 0x81020400) >> (25 - 7 jj)) & 127) - 64
      const int sh = 25 - 7 * jj;
      int32_t dg[32];
#pragma unroll
      for (int m = 0; m < 32; ++m) {
        const uint32_t j = (uint32_t)(l + 32 * m);
        const uint32_t e = (j - a) & 2047u;
        const uint32_t v = acc[e & 1023u];
        const uint32_t D = ((e & 1024u) ? (0u - v) : v) - acc[j];
        dg[m] = (int32_t)(((D + 0x81020400u) >> sh) & 127u) - 64;
      }
      // W > 1: every wave has read the accumulator before any adds to it
      if constexpr (W > 1) __syncthreads();
      uint64_t f[32];
      ntt_fwd_digits(dg, f, buf, opaque(tw_f), l);

      // W == 1: the rows of this level, loaded where they are used
      const gmem_u64* k_own = step_key + (size_t)((h * 3 + jj) * 2 + h) * RING_N + l * 2;
      const gmem_u64* k_oth = step_key + (size_t)(((1 - h) * 3 + jj) * 2 + h) * RING_N + l * 2;
#pragma unroll
      for (int sp = 0; sp < 16; ++sp) {
        uint64_t k0, k1, k2, k3;
        if constexpr (W > 1) {
          k0 = kpre[4 * sp];
          k1 = kpre[4 * sp + 1];
          k2 = kpre[4 * sp + 2];
          k3 = kpre[4 * sp + 3];
        } else {
          k0 = k_own[sp * 64];
          k1 = k_own[sp * 64 + 1];
          k2 = k_oth[sp * 64];
          k3 = k_oth[sp * 64 + 1];
        }
        // the other half holds the same level's transform of component 1-h
        const uint64_t g0 = from_other_half(f[2 * sp], lane), g1 = from_other_half(f[2 * sp + 1], lane);
        const uint64_t t0 = gl_mul_sum(f[2 * sp], k0, g0, k2);
        const uint64_t t1 = gl_mul_sum(f[2 * sp + 1], k1, g1, k3);
        if (W == 1 && jj > 0) {
          outv[2 * sp] = gl_add(outv[2 * sp], t0);
          outv[2 * sp + 1] = gl_add(outv[2 * sp + 1], t1);
        } else {
          outv[2 * sp] = t0;
          outv[2 * sp + 1] = t1;
        }
      }
    }

    if constexpr (W > 1) {
      // Each wave inverts its own level's partial product.  A partial is an
      // exact integer polynomial (|coefficient| < 2^49 < p/2), so its centred
      // lift mod 2^32 is exact, and adding the lifted partials of the W
      // levels in LDS gives the lift of their sum.
      ntt_inv(outv, buf, opaque(tw_i), l);
#pragma unroll
      for (int m = 0; m < 32; ++m) atomicAdd(&acc[l + 32 * m], gl_lift_u32(outv[m]));
      __syncthreads();
    } else {
      ntt_inv(outv, buf, opaque(tw_i), l);
#pragma unroll
      for (int m = 0; m < 32; ++m) acc[l + 32 * m] += gl_lift_u32(outv[m]);
      wave_fence();
    }
  }

  if (wave != 0) return;
  if (raw_acc) {
    uint32_t* o = ex_out + (size_t)J.out * (2 * RING_N) + h * RING_N;
#pragma unroll
    for (int m = 0; m < 32; ++m) o[l + 32 * m] = acc[l + 32 * m];
  } else {
    // sample extraction at coefficient 0: a'_0 = A_0, a'_j = -A_{N-j}, b' = B_0
    uint32_t* o = ex_out + (size_t)J.out * (RING_N + 1);
    if (h == 0) {
#pragma unroll
      for (int m = 0; m < 32; ++m) {
        const int j = l + 32 * m;
        if (j == 0) o[0] = acc[0];
        else o[RING_N - j] = 0u - acc[j];
      }
    } else if (l == 0) {
      o[RING_N] = acc[0];
    }
  }
}

// ---------------------------------------------------------------------------
// Blind rotation on two waves per bootstrap, one accumulator component per
// wave: wave c owns ACC_c (0 = mask A, 1 = body B) and runs whole-wave
// transforms (ntt64.h).  Output component o of a step is the sum over both
// input components c and the three gadget levels j of
// NTT(d_(c,j)) BSK[(c,j)][o], so each step wave c
//   1. forms D_c = X^a ACC_c - ACC_c, transforms the digits of every level
//      and accumulates its terms of both outputs, Q_(c->c) and Q_(c->1-c);
//   2. hands Q_(c->1-c) to the partner through LDS and adds the partner's
//      Q_(1-c->c) to its own: the full output component c, an exact
//      integer polynomial (|coefficient| < 2^50.6) in the NTT domain;
//   3. inverts it and adds its centred lift mod 2^32 to ACC_c.
// Every wave does a third of the forward transforms, half of the products
// and one inverse, with no accumulator shared between waves.  Sized for two
// waves per SIMD (four bootstraps per CU), the shape for levels of about
// one bootstrap per SIMD, where one wave per bootstrap leaves a SIMD a
// single wave to issue from.
//
// A wave's inbox (the partner's term) doubles as its transpose block
// between reading it and the partner's next write: the partner writes only
// after the first barrier of the next step, which this wave reaches after
// its inverse and its next forward transforms.
__global__ __launch_bounds__(128, 2) void blind_rotate_pair_kernel(
    const BrJob* __restrict__ jobs, int njobs, SrcBases src, uint32_t* __restrict__ ex_out,
    const uint64_t* const* __restrict__ bsk_tab, uint32_t* const* __restrict__ pool_tab, int n_lwe, int steps,
    int raw_acc, const uint64_t* __restrict__ tw_f, const uint64_t* __restrict__ tw_i) {
  __shared__ uint32_t s_acc[2][RING_N];
  __shared__ __align__(16) uint64_t s_in[2][RING_N];  // inbox of wave c
  __shared__ __align__(16) uint64_t s_twf[RING_N];    // forward twist table
  __shared__ uint16_t s_abar[MAX_LWE + 4];

  const int c = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, h = lane >> 5, l = lane & 31;
  const uint32_t h6 = 6u * (uint32_t)h;  // the lane's extra shift in a paired distance-1 stage
  const int job = blockIdx.x;
  if (job >= njobs) return;  // uniform over the block
  // entry 64 r + lane: the factor of register r of that lane in the pair
  // layout that the forward's first pass leaves
  for (int k = threadIdx.x; k < RING_N; k += 128) s_twf[k] = tw_f[pair_pos(k >> 6, (k >> 5) & 1) * 32 + (k & 31)];

  const BrJob J = jobs[job];
  {
    auto operand = [&](uint32_t r) -> const uint32_t* {
      if (r == REF_NONE) return nullptr;
      const uint32_t base = r >> REF_SHIFT;
      const uint32_t* b = base == KEY_POOL_BASE ? pool_tab[J.key] : src.p[base];
      return b + (size_t)(r & REF_INDEX_MASK) * (n_lwe + 1);
    };
    const uint32_t* in0 = operand(J.in0);
    const uint32_t* in1 = operand(J.in1);
    for (int k = threadIdx.x; k <= n_lwe; k += 128) {
      uint32_t v = (k == n_lwe) ? J.cst : 0u;
      if (in0) v += (uint32_t)J.c0 * in0[k];
      if (in1) v += (uint32_t)J.c1 * in1[k];
      s_abar[k] = (uint16_t)(((v + (1u << 20)) >> 21) & 2047u);
    }
  }
  __syncthreads();

  // ACC_0 = 0, ACC_1 = X^{-b} v (coefficient j: +1/8 if (j + b) mod 2N < N)
  uint32_t* acc = s_acc[c];
  const uint32_t bbar = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_abar[n_lwe]);
  for (int j = lane; j < RING_N; j += 64)
    acc[j] = c == 0 ? 0u : ((((uint32_t)j + bbar) & 2047u) < 1024u ? 0x20000000u : 0xE0000000u);
  wave_fence();

  uint64_t* inbox = s_in[c];
  uint64_t* outbox = s_in[1 - c];
  uint32_t* tbuf = reinterpret_cast<uint32_t*>(inbox);
  const gmem_u64* bsk = as_global(bsk_tab[J.key]);
  const int nsteps = steps < n_lwe ? steps : n_lwe;

  for (int i = 0; i < nsteps; ++i) {
    const uint32_t a = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_abar[i]);
    if (a == 0) continue;  // X^0 ACC - ACC = 0 decomposes to zero digits

    const gmem_u64* step_key = bsk + (size_t)i * 6 * 2 * RING_N;
    const gmem_u64* twi = as_global(opaque(tw_i)) + lane;  // twist64's reads
    uint64_t qo[16], qx[16];  // terms of output c and of output 1 - c
    // gadget level j: rows (c, j) of BSK_i, components c and 1 - c, at the
    // offsets of this lane's registers in the pair layout, 512 h + 64 (r & 7)
    // + 2 l + (r >> 3)
    auto level = [&](int j, auto first) {
      // the rows are loaded before the transform: the compiler keeps loads
      // where they are written, and after it they would be waited on at once
      const gmem_u64* ko = step_key + (size_t)((c * 3 + j) * 2 + c) * RING_N + 2 * l + 512 * h;
      const gmem_u64* kx = step_key + (size_t)((c * 3 + j) * 2 + (1 - c)) * RING_N + 2 * l + 512 * h;
      uint64_t k0[16], k1[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        k0[r] = ko[64 * (r & 7) + (r >> 3)];
        k1[r] = kx[64 * (r & 7) + (r >> 3)];
      }
      const int sh = 25 - 7 * j;
      int32_t dg[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const uint32_t k = (uint32_t)(l + 32 * (2 * s + h));
        const uint32_t e = (k - a) & 2047u;
        const uint32_t v = acc[e & 1023u];
        const uint32_t D = ((e & 1024u) ? (0u - v) : v) - acc[k];
        dg[s] = (int32_t)(((D + 0x81020400u) >> sh) & 127u) - 64;
      }
      // forward transform: both passes end in the paired distance-1 stage,
      // and the products and the inverse's input stay in the pair layout
      uint64_t f[16];
      fwd64_p1_digits(dg, f);
      // the lane's shift counts are formed here from h6, not held across
      // the step loop (which spills)
      uint32_t h6l = h6;
      asm volatile("" : "+v"(h6l));
      fwd64_p1_rest_pairs(f, h6l);
#pragma unroll
      for (int s = 0; s < 16; ++s) f[s] = gl_mul(f[s], s_twf[64 * s + lane]);
      transpose64_pairs(f, tbuf, h, l);
      fwd64_p2_pairs(f, h6l);
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        if constexpr (decltype(first)::value) {
          qo[s] = gl_mul(f[s], k0[s]);
          qx[s] = gl_mul(f[s], k1[s]);
        } else {
          qo[s] = gl_mac(qo[s], f[s], k0[s]);
          qx[s] = gl_mac(qx[s], f[s], k1[s]);
        }
      }
    };
    level(0, std::true_type{});
#pragma nounroll
    for (int j = 1; j < 3; ++j) level(j, std::false_type{});

    uint64_t w[16];  // inverse twist factors, loaded ahead of the barriers
#pragma unroll
    for (int s = 0; s < 16; ++s) w[s] = twi[s * 64];
    __syncthreads();  // the partner is done with its inbox of the previous step
#pragma unroll
    for (int s = 0; s < 16; ++s) outbox[64 * s + lane] = qx[s];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) qo[s] = gl_add(qo[s], inbox[64 * s + lane]);
    wave_fence();  // the inbox is read before it serves as the transpose block
    // inverse of the forward transform (1/1024 included), twist factors at
    // hand; each pass starts from the pair layout and ends interleaved
    uint32_t h6i = h6;
    asm volatile("" : "+v"(h6i));
    inv64_p2_pairs(qo, h6i);
#pragma unroll
    for (int s = 0; s < 16; ++s) qo[s] = gl_mul(qo[s], w[s]);
    transpose64_to_pairs(qo, tbuf, h, l);
    inv64_p1_pairs(qo, h6i);
#pragma unroll
    for (int s = 0; s < 16; ++s) acc[l + 32 * (2 * s + h)] += gl_lift_u32(qo[s]);
    wave_fence();
  }

  if (raw_acc) {
    uint32_t* o = ex_out + (size_t)J.out * (2 * RING_N) + c * RING_N;
    for (int j = lane; j < RING_N; j += 64) o[j] = acc[j];
  } else {
    // sample extraction at coefficient 0: a'_0 = A_0, a'_j = -A_{N-j}, b' = B_0
    uint32_t* o = ex_out + (size_t)J.out * (RING_N + 1);
    if (c == 0) {
      for (int j = lane; j < RING_N; j += 64) {
        if (j == 0) o[0] = acc[0];
        else o[RING_N - j] = 0u - acc[j];
      }
    } else if (lane == 0) {
      o[RING_N] = acc[0];
    }
  }
}

// KT > 0: the digit count t fixed at compile time; the KT x NROWS candidate
// rows of ring index i + 1 are requested while index i is applied, so a
// wave waits on the key-switching key once per index pair, not per digit.
template <int T, int BB, int KT>
__global__ __launch_bounds__(64) void keyswitch_kernel(const KsJob* __restrict__ jobs, int njobs,
                                                       const uint32_t* __restrict__ ex, DstBases dst,
                                                       const uint32_t* const* __restrict__ ksk_tab,
                                                       uint32_t* const* __restrict__ pool_tab, int n_lwe, int N,
                                                       int ks_t) {
  constexpr int NROWS = (1 << BB) - 1;
  const int lane = threadIdx.x;
  const int col = blockIdx.x * 64 + lane;
  const int j0 = blockIdx.y * T;
  const bool colok = col <= n_lwe;
  // lanes past the last column read column n_lwe (their sums are never
  // stored), so every key load is unconditional
  const uint32_t kcol = colok ? (uint32_t)col : (uint32_t)n_lwe;
  const uint32_t kbyte = kcol * 4u;  // a 32-bit offset, as the loads' scalar-base form takes
  const int w = n_lwe + 1;
  // the tile's key (one per tile), made uniform so that row addresses are
  // scalar
  const uint64_t kp = (uint64_t)ksk_tab[jobs[j0].key];
  const uint32_t* __restrict__ ksk = (const uint32_t*)(
      ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(kp >> 32)) << 32) |
      (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)kp));
  const uint32_t prec = 1u << (31 - BB * ks_t);
  const int isplit = gridDim.z;
  const int i_lo = (int)blockIdx.z * (N / isplit), i_hi = i_lo + N / isplit;

  uint32_t accv[T];
  const uint32_t* e0[T];
  const uint32_t* e1[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int jb = j0 + t;
    e0[t] = nullptr;
    e1[t] = nullptr;
    accv[t] = 0u;
    if (jb < njobs && jobs[jb].ex0 != REF_NONE) {
      const KsJob K = jobs[jb];
      e0[t] = ex + (size_t)K.ex0 * (N + 1);
      e1[t] = K.ex1 == REF_NONE ? nullptr : ex + (size_t)K.ex1 * (N + 1);
      if (col == n_lwe && isplit == 1) accv[t] = K.cst + e0[t][N] + (e1[t] ? e1[t][N] : 0u);
    }
  }

  for (int i0 = i_lo; i0 < i_hi; i0 += 64) {
    uint32_t av[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      uint32_t v = 0u;
      if (e0[t]) v = e0[t][i0 + lane] + (e1[t] ? e1[t][i0 + lane] : 0u) + prec;
      av[t] = v;
    }
    if constexpr (KT > 0) {
      constexpr int R = KT * NROWS;  // candidate rows of one ring index
      uint32_t picked[T];            // sums of the rows picked in this block
#pragma unroll
      for (int t = 0; t < T; ++t) picked[t] = 0u;
      // a uniform row pointer plus the lane's column, so that the loads take
      // a scalar base and share one offset register
      const gmem_u32* base = as_global(ksk) + (size_t)i0 * R * w;
      auto fetch = [&](uint32_t(&r)[R], int ii) {
        const gmem_u32* q = base + (size_t)ii * R * w;
        // the column offset re-enters here as a 32-bit value, so that its
        // widening is visible next to the loads
        uint32_t kb = kbyte;
        asm("" : "+v"(kb));
#pragma unroll
        for (int k = 0; k < R; ++k) {
          // each row's address stays a scalar pair (scalar adds), and the
          // load takes it as its base with the lane's column as offset,
          // instead of a chain of 64-bit vector adds
          const gmem_u32* row = q + (size_t)k * w;
          asm("" : "+s"(row));
          r[k] = *(const gmem_u32*)((__attribute__((address_space(1))) const char*)row + kb);
        }
      };
      auto apply = [&](const uint32_t(&r)[R], int ii) {
        uint32_t asc[T];
#pragma unroll
        for (int t = 0; t < T; ++t) asc[t] = (uint32_t)__builtin_amdgcn_readlane((int)av[t], ii);
#pragma unroll
        for (int j = 0; j < KT; ++j) {
          const int shift = 32 - (j + 1) * BB;
#pragma unroll
          for (int t = 0; t < T; ++t) {
            if constexpr (BB == 2) {
              // d = 2 b1 + b0 is uniform: each bit becomes an all-ones or
              // all-zero scalar word (one signed field extract), and two
              // bit-field selects of the rows pick row d (none for d = 0).
              // The picked rows are summed, and the sum subtracted at the end.
              // The masks are hidden from the optimizer, which would
              // otherwise turn them back into compares and lane masks.
              uint32_t m0 = (uint32_t)__builtin_amdgcn_sbfe((int)asc[t], shift, 1);
              uint32_t m1 = (uint32_t)__builtin_amdgcn_sbfe((int)asc[t], shift + 1, 1);
              asm("" : "+s"(m0), "+s"(m1));
              const uint32_t r1 = r[j * 3], r2 = r[j * 3 + 1], r3 = r[j * 3 + 2];
              uint32_t lo = r1 & m0;
              // kept apart from the last select, which could otherwise
              // fold it in and read two scalar masks in one instruction
              asm("" : "+v"(lo));
              const uint32_t hi = (r3 & m0) | (r2 & ~m0);
              picked[t] += (hi & m1) | (lo & ~m1);
            } else {
              // d is uniform: the row it selects is picked with scalar
              // masks, not a branch per digit
              const uint32_t d = (asc[t] >> shift) & (uint32_t)NROWS;
              uint32_t sub = 0u;
#pragma unroll
              for (int v = 1; v <= NROWS; ++v) sub |= r[j * NROWS + v - 1] & (0u - (uint32_t)(d == (uint32_t)v));
              picked[t] += sub;
            }
          }
          // one digit's masks at a time: hoisting them all ahead of the
          // selects spills scalar registers
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      uint32_t ra[R], rb[R];
      fetch(ra, 0);
      // the last pair is peeled so that the loop body has no branch
      for (int ii = 0; ii < 62; ii += 2) {
        fetch(rb, ii + 1);
        apply(ra, ii);
        fetch(ra, ii + 2);
        apply(rb, ii + 1);
      }
      fetch(rb, 63);
      apply(ra, 62);
      apply(rb, 63);
#pragma unroll
      for (int t = 0; t < T; ++t) accv[t] -= picked[t];
      continue;
    }
    for (int ii = 0; ii < 64; ++ii) {
      const int i = i0 + ii;
      uint32_t asc[T];
#pragma unroll
      for (int t = 0; t < T; ++t) asc[t] = (uint32_t)__builtin_amdgcn_readlane((int)av[t], ii);
      for (int j = 0; j < ks_t; ++j) {
        const uint32_t* rowp = ksk + ((size_t)(i * ks_t + j) * NROWS) * w + kcol;
        uint32_t r[NROWS + 1];
        r[0] = 0u;
#pragma unroll
        for (int v = 0; v < NROWS; ++v) r[v + 1] = rowp[(size_t)v * w];
        const int shift = 32 - (j + 1) * BB;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const uint32_t d = (asc[t] >> shift) & (uint32_t)NROWS;
          uint32_t sub = 0u;
#pragma unroll
          for (int v = 1; v <= NROWS; ++v) sub = (d == (uint32_t)v) ? r[v] : sub;
          accv[t] -= sub;
        }
      }
    }
  }

#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int jb = j0 + t;
    if (e0[t] && colok) {
      const uint32_t o = jobs[jb].out;
      uint32_t* b = (o >> REF_SHIFT) == KEY_POOL_BASE ? pool_tab[jobs[jb].key] : dst.p[o >> REF_SHIFT];
      uint32_t* p = b + (size_t)(o & REF_INDEX_MASK) * w + col;
      if (isplit == 1) *p = accv[t];
      else atomicAdd(p, accv[t]);  // accv already holds minus the partial sum
    }
  }
}

// Output of a split key switch before accumulation: (0, ..., 0, b'), with
// b' = cst + b(ex0) (+ b(ex1)).
__global__ void ks_init_kernel(const KsJob* __restrict__ jobs, int njobs, const uint32_t* __restrict__ ex,
                               DstBases dst, uint32_t* const* __restrict__ pool_tab, int n_lwe, int N) {
  const int jb = blockIdx.x;
  if (jb >= njobs) return;
  const KsJob K = jobs[jb];
  if (K.ex0 == REF_NONE) return;  // padding job
  const int w = n_lwe + 1;
  uint32_t* b = (K.out >> REF_SHIFT) == KEY_POOL_BASE ? pool_tab[K.key] : dst.p[K.out >> REF_SHIFT];
  uint32_t* o = b + (size_t)(K.out & REF_INDEX_MASK) * w;
  for (int c = threadIdx.x; c < w; c += blockDim.x) {
    uint32_t v = 0u;
    if (c == n_lwe) {
      v = K.cst + ex[(size_t)K.ex0 * (N + 1) + N];
      if (K.ex1 != REF_NONE) v += ex[(size_t)K.ex1 * (N + 1) + N];
    }
    o[c] = v;
  }
}

// ---------------------------------------------------------------------------
__global__ void make_batch_jobs_kernel(int nbr, uint32_t cst, int32_t c0, int32_t c1, int has_in1,
                                       size_t cnt, BrJob* __restrict__ br, KsJob* __restrict__ ks) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cnt) return;
  const uint32_t kk = (uint32_t)k;
  if (nbr == 1) {
    br[k] = BrJob{make_ref(0, kk), has_in1 ? make_ref(1, kk) : REF_NONE, c0, c1, cst, kk, 0u, 0u};
    ks[k] = KsJob{kk, REF_NONE, 0u, make_ref(0, kk), 0u, {0u, 0u, 0u}};
  } else {
    // MUX(sel = in0, t = in1, f = in2): (sel AND t), (NOT sel AND f)
    br[2 * k] = BrJob{make_ref(0, kk), make_ref(1, kk), 1, 1, 0xE0000000u, 2 * kk, 0u, 0u};
    br[2 * k + 1] = BrJob{make_ref(0, kk), make_ref(2, kk), -1, 1, 0xE0000000u, 2 * kk + 1, 0u, 0u};
    ks[k] = KsJob{2 * kk, 2 * kk + 1, 0x20000000u, make_ref(0, kk), 0u, {0u, 0u, 0u}};
  }
}

__global__ void lwe_scale_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, size_t words,
                                 int32_t sign) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < words) out[k] = (uint32_t)sign * in[k];
}

__global__ void gather_kernel(const uint32_t* __restrict__ refs, int cnt, SrcBases src, uint32_t index_offset,
                              uint32_t* __restrict__ out, int n_lwe) {
  const int j = blockIdx.x;
  if (j >= cnt) return;
  const uint32_t r = refs[j];
  const uint32_t* s = src.p[r >> REF_SHIFT] + (size_t)((r & REF_INDEX_MASK) + index_offset) * (n_lwe + 1);
  for (int c = threadIdx.x; c <= n_lwe; c += blockDim.x) out[(size_t)j * (n_lwe + 1) + c] = s[c];
}

__global__ __launch_bounds__(64) void debug_polymul_kernel(const int32_t* __restrict__ digits,
                                                           const uint64_t* __restrict__ poly,
                                                           uint32_t* __restrict__ out, int cnt,
                                                           const uint64_t* __restrict__ tw_f,
                                                           const uint64_t* __restrict__ tw_i) {
  __shared__ uint32_t s_buf[2][LDS_HALF];
  const int lane = threadIdx.x, h = lane >> 5, l = lane & 31;
  const int p = blockIdx.x;
  if (p >= cnt) return;
  int32_t dg[32];
#pragma unroll
  for (int m = 0; m < 32; ++m) dg[m] = digits[(size_t)p * RING_N + l + 32 * m];
  uint64_t f[32];
  ntt_fwd_digits(dg, f, s_buf[h], tw_f, l);
  const uint64_t* b = poly + (size_t)p * RING_N;
#pragma unroll
  for (int s = 0; s < 32; ++s) f[s] = gl_mul(f[s], b[ntt_pos(s, l)]);
  ntt_inv(f, s_buf[h], tw_i, l);
  if (h == 0) {
#pragma unroll
    for (int m = 0; m < 32; ++m) out[(size_t)p * RING_N + l + 32 * m] = gl_lift_u32(f[m]);
  }
}

// ---------------------------------------------------------------------------
// Launchers.

hipError_t launch_bsk_to_ntt(const uint32_t* d_src, uint64_t* d_dst, int npoly, Twiddles tw, hipStream_t s) {
  if (npoly <= 0) return hipSuccess;
  hipLaunchKernelGGL(bsk_to_ntt_kernel, dim3((npoly + 1) / 2), dim3(64), 0, s, d_src, d_dst, npoly, tw.fwd);
  return hipGetLastError();
}

hipError_t launch_blind_rotate(const BrJob* d_jobs, int njobs, const SrcBases& src, uint32_t* d_ex,
                               const uint64_t* const* d_bsk_tab, uint32_t* const* d_pool_tab, int n_lwe, int steps,
                               int raw_acc, Twiddles tw, int waves_per_job, hipStream_t s,
                               const SplitArea* split) {
  if (njobs <= 0) return hipSuccess;
  switch (waves_per_job) {
    case 1:
      hipLaunchKernelGGL(blind_rotate_kernel<1>, dim3(njobs), dim3(64), 0, s, d_jobs, njobs, src, d_ex, d_bsk_tab,
                         d_pool_tab, n_lwe, steps, raw_acc, tw.fwd, tw.inv);
      break;
    case 2:
      hipLaunchKernelGGL(blind_rotate_pair_kernel, dim3(njobs), dim3(128), 0, s, d_jobs, njobs, src, d_ex, d_bsk_tab,
                         d_pool_tab, n_lwe, steps, raw_acc, tw.fwd, tw.inv);
      break;
    case 3:
      hipLaunchKernelGGL(blind_rotate_kernel<3>, dim3(njobs), dim3(192), 0, s, d_jobs, njobs, src, d_ex, d_bsk_tab,
                         d_pool_tab, n_lwe, steps, raw_acc, tw.fwd, tw.inv);
      break;
    case 4:
      hipLaunchKernelGGL(blind_rotate_kernel<4>, dim3(njobs), dim3(256), 0, s, d_jobs, njobs, src, d_ex, d_bsk_tab,
                         d_pool_tab, n_lwe, steps, raw_acc, tw.fwd, tw.inv);
      break;
    case 5:
      hipLaunchKernelGGL(blind_rotate_kernel<5>, dim3(njobs), dim3(256), 0, s, d_jobs, njobs, src, d_ex, d_bsk_tab,
                         d_pool_tab, n_lwe, steps, raw_acc, tw.fwd, tw.inv);
      break;
    case 6:
    case 7:
      return launch_split(d_jobs, njobs, src, d_ex, d_bsk_tab, d_pool_tab, n_lwe, steps, raw_acc, tw, waves_per_job,
                          split, s);
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int T>
static hipError_t launch_ks_t(const KsJob* d_jobs, int njobs, const uint32_t* d_ex, const DstBases& dst,
                              const uint32_t* const* d_ksk_tab, uint32_t* const* pt, int n_lwe, int N, int ks_t,
                              int bb, int isplit, hipStream_t s) {
  dim3 grid((n_lwe + 1 + 63) / 64, (njobs + T - 1) / T, isplit);
  if (isplit > 1) {
    hipLaunchKernelGGL(ks_init_kernel, dim3(njobs), dim3(256), 0, s, d_jobs, njobs, d_ex, dst, pt, n_lwe, N);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // both parameter sets use base 2^2 with t = 8: that shape is compiled with
  // the digit count fixed; any other keeps the runtime loop
  if (bb == 2 && ks_t == 8) {
    hipLaunchKernelGGL((keyswitch_kernel<T, 2, 8>), grid, dim3(64), 0, s, d_jobs, njobs, d_ex, dst, d_ksk_tab, pt, n_lwe, N, ks_t);
    return hipGetLastError();
  }
  switch (bb) {
    case 1: hipLaunchKernelGGL((keyswitch_kernel<T, 1, 0>), grid, dim3(64), 0, s, d_jobs, njobs, d_ex, dst, d_ksk_tab, pt, n_lwe, N, ks_t); break;
    case 2: hipLaunchKernelGGL((keyswitch_kernel<T, 2, 0>), grid, dim3(64), 0, s, d_jobs, njobs, d_ex, dst, d_ksk_tab, pt, n_lwe, N, ks_t); break;
    case 3: hipLaunchKernelGGL((keyswitch_kernel<T, 3, 0>), grid, dim3(64), 0, s, d_jobs, njobs, d_ex, dst, d_ksk_tab, pt, n_lwe, N, ks_t); break;
    case 4: hipLaunchKernelGGL((keyswitch_kernel<T, 4, 0>), grid, dim3(64), 0, s, d_jobs, njobs, d_ex, dst, d_ksk_tab, pt, n_lwe, N, ks_t); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_keyswitch(const KsJob* d_jobs, int njobs, const uint32_t* d_ex, const DstBases& dst,
                            const uint32_t* const* d_ksk_tab, uint32_t* const* d_pool_tab, int n_lwe, int N,
                            int ks_t, int ks_base_bit, int tile, int isplit, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  if (isplit < 1 || N % (64 * isplit) != 0) return hipErrorInvalidValue;
  switch (tile) {
    case 1: return launch_ks_t<1>(d_jobs, njobs, d_ex, dst, d_ksk_tab, d_pool_tab, n_lwe, N, ks_t, ks_base_bit, isplit, s);
    case 4: return launch_ks_t<4>(d_jobs, njobs, d_ex, dst, d_ksk_tab, d_pool_tab, n_lwe, N, ks_t, ks_base_bit, isplit, s);
    case 8: return launch_ks_t<8>(d_jobs, njobs, d_ex, dst, d_ksk_tab, d_pool_tab, n_lwe, N, ks_t, ks_base_bit, isplit, s);
    case 16: return launch_ks_t<16>(d_jobs, njobs, d_ex, dst, d_ksk_tab, d_pool_tab, n_lwe, N, ks_t, ks_base_bit, isplit, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_make_batch_jobs(int nbr, uint32_t cst, int32_t c0, int32_t c1, int has_in1, size_t cnt, BrJob* d_br,
                                  KsJob* d_ks, hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(make_batch_jobs_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, nbr, cst, c0, c1,
                     has_in1, cnt, d_br, d_ks);
  return hipGetLastError();
}

hipError_t launch_lwe_scale(const uint32_t* d_in, uint32_t* d_out, size_t words, int32_t sign, hipStream_t s) {
  if (words == 0) return hipSuccess;
  hipLaunchKernelGGL(lwe_scale_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, d_in, d_out, words, sign);
  return hipGetLastError();
}

hipError_t launch_gather(const uint32_t* d_refs, int cnt, const SrcBases& src, uint32_t index_offset,
                         uint32_t* d_out, int n_lwe, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3(cnt), dim3(256), 0, s, d_refs, cnt, src, index_offset, d_out, n_lwe);
  return hipGetLastError();
}

hipError_t launch_debug_polymul(const int32_t* d_digits, const uint64_t* d_poly_ntt, uint32_t* d_out, int cnt,
                                Twiddles tw, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(debug_polymul_kernel, dim3(cnt), dim3(64), 0, s, d_digits, d_poly_ntt, d_out, cnt, tw.fwd,
                     tw.inv);
  return hipGetLastError();
}

}  // namespace lp
