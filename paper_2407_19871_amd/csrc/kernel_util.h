// Device helpers shared by the blind-rotation kernels (kernels.hip) and the
// split rotation (split.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lp {

constexpr int RING_N = 1024;
constexpr int ROW = 33;             // padded LDS row (32-bit words) of a 32 x 32 transpose
constexpr int LDS_HALF = 32 * ROW;  // words per half-wave transpose block
constexpr int MAX_LWE = 1024;

// Orders this wave's LDS accesses (DS operations of one wave execute in
// program order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Hides a (uniform) pointer's value from the optimizer so that loads
// through it stay inside the loop that uses them: hoisting the 64 twiddle
// loads out of the step loop would pin 128 VGPRs for the whole kernel.
template <typename T>
__device__ __forceinline__ const T* opaque(const T* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// The value held by lane ^ 32.
__device__ __forceinline__ uint64_t from_other_half(uint64_t v, int lane) {
  const int addr = (lane ^ 32) << 2;
  uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)v);
  uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// The bootstrapping key as a global-address-space pointer: the key table
// yields a generic pointer, and loads through it would otherwise be FLAT
// loads that also count against the LDS wait counter.
typedef __attribute__((address_space(1))) const uint64_t gmem_u64;
__device__ __forceinline__ const gmem_u64* as_global(const uint64_t* p) {
  return (const gmem_u64*)(const void*)p;
}
typedef __attribute__((address_space(1))) const uint32_t gmem_u32;
__device__ __forceinline__ const gmem_u32* as_global(const uint32_t* p) {
  return (const gmem_u32*)(const void*)p;
}

// ---- whole-wave transforms (layout of ntt64.h) ------------------------------
// 32 x 32 transposes of one polynomial held by a whole wave, through a
// 32 x 33 word block in two 32-bit passes.  From the pair layout of
// ntt64.h: on entry register r of lane (h, l) holds element (l, 16h +
// 2(r & 7) + (r >> 3)) of the matrix; on exit slot s holds element (2s + h,
// l).
__device__ __forceinline__ void transpose64_pairs(uint64_t (&a)[16], uint32_t* buf, int h, int l) {
  uint32_t lo[16];
  uint32_t* wr = buf + l * ROW + 16 * h;
#pragma unroll
  for (int r = 0; r < 16; ++r) wr[2 * (r & 7) + (r >> 3)] = (uint32_t)a[r];
  wave_fence();
#pragma unroll
  for (int s = 0; s < 16; ++s) lo[s] = buf[(2 * s + h) * ROW + l];
  wave_fence();
#pragma unroll
  for (int r = 0; r < 16; ++r) wr[2 * (r & 7) + (r >> 3)] = (uint32_t)(a[r] >> 32);
  wave_fence();
#pragma unroll
  for (int s = 0; s < 16; ++s) a[s] = ((uint64_t)buf[(2 * s + h) * ROW + l] << 32) | lo[s];
  wave_fence();
}

// Into the pair layout: on entry slot s of lane (h, l) holds element (l,
// 2s + h); on exit register r holds element (16h + 2(r & 7) + (r >> 3), l).
__device__ __forceinline__ void transpose64_to_pairs(uint64_t (&a)[16], uint32_t* buf, int h, int l) {
  uint32_t lo[16];
  const uint32_t* rd = buf + 16 * h * ROW + l;
#pragma unroll
  for (int s = 0; s < 16; ++s) buf[l * ROW + 2 * s + h] = (uint32_t)a[s];
  wave_fence();
#pragma unroll
  for (int r = 0; r < 16; ++r) lo[r] = rd[(2 * (r & 7) + (r >> 3)) * ROW];
  wave_fence();
#pragma unroll
  for (int s = 0; s < 16; ++s) buf[l * ROW + 2 * s + h] = (uint32_t)(a[s] >> 32);
  wave_fence();
#pragma unroll
  for (int r = 0; r < 16; ++r) a[r] = ((uint64_t)rd[(2 * (r & 7) + (r >> 3)) * ROW] << 32) | lo[r];
  wave_fence();
}

constexpr int T128_ROW = 36;  // u64 words per row of a two-wave transpose (bank spread)


__device__ __forceinline__ void vm_wait_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ void store_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t load_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace lp
