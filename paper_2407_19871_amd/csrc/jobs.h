// Work descriptors shared by the host scheduler and the device kernels.
//
// A ciphertext operand is a 32-bit reference: the top 4 bits select one of
// up to 8 base arrays passed to the kernel, the low 28 bits give the index
// of the ciphertext in that array.  Descriptors therefore hold no raw
// pointers, and a compiled query plan can be replayed on any buffers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lp {

constexpr uint32_t REF_NONE = 0xFFFFFFFFu;
constexpr int REF_SHIFT = 28;
constexpr uint32_t REF_INDEX_MASK = (1u << REF_SHIFT) - 1;
constexpr int MAX_BASES = 8;
// Base id selecting the pool of the job's key (table `pool_tab[key]`): the
// query server gives every request its own key and its own pool.
constexpr uint32_t KEY_POOL_BASE = 15;

__host__ __device__ inline uint32_t make_ref(uint32_t base, uint32_t index) { return (base << REF_SHIFT) | index; }

// One blind rotation: its input is the linear combination
//   (0, cst) + c0 * ref0 + c1 * ref1     (LWE_n samples, mod 2^32)
// and its output is the sample extracted from the accumulator (N+1 words)
// written to slot `out` of the extract buffer.  `key` indexes the table of
// bootstrapping keys.
struct BrJob {
  uint32_t in0, in1;
  int32_t c0, c1;
  uint32_t cst;
  uint32_t out;
  uint32_t key;
  uint32_t pad;
};

// One key switch: input (0, cst) + extract[ex0] (+ extract[ex1]), output an
// LWE_n sample at reference `out`; `key` indexes the table of KS keys.
// All jobs of one key-switch tile must share the same key.
struct KsJob {
  uint32_t ex0, ex1;
  uint32_t cst;
  uint32_t out;
  uint32_t key;
  uint32_t pad[3];
};

struct SrcBases {
  const uint32_t* p[MAX_BASES];
};
struct DstBases {
  uint32_t* p[MAX_BASES];
};

}  // namespace lp
