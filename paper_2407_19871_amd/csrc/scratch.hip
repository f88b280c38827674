// The library's static scratch area, for the gate-batch entry point that
// allocates nothing (lp_bootstrap_batch_noalloc).
//
// `scratch` is a file-scope device array of fixed size; every GPU the
// library runs on holds its own copy until the process ends.  In host code
// its name is only a host-side stand-in, so the device address of each copy
// is looked up once per device (hipGetSymbolAddress, with that device
// current) and kept; kernels and copies only ever see that address.
//
// Layout (byte offsets, each region 256-byte aligned):
//   sync  split-rotation control words for kNoAllocSplitJobs jobs
//   xbuf  split-rotation exchange slots for kNoAllocSplitJobs jobs
//   br    blind-rotation descriptors, 2 * kNoAllocMaxGates
//   ks    key-switch descriptors, kNoAllocMaxGates
//   ex    extracted samples (N+1 words), 2 * kNoAllocMaxGates
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "kernels.h"

namespace lp {

namespace {
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_ptr;  // device -> address of its copy of `scratch`

struct Offsets {
  size_t sync, xbuf, br, ks, ex, end;
};
Offsets layout() {
  Offsets o{};
  o.sync = 0;
  o.xbuf = align256(o.sync + split_sync_bytes(kNoAllocSplitJobs));
  o.br = align256(o.xbuf + split_xbuf_bytes(kNoAllocSplitJobs));
  o.ks = align256(o.br + 2 * (size_t)kNoAllocMaxGates * sizeof(BrJob));
  o.ex = align256(o.ks + (size_t)kNoAllocMaxGates * sizeof(KsJob));
  o.end = o.ex + 2 * (size_t)kNoAllocMaxGates * (RING_N_MAX + 1) * sizeof(uint32_t);
  return o;
}
}  // namespace

hipError_t noalloc_scratch(NoAllocScratch* out) {
  if (!out) return hipErrorInvalidValue;
  const Offsets o = layout();
  if (o.end > kNoAllocScratchBytes) return hipErrorInvalidValue;  // the regions above must fit the array
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return e;
      if (!p) return hipErrorInvalidSymbol;
      it = g_scratch_ptr.emplace(dev, static_cast<unsigned char*>(p)).first;
    }
    base = it->second;
  }
  out->split.sync = reinterpret_cast<uint32_t*>(base + o.sync);
  out->split.xbuf = reinterpret_cast<uint64_t*>(base + o.xbuf);
  out->split.max_jobs = kNoAllocSplitJobs;
  out->br = reinterpret_cast<BrJob*>(base + o.br);
  out->ks = reinterpret_cast<KsJob*>(base + o.ks);
  out->ex = reinterpret_cast<uint32_t*>(base + o.ex);
  return hipSuccess;
}

}  // namespace lp
