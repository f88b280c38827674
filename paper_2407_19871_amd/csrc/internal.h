// Internal declarations shared by the host sources of liblocpir: handle
// layouts, error reporting, launch-shape selection, device scoping and the
// per-launch event profiler.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/locpir.h"
#include "jobs.h"
#include "kernels.h"

struct lp_secret_key {
  lp_params P;
  std::vector<uint8_t> s;  // LWE key, n bits
  std::vector<uint8_t> S;  // ring key, N bits
};

struct lp_cloud_key {
  lp_params P;
  std::vector<uint32_t> bsk;  // [n][2l][2][N]
  std::vector<uint32_t> ksk;  // [N][t][base-1][n+1]
};

struct lp_device_key {
  lp_params P;
  int device = 0;
  uint64_t* bsk_ntt = nullptr;         // [n][2l][2][N] NTT domain
  uint32_t* ksk = nullptr;             // [N][t][base-1][n+1]
  const uint64_t** bsk_tab = nullptr;  // device array {bsk_ntt}
  const uint32_t** ksk_tab = nullptr;  // device array {ksk}
  lp::Twiddles tw{};
  size_t bytes = 0;
};

namespace lp {

// Records a message for lp_last_error() and returns code.
lp_status fail(lp_status code, const char* fmt, ...);

#define LP_HIP_TRY(expr)                                                                          \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return ::lp::fail(LP_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Twiddle tables of the current device (uploaded once per device).
lp_status device_twiddles(Twiddles* out);

// LP_EDEVICE with a message naming `stalls` split-rotation waits that ran
// out of polls (their jobs' outputs are undefined).
lp_status split_stall_error(const char* who, uint32_t stalls);

// Drops every cached query program that references dk.
void sched_forget_key(const lp_device_key* dk);

// Jobs of one bounding-box query shape (Algorithms 2-5), by depth level.
// Ciphertext operands are pool slots (make_ref(0, slot)); blind-rotation
// outputs and key-switch inputs index the level's extract buffer from 0.
// Input slots come first: x (l), y (l), bounds (N x 4 x l), payload (N x m).
struct Plan {
  uint32_t l = 0, N = 0, m = 0;
  int is_signed = 0;
  uint32_t n_inputs = 0, n_slots = 0;
  uint64_t n_br = 0, n_ks = 0;
  std::vector<std::vector<BrJob>> br;
  std::vector<std::vector<KsJob>> ks;
  std::vector<uint32_t> out_slots;
  int levels() const { return (int)br.size(); }
  size_t max_level_br() const {
    size_t mx = 0;
    for (auto& v : br) mx = v.size() > mx ? v.size() : mx;
    return mx;
  }
};
// Cached plan of a shape (thread-safe); xnor_early places the comparators'
// XNORs all at the first level instead of next to the MUX that uses them.
std::shared_ptr<const Plan> get_plan(uint32_t l, uint32_t N, uint32_t m, int is_signed, bool xnor_early);
// The XNOR placement a program of these query shapes gets on the current
// device (one entry per query: l, N, m, signed).
bool choose_xnor_early(const std::vector<std::tuple<uint32_t, uint32_t, uint32_t, int>>& shapes);
// Key-switch tile for a fused launch with per-key job counts.
int fused_ks_tile(const std::vector<size_t>& per_key, size_t total);

// ---- launch shapes ---------------------------------------------------------
// Each launch asks for its shapes by job count: a valid LOCPIR_BR_WAVES,
// LOCPIR_KS_TILE or LOCPIR_KS_SPLIT in the environment wins, then the
// current device's autotuned table (tune.cpp), then built-in defaults
// measured on MI355X.
inline int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return (v && *v) ? std::atoi(v) : dflt;
}
int pick_ks_tile(size_t njobs);
int pick_ks_split(size_t njobs, int tile, uint32_t n_lwe);
// Estimated rotation launch time (us) of njobs from the current device's
// timed table; false when there is none.
bool est_br_launch_us(size_t njobs, double* us);
// The narrowest bucket of the current device's timed table whose rotation
// time per job is within a factor 1 + tol of the table's best; 0 when the
// table has no timed row.
uint32_t throughput_knee(float tol);
// Waves per bootstrap; the built-in rule: 6 (split over two workgroups) up
// to kSplitMaxJobs, 7 (the same, two workgroups per CU) up to
// kSplitDualMaxJobs, 5 (levels summed, two-wave inverses, two rotations per
// CU) up to 768, 2 (one accumulator component per wave) up to 1280, else 1.
int pick_br_wpb(size_t njobs);
// Built-in defaults (no environment, no table).
int default_ks_tile(size_t njobs);
int default_ks_split(size_t njobs, int tile, uint32_t n_lwe);
int default_br_wpb(size_t njobs);
// Drops every cached query program (after the shape table changed).
void sched_forget_all();

struct ScopedDevice {
  int prev = -1;
  explicit ScopedDevice(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~ScopedDevice() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// ---- profiling -------------------------------------------------------------
enum ProfKind { kProfBR = 0, kProfKS = 1, kProfKinds = 2 };
struct ProfRecord {
  int kind;
  uint64_t jobs;
  int shape;  // waves per bootstrap (blind rotation) or jobs per tile (key switching)
  hipEvent_t start, stop;
};
extern std::mutex g_prof_mu;
extern bool g_prof_on;
extern std::vector<ProfRecord> g_prof;

// Brackets one launch (or one graph launch) with events when profiling is on.
struct ProfScope {
  bool on = false;
  ProfRecord rec{};
  hipStream_t s;
  ProfScope(int kind, uint64_t jobs, int shape, hipStream_t st) : s(st) {
    {
      std::lock_guard<std::mutex> lk(g_prof_mu);
      on = g_prof_on;
    }
    if (!on || jobs == 0) {
      on = false;
      return;
    }
    rec.kind = kind;
    rec.jobs = jobs;
    rec.shape = shape;
    if (hipEventCreate(&rec.start) != hipSuccess) {
      on = false;
      return;
    }
    if (hipEventCreate(&rec.stop) != hipSuccess) {
      (void)hipEventDestroy(rec.start);
      on = false;
      return;
    }
    (void)hipEventRecord(rec.start, s);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(rec.stop, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back(rec);
  }
};

}  // namespace lp
