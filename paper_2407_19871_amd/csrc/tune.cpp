// Launch-shape selection and its autotuner.
//
// Two shapes decide how a level of gates runs: the number of waves that
// cooperate on one blind rotation (1: independent bootstraps fill the GPU;
// 2: one accumulator component per wave, for levels of about one bootstrap
// per SIMD; 3: one gadget level per wave, for narrower levels; 4: the
// same with the levels summed in the NTT domain and one inverse per
// component on two waves; 5: the same sized for two bootstraps per CU; 6:
// the bootstrap split over two workgroups, one
// accumulator component each, for levels of at most kSplitMaxJobs jobs)
// and the key-switch tile and ring-index split.  The best choice depends on the
// job count, so the autotuner times every shape at a set of batch sizes on
// the device itself and installs the fastest per size as that device's
// table; every launch then looks its job count up in the table.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace lp {
namespace {

std::mutex g_tune_mu;
std::map<int, std::vector<lp_tune_entry>> g_tune;  // device -> rows sorted by jobs

constexpr uint32_t kMaxTuneJobs = 1u << 22;      // row bound
constexpr uint32_t kMaxTuneBucket = 1u << 16;    // batch size the autotuner times
const int kWaves[] = {1, 2, 3, 4, 5, 6, 7};
constexpr int kNumWaves = sizeof(kWaves) / sizeof(kWaves[0]);
const int kTiles[] = {1, 4, 8, 16};
const int kSplits[] = {1, 2, 4, 8, 16};

bool one_of(int v, const int* set, int n) {
  for (int i = 0; i < n; ++i)
    if (set[i] == v) return true;
  return false;
}

bool row_ok(const lp_tune_entry& r) {
  return r.jobs >= 1 && r.jobs <= kMaxTuneJobs && one_of(r.br_waves, kWaves, kNumWaves) && one_of(r.ks_tile, kTiles, 4) &&
         one_of(r.ks_split, kSplits, 5);
}

// Table key of the calling thread's current device (-1 on a host without
// one, so that the table logic also runs there).
int current_device() {
  int dev = 0;
  return hipGetDevice(&dev) == hipSuccess ? dev : -1;
}

// The current device's row for njobs, false without a table.
bool tuned_row(size_t njobs, lp_tune_entry* row) {
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(dev);
  if (it == g_tune.end() || it->second.empty()) return false;
  for (const auto& r : it->second)
    if (njobs <= r.jobs) {
      *row = r;
      return true;
    }
  *row = it->second.back();
  return true;
}

lp_status install(int dev, std::vector<lp_tune_entry> rows) {
  std::sort(rows.begin(), rows.end(), [](const lp_tune_entry& a, const lp_tune_entry& b) { return a.jobs < b.jobs; });
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (rows.empty()) g_tune.erase(dev);
    else g_tune[dev] = std::move(rows);
  }
  sched_forget_all();
  return LP_OK;
}

}  // namespace

// The key switch with t = 8 compiled in (its rows requested one ring index
// ahead) is fastest, on MI355X, at 4 jobs per wave from 16 jobs and 8 from
// 256 (16 needs 209 VGPRs), and with the ring split until a launch has
// 64 k blocks, at most 16 ways: 33 us for one job, 1.47 us per job at 128,
// 1.15 at 1024, 1.10 at 16384 (autotuner, split 16 up to 4096 and 4 at
// 16384).
int default_ks_tile(size_t njobs) { return njobs >= 256 ? 8 : njobs >= 16 ? 4 : 1; }

int default_ks_split(size_t njobs, int tile, uint32_t n_lwe) {
  const size_t blocks = ((n_lwe + 64) / 64) * ((njobs + tile - 1) / tile);
  int sp = 1;
  while (sp < 16 && blocks * sp < 65536) sp *= 2;
  return sp;
}

// MI355X, n = 630, gate batches with their key switch: split 5.9 ms up to
// 128 rotations; the split two workgroups per CU 10.1-10.7 ms at 129-256
// (four waves two per CU 12.5-12.6, one per CU 13.6-13.9); four waves two
// per CU 19.4-20.5 ms at 384-512 and 30.0-30.1 ms at 640-768 (two waves
// 28.9-30.2); two waves, one per component, 33.9 ms at 1024 (four waves
// 39.0, one wave 41.9) and 47.1 ms at 1280 (48.4, 58.5); one wave from 1536,
// where two waves per rotation need a second round.
int default_br_wpb(size_t njobs) {
  if (njobs <= (size_t)kSplitMaxJobs) return 6;
  if (njobs <= (size_t)kSplitDualMaxJobs) return 7;
  if (njobs <= 768) return 5;
  return njobs <= 1280 ? 2 : 1;
}

int pick_ks_tile(size_t njobs) {
  const int t = env_int("LOCPIR_KS_TILE", 0);
  if (one_of(t, kTiles, 4)) return t;
  lp_tune_entry r;
  if (tuned_row(njobs, &r)) return r.ks_tile;
  return default_ks_tile(njobs);
}

int pick_ks_split(size_t njobs, int tile, uint32_t n_lwe) {
  const int forced = env_int("LOCPIR_KS_SPLIT", 0);
  if (one_of(forced, kSplits, 5)) return forced;
  lp_tune_entry r;
  // a row's split was measured with its own tile; a launch whose tile was
  // lowered (per-key padding) falls back to the default rule
  if (tuned_row(njobs, &r) && r.ks_tile == tile) return r.ks_split;
  return default_ks_split(njobs, tile, n_lwe);
}

// A split shape applies up to split_max_jobs(w) jobs; a wider launch that
// looks it up (the table's last row, or a forced shape) takes the split
// sized for two workgroups per CU (7) where that fits, else four waves two
// per CU (5).
int pick_br_wpb(size_t njobs) {
  auto fit = [&](int w) {
    if (!is_split(w) || njobs <= (size_t)split_max_jobs(w)) return w;
    return njobs <= (size_t)kSplitDualMaxJobs ? 7 : 5;
  };
  const int forced = env_int("LOCPIR_BR_WAVES", 0);
  if (one_of(forced, kWaves, kNumWaves)) return fit(forced);
  lp_tune_entry r;
  if (tuned_row(njobs, &r)) return fit(r.br_waves);
  return default_br_wpb(njobs);
}

// Estimated duration (microseconds) of a rotation launch of njobs
// bootstraps from the current device's timed table: the row's per-job time
// times the jobs for one wave per bootstrap (throughput), or times the
// row's bucket for the latency shapes (a launch below the bucket takes
// about as long as the bucket).  False without a timed row.
bool est_br_launch_us(size_t njobs, double* us) {
  lp_tune_entry r;
  if (njobs == 0 || !tuned_row(njobs, &r) || !(r.br_us > 0.f)) return false;
  const int w = pick_br_wpb(njobs);
  *us = (double)r.br_us * (double)(w == 1 ? njobs : std::max<size_t>(njobs, r.jobs));
  return true;
}

uint32_t throughput_knee(float tol) {
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(dev);
  if (it == g_tune.end()) return 0;
  float best = 0.f;
  for (const auto& r : it->second)
    if (r.br_us > 0.f && (best == 0.f || r.br_us < best)) best = r.br_us;
  if (best == 0.f) return 0;
  for (const auto& r : it->second)  // sorted by jobs
    if (r.br_us > 0.f && r.br_us <= best * (1.f + tol)) return r.jobs;
  return 0;
}

}  // namespace lp

using lp::fail;

extern "C" lp_status lp_tune_set(const lp_tune_entry* rows, int n) {
  if (n < 0 || n > LP_TUNE_MAX_ROWS || (n > 0 && !rows)) return fail(LP_EINVAL, "lp_tune_set: bad row count %d", n);
  std::vector<lp_tune_entry> v(rows, rows + n);
  for (const auto& r : v)
    if (!lp::row_ok(r))
      return fail(LP_EINVAL, "lp_tune_set: invalid row (jobs %u, br_waves %d, ks_tile %d, ks_split %d)", r.jobs,
                  r.br_waves, r.ks_tile, r.ks_split);
  for (size_t i = 0; i < v.size(); ++i)
    for (size_t j = i + 1; j < v.size(); ++j)
      if (v[i].jobs == v[j].jobs) return fail(LP_EINVAL, "lp_tune_set: duplicate bound %u", v[i].jobs);
  return lp::install(lp::current_device(), std::move(v));
}

extern "C" lp_status lp_tune_get(lp_tune_entry* rows, int* n) {
  if (!n || *n < 0 || (*n > 0 && !rows)) return fail(LP_EINVAL, "lp_tune_get: bad arguments");
  const int dev = lp::current_device();
  std::lock_guard<std::mutex> lk(lp::g_tune_mu);
  auto it = lp::g_tune.find(dev);
  const int have = it == lp::g_tune.end() ? 0 : (int)it->second.size();
  const int m = std::min(have, *n);
  for (int i = 0; i < m; ++i) rows[i] = it->second[i];
  *n = m;
  return LP_OK;
}

extern "C" lp_status lp_tune_pick(uint32_t jobs, uint32_t n_lwe, lp_tune_entry* out) {
  if (!out || jobs == 0) return fail(LP_EINVAL, "lp_tune_pick: bad arguments");
  lp_tune_entry r{};
  r.jobs = jobs;
  r.br_waves = lp::pick_br_wpb(jobs);
  r.ks_tile = lp::pick_ks_tile(jobs);
  r.ks_split = lp::pick_ks_split(jobs, r.ks_tile, n_lwe);
  *out = r;
  return LP_OK;
}

namespace {

// SplitMix64 for the random timing inputs (their values do not matter).
uint64_t mix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct TuneBuffers {
  uint32_t *in = nullptr, *ex = nullptr, *out = nullptr;
  lp::BrJob* br = nullptr;
  lp::KsJob* ks = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  lp::SplitArea split;
  ~TuneBuffers() {
    for (void* p : {(void*)in, (void*)ex, (void*)out, (void*)br, (void*)ks})
      if (p) (void)hipFree(p);
    lp::split_area_free(&split);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  }
};

}  // namespace

extern "C" lp_status lp_autotune(const lp_device_key* dk, const uint32_t* bucket_jobs, int nbuckets,
                                 uint32_t br_steps, void* stream, lp_tune_entry* out) {
  if (!dk || !bucket_jobs) return fail(LP_EINVAL, "lp_autotune: null argument");
  if (nbuckets < 1 || nbuckets > LP_TUNE_MAX_ROWS) return fail(LP_EINVAL, "lp_autotune: %d buckets", nbuckets);
  const uint32_t n = dk->P.n, N = dk->P.N;
  if (br_steps < 1 || br_steps > n) return fail(LP_EINVAL, "lp_autotune: br_steps %u outside 1..%u", br_steps, n);
  std::vector<uint32_t> sizes(bucket_jobs, bucket_jobs + nbuckets);
  for (uint32_t b : sizes)
    if (b < 1 || b > lp::kMaxTuneBucket) return fail(LP_EINVAL, "lp_autotune: bucket size %u outside 1..65536", b);
  std::sort(sizes.begin(), sizes.end());
  if (std::adjacent_find(sizes.begin(), sizes.end()) != sizes.end())
    return fail(LP_EINVAL, "lp_autotune: duplicate bucket size");

  lp::ScopedDevice sd(dk->device);
  hipStream_t s = lp::as_stream(stream);
  const size_t maxB = sizes.back(), w = n + 1;
  TuneBuffers B;
  LP_HIP_TRY(hipMalloc(&B.in, 2 * maxB * w * 4));
  LP_HIP_TRY(hipMalloc(&B.ex, maxB * (N + 1) * 4));
  LP_HIP_TRY(hipMalloc(&B.out, maxB * w * 4));
  LP_HIP_TRY(hipMalloc(&B.br, maxB * sizeof(lp::BrJob)));
  LP_HIP_TRY(hipMalloc(&B.ks, maxB * sizeof(lp::KsJob)));
  LP_HIP_TRY(hipEventCreate(&B.t0));
  LP_HIP_TRY(hipEventCreate(&B.t1));
  if (sizes.front() <= (uint32_t)lp::kSplitDualMaxJobs)
    LP_HIP_TRY(lp::split_area_alloc(&B.split, (int)std::min<size_t>(maxB, lp::kSplitDualMaxJobs)));
  {
    std::vector<uint32_t> h(2 * maxB * w);
    uint64_t st = 0x5EED0F7A11ull;
    for (auto& v : h) v = (uint32_t)mix64(st);
    LP_HIP_TRY(hipMemcpyAsync(B.in, h.data(), h.size() * 4, hipMemcpyHostToDevice, s));
    // NAND jobs: in0 = sample k of the first half, in1 = sample k of the second
    LP_HIP_TRY(lp::launch_make_batch_jobs(1, 0x20000000u, -1, -1, 1, maxB, B.br, B.ks, s));
    LP_HIP_TRY(hipStreamSynchronize(s));  // h must outlive the copy
  }
  lp::SrcBases src{};
  src.p[0] = B.in;
  src.p[1] = B.in + maxB * w;
  lp::DstBases dst{};
  dst.p[0] = B.out;

  // mean duration (ms) of `reps` launches after one untimed launch
  auto time = [&](auto&& launch, int reps, float* ms) -> lp_status {
    LP_HIP_TRY(launch());
    LP_HIP_TRY(hipEventRecord(B.t0, s));
    for (int r = 0; r < reps; ++r) LP_HIP_TRY(launch());
    LP_HIP_TRY(hipEventRecord(B.t1, s));
    LP_HIP_TRY(hipEventSynchronize(B.t1));
    float t = 0.f;
    LP_HIP_TRY(hipEventElapsedTime(&t, B.t0, B.t1));
    *ms = t / (float)reps;
    return LP_OK;
  };

  std::vector<lp_tune_entry> rows;
  for (uint32_t jobs : sizes) {
    lp_tune_entry r{};
    r.jobs = jobs;
    float best = -1.f;
    for (int W : lp::kWaves) {
      if (lp::is_split(W) && jobs > (uint32_t)lp::split_max_jobs(W)) continue;
      // the split sized for two workgroups per CU serves launches too wide
      // for the one-per-CU split; up to that width the two tie within the
      // timing's noise over the timed steps, and over a whole rotation the
      // one-per-CU split is faster (5.45 against 5.65 ms at 128 in a query)
      if (W == 7 && jobs <= (uint32_t)lp::kSplitMaxJobs) continue;
      float ms = 0.f;
      lp_status st = time(
          [&] {
            return lp::launch_blind_rotate(B.br, (int)jobs, src, B.ex, dk->bsk_tab, nullptr, (int)n, (int)br_steps, 0,
                                           dk->tw, W, s, &B.split);
          },
          2, &ms);
      if (st != LP_OK) return st;
      if (best < 0.f || ms < best) {
        best = ms;
        r.br_waves = W;
      }
    }
    // microseconds per bootstrap over all n steps
    r.br_us = best * 1000.f / (float)jobs * (float)n / (float)br_steps;
    // A key-switch shape is scored with the blind rotation that follows it:
    // on MI355X a 16-way ring split leaves the caches in a state that slows
    // the next rotation by up to 40% when one wave per SIMD exposes its key
    // loads (1024 one-wave bootstraps), although the key switch alone is no
    // slower.  In a circuit every key switch is followed by a rotation.
    best = -1.f;
    for (int T : lp::kTiles)
      for (int S : lp::kSplits) {
        if (N % (64u * (uint32_t)S)) continue;
        float ms = 0.f;
        lp_status st = time(
            [&] {
              hipError_t e = lp::launch_keyswitch(B.ks, (int)jobs, B.ex, dst, dk->ksk_tab, nullptr, (int)n, (int)N,
                                                  (int)dk->P.ks_t, (int)dk->P.ks_base_bit, T, S, s);
              if (e != hipSuccess) return e;
              return lp::launch_blind_rotate(B.br, (int)jobs, src, B.ex, dk->bsk_tab, nullptr, (int)n, (int)br_steps,
                                             0, dk->tw, r.br_waves, s, &B.split);
            },
            2, &ms);
        if (st != LP_OK) return st;
        if (best < 0.f || ms < best) {
          best = ms;
          r.ks_tile = T;
          r.ks_split = S;
        }
      }
    {
      float ms = 0.f;
      lp_status st = time(
          [&] {
            return lp::launch_keyswitch(B.ks, (int)jobs, B.ex, dst, dk->ksk_tab, nullptr, (int)n, (int)N,
                                        (int)dk->P.ks_t, (int)dk->P.ks_base_bit, r.ks_tile, r.ks_split, s);
          },
          3, &ms);
      if (st != LP_OK) return st;
      r.ks_us = ms * 1000.f / (float)jobs;
    }
    rows.push_back(r);
  }
  lp_status st = lp::install(dk->device, rows);
  if (st != LP_OK) return st;
  if (out)
    for (size_t i = 0; i < rows.size(); ++i) out[i] = rows[i];
  return LP_OK;
}
