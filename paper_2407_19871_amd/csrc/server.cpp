// Query server: continuous batching of bounding-box queries from many
// clients, each request carrying its own keys.
//
// A scheduler thread owns one HIP stream.  Requests wait in a FIFO queue
// until the device bytes they need (keys, ciphertext pool, extract and job
// buffers) fit the configured budget; an admitted request gets its own device
// key and pool.  Every tick fuses the next depth level of every admitted
// request into one blind-rotation launch and one key-switch launch (jobs
// select their request's key and pool through per-tick tables), then
// advances each request by one level.  Requests that arrive while others are
// on the GPU join at the next tick, so their work shares launches with the
// requests already in flight.  A finished request's result is copied to the
// host and its device memory released.
//
// With a per-tick rotation cap, a tick runs at most that many blind
// rotations: requests with less of their level left than an equal share of
// the cap run all of it, the others split the rest, and a request whose
// level does not fit runs it over several ticks.  Gates within a level are
// independent, so results do not change; the tick time is bounded, which
// keeps a wide request from slowing every narrow one it shares ticks with.
//
// simulate = 1 runs the same admission and scheduling without touching a
// GPU (results are zero), which lets the host logic be tested on a CPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "jobs.h"
#include "kernels.h"

namespace {
using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  const lp_cloud_key* ck = nullptr;
  std::unique_ptr<lp_cloud_key> own_ck;  // the key deserialized from a submitted blob
  uint32_t l = 0, N = 0, m = 0;
  int is_signed = 0;
  std::vector<uint32_t> inputs;  // n_inputs * (n+1) words
  std::shared_ptr<const lp::Plan> plan;
  size_t bytes = 0;
  lp_device_key* dk = nullptr;
  uint32_t* pool = nullptr;
  int level = 0;
  size_t ks_pos = 0, br_pos = 0;  // jobs of the current level already run
  std::vector<uint32_t> out;
  lp_status status = LP_EAGAIN;
  std::string err;  // why the request failed (the scheduler thread's last error)
  bool cancel = false;
  Clock::time_point t_submit;
  double latency = 0.0;
};

template <typename T>
hipError_t grow(T** p, size_t* cap, size_t need) {
  if (need <= *cap) return hipSuccess;
  const size_t n = std::max(need, *cap * 2);
  if (*p) {
    hipError_t e = hipFree(*p);
    if (e != hipSuccess) return e;
  }
  *p = nullptr;
  *cap = 0;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e == hipSuccess) *cap = n;
  return e;
}
}  // namespace

struct lp_server {
  lp_server_config cfg{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> pending;
  std::vector<std::shared_ptr<Request>> active;
  std::map<uint64_t, std::shared_ptr<Request>> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  lp_server_stats st{};
  std::thread worker;
  hipStream_t stream = nullptr;
  // device buffers reused across ticks
  lp::BrJob* d_br = nullptr;
  size_t cap_br = 0;
  lp::KsJob* d_ks = nullptr;
  size_t cap_ks = 0;
  uint32_t* ex = nullptr;
  size_t cap_ex = 0;
  const uint64_t** d_bsk_tab = nullptr;
  size_t cap_bt = 0;
  const uint32_t** d_ksk_tab = nullptr;
  size_t cap_kt = 0;
  uint32_t** d_pool_tab = nullptr;
  size_t cap_pt = 0;
  lp::SplitArea split;  // exchange area of split rotations, made at first use
};

namespace {

size_t request_bytes(const lp_params& P, const lp::Plan& plan) {
  const size_t w = P.n + 1;
  const size_t key = lp_bsk_words(&P) * 8 + lp_ksk_words(&P) * 4;
  const size_t pool = (size_t)plan.n_slots * w * 4;
  const size_t lvl = plan.max_level_br();
  const size_t ex = lvl * (P.N + 1) * 4;
  const size_t jobs = lvl * (sizeof(lp::BrJob) + sizeof(lp::KsJob)) * 2;
  return key + pool + ex + jobs;
}

lp_status check_host_query(const lp_bbox_query_host* q) {
  if (!q) return lp::fail(LP_EINVAL, "null query");
  if (q->l == 0 || q->l > 64 || q->n_boxes == 0 || q->n_boxes > 4096 || q->m == 0 || q->m > 4096)
    return lp::fail(LP_EINVAL, "query shape out of range (l=%u, boxes=%u, m=%u)", q->l, q->n_boxes, q->m);
  if (!q->x || !q->y || !q->bounds || !q->payload) return lp::fail(LP_EINVAL, "null query input");
  return LP_OK;
}

void release(lp_server* S, Request& r) {
  if (!S->cfg.simulate) {
    if (r.pool) (void)hipFree(r.pool);
    if (r.dk) lp_device_key_free(r.dk);
  }
  r.pool = nullptr;
  r.dk = nullptr;
}

// Caller holds S->mu.
void finish_locked(lp_server* S, Request& r, lp_status status) {
  r.status = status;
  if (status != LP_OK && status != LP_ECANCELED && r.err.empty()) r.err = lp_last_error();
  r.latency = std::chrono::duration<double>(Clock::now() - r.t_submit).count();
  S->st.bytes_in_use -= r.bytes;
  if (status == LP_OK) S->st.completed++;
  else if (status == LP_ECANCELED) S->st.cancelled++;
  else S->st.failed++;
  r.inputs.clear();
  r.inputs.shrink_to_fit();
  if (r.own_ck) {
    r.ck = nullptr;
    r.own_ck.reset();
  }
  S->cv_done.notify_all();
}

lp_status setup_request(lp_server* S, Request& r) {
  if (r.ticket == S->cfg.fail_ticket) return lp::fail(LP_ENOMEM, "request %llu: injected allocation failure",
                                                       (unsigned long long)r.ticket);
  if (S->cfg.simulate) return LP_OK;
  lp_status st = lp_device_key_create(r.ck, S->stream, &r.dk);
  if (st != LP_OK) return st;
  const size_t w = r.ck->P.n + 1;
  hipError_t e = hipMalloc(&r.pool, (size_t)r.plan->n_slots * w * 4);
  if (e != hipSuccess) return lp::fail(LP_ENOMEM, "request pool: %s", hipGetErrorString(e));
  e = hipMemcpyAsync(r.pool, r.inputs.data(), r.inputs.size() * 4, hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return lp::fail(LP_EDEVICE, "request upload: %s", hipGetErrorString(e));
  return LP_OK;
}

// Requests fuse only with requests of the same LWE dimension and key-switching
// shape: a fused launch reads every request's pool with one sample stride.
bool same_shape(const lp_params& a, const lp_params& b) {
  return a.n == b.n && a.ks_t == b.ks_t && a.ks_base_bit == b.ks_base_bit;
}

// A request's part of a tick: key switches [k0, k1) of its current level
// and the rotations they read, [r0, r1).  The plan lists a level's
// rotations in the order of the key switches that read them (two for a MUX,
// one otherwise), and a rotation's output index is its place in the level,
// so both ranges are contiguous.
struct Chunk {
  size_t k0, k1, r0, r1;
};

// Rotations per request under a cap (0 = none) by water-filling over the
// rotations each has left in its level; every request gets at least one
// key switch.  LP_EINVAL if a level breaks the order above.
lp_status plan_chunks(const std::vector<std::shared_ptr<Request>>& act, uint32_t cap, std::vector<Chunk>* out) {
  const size_t n = act.size();
  std::vector<size_t> left(n), budget(n), order(n);
  for (size_t k = 0; k < n; ++k) {
    left[k] = act[k]->plan->br[act[k]->level].size() - act[k]->br_pos;
    order[k] = k;
  }
  if (cap == 0) {
    budget = left;
  } else {
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return left[a] < left[b]; });
    size_t rem = cap;
    for (size_t i = 0; i < n; ++i) {
      const size_t k = order[i];
      budget[k] = std::min(left[k], std::max<size_t>(rem / (n - i), 1));
      rem -= std::min(rem, budget[k]);
    }
  }
  out->assign(n, Chunk{});
  for (size_t k = 0; k < n; ++k) {
    const Request& r = *act[k];
    const std::vector<lp::KsJob>& ks = r.plan->ks[r.level];
    Chunk c{r.ks_pos, r.ks_pos, r.br_pos, r.br_pos};
    while (c.k1 < ks.size()) {
      const lp::KsJob& j = ks[c.k1];
      const size_t w = j.ex1 != lp::REF_NONE ? 2 : 1;
      if (j.ex0 != c.r1 || (w == 2 && j.ex1 != c.r1 + 1))
        return lp::fail(LP_EINVAL, "server: level %d of a plan is out of rotation order", r.level);
      if (c.k1 > c.k0 && c.r1 - c.r0 + w > budget[k]) break;
      c.r1 += w;
      ++c.k1;
    }
    (*out)[k] = c;
  }
  return LP_OK;
}

// The configured cap, LP_TICK_CAP_AUTO resolved: the narrowest width the
// timed table runs within 15 % of its best rate per rotation (wider ticks
// gain little throughput and cost latency), else kAutoTickCap.
constexpr uint32_t kAutoTickCap = 2048;
uint32_t tick_cap(uint32_t cfg) {
  if (cfg != LP_TICK_CAP_AUTO) return cfg;
  const uint32_t knee = lp::throughput_knee(0.15f);
  return knee ? knee : kAutoTickCap;
}

// One fused tick over admitted requests of one shape: each request's chunk
// of its current level.  (*stalled)[k] counts the jobs of request k whose
// split rotation gave up a wait in this tick (their outputs are undefined).
lp_status tick(lp_server* S, const std::vector<std::shared_ptr<Request>>& act, const std::vector<Chunk>& ch,
               uint64_t* n_br_out, std::vector<uint32_t>* stalled) {
  using lp::BrJob;
  using lp::KsJob;
  std::vector<BrJob> br;
  std::vector<KsJob> ks;
  std::vector<size_t> per_key;
  size_t ks_total = 0;
  std::vector<uint32_t> ex_base(act.size());
  uint32_t ex_cnt = 0;
  for (size_t k = 0; k < act.size(); ++k) {
    const lp::Plan& P = *act[k]->plan;
    const Chunk& c = ch[k];
    ex_base[k] = ex_cnt;
    for (size_t q = c.r0; q < c.r1; ++q) {
      BrJob j = P.br[act[k]->level][q];
      if (j.in0 != lp::REF_NONE) j.in0 = lp::make_ref(lp::KEY_POOL_BASE, j.in0 & lp::REF_INDEX_MASK);
      if (j.in1 != lp::REF_NONE) j.in1 = lp::make_ref(lp::KEY_POOL_BASE, j.in1 & lp::REF_INDEX_MASK);
      j.out = j.out - (uint32_t)c.r0 + ex_base[k];
      j.key = (uint32_t)k;
      br.push_back(j);
    }
    ex_cnt += (uint32_t)(c.r1 - c.r0);
    per_key.push_back(c.k1 - c.k0);
    ks_total += c.k1 - c.k0;
  }
  const int tile = lp::fused_ks_tile(per_key, ks_total);
  for (size_t k = 0; k < act.size(); ++k) {
    const lp::Plan& P = *act[k]->plan;
    const Chunk& c = ch[k];
    size_t cnt = 0;
    for (size_t q = c.k0; q < c.k1; ++q) {
      KsJob j = P.ks[act[k]->level][q];
      j.ex0 = j.ex0 - (uint32_t)c.r0 + ex_base[k];
      if (j.ex1 != lp::REF_NONE) j.ex1 = j.ex1 - (uint32_t)c.r0 + ex_base[k];
      j.out = lp::make_ref(lp::KEY_POOL_BASE, j.out & lp::REF_INDEX_MASK);
      j.key = (uint32_t)k;
      ks.push_back(j);
      ++cnt;
    }
    for (; cnt % tile; ++cnt) ks.push_back(KsJob{lp::REF_NONE, lp::REF_NONE, 0u, 0u, (uint32_t)k, {0, 0, 0}});
  }
  *n_br_out = br.size();
  stalled->assign(act.size(), 0);
  if (S->cfg.simulate) {
    std::this_thread::sleep_for(std::chrono::microseconds(200));
    return LP_OK;
  }
  const lp_params& Pp = act[0]->ck->P;
  std::vector<const uint64_t*> bt(act.size());
  std::vector<const uint32_t*> kt(act.size());
  std::vector<uint32_t*> pt(act.size());
  for (size_t k = 0; k < act.size(); ++k) {
    bt[k] = act[k]->dk->bsk_ntt;
    kt[k] = act[k]->dk->ksk;
    pt[k] = act[k]->pool;
  }
  hipError_t e = grow(&S->d_br, &S->cap_br, br.size());
  if (e == hipSuccess) e = grow(&S->d_ks, &S->cap_ks, ks.size());
  if (e == hipSuccess) e = grow(&S->ex, &S->cap_ex, (size_t)ex_cnt * (Pp.N + 1));
  if (e == hipSuccess) e = grow(&S->d_bsk_tab, &S->cap_bt, act.size());
  if (e == hipSuccess) e = grow(&S->d_ksk_tab, &S->cap_kt, act.size());
  if (e == hipSuccess) e = grow(&S->d_pool_tab, &S->cap_pt, act.size());
  if (e == hipSuccess) e = hipMemcpyAsync(S->d_br, br.data(), br.size() * sizeof(BrJob), hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(S->d_ks, ks.data(), ks.size() * sizeof(KsJob), hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(S->d_bsk_tab, bt.data(), bt.size() * 8, hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(S->d_ksk_tab, kt.data(), kt.size() * 8, hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(S->d_pool_tab, pt.data(), pt.size() * 8, hipMemcpyHostToDevice, S->stream);
  lp::SrcBases src{};
  lp::DstBases dst{};
  const lp::Twiddles tw = act[0]->dk->tw;
  const int waves = lp::pick_br_wpb(br.size());
  if (e == hipSuccess && lp::is_split(waves) && S->split.max_jobs < (int)br.size()) {
    // ticks run one at a time, so the previous area is idle once the stream is
    e = hipStreamSynchronize(S->stream);
    if (e == hipSuccess) {
      lp::split_area_free(&S->split);
      e = lp::split_area_alloc(&S->split, lp::kSplitDualMaxJobs);
    }
  }
  if (e == hipSuccess) {
    lp::ProfScope ps(lp::kProfBR, br.size(), waves, S->stream);
    e = lp::launch_blind_rotate(S->d_br, (int)br.size(), src, S->ex, S->d_bsk_tab, S->d_pool_tab, (int)Pp.n, (int)Pp.n,
                                0, tw, waves, S->stream, &S->split);
  }
  if (e == hipSuccess) {
    lp::ProfScope ps(lp::kProfKS, ks.size(), tile, S->stream);
    e = lp::launch_keyswitch(S->d_ks, (int)ks.size(), S->ex, dst, S->d_ksk_tab, S->d_pool_tab, (int)Pp.n, (int)Pp.N,
                             (int)Pp.ks_t, (int)Pp.ks_base_bit, tile, lp::pick_ks_split(ks.size(), tile, Pp.n),
                             S->stream);
  }
  // the host job arrays must outlive every copy queued above, also on failure
  const hipError_t es = hipStreamSynchronize(S->stream);
  if (e == hipSuccess) e = es;
  if (e == hipSuccess && lp::is_split(waves)) {
    // split waits that ran out: only the requests owning those jobs fail
    uint32_t n_stalls = 0;
    std::vector<int> jobs;
    e = lp::split_area_take_stalls(&S->split, S->stream, &n_stalls, &jobs);
    for (int j : jobs)
      if (j < (int)br.size()) (*stalled)[br[j].key] += 1;
  }
  if (e != hipSuccess) return lp::fail(LP_EDEVICE, "server tick: %s", hipGetErrorString(e));
  return LP_OK;
}

lp_status collect_output(lp_server* S, Request& r) {
  const size_t w = r.ck->P.n + 1;
  r.out.assign((size_t)r.m * w, 0u);
  if (S->cfg.simulate) return LP_OK;
  for (uint32_t j = 0; j < r.m; ++j) {
    hipError_t e = hipMemcpyAsync(r.out.data() + (size_t)j * w, r.pool + (size_t)r.plan->out_slots[j] * w, w * 4,
                                  hipMemcpyDeviceToHost, S->stream);
    if (e != hipSuccess) return lp::fail(LP_EDEVICE, "result copy: %s", hipGetErrorString(e));
  }
  hipError_t e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return lp::fail(LP_EDEVICE, "result copy: %s", hipGetErrorString(e));
  return LP_OK;
}

void worker_main(lp_server* S) {
  if (!S->cfg.simulate) (void)hipSetDevice(S->device);
  for (;;) {
    std::vector<std::shared_ptr<Request>> admit, act;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty() || !S->active.empty(); });
      if (S->stop && S->pending.empty() && S->active.empty()) break;
      // FIFO admission by budget and slot count
      while (!S->pending.empty()) {
        auto& r = S->pending.front();
        if (r->cancel) {
          S->st.bytes_in_use += r->bytes;  // finish_locked releases it
          finish_locked(S, *r, LP_ECANCELED);
          S->pending.pop_front();
          continue;
        }
        if (S->cfg.max_inflight && S->active.size() + admit.size() >= S->cfg.max_inflight) break;
        if (S->st.bytes_in_use + r->bytes > S->cfg.hbm_budget) break;
        S->st.bytes_in_use += r->bytes;
        S->st.peak_bytes = std::max(S->st.peak_bytes, S->st.bytes_in_use);
        admit.push_back(r);
        S->pending.pop_front();
      }
    }
    for (auto& r : admit) {
      lp_status st = setup_request(S, *r);
      std::lock_guard<std::mutex> lk(S->mu);
      if (st != LP_OK) {
        release(S, *r);
        finish_locked(S, *r, st);
      } else {
        S->active.push_back(r);
        S->st.admitted++;
      }
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (auto it = S->active.begin(); it != S->active.end();) {
        if ((*it)->cancel) {
          release(S, **it);
          finish_locked(S, **it, LP_ECANCELED);
          it = S->active.erase(it);
        } else {
          ++it;
        }
      }
      act = S->active;
      S->st.active = (uint32_t)act.size();
      S->st.pending = (uint32_t)S->pending.size();
    }
    if (act.empty()) continue;
    std::vector<std::vector<std::shared_ptr<Request>>> groups;
    for (auto& r : act) {
      auto g = std::find_if(groups.begin(), groups.end(), [&](const std::vector<std::shared_ptr<Request>>& v) {
        return same_shape(v[0]->ck->P, r->ck->P);
      });
      if (g == groups.end()) groups.push_back({r});
      else g->push_back(r);
    }
    uint64_t nbr = 0;
    std::vector<std::shared_ptr<Request>> done;
    std::vector<lp_status> done_st;
    uint64_t widest = 0;
    for (auto& g : groups) {
      uint64_t n = 0;
      std::vector<Chunk> ch;
      std::vector<uint32_t> stalled(g.size(), 0);
      lp_status st = plan_chunks(g, tick_cap(S->cfg.max_tick_rotations), &ch);
      if (st == LP_OK) st = tick(S, g, ch, &n, &stalled);
      nbr += n;
      widest = std::max(widest, n);
      for (size_t i = 0; i < g.size(); ++i) {
        Request& r = *g[i];
        if (st == LP_OK && stalled[i]) {
          done.push_back(g[i]);
          done_st.push_back(lp::split_stall_error("server request", stalled[i]));
          r.err = lp_last_error();
          continue;
        }
        if (st == LP_OK) {
          r.ks_pos = ch[i].k1;
          r.br_pos = ch[i].r1;
          if (r.ks_pos < r.plan->ks[r.level].size()) continue;  // the level goes on next tick
          r.ks_pos = r.br_pos = 0;
          if (++r.level < r.plan->levels()) continue;
        }
        done.push_back(g[i]);
        done_st.push_back(st == LP_OK ? collect_output(S, r) : st);
        if (done_st.back() != LP_OK) r.err = lp_last_error();
      }
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->st.ticks += groups.size();
    S->st.fused_bootstraps += nbr;
    S->st.widest_tick = std::max(S->st.widest_tick, widest);
    for (size_t i = 0; i < done.size(); ++i) {
      release(S, *done[i]);
      finish_locked(S, *done[i], done_st[i]);
      S->active.erase(std::find(S->active.begin(), S->active.end(), done[i]));
    }
  }
}
}  // namespace

extern "C" lp_status lp_server_create(const lp_server_config* cfg, lp_server** out) {
  if (!cfg || !out) return lp::fail(LP_EINVAL, "lp_server_create: null argument");
  if (cfg->hbm_budget == 0) return lp::fail(LP_EINVAL, "lp_server_create: zero budget");
  auto S = std::make_unique<lp_server>();
  S->cfg = *cfg;
  if (!cfg->simulate) {
    LP_HIP_TRY(hipGetDevice(&S->device));
    LP_HIP_TRY(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
  }
  lp_server* raw = S.release();
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return LP_OK;
}

extern "C" lp_status lp_server_request_bytes(const lp_cloud_key* ck, const lp_bbox_query_host* q, size_t* bytes) {
  if (!ck || !bytes) return lp::fail(LP_EINVAL, "lp_server_request_bytes: null argument");
  lp_status st = check_host_query(q);
  if (st != LP_OK) return st;
  *bytes = request_bytes(ck->P, *lp::get_plan(q->l, q->n_boxes, q->m, q->is_signed ? 1 : 0, false));
  return LP_OK;
}

namespace {
// Queues a request under key ck (owned by the request when `owned` holds
// it); t0 is the moment the request arrived.
lp_status submit(lp_server* S, const char* who, const lp_cloud_key* ck, std::unique_ptr<lp_cloud_key> owned,
                 const lp_bbox_query_host* q, uint64_t* ticket, Clock::time_point t0) {
  if (!S->cfg.simulate && (ck->P.N != 1024 || ck->P.l != 3 || ck->P.bg_bit != 7 || ck->P.n > 1024))
    return lp::fail(LP_EUNSUPPORTED, "%s: parameters the GPU kernels do not handle", who);
  auto r = std::make_shared<Request>();
  r->ck = ck;
  r->own_ck = std::move(owned);
  r->l = q->l;
  r->N = q->n_boxes;
  r->m = q->m;
  r->is_signed = q->is_signed ? 1 : 0;
  r->plan = lp::get_plan(r->l, r->N, r->m, r->is_signed, false);
  r->bytes = request_bytes(ck->P, *r->plan);
  if (r->bytes > S->cfg.hbm_budget)
    return lp::fail(LP_EBUDGET, "%s: request needs %zu bytes, budget is %zu", who, r->bytes, S->cfg.hbm_budget);
  const size_t w = ck->P.n + 1, l = q->l, N = q->n_boxes, m = q->m;
  r->inputs.resize((size_t)r->plan->n_inputs * w);
  uint32_t* p = r->inputs.data();
  std::memcpy(p, q->x, l * w * 4);
  std::memcpy(p + l * w, q->y, l * w * 4);
  std::memcpy(p + 2 * l * w, q->bounds, 4 * l * N * w * 4);
  std::memcpy(p + (2 * l + 4 * l * N) * w, q->payload, N * m * w * 4);
  r->t_submit = t0;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return lp::fail(LP_EINVAL, "%s: server is shutting down", who);
    r->ticket = S->next_ticket++;
    S->all[r->ticket] = r;
    S->pending.push_back(r);
    S->st.submitted++;
    S->st.pending = (uint32_t)S->pending.size();
  }
  S->cv_work.notify_one();
  *ticket = r->ticket;
  return LP_OK;
}
}  // namespace

extern "C" lp_status lp_server_submit(lp_server* S, const lp_cloud_key* ck, const lp_bbox_query_host* q,
                                      uint64_t* ticket) {
  const Clock::time_point t0 = Clock::now();
  if (!S || !ck || !ticket) return lp::fail(LP_EINVAL, "lp_server_submit: null argument");
  lp_status st = check_host_query(q);
  if (st != LP_OK) return st;
  return submit(S, "lp_server_submit", ck, nullptr, q, ticket, t0);
}

extern "C" lp_status lp_server_submit_blob(lp_server* S, const void* key_blob, size_t key_len,
                                           const lp_bbox_query_host* q, uint64_t* ticket) {
  const Clock::time_point t0 = Clock::now();
  if (!S || !key_blob || !ticket) return lp::fail(LP_EINVAL, "lp_server_submit_blob: null argument");
  lp_status st = check_host_query(q);
  if (st != LP_OK) return st;
  lp_cloud_key* ck = nullptr;
  st = lp_cloud_key_deserialize(key_blob, key_len, &ck);
  if (st != LP_OK) return st;
  std::unique_ptr<lp_cloud_key> own(ck);
  return submit(S, "lp_server_submit_blob", ck, std::move(own), q, ticket, t0);
}

extern "C" lp_status lp_server_poll(lp_server* S, uint64_t ticket, int wait, uint32_t* out, double* latency_s) {
  if (!S) return lp::fail(LP_EINVAL, "lp_server_poll: null server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return lp::fail(LP_EINVAL, "lp_server_poll: unknown ticket %llu", (unsigned long long)ticket);
  std::shared_ptr<Request> r = it->second;
  if (r->status == LP_EAGAIN) {
    if (!wait) return LP_EAGAIN;
    S->cv_done.wait(lk, [&] { return r->status != LP_EAGAIN; });
  }
  if (latency_s) *latency_s = r->latency;
  const lp_status st = r->status;
  if (st == LP_OK && out) std::memcpy(out, r->out.data(), r->out.size() * 4);
  S->all.erase(ticket);
  if (st != LP_OK)
    return lp::fail(st, "request %llu ended with status %d%s%s", (unsigned long long)ticket, (int)st,
                    r->err.empty() ? "" : ": ", r->err.c_str());
  return LP_OK;
}

extern "C" lp_status lp_server_cancel(lp_server* S, uint64_t ticket) {
  if (!S) return lp::fail(LP_EINVAL, "lp_server_cancel: null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return lp::fail(LP_EINVAL, "lp_server_cancel: unknown ticket");
  it->second->cancel = true;
  S->cv_work.notify_one();
  return LP_OK;
}

extern "C" lp_status lp_server_stats_get(lp_server* S, lp_server_stats* out) {
  if (!S || !out) return lp::fail(LP_EINVAL, "lp_server_stats_get: null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  out->pending = (uint32_t)S->pending.size();
  out->active = (uint32_t)S->active.size();
  return LP_OK;
}

extern "C" void lp_server_free(lp_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  if (!S->cfg.simulate) {
    for (void* p : {(void*)S->d_br, (void*)S->d_ks, (void*)S->ex, (void*)S->d_bsk_tab, (void*)S->d_ksk_tab,
                    (void*)S->d_pool_tab})
      if (p) (void)hipFree(p);
    lp::split_area_free(&S->split);
    if (S->stream) (void)hipStreamDestroy(S->stream);
  }
  delete S;
}
