// The bounding-box circuit (Algorithms 2-5) as a DAG of gates, cut into
// depth levels, and the engine that runs one or many queries together:
// level L of every query goes into one blind-rotation launch and one
// key-switch launch, each job carrying the index of its query's key.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"
#include "jobs.h"
#include "kernels.h"

namespace lp {
namespace {

// ---------------------------------------------------------------- circuit
// A ciphertext of the circuit: an input or gate-output slot, possibly
// negated (HomNOT negates the sample and needs no bootstrap), or the
// noiseless trivial sample (0, tval).
struct CRef {
  int32_t slot = -1;  // -1: trivial sample
  bool neg = false;
  uint32_t tval = 0;
  int level = 0;
};

struct Gate {
  int kind;  // LP_GATE_AND, LP_GATE_XNOR, LP_GATE_XOR or LP_GATE_MUX
  CRef in[3];
  int level;
  int32_t out;
};

CRef cnot(CRef r) {
  if (r.slot < 0) r.tval = 0u - r.tval;
  else r.neg = !r.neg;
  return r;
}

struct Circuit {
  int32_t n_slots = 0;
  std::vector<Gate> gates;
  std::vector<CRef> outputs;

  CRef input() {
    CRef r;
    r.slot = n_slots++;
    return r;
  }
  CRef gate(int kind, CRef a, CRef b, CRef c = CRef()) {
    Gate g;
    g.kind = kind;
    g.in[0] = a;
    g.in[1] = b;
    g.in[2] = c;
    g.level = 1 + std::max({a.level, b.level, kind == LP_GATE_MUX ? c.level : 0});
    g.out = n_slots++;
    gates.push_back(g);
    CRef r;
    r.slot = g.out;
    r.level = g.level;
    return r;
  }
  // Algorithm 2 (HomCompS): Enc(1) iff a < b.  t0 starts as the trivial
  // Enc(0) = (0, -1/8); signed inputs flip both MSBs first; then per bit
  // from the LSB: t1 = XNOR(a_i, b_i), t0 = MUX(t1, t0, b_i).
  CRef comp_s(std::vector<CRef> a, std::vector<CRef> b, bool is_signed) {
    const size_t l = a.size();
    if (is_signed) {
      a[l - 1] = cnot(a[l - 1]);
      b[l - 1] = cnot(b[l - 1]);
    }
    CRef t0;
    t0.tval = 0xE0000000u;
    for (size_t i = 0; i < l; ++i) {
      CRef t1 = gate(LP_GATE_XNOR, a[i], b[i]);
      t0 = gate(LP_GATE_MUX, t1, t0, b[i]);
    }
    return t0;
  }
};

// Algorithm 3 (LocPIR) with Algorithm 4 (bitwiseAND) and Algorithm 5
// (HomAddXOR as a balanced tree).  Input slots in order: x (l), y (l),
// bounds (N x {x1, x2, y1, y2} x l), payload (N x m).
Circuit build_bbox(uint32_t l, uint32_t N, uint32_t m, bool is_signed) {
  Circuit C;
  std::vector<CRef> X(l), Y(l);
  for (auto& r : X) r = C.input();
  for (auto& r : Y) r = C.input();
  std::vector<std::vector<CRef>> B(4 * (size_t)N, std::vector<CRef>(l));
  for (auto& v : B)
    for (auto& r : v) r = C.input();
  std::vector<CRef> S((size_t)N * m);
  for (auto& r : S) r = C.input();
  std::vector<std::vector<CRef>> T(m);
  for (uint32_t bi = 0; bi < N; ++bi) {
    // x_l = HomCompLE(x1, x) = NOT HomCompS(x, x1);  x_r = HomCompS(x, x2)
    CRef xl = cnot(C.comp_s(X, B[4 * bi + 0], is_signed));
    CRef xr = C.comp_s(X, B[4 * bi + 1], is_signed);
    CRef yl = cnot(C.comp_s(Y, B[4 * bi + 2], is_signed));
    CRef yr = C.comp_s(Y, B[4 * bi + 3], is_signed);
    CRef v1 = C.gate(LP_GATE_AND, xl, xr);
    CRef v2 = C.gate(LP_GATE_AND, yl, yr);
    CRef f = C.gate(LP_GATE_AND, v1, v2);
    for (uint32_t j = 0; j < m; ++j) T[j].push_back(C.gate(LP_GATE_AND, f, S[(size_t)bi * m + j]));
  }
  // pairs taken left to right, an odd last element carried to the next round
  for (uint32_t j = 0; j < m; ++j) {
    std::vector<CRef> cur = T[j];
    while (cur.size() > 1) {
      std::vector<CRef> nxt;
      for (size_t k = 0; k + 1 < cur.size(); k += 2) nxt.push_back(C.gate(LP_GATE_XOR, cur[k], cur[k + 1]));
      if (cur.size() & 1) nxt.push_back(cur.back());
      cur.swap(nxt);
    }
    C.outputs.push_back(cur[0]);
  }
  return C;
}

// Linear pre-combination (constant, coefficient of input 0, of input 1) of
// the bootstrapped gates used by the circuit; MUX is handled apart.
void combo(int kind, uint32_t* cst, int32_t* c0, int32_t* c1) {
  switch (kind) {
    case LP_GATE_AND: *cst = 0xE0000000u; *c0 = 1; *c1 = 1; return;      // -1/8 + a + b
    case LP_GATE_XOR: *cst = 0x40000000u; *c0 = 2; *c1 = 2; return;      // 1/4 + 2(a + b)
    case LP_GATE_XNOR: *cst = 0xC0000000u; *c0 = -2; *c1 = -2; return;   // -1/4 - 2(a + b)
    default: *cst = 0; *c0 = 0; *c1 = 0; return;
  }
}

// ---------------------------------------------------------------- plans
std::shared_ptr<const Plan> make_plan(uint32_t l, uint32_t N, uint32_t m, int is_signed, bool xnor_early) {
  Circuit C = build_bbox(l, N, m, is_signed != 0);
  auto P = std::make_shared<Plan>();
  P->l = l;
  P->N = N;
  P->m = m;
  P->is_signed = is_signed;
  P->n_inputs = 2 * l + 4 * l * N + N * m;
  P->n_slots = (uint32_t)C.n_slots;
  int depth = 0;
  for (auto& g : C.gates) depth = std::max(depth, g.level);
  // Two placements of the gates off the critical path (the comparators'
  // XNORs; every other gate has no slack), with the same depth:
  //   early (as soon as possible, the level from the inputs): every XNOR at
  //     level 1, then l levels of MUXes alone (2 bootstraps per comparator);
  //   late (as late as possible: depth + 1 - the longest path from the gate
  //     to an output, in gates): the XNOR of comparator bit i joins the
  //     level of the MUX of bit i-1, so no level is wider than 3 bootstraps
  //     per comparator.
  // Early suits a device on which the narrower MUX levels run faster per
  // launch than the mixed ones (split rotations); late keeps every level
  // narrow.  Gates are stored in topological order.
  if (!xnor_early) {
    std::vector<int> producer((size_t)C.n_slots, -1);
    for (size_t k = 0; k < C.gates.size(); ++k) producer[(size_t)C.gates[k].out] = (int)k;
    std::vector<int> height(C.gates.size(), 1);
    for (size_t k = C.gates.size(); k-- > 0;) {
      const Gate& g = C.gates[k];
      for (int r = 0; r < (g.kind == LP_GATE_MUX ? 3 : 2); ++r) {
        if (g.in[r].slot < 0) continue;
        const int pk = producer[(size_t)g.in[r].slot];
        if (pk >= 0) height[(size_t)pk] = std::max(height[(size_t)pk], height[k] + 1);
      }
    }
    for (size_t k = 0; k < C.gates.size(); ++k) C.gates[k].level = depth + 1 - height[k];
  }
  P->br.resize(depth);
  P->ks.resize(depth);
  auto put = [](BrJob& j, int which, const CRef& r, int32_t coef) {
    if (r.slot < 0) {  // trivial sample folds into the constant
      j.cst += (uint32_t)coef * r.tval;
      return;
    }
    const uint32_t ref = make_ref(0, (uint32_t)r.slot);
    const int32_t c = r.neg ? -coef : coef;
    if (which == 0) {
      j.in0 = ref;
      j.c0 = c;
    } else {
      j.in1 = ref;
      j.c1 = c;
    }
  };
  for (const Gate& g : C.gates) {
    auto& br = P->br[g.level - 1];
    auto& ks = P->ks[g.level - 1];
    BrJob j{REF_NONE, REF_NONE, 0, 0, 0u, 0u, 0u, 0u};
    KsJob k{REF_NONE, REF_NONE, 0u, make_ref(0, (uint32_t)g.out), 0u, {0, 0, 0}};
    if (g.kind == LP_GATE_MUX) {
      // MUX(s, t, f) = KS((0, 1/8) + BR((0, -1/8) + s + t) + BR((0, -1/8) - s + f))
      BrJob j1 = j, j2 = j;
      j1.cst = j2.cst = 0xE0000000u;
      put(j1, 0, g.in[0], 1);
      put(j1, 1, g.in[1], 1);
      put(j2, 0, g.in[0], -1);
      put(j2, 1, g.in[2], 1);
      j1.out = (uint32_t)br.size();
      br.push_back(j1);
      j2.out = (uint32_t)br.size();
      br.push_back(j2);
      k.ex0 = j1.out;
      k.ex1 = j2.out;
      k.cst = 0x20000000u;
      P->n_br += 2;
    } else {
      int32_t c0, c1;
      combo(g.kind, &j.cst, &c0, &c1);
      put(j, 0, g.in[0], c0);
      put(j, 1, g.in[1], c1);
      j.out = (uint32_t)br.size();
      br.push_back(j);
      k.ex0 = j.out;
      P->n_br += 1;
    }
    ks.push_back(k);
    P->n_ks += 1;
  }
  for (auto& o : C.outputs) P->out_slots.push_back((uint32_t)o.slot);
  return P;
}

std::mutex g_plan_mu;
std::map<std::tuple<uint32_t, uint32_t, uint32_t, int, bool>, std::shared_ptr<const Plan>> g_plans;
}  // namespace

std::shared_ptr<const Plan> get_plan(uint32_t l, uint32_t N, uint32_t m, int is_signed, bool xnor_early) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto key = std::make_tuple(l, N, m, is_signed, xnor_early);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) return it->second;
  auto P = make_plan(l, N, m, is_signed, xnor_early);
  g_plans[key] = P;
  return P;
}

// XNOR placement of a program (one query, or many fused level by level).
// With a timed shape table on the device: early when its levels' estimated
// rotation launch times sum at least 2 % lower than late's (late keeps the
// widest level, and so the extract buffer, smaller).  Without one: a
// lone query goes early exactly when that lets its MUX levels (2
// bootstraps per comparator, 4N comparators) run as split rotations, which
// the mixed levels (3 per comparator) cannot -- on MI355X a split launch
// takes about 0.73 of a one-level-per-wave one, more than paying for the
// wider first level -- and fused queries stay late.  LOCPIR_XNOR_EARLY = 0
// or 1 overrides.
bool choose_xnor_early(const std::vector<std::tuple<uint32_t, uint32_t, uint32_t, int>>& shapes) {
  const int forced = env_int("LOCPIR_XNOR_EARLY", -1);
  if (forced == 0 || forced == 1) return forced == 1;
  if (shapes.empty()) return false;
  double cost[2] = {0.0, 0.0};
  bool timed = true;
  for (int early = 0; early < 2 && timed; ++early) {
    std::vector<size_t> width;
    for (const auto& q : shapes) {
      auto P = get_plan(std::get<0>(q), std::get<1>(q), std::get<2>(q), std::get<3>(q), early == 1);
      if (width.size() < P->br.size()) width.resize(P->br.size(), 0);
      for (size_t L = 0; L < P->br.size(); ++L) width[L] += P->br[L].size();
    }
    for (size_t w : width) {
      double us = 0.0;
      if (w > 0 && !est_br_launch_us(w, &us)) {
        timed = false;
        break;
      }
      cost[early] += us;
    }
  }
  if (timed) return cost[1] < 0.98 * cost[0];
  if (shapes.size() != 1) return false;
  const uint32_t l = std::get<0>(shapes[0]);
  const size_t comparators = 4 * (size_t)std::get<1>(shapes[0]);
  return l >= 2 && pick_br_wpb(2 * comparators) == 6 && pick_br_wpb(3 * comparators) != 6;
}

namespace {

// ---------------------------------------------------------------- programs
// Queries (each under its own key) fused level by level, with device job
// arrays, the ciphertext pool, the extract buffer and optionally one pair of
// graphs (blind rotation, key switching) per level.
struct Program {
  int device = 0;
  uint32_t n_lwe = 0, Nr = 0, ks_t = 0, ks_bb = 0;
  std::vector<const lp_device_key*> keys;
  std::vector<std::shared_ptr<const Plan>> plans;
  std::vector<uint32_t> pool_off;  // first pool slot of each query
  std::vector<uint32_t> out_off;   // first output reference of each query
  size_t pool_slots = 0, ex_slots = 0;
  uint64_t n_br = 0, n_ks = 0;
  std::vector<int> br_off, br_cnt, br_waves, ks_off, ks_cnt, ks_tile, ks_split;
  BrJob* d_br = nullptr;
  KsJob* d_ks = nullptr;
  const uint64_t** d_bsk_tab = nullptr;
  const uint32_t** d_ksk_tab = nullptr;
  uint32_t* d_out_refs = nullptr;
  uint32_t* pool = nullptr;
  uint32_t* ex = nullptr;
  Twiddles tw{};
  SplitArea split;  // exchange area of the levels that run split rotations
  hipStream_t capture = nullptr;
  std::vector<hipGraphExec_t> g_br, g_ks;
  bool graphs_ready = false;
  std::mutex mu;

  int levels() const { return (int)br_cnt.size(); }
  ~Program() {
    for (auto g : g_br) (void)hipGraphExecDestroy(g);
    for (auto g : g_ks) (void)hipGraphExecDestroy(g);
    if (capture) (void)hipStreamDestroy(capture);
    for (void* p : {(void*)d_br, (void*)d_ks, (void*)d_bsk_tab, (void*)d_ksk_tab, (void*)d_out_refs, (void*)pool,
                    (void*)ex})
      if (p) (void)hipFree(p);
    split_area_free(&split);
  }
};

}  // namespace

// Tile of a fused key-switch launch: the default for the level's size,
// halved while per-key padding would waste more than a quarter of it.
int fused_ks_tile(const std::vector<size_t>& per_key, size_t total) {
  int t = pick_ks_tile(total);
  while (t > 1) {
    size_t padded = 0;
    for (size_t c : per_key) padded += (c + t - 1) / t * t;
    if (padded * 4 <= total * 5) break;
    t = t == 16 ? 8 : t == 8 ? 4 : 1;
  }
  return t;
}

namespace {

lp_status build_program(const std::vector<const lp_device_key*>& keys,
                        const std::vector<std::shared_ptr<const Plan>>& plans, std::shared_ptr<Program>* out) {
  auto G = std::make_shared<Program>();
  const size_t nq = keys.size();
  G->device = keys[0]->device;
  G->n_lwe = keys[0]->P.n;
  G->Nr = keys[0]->P.N;
  G->ks_t = keys[0]->P.ks_t;
  G->ks_bb = keys[0]->P.ks_base_bit;
  G->keys = keys;
  G->plans = plans;
  G->tw = keys[0]->tw;
  int depth = 0;
  std::vector<uint32_t> out_refs;
  for (size_t k = 0; k < nq; ++k) {
    G->pool_off.push_back((uint32_t)G->pool_slots);
    G->out_off.push_back((uint32_t)out_refs.size());
    for (uint32_t s : plans[k]->out_slots) out_refs.push_back(make_ref(0, (uint32_t)G->pool_slots + s));
    G->pool_slots += plans[k]->n_slots;
    depth = std::max(depth, plans[k]->levels());
    G->n_br += plans[k]->n_br;
    G->n_ks += plans[k]->n_ks;
  }
  if (G->pool_slots > REF_INDEX_MASK) return fail(LP_EINVAL, "queries too large for one program");
  std::vector<BrJob> br;
  std::vector<KsJob> ks;
  for (int L = 0; L < depth; ++L) {
    G->br_off.push_back((int)br.size());
    G->ks_off.push_back((int)ks.size());
    std::vector<uint32_t> ex_base(nq, 0);
    uint32_t ex_cnt = 0;
    std::vector<size_t> per_key;
    size_t ks_total = 0;
    for (size_t k = 0; k < nq; ++k) {
      if (L >= plans[k]->levels()) continue;
      ex_base[k] = ex_cnt;
      for (BrJob j : plans[k]->br[L]) {
        if (j.in0 != REF_NONE) j.in0 = make_ref(0, G->pool_off[k] + (j.in0 & REF_INDEX_MASK));
        if (j.in1 != REF_NONE) j.in1 = make_ref(0, G->pool_off[k] + (j.in1 & REF_INDEX_MASK));
        j.out += ex_base[k];
        j.key = (uint32_t)k;
        br.push_back(j);
      }
      ex_cnt += (uint32_t)plans[k]->br[L].size();
      per_key.push_back(plans[k]->ks[L].size());
      ks_total += plans[k]->ks[L].size();
    }
    const int tile = fused_ks_tile(per_key, ks_total);
    for (size_t k = 0; k < nq; ++k) {
      if (L >= plans[k]->levels()) continue;
      size_t cnt = 0;
      for (KsJob j : plans[k]->ks[L]) {
        j.ex0 += ex_base[k];
        if (j.ex1 != REF_NONE) j.ex1 += ex_base[k];
        j.out = make_ref(0, G->pool_off[k] + (j.out & REF_INDEX_MASK));
        j.key = (uint32_t)k;
        ks.push_back(j);
        ++cnt;
      }
      for (; cnt % tile; ++cnt) ks.push_back(KsJob{REF_NONE, REF_NONE, 0u, 0u, (uint32_t)k, {0, 0, 0}});
    }
    G->br_cnt.push_back((int)br.size() - G->br_off.back());
    G->ks_cnt.push_back((int)ks.size() - G->ks_off.back());
    G->br_waves.push_back(pick_br_wpb(G->br_cnt.back()));
    G->ks_tile.push_back(tile);
    G->ks_split.push_back(pick_ks_split(G->ks_cnt.back(), tile, G->n_lwe));
    G->ex_slots = std::max<size_t>(G->ex_slots, ex_cnt);
  }
  std::vector<const uint64_t*> bsk_tab(nq);
  std::vector<const uint32_t*> ksk_tab(nq);
  for (size_t k = 0; k < nq; ++k) {
    bsk_tab[k] = keys[k]->bsk_ntt;
    ksk_tab[k] = keys[k]->ksk;
  }
  const size_t w = G->n_lwe + 1;
  LP_HIP_TRY(hipMalloc(&G->d_br, std::max<size_t>(1, br.size()) * sizeof(BrJob)));
  LP_HIP_TRY(hipMalloc(&G->d_ks, std::max<size_t>(1, ks.size()) * sizeof(KsJob)));
  LP_HIP_TRY(hipMalloc((void**)&G->d_bsk_tab, nq * sizeof(void*)));
  LP_HIP_TRY(hipMalloc((void**)&G->d_ksk_tab, nq * sizeof(void*)));
  LP_HIP_TRY(hipMalloc(&G->d_out_refs, std::max<size_t>(1, out_refs.size()) * 4));
  LP_HIP_TRY(hipMalloc(&G->pool, G->pool_slots * w * 4));
  LP_HIP_TRY(hipMalloc(&G->ex, std::max<size_t>(1, G->ex_slots) * (G->Nr + 1) * 4));
  LP_HIP_TRY(hipMemcpy(G->d_br, br.data(), br.size() * sizeof(BrJob), hipMemcpyHostToDevice));
  LP_HIP_TRY(hipMemcpy(G->d_ks, ks.data(), ks.size() * sizeof(KsJob), hipMemcpyHostToDevice));
  LP_HIP_TRY(hipMemcpy(G->d_bsk_tab, bsk_tab.data(), nq * sizeof(void*), hipMemcpyHostToDevice));
  LP_HIP_TRY(hipMemcpy(G->d_ksk_tab, ksk_tab.data(), nq * sizeof(void*), hipMemcpyHostToDevice));
  LP_HIP_TRY(hipMemcpy(G->d_out_refs, out_refs.data(), out_refs.size() * 4, hipMemcpyHostToDevice));
  int split_jobs = 0;
  for (int L = 0; L < depth; ++L)
    if (is_split(G->br_waves[L])) split_jobs = std::max(split_jobs, G->br_cnt[L]);
  if (split_jobs > 0) LP_HIP_TRY(split_area_alloc(&G->split, split_jobs));
  *out = G;
  return LP_OK;
}

hipError_t launch_level_br(const Program& G, int L, hipStream_t s) {
  SrcBases src{};
  src.p[0] = G.pool;
  return launch_blind_rotate(G.d_br + G.br_off[L], G.br_cnt[L], src, G.ex, G.d_bsk_tab, nullptr, (int)G.n_lwe,
                             (int)G.n_lwe, 0, G.tw, G.br_waves[L], s, &G.split);
}

hipError_t launch_level_ks(const Program& G, int L, hipStream_t s) {
  DstBases dst{};
  dst.p[0] = G.pool;
  return launch_keyswitch(G.d_ks + G.ks_off[L], G.ks_cnt[L], G.ex, dst, G.d_ksk_tab, nullptr, (int)G.n_lwe, (int)G.Nr,
                          (int)G.ks_t, (int)G.ks_bb, G.ks_tile[L], G.ks_split[L], s);
}

// Captures one graph per level for the blind rotation and one for the key
// switching, on a private stream (the caller's may be the null stream).
lp_status capture_graphs(Program& G) {
  LP_HIP_TRY(hipStreamCreateWithFlags(&G.capture, hipStreamNonBlocking));
  for (int L = 0; L < G.levels(); ++L) {
    for (int part = 0; part < 2; ++part) {
      hipGraph_t graph = nullptr;
      LP_HIP_TRY(hipStreamBeginCapture(G.capture, hipStreamCaptureModeThreadLocal));
      hipError_t e = part == 0 ? launch_level_br(G, L, G.capture) : launch_level_ks(G, L, G.capture);
      hipError_t e2 = hipStreamEndCapture(G.capture, &graph);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(LP_EDEVICE, "graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
      }
      hipGraphExec_t exec = nullptr;
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return fail(LP_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
      (part == 0 ? G.g_br : G.g_ks).push_back(exec);
    }
  }
  G.graphs_ready = true;
  return LP_OK;
}

// Captures the program's graphs ahead of its first run (when graphs are on).
lp_status prepare_program(Program& G) {
  std::lock_guard<std::mutex> lk(G.mu);
  if (env_int("LOCPIR_GRAPHS", 1) != 0 && !G.graphs_ready) return capture_graphs(G);
  return LP_OK;
}

// Copies the queries' inputs into the pool, runs every level and gathers
// each query's m outputs.
lp_status run_program(Program& G, const lp_bbox_query* qs, uint32_t* const* d_outs, hipStream_t s) {
  std::lock_guard<std::mutex> lk(G.mu);
  const bool use_graphs = env_int("LOCPIR_GRAPHS", 1) != 0;
  if (use_graphs && !G.graphs_ready) {
    lp_status st = capture_graphs(G);
    if (st != LP_OK) return st;
  }
  const size_t w = G.n_lwe + 1;
  for (size_t k = 0; k < G.keys.size(); ++k) {
    const Plan& P = *G.plans[k];
    const size_t l = P.l, N = P.N, m = P.m;
    size_t off = G.pool_off[k];
    auto put = [&](const uint32_t* src, size_t cts) -> hipError_t {
      hipError_t e = hipMemcpyAsync(G.pool + off * w, src, cts * w * 4, hipMemcpyDeviceToDevice, s);
      off += cts;
      return e;
    };
    LP_HIP_TRY(put(qs[k].d_x, l));
    LP_HIP_TRY(put(qs[k].d_y, l));
    LP_HIP_TRY(put(qs[k].d_bounds, 4 * l * N));
    LP_HIP_TRY(put(qs[k].d_payload, N * m));
  }
  for (int L = 0; L < G.levels(); ++L) {
    {
      ProfScope ps(kProfBR, (uint64_t)G.br_cnt[L], G.br_waves[L], s);
      LP_HIP_TRY(use_graphs ? hipGraphLaunch(G.g_br[L], s) : launch_level_br(G, L, s));
    }
    {
      ProfScope ps(kProfKS, (uint64_t)G.ks_cnt[L], G.ks_tile[L], s);
      LP_HIP_TRY(use_graphs ? hipGraphLaunch(G.g_ks[L], s) : launch_level_ks(G, L, s));
    }
  }
  SrcBases src{};
  src.p[0] = G.pool;
  for (size_t k = 0; k < G.keys.size(); ++k)
    LP_HIP_TRY(launch_gather(G.d_out_refs + G.out_off[k], (int)G.plans[k]->m, src, 0, d_outs[k], (int)G.n_lwe, s));
  // a program with split rotations waits for its end and reads the
  // exchange area's give-up record: a wait that ran out leaves its job's
  // output undefined, so the whole call fails
  if (G.split.sync) {
    uint32_t stalls = 0;
    LP_HIP_TRY(split_area_take_stalls(&G.split, s, &stalls, nullptr));
    if (stalls) return split_stall_error("bounding-box query", stalls);
  }
  return LP_OK;
}

// ---------------------------------------------------------------- cache
struct ProgKey {
  hipStream_t stream;
  std::vector<std::tuple<const lp_device_key*, uint32_t, uint32_t, uint32_t, int>> items;
  bool operator<(const ProgKey& o) const { return std::tie(stream, items) < std::tie(o.stream, o.items); }
  bool operator==(const ProgKey& o) const { return stream == o.stream && items == o.items; }
};
std::mutex g_prog_mu;
std::map<ProgKey, std::shared_ptr<Program>> g_progs;
std::vector<ProgKey> g_prog_order;  // oldest first
constexpr size_t kMaxPrograms = 16;

lp_status get_program(const std::vector<const lp_device_key*>& keys, const lp_bbox_query* qs, hipStream_t s,
                      std::shared_ptr<Program>* out) {
  ProgKey key;
  key.stream = s;
  for (size_t k = 0; k < keys.size(); ++k)
    key.items.emplace_back(keys[k], qs[k].l, qs[k].n_boxes, qs[k].m, qs[k].is_signed ? 1 : 0);
  std::lock_guard<std::mutex> lk(g_prog_mu);
  auto it = g_progs.find(key);
  if (it != g_progs.end()) {
    *out = it->second;
    return LP_OK;
  }
  std::vector<std::tuple<uint32_t, uint32_t, uint32_t, int>> shapes;
  for (size_t k = 0; k < keys.size(); ++k)
    shapes.emplace_back(qs[k].l, qs[k].n_boxes, qs[k].m, qs[k].is_signed ? 1 : 0);
  const bool early = choose_xnor_early(shapes);
  std::vector<std::shared_ptr<const Plan>> plans;
  for (size_t k = 0; k < keys.size(); ++k)
    plans.push_back(get_plan(qs[k].l, qs[k].n_boxes, qs[k].m, qs[k].is_signed ? 1 : 0, early));
  std::shared_ptr<Program> G;
  lp_status st = build_program(keys, plans, &G);
  if (st != LP_OK) return st;
  if (g_progs.size() >= kMaxPrograms) {
    g_progs.erase(g_prog_order.front());
    g_prog_order.erase(g_prog_order.begin());
  }
  g_progs[key] = G;
  g_prog_order.push_back(key);
  *out = G;
  return LP_OK;
}

lp_status check_query(const lp_bbox_query& q) {
  if (q.l == 0 || q.l > 64 || q.n_boxes == 0 || q.m == 0 || q.n_boxes > (1u << 16) || q.m > 4096)
    return fail(LP_EINVAL, "empty or oversized query shape (l=%u, boxes=%u, m=%u)", q.l, q.n_boxes, q.m);
  if (!q.d_x || !q.d_y || !q.d_bounds || !q.d_payload) return fail(LP_EINVAL, "null query input");
  return LP_OK;
}

}  // namespace

void sched_forget_all() {
  std::lock_guard<std::mutex> lk(g_prog_mu);
  g_progs.clear();
  g_prog_order.clear();
}

void sched_forget_key(const lp_device_key* dk) {
  std::lock_guard<std::mutex> lk(g_prog_mu);
  for (auto it = g_progs.begin(); it != g_progs.end();) {
    bool uses = false;
    for (auto& item : it->first.items) uses |= std::get<0>(item) == dk;
    if (uses) {
      g_prog_order.erase(std::find(g_prog_order.begin(), g_prog_order.end(), it->first));
      it = g_progs.erase(it);
    } else {
      ++it;
    }
  }
}

// Host-side plan statistics for the server and the counts entry point.
void plan_counts(uint32_t l, uint32_t N, uint32_t m, uint64_t* n_br, uint64_t* n_ks, uint32_t* levels) {
  auto P = get_plan(l, N, m, 1, false);
  if (n_br) *n_br = P->n_br;
  if (n_ks) *n_ks = P->n_ks;
  if (levels) *levels = (uint32_t)P->levels();
}

}  // namespace lp

extern "C" lp_status lp_bbox_counts(uint32_t l, uint32_t n_boxes, uint32_t m, uint64_t* n_br, uint64_t* n_ks,
                                    uint32_t* n_levels) {
  if (l == 0 || l > 64 || n_boxes == 0 || m == 0) return lp::fail(LP_EINVAL, "lp_bbox_counts: empty shape");
  lp::plan_counts(l, n_boxes, m, n_br, n_ks, n_levels);
  return LP_OK;
}

extern "C" lp_status lp_bbox_level_widths(uint32_t l, uint32_t n_boxes, uint32_t m, uint32_t* widths,
                                          uint32_t* n_levels) {
  if (l == 0 || l > 64 || n_boxes == 0 || m == 0) return lp::fail(LP_EINVAL, "lp_bbox_level_widths: empty shape");
  if (!n_levels || (*n_levels > 0 && !widths)) return lp::fail(LP_EINVAL, "lp_bbox_level_widths: null argument");
  auto P = lp::get_plan(l, n_boxes, m, 1, lp::choose_xnor_early({std::make_tuple(l, n_boxes, m, 1)}));
  const uint32_t depth = (uint32_t)P->levels();
  for (uint32_t k = 0; k < depth && k < *n_levels; ++k) widths[k] = (uint32_t)P->br[k].size();
  *n_levels = depth;
  return LP_OK;
}

namespace {
// Validation shared by the batch call and its prepare step.
lp_status check_batch(const char* who, const lp_device_key* const* keys, const lp_bbox_query* queries, size_t nq,
                      uint32_t* const* d_outs, std::vector<const lp_device_key*>* ks) {
  if (!keys || !queries) return lp::fail(LP_EINVAL, "%s: null argument", who);
  ks->assign(keys, keys + nq);
  for (size_t k = 0; k < nq; ++k) {
    if (!(*ks)[k]) return lp::fail(LP_EINVAL, "%s: null key %zu", who, k);
    if (d_outs && !d_outs[k]) return lp::fail(LP_EINVAL, "%s: null output %zu", who, k);
    const lp_device_key* a = (*ks)[k];
    const lp_device_key* b = (*ks)[0];
    if (a->device != b->device || a->P.n != b->P.n || a->P.ks_t != b->P.ks_t || a->P.ks_base_bit != b->P.ks_base_bit)
      return lp::fail(LP_EINVAL, "%s: keys differ in device or parameters", who);
    lp_status st = lp::check_query(queries[k]);
    if (st != LP_OK) return st;
  }
  return LP_OK;
}
}  // namespace

extern "C" lp_status lp_eval_bbox_batch(const lp_device_key* const* keys, const lp_bbox_query* queries, size_t nq,
                                        uint32_t* const* d_outs, void* stream) {
  if (nq == 0) return LP_OK;
  if (!d_outs) return lp::fail(LP_EINVAL, "lp_eval_bbox_batch: null argument");
  std::vector<const lp_device_key*> ks;
  lp_status st = check_batch("lp_eval_bbox_batch", keys, queries, nq, d_outs, &ks);
  if (st != LP_OK) return st;
  lp::ScopedDevice sd(ks[0]->device);
  hipStream_t s = lp::as_stream(stream);
  std::shared_ptr<lp::Program> G;
  st = lp::get_program(ks, queries, s, &G);
  if (st != LP_OK) return st;
  return lp::run_program(*G, queries, d_outs, s);
}

extern "C" lp_status lp_eval_bbox_prepare(const lp_device_key* const* keys, const lp_bbox_query* queries, size_t nq,
                                          void* stream) {
  if (nq == 0) return LP_OK;
  std::vector<const lp_device_key*> ks;
  lp_status st = check_batch("lp_eval_bbox_prepare", keys, queries, nq, nullptr, &ks);
  if (st != LP_OK) return st;
  lp::ScopedDevice sd(ks[0]->device);
  std::shared_ptr<lp::Program> G;
  st = lp::get_program(ks, queries, lp::as_stream(stream), &G);
  if (st != LP_OK) return st;
  return lp::prepare_program(*G);
}

extern "C" lp_status lp_eval_bbox_query(const lp_device_key* dk, const lp_bbox_query* q, uint32_t* d_out,
                                        void* stream) {
  if (!dk || !q || !d_out) return lp::fail(LP_EINVAL, "lp_eval_bbox_query: null argument");
  return lp_eval_bbox_batch(&dk, q, 1, &d_out, stream);
}
