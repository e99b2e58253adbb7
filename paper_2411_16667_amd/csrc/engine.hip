// Host runtime of the library: C ABI, graph upload, device-resident query
// slots, admission by memory reservation, the step loop, batch and server.
//
// One Engine owns a device arena and a table of slots.  Every tick it
//   1. admits queued queries into free slots whose reservation fits the arena
//      (first fit), computes their heuristics and seeds their start labels,
//   2. replays a captured hipGraph of K batched label steps over all slots,
//   3. reads the slot table back and harvests finished queries (results and
//      witness paths are copied to host memory; the reservation is released).
// mos_solve is a one-query batch; mos_solve_batch feeds a queue of queries
// through the same engine (continuous batching); the server runs the same
// ticks on a thread fed by a request queue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "front.h"
#include "graph_internal.h"
#include "kernels.h"
#include "layout.h"
#include "mos.h"

using namespace mos;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

struct MosError : std::runtime_error {
  mos_status st;
  MosError(mos_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

static void hip_check(hipError_t e, const char* what, int line) {
  if (e != hipSuccess) {
    hipGetLastError();
    throw MosError(e == hipErrorOutOfMemory ? MOS_E_OUT_OF_MEMORY : MOS_E_DEVICE,
                   std::string(what) + " failed at engine line " + std::to_string(line) + ": " +
                       hipGetErrorString(e));
  }
}
// line of the HIP call in progress (or last finished), for errors raised
// inside the runtime as C++ exceptions
static thread_local int g_site = 0;
#define HIPCHK(x) (g_site = __LINE__, hip_check((x), #x, __LINE__))

static mos_status set_err(mos_status s, const std::string& m) {
  g_last_error = m;
  return s;
}

mos_status mos_internal_set_error(mos_status s, const std::string& m) { return set_err(s, m); }

void mos_internal_stats_of(const Slot& d, mos_stats* o) {
  o->pops = d.st[ST_POPS];
  o->goal_pops = d.st[ST_GOAL_POPS];
  o->candidates = d.st[ST_CANDS];
  o->p_pairs = d.st[ST_PPAIRS];
  o->group_pairs = d.st[ST_GPAIRS];
  o->frontier_pairs = d.st[ST_FPAIRS];
  o->inserted = d.st[ST_INSERTED];
  o->pruned = d.st[ST_PRUNED];
  o->steps = d.st[ST_STEPS];
  o->front = d.P_n - d.P_dead;
  o->frontier_bytes = d.st[ST_FBYTES];
  o->killed = d.st[ST_KILLED];
  o->frontier_bytes_onepass = d.st[ST_FBYTES_WAVE];
  o->pairs_onepass = d.st[ST_PAIRS_WAVE];
  o->near_scanned = d.st[ST_NEAR_SCAN];
  o->far_scanned = d.st[ST_FAR_SCAN];
  o->tie_entries = d.st[ST_TIE];
  o->front_reads = d.st[ST_PREAD];
  o->search_ms = 0;
  o->heuristic_ms = 0;
  o->open_min_f1 = d.status == S_DONE ? INT32_MAX : -1;
}

template <class F>
static mos_status guarded(F&& f) {
  try {
    return f();
  } catch (const MosError& e) {
    return set_err(e.st, e.what());
  } catch (const std::bad_alloc&) {
    return set_err(MOS_E_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    return set_err(MOS_E_DEVICE, std::string(e.what()) + " (raised inside the HIP runtime; last "
                                     "HIP call at engine line " + std::to_string(g_site) + ")");
  }
}

// ------------------------------------------------------------- allocation
struct AllocHooks {
  void* (*alloc)(size_t, void*, void*) = nullptr;
  void (*release)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
static std::mutex g_hooks_mu;
static AllocHooks g_hooks;

// Device buffer that remembers which allocator made it.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  AllocHooks h;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  void alloc(size_t n, hipStream_t st) {
    reset();
    if (n == 0) n = 256;
    {
      std::lock_guard<std::mutex> lk(g_hooks_mu);
      h = g_hooks;
    }
    if (h.alloc) {
      p = h.alloc(n, (void*)st, h.ctx);
      if (!p) throw MosError(MOS_E_OUT_OF_MEMORY, "allocator hook returned NULL");
    } else {
      hipError_t e = hipMalloc(&p, n);
      if (e != hipSuccess) {
        hipGetLastError();
        p = nullptr;
        throw MosError(MOS_E_OUT_OF_MEMORY,
                       "hipMalloc of " + std::to_string(n) + " bytes failed");
      }
    }
    bytes = n;
  }
  void reset() {
    if (p) {
      if (h.release) h.release(p, h.ctx);
      else hipFree(p);
    }
    p = nullptr;
    bytes = 0;
  }
  ~DevBuf() { reset(); }
  template <class T>
  T* as() const { return (T*)p; }
};

static int ensure_device() {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) {
    hipGetLastError();
    throw MosError(MOS_E_NO_DEVICE, "no HIP device is visible");
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  return dev;
}

// ------------------------------------------------------------------ graph
class Engine;

// Engines are cached per graph and reused by later solves with the same
// configuration (arena, slot table and captured step graph stay allocated).
struct EngineKey {
  int S;
  int dm;
  int64_t budget;
  void* stream;
  int B;
  int64_t label_limit;
  bool paths;
  int steps;
  bool pipelined;  // not part of the match: a cached engine switches mode per call
  bool operator==(const EngineKey& o) const {
    return S == o.S && dm == o.dm && budget == o.budget && stream == o.stream && B == o.B &&
           label_limit == o.label_limit && paths == o.paths && steps == o.steps;
  }
};

struct mos_graph {
  int32_t n = 0, D = 0, maxdeg = 0, device = 0;
  int64_t m = 0;
  int32_t csum[MAXD] = {};
  DevBuf row_ptr, col, cost, rrow, rsrc, rarc;
  std::mutex pool_mu;
  std::vector<std::pair<EngineKey, Engine*>> pool;  // idle engines, oldest first
  GraphDev view() const {
    GraphDev g;
    g.n = n;
    g.m = (int32_t)m;
    g.D = D;
    g.maxdeg = maxdeg;
    for (int k = 0; k < MAXD; ++k) g.csum[k] = csum[k];
    g.row_ptr = row_ptr.as<int32_t>();
    g.col = col.as<int32_t>();
    g.cost = cost.as<int32_t>();
    g.rrow = rrow.as<int32_t>();
    g.rsrc = rsrc.as<int32_t>();
    g.rarc = rarc.as<int32_t>();
    return g;
  }
};

GraphDev mos_internal_graph_view(const mos_graph* g) { return g->view(); }
int mos_internal_graph_device(const mos_graph* g) { return g->device; }

// ----------------------------------------------------------------- result
struct mos_result {
  int32_t d = 0;
  int64_t size = 0;
  bool complete = true;  // false: the exact part below stats.open_min_f1 only
  std::vector<int32_t> costs;     // size*d, lexicographically ascending
  std::vector<int64_t> path_off;  // size+1 (empty when paths were not requested)
  std::vector<int32_t> arcs;
  mos_stats stats{};
};

// --------------------------------------------------------- range allocator
// First-fit allocator over [0, total) of the arena (256-byte units).
struct RangeAlloc {
  std::map<int64_t, int64_t> free_;  // offset -> length
  int64_t total = 0;
  void init(int64_t t) {
    total = t;
    free_.clear();
    free_[0] = t;
  }
  bool take(int64_t len, int64_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        *off = it->first;
        int64_t rest = it->second - len;
        int64_t noff = it->first + len;
        free_.erase(it);
        if (rest > 0) free_[noff] = rest;
        return true;
      }
    }
    return false;
  }
  void give(int64_t off, int64_t len) {
    auto it = free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int64_t largest() const {
    int64_t b = 0;
    for (auto& kv : free_) b = std::max(b, kv.second);
    return b;
  }
};

// ----------------------------------------------------------- slot layout
static bool plan_layout(const mos_graph* g, int d, int B, int64_t budget, int64_t label_limit,
                        Layout* L) {
  return plan_slot_layout(g->n, g->maxdeg, d, B, budget, label_limit, L);
}

static void carve(Slot& s, char* base, const Layout& L, int64_t n, int d) {
  if (!carve_slot(s, base, L, n, d)) throw MosError(MOS_E_DEVICE, "slot layout overrun");
}

// ------------------------------------------------------------------ engine

struct QueryReq {
  int64_t id = 0;
  int32_t start = 0, goal = 0, d = 0;
  int32_t heur_factor = kDefaultHeurFactor;  // 0 = exact heuristic on the whole graph
  int64_t reserve = 0;  // bytes of the next admission attempt
  int attempts = 0;
  int64_t step_budget = 0;  // steps after which the exact prefix is returned (0 = none)
  int32_t pop_order = 0;    // MOS_POP_*
  int32_t eps_ppm = 0;      // approximate mode (0 = exact)
  int32_t eager_goal = 0;
  int32_t solo = 0;         // steps run in one workgroup of its own (persistent_query)
};

struct Finished {
  int64_t id;
  mos_status st;
  mos_result* res;
  std::string msg;
};

struct SlotHost {
  bool busy = false;
  QueryReq q;
  int64_t off = 0, len = 0;
  Layout L{};
  double search_ms = 0, heur_ms = 0;
  bool cancel = false;
};

class Engine {
 public:
  Engine(const mos_graph* g, int nslots, int dm, int64_t budget, hipStream_t user_stream, int B,
         int64_t label_limit, bool want_paths, int steps_per_poll)
      : g_(g), S_(nslots), DM_(dm), B_(B), label_limit_(label_limit), want_paths_(want_paths),
        K_(steps_per_poll) {
    HIPCHK(hipSetDevice(g->device));
    if (user_stream) {
      st_ = user_stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
      own_stream_ = true;
    }
    budget = std::max<int64_t>(budget, 1 << 20);
    arena_.alloc((size_t)budget, st_);
    ra_.init(budget / 256);
    slots_.alloc(sizeof(Slot) * S_, st_);
    HIPCHK(hipHostMalloc((void**)&hslots_, sizeof(Slot) * S_, hipHostMallocDefault));
    std::memset(hslots_, 0, sizeof(Slot) * S_);
    HIPCHK(hipMemcpyAsync(slots_.p, hslots_, sizeof(Slot) * S_, hipMemcpyHostToDevice, st_));
    hist_.alloc((size_t)S_ * NB * 4, st_);
    HIPCHK(hipMemsetAsync(hist_.p, 0, (size_t)S_ * NB * 4, st_));
    sh_.resize(S_);
    gx_ = std::max(1, 2048 / S_);
    // tuning knobs of the step's launch shape (defaults otherwise):
    // MOS_GX workgroups per slot of the tiled kernels, MOS_BIG_WORK pair
    // checks above which a group is split into pair tiles
    if (const char* x = std::getenv("MOS_GX")) gx_ = std::max(1, std::min(65535, std::atoi(x)));
    if (const char* x = std::getenv("MOS_BIG_WORK")) big_work_ = std::max(64, std::atoi(x));
    // tail widening (see widen_slots): a slot's batch capacity is planned for
    // `widen_` times the batch width; MOS_WIDEN=1 turns it off
    widen_ = S_ > 1 ? 4 : 1;
    if (const char* x = std::getenv("MOS_WIDEN")) widen_ = std::max(1, std::min(64, std::atoi(x)));
    Bplan_ = (int)std::min<int64_t>((int64_t)B_ * widen_, BATCH_MAX);
    HIPCHK(hipEventCreate(&ev0_));
    HIPCHK(hipEventCreate(&ev1_));
    HIPCHK(hipStreamSynchronize(st_));
    // MOS_HIPGRAPH=0 launches the step kernels one by one instead of replaying
    // a captured graph (same kernels, same order).
    const char* e = std::getenv("MOS_HIPGRAPH");
    use_graph_ = !(e && e[0] == '0');
    // MOS_PROGRESS=1 prints the state of resident queries every few seconds
    // from the poll loop (long single solves otherwise run silently).
    const char* pr = std::getenv("MOS_PROGRESS");
    progress_ = pr && (pr[0] == '1' || pr[0] == '2');
    progress_level_ = progress_ ? pr[0] - '0' : 0;
    t_last_ = std::chrono::steady_clock::now();
  }

  ~Engine() {
    hipStreamSynchronize(st_);
    if (st2_) {
      hipStreamSynchronize(st2_);
      hipStreamDestroy(st2_);
      hipEventDestroy(fork_);
      hipEventDestroy(join_);
    }
    for (auto& e : pev_) hipEventDestroy(e);
    if (graph_exec_) hipGraphExecDestroy(graph_exec_);

    if (hslots_) hipHostFree(hslots_);
    hipEventDestroy(ev0_);
    hipEventDestroy(ev1_);
    hipStreamSynchronize(st_);
    arena_.reset();
    slots_.reset();
    hist_.reset();
    hscr_.reset();
    hcnt_.reset();
    hjob_.reset();
    omin_.reset();
    if (own_stream_) hipStreamDestroy(st_);
  }

  // Pipelined steps (set while no query is resident): the goal-front filter
  // of a step's new labels runs beside the next step's pop, on a second
  // stream.  A change of mode drops the captured step graph.
  void set_pipelined(bool p) {
    if (p != pipelined_ && graph_exec_) {
      HIPCHK(hipGraphExecDestroy(graph_exec_));
      graph_exec_ = nullptr;
      graph_failed_ = false;
    }
    pipelined_ = p;
    if (p && !st2_) {
      HIPCHK(hipStreamCreateWithFlags(&st2_, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&fork_, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&join_, hipEventDisableTiming));
    }
  }

  int64_t arena_bytes() const { return ra_.total * 256; }
  int busy_count() const {
    int c = 0;
    for (auto& s : sh_) c += s.busy;
    return c;
  }
  int slots() const { return S_; }

  // Default reservation for a query: an equal share of the arena.
  int64_t default_reserve() const { return std::max<int64_t>(arena_bytes() / S_, 1 << 20); }

  void cancel_query(int64_t id) {
    for (int s = 0; s < S_; ++s)
      if (sh_[s].busy && sh_[s].q.id == id) sh_[s].cancel = true;
  }

  // Admit, step, harvest.  Returns finished queries through `done`.
  void tick(std::deque<QueryReq>& pending, std::vector<Finished>& done) {
    cancellations(done);
    std::vector<int> fresh = admit(pending, done);
    if (!fresh.empty()) run_heuristics(fresh);
    if (busy_count() > 0) {
      widen_slots(pending.empty());
      advance(K_);
      collect(pending, done);
    }
  }

  // Tail widening.  With no query waiting and so few queries resident that
  // a step pops fewer than kWidenLabels labels in all (a step of that size
  // costs little more than its fixed sequence of launches), each resident
  // query pops up to kWidenLabels / busy labels per step (at most its planned
  // capacity, widen_ times the batch width), so the last queries of a batch
  // need fewer steps.  The front does not depend on the pop order.  A query
  // with a step budget keeps the plain width: its exact prefix after that
  // many steps then does not depend on the other queries.
  static constexpr int kWidenLabels = 16384;
  // steps a one-workgroup query runs per launch (at least the steps per poll)
  static constexpr int kSoloSteps = 32;
  void widen_slots(bool none_waiting) {
    const int busy = busy_count();
    if (busy == 0) return;
    int target = B_;
    if (none_waiting && (int64_t)busy * B_ < kWidenLabels)
      target = (int)std::min<int64_t>(std::max(B_, kWidenLabels / busy), Bplan_);
    for (int s = 0; s < S_; ++s) {
      if (!sh_[s].busy) continue;
      const int b = sh_[s].q.step_budget > 0 ? B_ : std::min(target, sh_[s].L.batch_cap);
      if (hslots_[s].B != b) {
        hslots_[s].B = b;
        HIPCHK(hipMemcpyAsync((char*)slots_.p + (size_t)s * sizeof(Slot) + offsetof(Slot, B),
                              &hslots_[s].B, sizeof(int32_t), hipMemcpyHostToDevice, st_));
      }
    }
  }

  // Cancelled resident queries leave their slot at once.
  void cancellations(std::vector<Finished>& done) {
    for (int s = 0; s < S_; ++s) {
      if (sh_[s].busy && sh_[s].cancel) {
        int32_t idle = S_IDLE;
        HIPCHK(hipMemcpyAsync((char*)slots_.p + (size_t)s * sizeof(Slot) + offsetof(Slot, status),
                              &idle, sizeof(idle), hipMemcpyHostToDevice, st_));
        HIPCHK(hipStreamSynchronize(st_));
        release(s);
        done.push_back({sh_[s].q.id, MOS_E_CANCELLED, nullptr, "cancelled"});
      }
    }
  }

  // Admission, first fit in queue order: a query enters a free slot when its
  // reservation fits into the arena; the head of the queue waits otherwise.
  std::vector<int> admit(std::deque<QueryReq>& pending, std::vector<Finished>& done) {
    std::vector<int> fresh;
    while (!pending.empty()) {
      int free_slot = -1;
      for (int s = 0; s < S_; ++s)
        if (!sh_[s].busy) {
          free_slot = s;
          break;
        }
      if (free_slot < 0) break;
      QueryReq q = pending.front();
      q.reserve = std::min<int64_t>(q.reserve, arena_bytes());
      Layout L;
      if (!plan_layout(g_, q.d, Bplan_, q.reserve, label_limit_, &L)) {
        pending.pop_front();
        done.push_back({q.id, MOS_E_LABEL_LIMIT, nullptr,
                        "memory budget too small for one query of this graph"});
        continue;
      }
      int64_t off;
      if (!ra_.take((L.bytes + 255) / 256, &off)) {
        if (busy_count() == 0 && ra_.largest() * 256 < L.bytes) {
          pending.pop_front();
          done.push_back({q.id, MOS_E_LABEL_LIMIT, nullptr, "reservation exceeds the arena"});
          continue;
        }
        break;  // wait for resident queries to leave
      }
      pending.pop_front();
      SlotHost& h = sh_[free_slot];
      h.busy = true;
      h.cancel = false;
      h.q = q;
      h.off = off;
      h.len = (L.bytes + 255) / 256;
      h.L = L;
      h.search_ms = h.heur_ms = 0;
      Slot& s = hslots_[free_slot];
      std::memset(&s, 0, sizeof(Slot));
      s.status = S_IDLE;
      s.start = q.start;
      s.goal = q.goal;
      s.d = q.d;
      s.B = B_;  // widen_slots may raise it up to the planned capacity
      s.big_work = big_work_;
      s.batch_cap = L.batch_cap;
      s.cand_cap = L.cand_cap;
      s.tie_cap = L.tie_cap;
      s.pool_cap = L.pool_cap;
      s.open_cap = L.open_cap;
      s.P_cap = L.P_cap;
      s.fw_cap = L.fw_cap;
      s.query_id = (int32_t)q.id;
      s.heur_factor = q.heur_factor;
      s.hn = g_->n;
      s.pop_fifo = q.pop_order == MOS_POP_GENERATION ? 1 : 0;
      s.eps_ppm = q.eps_ppm;
      s.eager_goal = q.eager_goal;
      s.pipelined = pipelined_ ? 1 : 0;
      s.solo = q.solo;
      carve(s, arena_.as<char>() + off * 256, L, g_->n, q.d);
      HIPCHK(hipMemcpyAsync((char*)slots_.p + (size_t)free_slot * sizeof(Slot), &s, sizeof(Slot),
                            hipMemcpyHostToDevice, st_));
      fresh.push_back(free_slot);
    }
    return fresh;
  }

  // Run n label steps over every resident slot, then read the slot table back.
  void advance(int64_t n) {
    HIPCHK(hipEventRecord(ev0_, st_));
    launch_steps(n);
    HIPCHK(hipEventRecord(ev1_, st_));
    HIPCHK(hipMemcpyAsync(hslots_, slots_.p, sizeof(Slot) * S_, hipMemcpyDeviceToHost, st_));
    HIPCHK(hipStreamSynchronize(st_));
    if (profile_) drain_profile();
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ev0_, ev1_));
    for (int s = 0; s < S_; ++s)
      if (sh_[s].busy) sh_[s].search_ms += ms;
    if (progress_) report_progress();
  }

  // Harvest finished slots; re-queue overflowed ones with a larger reservation.
  void collect(std::deque<QueryReq>& pending, std::vector<Finished>& done) {
    for (int s = 0; s < S_; ++s) {
      if (!sh_[s].busy) continue;
      const Slot& d = hslots_[s];
      if (d.status == S_SOLO_QUIT) {
        // more labels of one F1 than a one-workgroup batch holds: run again by
        // the multi-kernel step
        QueryReq q = sh_[s].q;
        release(s);
        q.solo = 0;
        pending.push_front(q);
        continue;
      }
      if (d.status == S_RUN || d.status == S_SOLO) {
        const int64_t budget = sh_[s].q.step_budget;
        if (budget > 0 && d.st[ST_STEPS] >= budget) {
          Finished f{sh_[s].q.id, MOS_E_STEP_LIMIT, nullptr,
                     "step budget reached: the result is the exact front below stats.open_min_f1"};
          f.res = harvest_prefix(s);
          release(s);
          done.push_back(f);
        }
        continue;
      }
      if (d.status == S_DONE) {
        Finished f{sh_[s].q.id, MOS_OK, nullptr, ""};
        f.res = harvest(s);
        release(s);
        done.push_back(f);
      } else {
        QueryReq q = sh_[s].q;
        const Layout L = sh_[s].L;
        release(s);
        if ((label_limit_ > 0 && L.pool_cap >= label_limit_) || q.reserve >= arena_bytes()) {
          done.push_back({q.id, MOS_E_LABEL_LIMIT, nullptr,
                          "search state outgrew the label limit or memory budget"});
        } else {
          q.reserve = std::min<int64_t>(arena_bytes(), q.reserve * 4);
          q.attempts++;
          readmissions_++;
          pending.push_front(q);
        }
      }
    }
  }

  // ---- single-query sessions (stepped on demand)
  mos_status session_admit(const QueryReq& q0, std::string* msg) {
    std::deque<QueryReq> p{q0};
    std::vector<Finished> d;
    std::vector<int> fresh = admit(p, d);
    if (!d.empty()) {
      *msg = d[0].msg;
      return d[0].st;
    }
    if (fresh.empty()) {
      *msg = "query does not fit the arena";
      return MOS_E_LABEL_LIMIT;
    }
    run_heuristics(fresh);
    HIPCHK(hipMemcpyAsync(hslots_, slots_.p, sizeof(Slot) * S_, hipMemcpyDeviceToHost, st_));
    HIPCHK(hipStreamSynchronize(st_));
    return MOS_OK;
  }
  const Slot& slot0() const { return hslots_[0]; }
  const SlotHost& host0() const { return sh_[0]; }
  void set_profile(uint32_t mask) {
    drain_profile();
    profile_ = mask;
  }
  int64_t graph_replays() const { return graph_replays_; }
  int64_t direct_steps() const { return direct_steps_; }
  int steps_per_replay() const { return K_; }
  double kernel_ms(int i) const { return kms_[i]; }
  int64_t kernel_launches(int i) const { return klaunch_[i]; }
  mos_result* harvest_slot0() {
    mos_result* r = harvest(0);
    release(0);
    return r;
  }
  // The goal front of slot 0 so far and the smallest F1 left in OPEN.
  mos_result* front_so_far0(int32_t* m) {
    *m = open_min_f1(0);
    mos_result* r = harvest(0);
    r->stats.open_min_f1 = *m;
    r->complete = false;
    return r;
  }
  mos_stats stats_of(int s) const {
    mos_stats o{};
    mos_internal_stats_of(hslots_[s], &o);
    o.search_ms = sh_[s].search_ms;
    o.heuristic_ms = sh_[s].heur_ms;
    return o;
  }

  int64_t readmissions() const { return readmissions_; }
  std::vector<int64_t> resident_ids() const {
    std::vector<int64_t> v;
    for (auto& h : sh_)
      if (h.busy) v.push_back(h.q.id);
    return v;
  }

  void report_progress() {
    const auto now = std::chrono::steady_clock::now();
    if (std::chrono::duration<double>(now - t_last_).count() < 5.0) return;
    t_last_ = now;
    int shown = 0;
    for (int s = 0; s < S_ && shown < 4; ++s) {
      if (!sh_[s].busy) continue;
      const Slot& d = hslots_[s];
      std::fprintf(stderr,
                   "[mos] slot %d query %lld: steps %lld pops %lld labels %d open %d+%d front %d "
                   "frontier words %lld/%lld search %.0f ms\n",
                   s, (long long)sh_[s].q.id, (long long)d.st[ST_STEPS], (long long)d.st[ST_POPS],
                   d.n_labels, d.open_n, d.far_n, d.P_n, (long long)d.fw_top, (long long)d.fw_cap,
                   sh_[s].search_ms);
      ++shown;
    }
    if (progress_level_ > 1) {
      const Slot& d = hslots_[0];
      std::fprintf(stderr, "[mos] phase ticks:");
      for (int i = 0; i < 8; ++i) std::fprintf(stderr, " %lld", (long long)d.st[ST_T0 + i]);
      std::fprintf(stderr, " | near %lld far %lld tie %lld front-reads %lld\n",
                   (long long)d.st[ST_NEAR_SCAN], (long long)d.st[ST_FAR_SCAN],
                   (long long)d.st[ST_TIE], (long long)d.st[ST_PREAD]);
    }
    std::fprintf(stderr, "[mos] resident %d\n", busy_count());
    std::fflush(stderr);
  }

  // Heuristic only: h planes of one goal (used by mos_heuristic).
  void heuristic_only(int32_t goal, int d, int32_t* out) {
    Layout L;
    if (!plan_layout(g_, d, B_, arena_bytes(), 16, &L))
      throw MosError(MOS_E_OUT_OF_MEMORY, "arena too small");
    int64_t off;
    if (!ra_.take((L.bytes + 255) / 256, &off)) throw MosError(MOS_E_OUT_OF_MEMORY, "arena full");
    Slot& s = hslots_[0];
    std::memset(&s, 0, sizeof(Slot));
    s.goal = goal;
    s.start = goal;
    s.d = d;
    s.pool_cap = L.pool_cap;
    carve(s, arena_.as<char>() + off * 256, L, g_->n, d);
    HIPCHK(hipMemcpyAsync(slots_.p, &s, sizeof(Slot), hipMemcpyHostToDevice, st_));
    sh_[0].busy = true;
    std::vector<int> one{0};
    run_heuristics(one, /*seed=*/false);
    HIPCHK(hipMemcpyAsync(out, s.h, sizeof(int32_t) * (size_t)d * g_->n, hipMemcpyDeviceToHost,
                          st_));
    HIPCHK(hipStreamSynchronize(st_));
    sh_[0].busy = false;
    ra_.give(off, (L.bytes + 255) / 256);
  }

 private:
  void release(int s) {
    ra_.give(sh_[s].off, sh_[s].len);
    sh_[s].busy = false;
    sh_[s].cancel = false;
  }

  void run_heuristics(const std::vector<int>& fresh, bool seed = true) {
    const int nj = (int)fresh.size();
    const size_t per = (size_t)MAXD * 3 * g_->n * 4;
    if (hscr_.bytes < per * nj) hscr_.alloc(per * nj, st_);
    if (hcnt_.bytes < (size_t)nj * MAXD * 3 * 4) hcnt_.alloc((size_t)nj * MAXD * 3 * 4, st_);
    if (hjob_.bytes < (size_t)nj * 4) hjob_.alloc((size_t)nj * 4, st_);
    HIPCHK(hipMemcpyAsync(hjob_.p, fresh.data(), nj * 4, hipMemcpyHostToDevice, st_));
    const GraphDev G = g_->view();
    HIPCHK(hipEventRecord(ev0_, st_));
    std::vector<int32_t> cnt((size_t)nj * MAXD * 3);
    const int rc = run_heuristic(slots_.as<Slot>(), hjob_.as<int32_t>(), nj, G, hscr_.as<int32_t>(),
                                 hcnt_.as<int32_t>(), cnt.data(), st_);
    if (rc == -2) throw MosError(MOS_E_DEVICE, "heuristic did not converge");
    if (rc != 0) throw MosError(MOS_E_DEVICE, "heuristic: a HIP call failed");
    HIPCHK(hipGetLastError());
    if (seed)
      for (int s : fresh) launch_slot_init(slots_.as<Slot>(), s, G, st_);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(ev1_, st_));
    HIPCHK(hipStreamSynchronize(st_));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ev0_, ev1_));
    for (int s : fresh) sh_[s].heur_ms += ms;
  }

  StepArgs step_args() const {
    StepArgs a;
    a.slots = slots_.as<Slot>();
    a.hist = hist_.as<int32_t>();
    a.G = g_->view();
    a.nslots = S_;
    a.gx = gx_;
    {
      const int64_t cand = (int64_t)std::min(2 * Bplan_, BATCH_MAX) * std::max(1, g_->maxdeg);
      a.gc = (int)std::max<int64_t>(1, std::min<int64_t>(gx_, (cand + 255) / 256));
    }
    a.dm = DM_;
    a.pipelined = pipelined_ ? 1 : 0;
    a.st2 = st2_;
    a.fork = fork_;
    a.join = join_;
    return a;
  }

  // Capture K_ steps into an executable graph (nullptr when capture is not
  // possible).
  hipGraphExec_t capture_steps(const StepArgs& a) {
    hipGraph_t gr = nullptr;
    hipGraphExec_t ex = nullptr;
    if (hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      for (int k = 0; k < K_; ++k) launch_step(a, st_);
      if (hipStreamEndCapture(st_, &gr) != hipSuccess || !gr ||
          hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) != hipSuccess)
        ex = nullptr;
      if (gr) hipGraphDestroy(gr);
    }
    hipGetLastError();
    return ex;
  }

  // K_ steps are captured once into a graph and replayed; the remainder is
  // launched directly, and so is every step in profile mode.
  void launch_steps(int64_t n) {
    const StepArgs a = step_args();
    int nsolo = 0, nreg = 0;
    for (int s = 0; s < S_; ++s)
      if (sh_[s].busy) (sh_[s].q.solo ? nsolo : nreg)++;
    if (nsolo > 0) {
      // each such query advances up to this many steps in its own workgroup
      launch_solo(slots_.as<Slot>(), S_, a.G, DM_, (int)std::max<int64_t>(n, kSoloSteps), st_);
      HIPCHK(hipGetLastError());
    }
    if (nreg == 0) return;
    if (profile_) {
      // events bracketing kernels are not timed when recorded inside a
      // captured graph on this runtime, so profiled steps launch directly
      for (; n > 0; --n) profiled_step(a);
      return;
    }
    if (use_graph_ && !graph_exec_ && !graph_failed_ && n >= K_) {
      graph_exec_ = capture_steps(a);
      graph_failed_ = graph_exec_ == nullptr;
    }
    if (graph_exec_) {
      for (; n >= K_; n -= K_) {
        HIPCHK(hipGraphLaunch(graph_exec_, st_));
        ++graph_replays_;
      }
    }
    for (; n > 0; --n) {
      launch_step(a, st_);
      ++direct_steps_;
    }
    HIPCHK(hipGetLastError());
  }

  // Profile mode: every kernel of every step is bracketed by events; a ring of
  // event sets is drained as it wraps and at every poll.
  static constexpr int RING = 32;
  void profiled_step(const StepArgs& a) {
    constexpr int NE = 2 * kStepKernels + 1;
    if (pev_.empty()) {
      pev_.resize((size_t)RING * NE);
      for (auto& e : pev_) HIPCHK(hipEventCreate(&e));
    }
    if (ring_used_ == RING) drain_one();
    hipEvent_t* set = &pev_[(size_t)((ring_head_ + ring_used_) % RING) * NE];
    launch_step(a, st_, set, profile_);
    HIPCHK(hipGetLastError());
    ++ring_used_;
    ++direct_steps_;
  }
  void drain_one() {
    constexpr int NE = 2 * kStepKernels + 1;
    hipEvent_t* set = &pev_[(size_t)ring_head_ * NE];
    HIPCHK(hipEventSynchronize(set[2 * kStepKernels]));
    for (int i = 0; i < kStepKernels; ++i) {
      if (!((profile_ >> i) & 1u)) continue;
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, set[2 * i], set[2 * i + 1]));
      kms_[i] += ms;
      klaunch_[i]++;
    }
    ring_head_ = (ring_head_ + 1) % RING;
    --ring_used_;
  }
  void drain_profile() {
    while (ring_used_ > 0) drain_one();
  }

  // Smallest F1 left in slot s's OPEN (INT32_MAX when empty).
  int32_t open_min_f1(int s) {
    if (omin_.bytes < 4) omin_.alloc(256, st_);
    launch_open_min(slots_.as<Slot>(), s, omin_.as<int32_t>(), st_);
    HIPCHK(hipGetLastError());
    int32_t m = INT32_MAX;
    HIPCHK(hipMemcpyAsync(&m, omin_.p, 4, hipMemcpyDeviceToHost, st_));
    HIPCHK(hipStreamSynchronize(st_));
    return m;
  }

  // An unfinished query's exact part of the front: the sorted goal front so
  // far cut to the entries whose first objective lies below the smallest F1
  // left in OPEN (every later goal label costs at least that much there, so
  // these entries are final and no other final entry lies below the bound).
  mos_result* harvest_prefix(int s) {
    const int32_t m = open_min_f1(s);
    mos_result* r = harvest(s);
    int64_t k = 0;
    while (k < r->size && r->costs[(size_t)k * r->d] < m) ++k;
    r->size = k;
    r->costs.resize((size_t)k * r->d);
    if (!r->path_off.empty()) {
      r->path_off.resize(k + 1);
      r->arcs.resize(r->path_off[k]);
    }
    r->stats.front = k;
    r->stats.open_min_f1 = m;
    r->complete = false;
    return r;
  }

  // The goal front of slot s: live entries (tombstones dropped), sorted
  // lexicographically ascending on the device, with their witness paths.
  mos_result* harvest(int s) {
    const Slot& d = hslots_[s];
    std::unique_ptr<mos_result> r(new mos_result());
    const int dd = d.d;
    const int nall = d.P_n;
    // read-out scratch, carved from a grow-only buffer of the engine (results
    // are read out one at a time on the engine's stream)
    const auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_fsw = al(front_sort_scratch_bytes(std::max(nall, 1)));
    const size_t b_rows = al((size_t)std::max(nall, 1) * dd * 4), b_labs = al((size_t)std::max(nall, 1) * 4);
    const size_t b_len = b_labs, b_off = al(((size_t)std::max(nall, 1) + 1) * 8);
    char* hv = (char*)grow(hv_, b_fsw + b_rows + b_labs + b_len + b_off);
    void* fsw = hv;
    int32_t* rows = (int32_t*)(hv + b_fsw);
    int32_t* labs = (int32_t*)(hv + b_fsw + b_rows);
    int32_t* lenp = (int32_t*)(hv + b_fsw + b_rows + b_labs);
    int64_t* offp = (int64_t*)(hv + b_fsw + b_rows + b_labs + b_len);
    int np = 0;
    if (nall > 0) {
      np = front_sort(d.Pg[d.P_sel], d.P_cap, d.Plab[d.P_sel], dd, nall, fsw, rows, labs, st_);
      if (np < 0) HIPCHK(hipGetLastError());
      if (np < 0) throw MosError(MOS_E_DEVICE, "front sort failed");
    }
    r->d = dd;
    r->size = np;
    r->costs.resize((size_t)np * dd);
    if (np > 0)
      HIPCHK(hipMemcpyAsync(r->costs.data(), rows, (size_t)np * dd * 4, hipMemcpyDeviceToHost,
                            st_));
    HIPCHK(hipStreamSynchronize(st_));
    if (want_paths_ && np > 0) {
      launch_path_len(slots_.as<Slot>(), s, labs, (int)np, lenp, st_);
      std::vector<int32_t> hl(np);
      HIPCHK(hipMemcpyAsync(hl.data(), lenp, np * 4, hipMemcpyDeviceToHost, st_));
      HIPCHK(hipStreamSynchronize(st_));
      r->path_off.assign(np + 1, 0);
      for (int64_t i = 0; i < np; ++i) r->path_off[i + 1] = r->path_off[i] + hl[i];
      const int64_t tot = r->path_off[np];
      r->arcs.resize(tot);
      if (tot > 0) {
        int32_t* arcs = (int32_t*)grow(ha_, (size_t)tot * 4);
        HIPCHK(hipMemcpyAsync(offp, r->path_off.data(), (np + 1) * 8, hipMemcpyHostToDevice, st_));
        launch_path_write(slots_.as<Slot>(), s, labs, (int)np, offp, arcs, st_);
        HIPCHK(hipMemcpyAsync(r->arcs.data(), arcs, tot * 4, hipMemcpyDeviceToHost, st_));
      }
      HIPCHK(hipStreamSynchronize(st_));
    } else if (want_paths_) {
      r->path_off.assign(1, 0);
    }
    r->stats = stats_of(s);
    r->stats.front = np;
    return r.release();
  }

  const mos_graph* g_;
  int S_, DM_, B_;
  int widen_ = 1, Bplan_ = 1;  // tail widening factor; batch width the slot layouts allow
  bool pipelined_ = false;
  hipStream_t st2_ = nullptr;  // pipelined steps: the pop's stream
  hipEvent_t fork_ = nullptr, join_ = nullptr;
  int64_t label_limit_;
  bool want_paths_;
  int K_;
  hipStream_t st_ = nullptr;
  bool own_stream_ = false;
  DevBuf arena_, slots_, hist_, hscr_, hcnt_, hjob_, omin_;
  DevBuf hv_, ha_;  // result read-out scratch (front sort, rows, path offsets; path arcs)
  // b with at least n bytes (grown by doubling; the engine's stream is idle
  // between read-outs, so the old contents need not survive)
  void* grow(DevBuf& b, size_t n) {
    if (b.bytes < n) b.alloc(std::max(n, 2 * b.bytes), st_);
    return b.p;
  }
  Slot* hslots_ = nullptr;
  RangeAlloc ra_;
  std::vector<SlotHost> sh_;
  int gx_ = 1;
  int big_work_ = (int)BIG_WORK;
  hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
  hipGraphExec_t graph_exec_ = nullptr;
  bool graph_failed_ = false;
  int64_t graph_replays_ = 0, direct_steps_ = 0;
  bool use_graph_ = true;
  bool progress_ = false;
  int progress_level_ = 0;
  uint32_t profile_ = 0;  // kernels of the step timed with events (bit i = kernel i)
  std::vector<hipEvent_t> pev_;
  int ring_head_ = 0, ring_used_ = 0;
  double kms_[kStepKernels] = {};
  int64_t klaunch_[kStepKernels] = {};
  std::chrono::steady_clock::time_point t_last_;
  int64_t readmissions_ = 0;
};

// ------------------------------------------------------------- engine cache
static Engine* acquire_engine(const mos_graph* gc, const EngineKey& k, int64_t budget,
                              hipStream_t stream) {
  mos_graph* g = const_cast<mos_graph*>(gc);
  {
    std::lock_guard<std::mutex> lk(g->pool_mu);
    for (size_t i = 0; i < g->pool.size(); ++i)
      if (g->pool[i].first == k) {
        Engine* e = g->pool[i].second;
        g->pool.erase(g->pool.begin() + i);
        e->set_pipelined(k.pipelined);
        return e;
      }
  }
  Engine* e = new Engine(g, k.S, k.dm, budget, stream, k.B, k.label_limit, k.paths, k.steps);
  e->set_pipelined(k.pipelined);
  return e;
}

static void release_engine(const mos_graph* gc, const EngineKey& k, Engine* e) {
  mos_graph* g = const_cast<mos_graph*>(gc);
  Engine* evict = nullptr;
  {
    std::lock_guard<std::mutex> lk(g->pool_mu);
    g->pool.emplace_back(k, e);
    if (g->pool.size() > 2) {
      evict = g->pool.front().second;
      g->pool.erase(g->pool.begin());
    }
  }
  delete evict;
}

// ------------------------------------------------------------ option helpers
using Opts = MosOpts;

mos_status mos_internal_read_options(const mos_options* o, MosOpts* out) {
  Opts r;
  if (o) {
    if (o->struct_size < offsetof(mos_options, costs_only))
      return set_err(MOS_E_INVALID_ARG, "mos_options.struct_size too small");
    r.n_objectives = o->n_objectives;
    if (o->batch_width) r.B = o->batch_width;
    r.max_slots = o->max_slots;
    r.label_limit = o->label_limit;
    r.mem_budget = o->mem_budget;
    r.stream = o->stream;
    if (o->struct_size >= offsetof(mos_options, steps_per_poll)) r.want_paths = o->costs_only ? 0 : 1;
    if (o->struct_size >= offsetof(mos_options, profile_kernels) && o->steps_per_poll > 0)
      r.steps = o->steps_per_poll;
    if (o->struct_size >= offsetof(mos_options, heuristic_radius)) r.profile = (uint32_t)o->profile_kernels;
    if (o->struct_size >= offsetof(mos_options, step_budget))
      r.heur_factor = o->heuristic_radius == 0 ? kDefaultHeurFactor
                                               : (o->heuristic_radius < 0 ? 0 : o->heuristic_radius);
    if (o->struct_size >= offsetof(mos_options, step_budget) + sizeof(int64_t))
      r.step_budget = o->step_budget;
    if (o->struct_size >= offsetof(mos_options, pop_order) + sizeof(int32_t))
      r.pop_order = o->pop_order;
    if (o->struct_size >= offsetof(mos_options, epsilon_ppm) + sizeof(int32_t))
      r.eps_ppm = o->epsilon_ppm;
    if (o->struct_size >= offsetof(mos_options, eager_goal) + sizeof(int32_t))
      r.eager_goal = o->eager_goal ? 1 : 0;
    if (o->struct_size >= offsetof(mos_options, pipelined) + sizeof(int32_t))
      r.pipelined = o->pipelined ? 1 : 0;
    if (o->struct_size >= offsetof(mos_options, persistent_query) + sizeof(int32_t))
      r.persistent_query = o->persistent_query ? 1 : 0;
  }
  if (r.B < 1 || r.B > BATCH_MAX)
    return set_err(MOS_E_INVALID_ARG, "batch_width must lie in [1, 32768]");
  if (r.max_slots < 0 || r.label_limit < 0 || r.mem_budget < 0 || r.n_objectives < 0)
    return set_err(MOS_E_INVALID_ARG, "negative option");
  if (r.steps > 1024) return set_err(MOS_E_INVALID_ARG, "steps_per_poll too large");
  if (r.step_budget < 0) return set_err(MOS_E_INVALID_ARG, "negative step_budget");
  if (r.pop_order != MOS_POP_LEXICOGRAPHIC && r.pop_order != MOS_POP_GENERATION)
    return set_err(MOS_E_INVALID_ARG, "unknown pop_order");
  if (r.eps_ppm < 0 || r.eps_ppm > 1000000000)
    return set_err(MOS_E_INVALID_ARG, "epsilon_ppm must lie in [0, 10^9]");
  *out = r;
  return MOS_OK;
}

static int64_t default_budget(int64_t want) {
  size_t fr = 0, tot = 0;
  HIPCHK(hipMemGetInfo(&fr, &tot));
  int64_t cap = (int64_t)(fr * 0.7);
  if (want > 0) {
    if (want > cap) throw MosError(MOS_E_OUT_OF_MEMORY, "mem_budget exceeds free device memory");
    return want;
  }
  return std::min<int64_t>(cap, (int64_t)48 << 30);
}

mos_status mos_internal_check_query(const mos_graph* g, int32_t s, int32_t t, int32_t nobj, int* d) {
  if (s < 0 || s >= g->n || t < 0 || t >= g->n)
    return set_err(MOS_E_INVALID_ARG, "start or goal out of range");
  if (nobj < 0 || nobj > g->D) return set_err(MOS_E_INVALID_ARG, "n_objectives out of range");
  *d = nobj == 0 ? g->D : nobj;
  return MOS_OK;
}

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* mos_status_string(mos_status s) {
  switch (s) {
    case MOS_OK: return "ok";
    case MOS_E_INVALID_ARG: return "invalid argument";
    case MOS_E_NEGATIVE_COST: return "negative cost";
    case MOS_E_OVERFLOW_RISK: return "int32 overflow risk";
    case MOS_E_NO_DEVICE: return "no device";
    case MOS_E_DEVICE: return "device error";
    case MOS_E_OUT_OF_MEMORY: return "out of memory";
    case MOS_E_LABEL_LIMIT: return "label limit";
    case MOS_E_CANCELLED: return "cancelled";
    case MOS_E_NOT_READY: return "not ready";
    case MOS_E_STEP_LIMIT: return "step budget reached (exact prefix returned)";
  }
  return "unknown status";
}

const char* mos_last_error(void) { return g_last_error.c_str(); }

mos_status mos_set_allocator(void* (*alloc)(size_t, void*, void*), void (*release)(void*, void*),
                             void* ctx) {
  if ((alloc == nullptr) != (release == nullptr))
    return set_err(MOS_E_INVALID_ARG, "alloc and release must both be set or both be NULL");
  std::lock_guard<std::mutex> lk(g_hooks_mu);
  g_hooks.alloc = alloc;
  g_hooks.release = release;
  g_hooks.ctx = ctx;
  return MOS_OK;
}

mos_status mos_graph_create(int32_t n, int64_t m, int32_t D, const int64_t* row_ptr,
                            const int32_t* col, const int32_t* cost, mos_graph** out) {
  // ---- validation (no device call before it passes)
  if (!out) return set_err(MOS_E_INVALID_ARG, "out is NULL");
  if (n < 1 || m < 0 || m >= ((int64_t)1 << 31) - 1)
    return set_err(MOS_E_INVALID_ARG, "n_nodes must be >= 1 and n_arcs in [0, 2^31-1)");
  if (D < 1 || D > MOS_MAX_OBJECTIVES) return set_err(MOS_E_INVALID_ARG, "D must lie in [1, 12]");
  if (!row_ptr || (m > 0 && (!col || !cost))) return set_err(MOS_E_INVALID_ARG, "NULL array");
  if (row_ptr[0] != 0 || row_ptr[n] != m) return set_err(MOS_E_INVALID_ARG, "row_ptr ends");
  int32_t maxdeg = 0;
  for (int32_t v = 0; v < n; ++v) {
    const int64_t a = row_ptr[v], b = row_ptr[v + 1];
    if (b < a) return set_err(MOS_E_INVALID_ARG, "row_ptr not non-decreasing");
    maxdeg = (int32_t)std::max<int64_t>(maxdeg, b - a);
  }
  for (int64_t e = 0; e < m; ++e)
    if (col[e] < 0 || col[e] >= n) return set_err(MOS_E_INVALID_ARG, "arc target out of range");
  int32_t csum[MAXD] = {};
  for (int32_t k = 0; k < D; ++k) {
    int64_t sum = 0, mx = 0;
    for (int64_t e = 0; e < m; ++e) {
      const int64_t c = cost[e * D + k];
      if (c < 0) return set_err(MOS_E_NEGATIVE_COST, "negative arc cost");
      sum += c;
      mx = std::max(mx, c);
    }
    if (2 * sum + mx >= (int64_t)INT32_MAX)
      return set_err(MOS_E_OVERFLOW_RISK, "2*sum+max of an objective reaches INT32_MAX");
    csum[k] = (int32_t)sum;
  }
  return guarded([&]() -> mos_status {
    const int dev = ensure_device();
    std::unique_ptr<mos_graph> g(new mos_graph());
    g->n = n;
    g->m = m;
    g->D = D;
    g->maxdeg = maxdeg;
    g->device = dev;
    for (int k = 0; k < MAXD; ++k) g->csum[k] = csum[k];
    std::vector<int32_t> rp(n + 1), planes((size_t)D * std::max<int64_t>(m, 1));
    for (int32_t v = 0; v <= n; ++v) rp[v] = (int32_t)row_ptr[v];
    for (int64_t e = 0; e < m; ++e)
      for (int k = 0; k < D; ++k) planes[(size_t)k * m + e] = cost[e * D + k];
    // reverse CSR
    std::vector<int32_t> rrow(n + 1, 0), rsrc(std::max<int64_t>(m, 1)), rarc(std::max<int64_t>(m, 1));
    for (int64_t e = 0; e < m; ++e) rrow[col[e] + 1]++;
    for (int32_t v = 0; v < n; ++v) rrow[v + 1] += rrow[v];
    std::vector<int32_t> fill(rrow.begin(), rrow.end() - 1);
    for (int32_t u = 0; u < n; ++u)
      for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
        const int32_t p = fill[col[e]]++;
        rsrc[p] = u;
        rarc[p] = (int32_t)e;
      }
    hipStream_t st = nullptr;
    g->row_ptr.alloc((n + 1) * 4, st);
    g->col.alloc(std::max<int64_t>(m, 1) * 4, st);
    g->cost.alloc(planes.size() * 4, st);
    g->rrow.alloc((n + 1) * 4, st);
    g->rsrc.alloc(rsrc.size() * 4, st);
    g->rarc.alloc(rarc.size() * 4, st);
    HIPCHK(hipMemcpy(g->row_ptr.p, rp.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    if (m > 0) HIPCHK(hipMemcpy(g->col.p, col, m * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->cost.p, planes.data(), planes.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->rrow.p, rrow.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->rsrc.p, rsrc.data(), rsrc.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->rarc.p, rarc.data(), rarc.size() * 4, hipMemcpyHostToDevice));
    *out = g.release();
    return MOS_OK;
  });
}

void mos_graph_destroy(mos_graph* g) {
  if (!g) return;
  for (auto& kv : g->pool) delete kv.second;
  g->pool.clear();
  delete g;
}


// Whether a query of these options runs its steps in one workgroup of its own
// (mos_options.persistent_query): not with a step budget (its exact prefix
// is defined by the multi-kernel step's pops), the generation order or the
// approximate mode, nor on a graph whose out-degree exceeds the one-workgroup
// candidate sort.
static int32_t solo_for(const mos_graph* g, const Opts& o) {
  return o.persistent_query && o.step_budget == 0 && o.pop_order == MOS_POP_LEXICOGRAPHIC &&
                 o.eps_ppm == 0 && g->maxdeg <= kSoloMaxDeg
             ? 1
             : 0;
}

mos_status mos_solve_batch(const mos_graph* g, int32_t nq, const int32_t* starts,
                           const int32_t* goals, const int32_t* n_objectives,
                           const mos_options* opt, mos_result** out, mos_status* st) {
  if (!g || nq < 0 || (nq > 0 && (!starts || !goals || !out || !st)))
    return set_err(MOS_E_INVALID_ARG, "NULL argument or negative count");
  Opts o;
  mos_status rs = mos_internal_read_options(opt, &o);
  if (rs != MOS_OK) return rs;
  std::vector<int> dq(nq);
  for (int32_t i = 0; i < nq; ++i) {
    int32_t nobj = n_objectives ? n_objectives[i] : o.n_objectives;
    rs = mos_internal_check_query(g, starts[i], goals[i], nobj, &dq[i]);
    if (rs != MOS_OK) return rs;
  }
  if (nq == 0) return MOS_OK;
  return guarded([&]() -> mos_status {
    HIPCHK(hipSetDevice(g->device));
    // engines are cached per graph: slot counts are rounded up to a power of
    // two and the kernels are built for the graph's objective count (queries
    // with fewer objectives run in the same engine), so repeated calls with
    // varying sizes and objective counts reuse one engine and its arena
    const int want = o.max_slots > 0 ? std::min(o.max_slots, nq) : std::min(nq, 256);
    int S = 1;
    while (S < want) S <<= 1;
    const EngineKey key{S, dm_for(g->D), o.mem_budget, (void*)o.stream, o.B, o.label_limit,
                        o.want_paths != 0, o.steps, o.pipelined != 0};
    Engine* ep = acquire_engine(g, key, default_budget(o.mem_budget), (hipStream_t)o.stream);
    std::unique_ptr<Engine> guard(ep);
    Engine& eng = *ep;
    std::deque<QueryReq> pending;
    for (int32_t i = 0; i < nq; ++i) {
      QueryReq q;
      q.id = i;
      q.start = starts[i];
      q.goal = goals[i];
      q.d = dq[i];
      q.heur_factor = o.heur_factor;
      q.step_budget = o.step_budget;
      q.pop_order = o.pop_order;
      q.eps_ppm = o.eps_ppm;
      q.eager_goal = o.eager_goal;
      q.solo = solo_for(g, o);
      q.reserve = eng.default_reserve();
      pending.push_back(q);
      out[i] = nullptr;
      st[i] = MOS_E_NOT_READY;
    }
    std::vector<Finished> done;
    int64_t left = nq;
    mos_status first_bad = MOS_OK;
    std::string msg;
    while (left > 0) {
      done.clear();
      eng.tick(pending, done);
      for (auto& f : done) {
        out[f.id] = f.res;
        st[f.id] = f.st;
        if (f.st != MOS_OK && first_bad == MOS_OK) {
          first_bad = f.st;
          msg = f.msg;
        }
        --left;
      }
      if (pending.empty() && eng.busy_count() == 0 && left > 0)
        throw MosError(MOS_E_DEVICE, "engine stalled");
    }
    release_engine(g, key, guard.release());
    if (first_bad != MOS_OK) return set_err(first_bad, msg);
    return MOS_OK;
  });
}

mos_status mos_solve(const mos_graph* g, int32_t start, int32_t goal, const mos_options* opt,
                     mos_result** out) {
  if (!g || !out) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  Opts o;
  mos_status rs = mos_internal_read_options(opt, &o);
  if (rs != MOS_OK) return rs;
  int d;
  rs = mos_internal_check_query(g, start, goal, o.n_objectives, &d);
  if (rs != MOS_OK) return rs;
  mos_options o1{};
  if (opt) std::memcpy(&o1, opt, std::min<size_t>(opt->struct_size, sizeof(mos_options)));
  o1.struct_size = sizeof(mos_options);
  o1.max_slots = 1;
  mos_status st1 = MOS_E_NOT_READY;
  mos_result* r = nullptr;
  rs = mos_solve_batch(g, 1, &start, &goal, nullptr, &o1, &r, &st1);
  if (rs == MOS_E_STEP_LIMIT && r) {
    *out = r;  // the exact prefix (see mos_options.step_budget)
    return rs;
  }
  if (rs != MOS_OK) return rs;
  *out = r;
  return MOS_OK;
}

int64_t mos_result_size(const mos_result* r) { return r ? r->size : 0; }
int32_t mos_result_dim(const mos_result* r) { return r ? r->d : 0; }

mos_status mos_result_costs(const mos_result* r, int32_t* out) {
  if (!r || (!out && r->size > 0)) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  if (!r->costs.empty()) std::memcpy(out, r->costs.data(), r->costs.size() * 4);
  return MOS_OK;
}

mos_status mos_result_path(const mos_result* r, int64_t i, int32_t* arcs, int64_t cap,
                           int64_t* len) {
  if (!r || !len || i < 0 || i >= r->size || cap < 0 || (cap > 0 && !arcs))
    return set_err(MOS_E_INVALID_ARG, "bad path request");
  if (r->path_off.empty()) return set_err(MOS_E_INVALID_ARG, "paths were not requested");
  const int64_t a = r->path_off[i], b = r->path_off[i + 1];
  *len = b - a;
  const int64_t c = std::min(cap, b - a);
  if (c > 0) std::memcpy(arcs, r->arcs.data() + a, c * 4);
  return MOS_OK;
}

mos_status mos_result_stats(const mos_result* r, mos_stats* out) {
  if (!r || !out) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  *out = r->stats;
  return MOS_OK;
}

void mos_result_destroy(mos_result* r) { delete r; }

mos_status mos_heuristic(const mos_graph* g, int32_t goal, int32_t n_objectives, int32_t* h) {
  if (!g || !h) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  int d;
  mos_status rs = mos_internal_check_query(g, goal, goal, n_objectives, &d);
  if (rs != MOS_OK) return rs;
  return guarded([&]() -> mos_status {
    HIPCHK(hipSetDevice(g->device));
    Layout L;
    int64_t need = 0;
    for (int64_t b = 1 << 22;; b *= 2) {
      if (plan_layout(g, d, 1, b, 16, &L)) {
        need = b;
        break;
      }
      if (b > ((int64_t)1 << 40)) throw MosError(MOS_E_OUT_OF_MEMORY, "graph too large");
    }
    Engine eng(g, 1, dm_for(d), need, nullptr, 1, 16, false, 1);
    eng.heuristic_only(goal, d, h);
    return MOS_OK;
  });
}

}  // extern "C"

// ----------------------------------------------------------------- session
struct mos_session {
  const mos_graph* g = nullptr;
  std::unique_ptr<Engine> eng;
  bool finished = false;
};

extern "C" {

mos_status mos_session_create(const mos_graph* g, int32_t start, int32_t goal,
                              const mos_options* opt, mos_session** out) {
  if (!g || !out) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  Opts o;
  mos_status rs = mos_internal_read_options(opt, &o);
  if (rs != MOS_OK) return rs;
  int d;
  rs = mos_internal_check_query(g, start, goal, o.n_objectives, &d);
  if (rs != MOS_OK) return rs;
  return guarded([&]() -> mos_status {
    HIPCHK(hipSetDevice(g->device));
    std::unique_ptr<mos_session> s(new mos_session());
    s->g = g;
    s->eng.reset(new Engine(g, 1, dm_for(d), default_budget(o.mem_budget), (hipStream_t)o.stream, o.B,
                            o.label_limit, o.want_paths != 0, o.steps));
    s->eng->set_pipelined(o.pipelined != 0);
    s->eng->set_profile(o.profile);
    QueryReq q;
    q.id = 0;
    q.start = start;
    q.goal = goal;
    q.d = d;
    q.heur_factor = o.heur_factor;
    q.pop_order = o.pop_order;
    q.eps_ppm = o.eps_ppm;
    q.eager_goal = o.eager_goal;
    q.reserve = s->eng->arena_bytes();
    std::string msg;
    mos_status st = s->eng->session_admit(q, &msg);
    if (st != MOS_OK) return set_err(st, msg);
    *out = s.release();
    return MOS_OK;
  });
}

mos_status mos_session_step(mos_session* s, int64_t nsteps, int32_t* done) {
  if (!s || !done || nsteps < 0) return set_err(MOS_E_INVALID_ARG, "bad session step");
  return guarded([&]() -> mos_status {
    HIPCHK(hipSetDevice(s->g->device));
    const int32_t st = s->eng->slot0().status;
    if (st == S_RUN && nsteps > 0) s->eng->advance(nsteps);
    const int32_t st2 = s->eng->slot0().status;
    if (st2 == S_OVERFLOW) return set_err(MOS_E_LABEL_LIMIT, "search state outgrew the reservation");
    *done = st2 == S_RUN ? 0 : 1;
    return MOS_OK;
  });
}

mos_status mos_session_stats(const mos_session* s, mos_stats* out) {
  if (!s || !out) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  *out = s->eng->stats_of(0);
  return MOS_OK;
}

mos_status mos_session_result(mos_session* s, mos_result** out) {
  if (!s || !out) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  if (s->finished) return set_err(MOS_E_INVALID_ARG, "result already taken");
  return guarded([&]() -> mos_status {
    HIPCHK(hipSetDevice(s->g->device));
    while (s->eng->slot0().status == S_RUN) s->eng->advance(64);
    if (s->eng->slot0().status != S_DONE)
      return set_err(MOS_E_LABEL_LIMIT, "search state outgrew the reservation");
    *out = s->eng->harvest_slot0();
    s->finished = true;
    return MOS_OK;
  });
}

mos_status mos_session_front(mos_session* s, int32_t* open_min_f1, mos_result** out) {
  if (!s || !open_min_f1 || !out) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  if (s->finished) return set_err(MOS_E_INVALID_ARG, "result already taken");
  return guarded([&]() -> mos_status {
    HIPCHK(hipSetDevice(s->g->device));
    if (s->eng->slot0().status == S_OVERFLOW)
      return set_err(MOS_E_LABEL_LIMIT, "search state outgrew the reservation");
    int32_t m = INT32_MAX;
    mos_result* r = s->eng->front_so_far0(&m);
    *open_min_f1 = m;
    *out = r;
    return MOS_OK;
  });
}

int32_t mos_session_kernel_count(void) { return kStepKernels; }

mos_status mos_session_launch_counts(const mos_session* s, int64_t* graph_replays,
                                     int64_t* steps_per_replay, int64_t* direct_steps) {
  if (!s || !graph_replays || !steps_per_replay || !direct_steps)
    return set_err(MOS_E_INVALID_ARG, "NULL argument");
  *graph_replays = s->eng->graph_replays();
  *steps_per_replay = s->eng->steps_per_replay();
  *direct_steps = s->eng->direct_steps();
  return MOS_OK;
}

mos_status mos_session_set_profile(mos_session* s, int32_t mask) {
  if (!s) return set_err(MOS_E_INVALID_ARG, "NULL session");
  return guarded([&]() -> mos_status {
    HIPCHK(hipSetDevice(s->g->device));
    s->eng->set_profile((uint32_t)mask);
    return MOS_OK;
  });
}

mos_status mos_session_kernel_times(const mos_session* s, int32_t i, const char** name, double* ms,
                                    int64_t* launches) {
  if (!s || i < 0 || i >= kStepKernels || !name || !ms || !launches)
    return set_err(MOS_E_INVALID_ARG, "bad kernel index or NULL argument");
  *name = kStepKernelNames[i];
  *ms = s->eng->kernel_ms(i);
  *launches = s->eng->kernel_launches(i);
  return MOS_OK;
}

void mos_session_destroy(mos_session* s) { delete s; }

}  // extern "C"

// ------------------------------------------------------------------ server
struct mos_server {
  const mos_graph* g = nullptr;
  std::unique_ptr<Engine> eng;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<QueryReq> inbox;
  std::map<uint64_t, Finished> finished;
  std::map<uint64_t, bool> known;  // ticket -> collected
  bool stop = false;
  uint64_t next = 1;
  int64_t submitted = 0, nfinished = 0, ticks = 0;
  std::atomic<int64_t> resident{0}, queued{0};
  std::vector<uint64_t> cancels;
  std::string fatal;
  mos_status fatal_st = MOS_OK;
  int64_t fail_at_tick = -1;  // test hook (MOS_SERVER_FAIL_AT_TICK): throw before this tick
  int32_t heur_factor = kDefaultHeurFactor;
  int64_t step_budget = 0;
  int32_t pop_order = 0;
  int32_t eps_ppm = 0;
  int32_t eager_goal = 0;
  int32_t solo = 0;

  // The loop cannot go on (a device error): every query that has not been
  // reported yet -- finished this tick, resident in a slot, queued here or
  // still in the inbox -- gets an error entry, so that no wait blocks forever.
  void fail_all(std::deque<QueryReq>& pending, std::vector<Finished>& done, mos_status st,
                const std::string& what) {
    std::lock_guard<std::mutex> lk(mu);
    fatal = what;
    fatal_st = st;
    auto put = [&](int64_t id, const Finished& f) {
      if (finished.count((uint64_t)id) == 0 && !known[(uint64_t)id]) {
        finished[(uint64_t)id] = f;
        nfinished++;
      }
    };
    for (auto& f : done) put(f.id, f);
    done.clear();
    for (int64_t id : eng->resident_ids()) put(id, Finished{id, st, nullptr, what});
    for (auto& q : pending) put(q.id, Finished{q.id, st, nullptr, what});
    for (auto& q : inbox) put(q.id, Finished{q.id, st, nullptr, what});
    pending.clear();
    inbox.clear();
    resident = 0;
    queued = 0;
    stop = true;
    cv_done.notify_all();
  }

  void loop() {
    hipSetDevice(g->device);
    std::deque<QueryReq> pending;
    std::vector<Finished> done;
    for (;;) {
      std::vector<uint64_t> cs;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || !inbox.empty() || !pending.empty() || eng->busy_count() > 0 || !cancels.empty(); });
        if (stop) return;
        while (!inbox.empty()) {
          pending.push_back(inbox.front());
          inbox.pop_front();
        }
        cs.swap(cancels);
      }
      for (uint64_t t : cs) {
        bool was_pending = false;
        for (auto it = pending.begin(); it != pending.end(); ++it)
          if ((uint64_t)it->id == t) {
            pending.erase(it);
            was_pending = true;
            break;
          }
        if (was_pending) {
          std::lock_guard<std::mutex> lk(mu);
          finished[t] = Finished{(int64_t)t, MOS_E_CANCELLED, nullptr, "cancelled"};
          nfinished++;
          cv_done.notify_all();
        } else {
          eng->cancel_query((int64_t)t);
        }
      }
      done.clear();
      try {
        if (fail_at_tick >= 0 && ticks >= fail_at_tick)
          throw MosError(MOS_E_DEVICE, "injected server failure (test hook)");
        eng->tick(pending, done);
      } catch (const std::exception& e) {
        const MosError* me = dynamic_cast<const MosError*>(&e);
        fail_all(pending, done, me ? me->st : MOS_E_DEVICE, e.what());
        return;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        ticks++;
        for (auto& f : done) {
          finished[(uint64_t)f.id] = f;
          nfinished++;
        }
        resident = eng->busy_count();
        queued = (int64_t)pending.size() + (int64_t)inbox.size();
        if (!done.empty()) cv_done.notify_all();
      }
    }
  }
};

extern "C" {

mos_status mos_server_create_ex(const mos_graph* g, int64_t mem_budget, int32_t max_slots,
                                const mos_options* opt, mos_server** out) {
  if (!g || !out || mem_budget < 0 || max_slots < 0)
    return set_err(MOS_E_INVALID_ARG, "bad server arguments");
  MosOpts o;
  if (opt) {
    mos_status rs = mos_internal_read_options(opt, &o);
    if (rs != MOS_OK) return rs;
  } else {
    o.steps = 4;
  }
  return guarded([&]() -> mos_status {
    HIPCHK(hipSetDevice(g->device));
    std::unique_ptr<mos_server> s(new mos_server());
    s->g = g;
    s->heur_factor = o.heur_factor;
    s->step_budget = o.step_budget;
    s->pop_order = o.pop_order;
    s->eps_ppm = o.eps_ppm;
    s->eager_goal = o.eager_goal;
    s->solo = solo_for(g, o);
    const int S = max_slots > 0 ? max_slots : 64;
    s->eng.reset(new Engine(g, S, dm_for(g->D), default_budget(mem_budget), nullptr, o.B,
                            o.label_limit, o.want_paths != 0, o.steps));
    s->eng->set_pipelined(o.pipelined != 0);
    if (const char* x = std::getenv("MOS_SERVER_FAIL_AT_TICK")) s->fail_at_tick = std::atoll(x);
    s->th = std::thread([p = s.get()] { p->loop(); });
    *out = s.release();
    return MOS_OK;
  });
}

mos_status mos_server_create(const mos_graph* g, int64_t mem_budget, int32_t max_slots,
                             mos_server** out) {
  return mos_server_create_ex(g, mem_budget, max_slots, nullptr, out);
}

mos_status mos_server_submit(mos_server* s, int32_t start, int32_t goal, int32_t n_objectives,
                             uint64_t* ticket) {
  if (!s || !ticket) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  int d;
  mos_status rs = mos_internal_check_query(s->g, start, goal, n_objectives, &d);
  if (rs != MOS_OK) return rs;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return set_err(s->fatal_st == MOS_OK ? MOS_E_DEVICE : s->fatal_st, "server stopped: " + s->fatal);
  QueryReq q;
  q.id = (int64_t)s->next++;
  q.start = start;
  q.goal = goal;
  q.d = d;
  q.heur_factor = s->heur_factor;
  q.step_budget = s->step_budget;
  q.pop_order = s->pop_order;
  q.eps_ppm = s->eps_ppm;
  q.eager_goal = s->eager_goal;
  q.solo = s->solo;
  q.reserve = s->eng->default_reserve();
  s->inbox.push_back(q);
  s->known[(uint64_t)q.id] = false;
  s->submitted++;
  *ticket = (uint64_t)q.id;
  s->cv.notify_all();
  return MOS_OK;
}

static mos_status collect(mos_server* s, uint64_t ticket, mos_result** out) {
  auto it = s->finished.find(ticket);
  if (it == s->finished.end()) {
    // a stopped server finishes nothing more: report why instead of NOT_READY
    if (s->stop)
      return set_err(s->fatal_st == MOS_OK ? MOS_E_DEVICE : s->fatal_st,
                     "server stopped: " + s->fatal);
    return MOS_E_NOT_READY;
  }
  Finished f = it->second;
  s->finished.erase(it);
  s->known[ticket] = true;
  if (f.st == MOS_E_STEP_LIMIT && f.res) {
    *out = f.res;  // the exact prefix
    return set_err(f.st, f.msg);
  }
  if (f.st != MOS_OK) return set_err(f.st, f.msg);
  *out = f.res;
  return MOS_OK;
}

mos_status mos_server_poll(mos_server* s, uint64_t ticket, mos_result** out) {
  if (!s || !out) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto k = s->known.find(ticket);
  if (k == s->known.end() || k->second) return set_err(MOS_E_INVALID_ARG, "unknown ticket");
  return collect(s, ticket, out);
}

mos_status mos_server_wait(mos_server* s, uint64_t ticket, int64_t timeout_ms, mos_result** out) {
  if (!s || !out) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto k = s->known.find(ticket);
  if (k == s->known.end() || k->second) return set_err(MOS_E_INVALID_ARG, "unknown ticket");
  auto ready = [&] { return s->finished.count(ticket) > 0 || s->stop; };
  if (timeout_ms < 0) s->cv_done.wait(lk, ready);
  else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
    return MOS_E_NOT_READY;
  return collect(s, ticket, out);
}

mos_status mos_server_cancel(mos_server* s, uint64_t ticket) {
  if (!s) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto k = s->known.find(ticket);
  if (k == s->known.end() || k->second) return set_err(MOS_E_INVALID_ARG, "unknown ticket");
  if (s->finished.count(ticket)) return MOS_OK;  // already done: nothing to cancel
  for (auto it = s->inbox.begin(); it != s->inbox.end(); ++it)
    if ((uint64_t)it->id == ticket) {
      s->inbox.erase(it);
      s->finished[ticket] = Finished{(int64_t)ticket, MOS_E_CANCELLED, nullptr, "cancelled"};
      s->nfinished++;
      s->cv_done.notify_all();
      return MOS_OK;
    }
  s->cancels.push_back(ticket);
  s->cv.notify_all();
  return MOS_OK;
}

mos_status mos_server_counters(mos_server* s, int64_t* out6) {
  if (!s || !out6) return set_err(MOS_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out6[0] = s->submitted;
  out6[1] = s->nfinished;
  out6[2] = s->resident;
  out6[3] = s->queued;
  out6[4] = s->ticks;
  out6[5] = s->eng ? s->eng->readmissions() : 0;
  return MOS_OK;
}

void mos_server_destroy(mos_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  for (auto& kv : s->finished) delete kv.second.res;
  s->eng.reset();
  delete s;
}

}  // extern "C"
