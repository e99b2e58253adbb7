// mos_solve_noalloc: the exact front of one query with no device allocation.
//
// For callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid hipMalloc): every device byte the
// search needs -- the slot descriptor, the OPEN histogram, the heuristic's
// worklists, the query's label state and the sorted front -- is carved from
// one file-scope device array of kScratchBytes per GPU.  The search itself is
// the same step (the same kernels, launched one by one on the caller's stream)
// that mos_solve runs.  Calls on one device share its array and are serialised
// by a per-device lock; nothing survives from one call to the next.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <mutex>
#include <string>

#include "front.h"
#include "graph_internal.h"
#include "kernels.h"
#include "layout.h"
#include "mos.h"

namespace mos {

constexpr size_t kScratchBytes = (size_t)256 << 20;  // per GPU, held until the process ends
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

// device address of `scratch` on each device (the array's name in host code
// is only a host-side stand-in for the symbol)
static void* g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu[kMaxDevices];

static hipError_t scratch_on(int dev, char** out) {
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = (char*)g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace mos

using namespace mos;

namespace {

struct Fail {
  mos_status st;
  std::string msg;
};

inline void hipok(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    hipGetLastError();
    throw Fail{MOS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e)};
  }
}

// Carve bump-style from the scratch array.
struct Carver {
  char* base;
  size_t used, cap;
  char* take(size_t bytes) {
    const size_t b = (bytes + 255) & ~size_t(255);
    if (used + b > cap) return nullptr;
    char* r = base + used;
    used += b;
    return r;
  }
};

}  // namespace

extern "C" mos_status mos_solve_noalloc(const mos_graph* g, int32_t start, int32_t goal,
                                        const mos_options* opt, int32_t* costs, int64_t cap,
                                        int64_t* size, mos_stats* stats) {
  if (!g || !size || cap < 0 || (cap > 0 && !costs))
    return mos_internal_set_error(MOS_E_INVALID_ARG, "NULL argument or negative capacity");
  MosOpts o;
  mos_status rs = mos_internal_read_options(opt, &o);
  if (rs != MOS_OK) return rs;
  int d = 0;
  rs = mos_internal_check_query(g, start, goal, o.n_objectives, &d);
  if (rs != MOS_OK) return rs;
  const GraphDev G = mos_internal_graph_view(g);
  const int dev = mos_internal_graph_device(g);
  if (dev < 0 || dev >= kMaxDevices) return mos_internal_set_error(MOS_E_DEVICE, "device id");
  std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
  try {
    hipok(hipSetDevice(dev), "hipSetDevice");
    hipStream_t st = (hipStream_t)o.stream;
    char* base = nullptr;
    hipok(scratch_on(dev, &base), "hipGetSymbolAddress(scratch)");
    Carver c{base, 0, kScratchBytes};
    // fixed parts: slot table of one slot, OPEN histogram, heuristic counters and job
    Slot* dslot = (Slot*)c.take(sizeof(Slot));
    int32_t* hist = (int32_t*)c.take((size_t)NB * 4);
    int32_t* hcnt = (int32_t*)c.take((size_t)MAXD * 3 * 4);
    int32_t* hjob = (int32_t*)c.take(4);
    // the phase area: the heuristic's worklists first, the front readout at the end
    const size_t heur_bytes = (size_t)MAXD * 3 * G.n * 4;
    const size_t left = kScratchBytes - c.used;
    Layout L{};
    size_t phase = heur_bytes;
    bool planned = false;
    for (int it = 0; it < 3 && !planned; ++it) {
      if (phase + 4096 >= left) break;
      if (!plan_slot_layout(G.n, G.maxdeg, d, o.B, (int64_t)(left - phase - 4096), o.label_limit,
                            &L))
        break;
      const size_t readout = (size_t)L.P_cap * (d + 1) * 4 + front_sort_scratch_bytes(L.P_cap) + 1024;
      if (readout <= phase) planned = true;
      else phase = readout;
    }
    if (!planned)
      throw Fail{MOS_E_INVALID_ARG,
                 "graph too large for mos_solve_noalloc: its per-node search state and "
                 "heuristic worklists do not fit the " +
                     std::to_string(kScratchBytes >> 20) + " MiB scratch array"};
    char* area = c.take(phase);
    char* resv = c.take((size_t)L.bytes);
    if (!area || !resv) throw Fail{MOS_E_INVALID_ARG, "scratch array too small for this query"};

    // the slot descriptor, as the engine's admission writes it
    Slot hs;
    std::memset(&hs, 0, sizeof(Slot));
    hs.status = S_IDLE;
    hs.start = start;
    hs.goal = goal;
    hs.d = d;
    hs.B = L.B;
    hs.big_work = (int32_t)BIG_WORK;
    hs.batch_cap = L.batch_cap;
    hs.cand_cap = L.cand_cap;
    hs.tie_cap = L.tie_cap;
    hs.pool_cap = L.pool_cap;
    hs.open_cap = L.open_cap;
    hs.P_cap = L.P_cap;
    hs.fw_cap = L.fw_cap;
    hs.heur_factor = o.heur_factor;
    hs.hn = G.n;
    hs.pop_fifo = o.pop_order == MOS_POP_GENERATION ? 1 : 0;
    hs.eps_ppm = o.eps_ppm;
    hs.eager_goal = o.eager_goal;
    if (!carve_slot(hs, resv, L, G.n, d)) throw Fail{MOS_E_DEVICE, "slot layout overrun"};
    hipok(hipMemcpyAsync(dslot, &hs, sizeof(Slot), hipMemcpyHostToDevice, st), "slot upload");
    // the array keeps the previous call's contents: the histogram must start at zero
    hipok(hipMemsetAsync(hist, 0, (size_t)NB * 4, st), "histogram clear");
    const int32_t job0 = 0;
    hipok(hipMemcpyAsync(hjob, &job0, 4, hipMemcpyHostToDevice, st), "job upload");
    int32_t cnt_host[MAXD * 3];
    const auto t_heur = std::chrono::steady_clock::now();
    const int hr = run_heuristic(dslot, hjob, 1, G, (int32_t*)area, hcnt, cnt_host, st);
    if (hr == -2) throw Fail{MOS_E_DEVICE, "heuristic did not converge"};
    if (hr != 0) hipok(hipErrorUnknown, "heuristic");
    launch_slot_init(dslot, 0, G, st);
    hipok(hipGetLastError(), "slot init");

    StepArgs a;
    a.slots = dslot;
    a.hist = hist;
    a.G = G;
    a.nslots = 1;
    a.gx = 2048;
    {
      const int64_t cand = (int64_t)L.batch_cap * std::max(1, G.maxdeg);
      a.gc = (int)std::max<int64_t>(1, std::min<int64_t>(a.gx, (cand + 255) / 256));
    }
    a.dm = dm_for(d);
    hipok(hipStreamSynchronize(st), "heuristic sync");
    const auto t_search = std::chrono::steady_clock::now();
    const int K = o.steps;
    for (;;) {
      hipok(hipMemcpyAsync(&hs, dslot, sizeof(Slot), hipMemcpyDeviceToHost, st), "status read");
      hipok(hipStreamSynchronize(st), "step sync");
      if (hs.status != S_RUN) break;
      for (int k = 0; k < K; ++k) launch_step(a, st);
      hipok(hipGetLastError(), "step launch");
    }
    const auto t_end = std::chrono::steady_clock::now();
    if (hs.status != S_DONE)
      throw Fail{MOS_E_LABEL_LIMIT, "search state outgrew the " +
                                        std::to_string(kScratchBytes >> 20) + " MiB scratch array"};
    // sorted front, read into the phase area (the worklists are no longer needed)
    int np = 0;
    if (hs.P_n > 0) {
      int32_t* rows = (int32_t*)area;
      char* fsw = area + (((size_t)hs.P_n * d * 4 + 255) & ~size_t(255));
      np = front_sort(hs.Pg[hs.P_sel], hs.P_cap, nullptr, d, hs.P_n, fsw, rows, nullptr, st);
      if (np < 0) hipok(hipErrorUnknown, "front sort");
      if (np > cap)
        throw Fail{MOS_E_INVALID_ARG, "the front has " + std::to_string(np) +
                                          " entries, more than cap = " + std::to_string(cap)};
      if (np > 0)
        hipok(hipMemcpyAsync(costs, rows, (size_t)np * d * 4, hipMemcpyDeviceToHost, st),
              "front read");
      hipok(hipStreamSynchronize(st), "front sync");
    }
    *size = np;
    if (stats) {
      mos_internal_stats_of(hs, stats);
      stats->front = np;
      stats->heuristic_ms = std::chrono::duration<double, std::milli>(t_search - t_heur).count();
      stats->search_ms = std::chrono::duration<double, std::milli>(t_end - t_search).count();
    }
    return MOS_OK;
  } catch (const Fail& f) {
    return mos_internal_set_error(f.st, f.msg);
  }
}
