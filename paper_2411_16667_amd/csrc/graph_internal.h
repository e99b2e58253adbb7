// Internal interface between the C ABI's translation units (the engine and
// the allocation-free entry point): options, query checks, the device view
// of a graph, errors and counters.  Not part of the public ABI.
#pragma once

#include <string>

#include "mos.h"
#include "mos_core.h"

constexpr int kDefaultHeurFactor = 4;  // heuristic radius: 4 x h(start), per objective

struct MosOpts {
  int n_objectives = 0, B = 256, max_slots = 0, want_paths = 1, steps = 8;
  int heur_factor = kDefaultHeurFactor;
  uint32_t profile = 0;
  int64_t label_limit = 0, mem_budget = 0;
  int64_t step_budget = 0;
  int32_t pop_order = 0;  // MOS_POP_*
  int32_t eps_ppm = 0;    // approximate mode (0 = exact)
  int32_t eager_goal = 0;
  int32_t pipelined = 0;
  int32_t persistent_query = 0;
  void* stream = nullptr;  // hipStream_t
};

// Validate and read options (NULL = defaults); sets the thread's last error.
mos_status mos_internal_read_options(const mos_options* o, MosOpts* out);
// Start, goal and objective count in range; *d = the query's objective count.
mos_status mos_internal_check_query(const mos_graph* g, int32_t s, int32_t t, int32_t nobj, int* d);
mos::GraphDev mos_internal_graph_view(const mos_graph* g);
int mos_internal_graph_device(const mos_graph* g);
// Record the message behind mos_last_error() and return s.
mos_status mos_internal_set_error(mos_status s, const std::string& msg);
// Counters of a slot descriptor read back from the device (times left 0).
void mos_internal_stats_of(const mos::Slot& s, mos_stats* out);
