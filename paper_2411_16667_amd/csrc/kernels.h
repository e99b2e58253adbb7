// Host-side launchers of the device kernels (the only symbols the host engine uses).
#pragma once

#include <algorithm>

#include "mos_core.h"

namespace mos {

struct StepArgs {
  Slot* slots;
  int32_t* hist;
  GraphDev G;
  int nslots;
  int gx;  // workgroups per slot of the tiled kernels
  int gc;  // workgroups per slot of the per-candidate kernels (enough for one candidate per thread)
  int dm;  // compile-time bound on the objectives of every slot (2,3,4,5,6,8)
  // pipelined step: the pop runs on st2 beside the previous step's goal-front
  // filter on the main stream (fork and join through the two events)
  int pipelined = 0;
  hipStream_t st2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

// Smallest supported compile-time objective bound >= d.
int dm_for(int d);

// One batched label step over every resident slot: a fixed set of
// kStepKernels kernels.  Synchronous order: pop, goal step, expansion,
// frontier checks, insertion, goal-front filter of the new labels, step end.
// Pipelined (a.pipelined): the previous step's goal-front filter runs beside
// this step's pop (two streams), then the rest in order; in profile mode the
// same order on one stream.  With ev != nullptr, the kernels i whose bit is set
// in `mask` are bracketed by events ev[2i] (before) and ev[2i + 1] (after);
// ev[2 * kStepKernels] is always recorded after the last kernel.
constexpr int kStepKernels = 22 + NPASS;
extern const char* const kStepKernelNames[kStepKernels];
void launch_step(const StepArgs& a, hipStream_t st, hipEvent_t* ev = nullptr,
                 uint32_t mask = 0xffffffffu);

// Per-query persistent step: one workgroup per slot runs up to max_steps label
// steps of its query (slots in state S_SOLO only; the others are left alone).
// Queries of a graph whose out-degree exceeds kSoloMaxDeg are not run this way.
constexpr int kSoloMaxDeg = 1024;
void launch_solo(Slot* slots, int nslots, const GraphDev& G, int dm, int max_steps,
                 hipStream_t st);

void launch_heur_init(Slot* slots, const int32_t* slot_of, int njobs, const GraphDev& G,
                      int32_t* hs, int32_t* cnt, hipStream_t st);
void launch_heur_round(Slot* slots, const int32_t* slot_of, int njobs, const GraphDev& G,
                       int32_t* hs, int32_t* cnt, int r, int gx, hipStream_t st);
void launch_heur_clamp(Slot* slots, const int32_t* slot_of, int njobs, const GraphDev& G,
                       hipStream_t st);
void launch_slot_init(Slot* slots, int s, const GraphDev& G, hipStream_t st);
// The whole heuristic of the slots slot_of[0 .. njobs): init, relaxation
// rounds until no worklist is left, clamp.  The rounds run in one workgroup
// per (query, objective) instance; one whose worklist outgrows its workgroup
// continues in grid-wide rounds (the host reads the counters into
// cnt_host[njobs * MAXD * 3] after the workgroups and every 8 grid-wide
// rounds).  hs: njobs * MAXD * 3 * n
// ints of device scratch; cnt: njobs * MAXD * 3 device ints.  0 on success,
// -1 on a HIP error, -2 if the rounds did not converge.
int run_heuristic(Slot* slots, const int32_t* slot_of, int njobs, const GraphDev& G, int32_t* hs,
                  int32_t* cnt, int32_t* cnt_host, hipStream_t st);
void launch_open_min(const Slot* slots, int s, int32_t* out, hipStream_t st);
void launch_path_len(const Slot* slots, int s, const int32_t* labs, int np, int32_t* len,
                     hipStream_t st);
void launch_path_write(const Slot* slots, int s, const int32_t* labs, int np, const int64_t* off,
                       int32_t* arcs, hipStream_t st);

}  // namespace mos
