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
};

// One batched label step over every resident slot (13 kernel launches).
void launch_step(const StepArgs& a, hipStream_t st);

void launch_heur_init(Slot* slots, const int32_t* slot_of, int njobs, const GraphDev& G,
                      int32_t* hs, int32_t* cnt, hipStream_t st);
void launch_heur_round(Slot* slots, const int32_t* slot_of, int njobs, const GraphDev& G,
                       int32_t* hs, int32_t* cnt, int r, int gx, hipStream_t st);
void launch_slot_init(Slot* slots, int s, const GraphDev& G, hipStream_t st);
void launch_path_len(const Slot* slots, int s, int np, int32_t* len, hipStream_t st);
void launch_path_write(const Slot* slots, int s, int np, const int64_t* off, int32_t* arcs,
                       hipStream_t st);

}  // namespace mos
