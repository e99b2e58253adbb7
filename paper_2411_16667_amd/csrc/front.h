// Device-side readout of a goal front in lexicographic order.
#pragma once

#include <algorithm>

#include "mos_core.h"

namespace mos {

// Device bytes of scratch front_sort needs for a front array of n entries.
size_t front_sort_scratch_bytes(int n);

// Sort the live entries (plane 0 != INT32_MAX) of the front P (d planes of
// `stride` entries, entries [0, n)) lexicographically ascending, objective 0
// first.  Writes rows[np * d] (row-major) and, when labs != nullptr, the label
// id lab[e] of each row, all device memory; `scratch` is device memory of
// front_sort_scratch_bytes(n) bytes.  Synchronises the stream once (to read the
// live count).  Returns the number of live entries np, or -1 on a HIP error.
int front_sort(const int32_t* P, int64_t stride, const int32_t* lab, int d, int n, void* scratch,
               int32_t* rows, int32_t* labs, hipStream_t st);

}  // namespace mos
