// The batched label step on gfx950: one pass of the search over every resident query.
//
// A step follows the paper's Algorithm 1 body (NAMOA*), applied to a batch of
// labels popped in lexicographic order as Algorithm 2 (OPMOS) does:
//   pop      k_open_hist, k_open_threshold, k_open_scatter, k_batch_finalize,
//            k_split_count, k_split_scan: the B lexicographically smallest live
//            OPEN labels (labels pruned since they were queued are skipped
//            lazily, Section 5.1), split into goal and regular labels
//   goal     k_goal_pairs, k_goal_merge: Prune(P, l) and NotDominated(l, P),
//            P <- minimal(P + goal labels)
//   prune    k_popcheck: PruneOPEN applied to the popped labels
//   expand   k_expand: g' = g + c, F' = g' + h over the out-arcs
//   group    k_group_count, k_group_offsets, k_group_scatter: candidates by node
//   check    k_group_process (one wave per group, one streamed pass over the
//            node's frontier) or k_group_pairs + k_group_finish (large groups
//            split into pair tiles): Duplicate, NotDominated and Prune against
//            the node's labels (G_OP and G_CL together) plus dominance among the
//            candidates of the same step
//   insert   k_accept_count, k_accept_scan, k_insert, k_step_end: new labels
//            into OPEN and G_OP
//   filter   k_pfilter: NotDominated(F', P) for the labels inserted this step
//
// All arithmetic is exact int32.  Tiled kernels run on a (workgroups, slots)
// grid and grid-stride over the slot's items; per-slot kernels run one
// 1024-thread workgroup per slot.  Each kernel copies its slot descriptor once (scalar
// registers); writes to descriptor fields go through the pointer.  Objective
// loops are unrolled to the engine's compile-time bound DM (d <= DM).
#include "kernels.h"

namespace mos {

constexpr int NT_SLOT = 1024;  // threads of the one-workgroup-per-slot kernels
constexpr int NT_TILE = 256;   // threads of the tiled kernels
constexpr int GP_WAVES = NT_TILE / WAVE;
constexpr int HOLECAP = 1024;  // holes a large group's in-place compaction lists in LDS
constexpr int PCH = 256;       // goal-front entries per LDS chunk (one per tiled thread)
constexpr int BT_U = 4;        // frontier entries per lane in a pair tile of a large group
constexpr int BT_ENTRIES = BT_U * WAVE;
static_assert(PCH == NT_TILE, "goal tiles map one label to one thread");
static_assert(kStepKernels == 22 + NPASS, "one kernel-name entry per pair pass");
static_assert(ACC_TILE % NT_TILE == 0, "an accept tile is whole chunks of one workgroup");
static_assert(SPLIT_TILE % NT_TILE == 0, "a split tile is whole chunks of one workgroup");

#define FOR_K(k) _Pragma("unroll") for (int k = 0; k < DM; ++k) if (k < d)

// per goal label flags of the goal step (bits of c_rej, set at the pop)
constexpr int GF_REJECTED = 1;     // an entry of P or another goal label is <= it
constexpr int GF_EPS_COVERED = 2;  // approximate mode: an entry of P is <= (1 + eps) it
constexpr int GF_PRUNER = 4;       // it is strictly below an entry of P

// Exclusive scan of one value per thread across a workgroup of NT threads.
// Four exclusive scans at once (one set of barriers for all four).
template <int NT>
__device__ int4 block_exscan4(int4 v, int4* total, int4* tmp /* >= NT/64 int4 */) {
  const int lane = lane_id(), w = threadIdx.x / WAVE;
  int4 x = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int4 y = make_int4(__shfl_up(x.x, o), __shfl_up(x.y, o), __shfl_up(x.z, o),
                             __shfl_up(x.w, o));
    if (lane >= o) x = make_int4(x.x + y.x, x.y + y.y, x.z + y.z, x.w + y.w);
  }
  if (lane == WAVE - 1) tmp[w] = x;
  __syncthreads();
  if (w == 0) {
    constexpr int NW = NT / WAVE;
    int4 t = lane < NW ? tmp[lane] : make_int4(0, 0, 0, 0);
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const int4 y = make_int4(__shfl_up(t.x, o), __shfl_up(t.y, o), __shfl_up(t.z, o),
                               __shfl_up(t.w, o));
      if (lane >= o) t = make_int4(t.x + y.x, t.y + y.y, t.z + y.z, t.w + y.w);
    }
    if (lane < NW) tmp[lane] = t;
  }
  __syncthreads();
  const int4 before = w > 0 ? tmp[w - 1] : make_int4(0, 0, 0, 0);
  *total = tmp[NT / WAVE - 1];
  __syncthreads();
  return make_int4(before.x + x.x - v.x, before.y + x.y - v.y, before.z + x.z - v.z,
                   before.w + x.w - v.w);
}

template <int NT>
__device__ int block_exscan(int v, int* total, int* tmp /* >= NT/64 ints */) {
  const int lane = lane_id(), w = threadIdx.x / WAVE;
  int x = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == WAVE - 1) tmp[w] = x;
  __syncthreads();
  if (w == 0) {
    constexpr int NW = NT / WAVE;
    int t = lane < NW ? tmp[lane] : 0;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      int y = __shfl_up(t, o);
      if (lane >= o) t += y;
    }
    if (lane < NW) tmp[lane] = t;
  }
  __syncthreads();
  int before = w > 0 ? tmp[w - 1] : 0;
  *total = tmp[NT / WAVE - 1];
  __syncthreads();
  return before + x - v;
}

// Wave-aggregated append to an LDS counter: lanes with p get consecutive
// positions (in no particular order across waves); -1 for !p.
__device__ __forceinline__ int lds_append(int* ctr, bool p) {
  const uint64_t m = ballot(p);
  if (m == 0) return -1;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane_id() == leader) base = atomicAdd(ctr, __popcll(m));
  base = __shfl(base, leader);
  return p ? base + rank_below(m) : -1;
}

// Workgroup-aggregated append of NQ flags per thread: one atomic per counter
// and workgroup; pos[q] is the thread's position for counter q (-1 if !p[q]).
// Every thread of the workgroup calls it (it synchronises the workgroup).
template <int NQ>
__device__ __forceinline__ void block_append(int32_t* const (&ctr)[NQ], const bool (&p)[NQ],
                                             int (&pos)[NQ]) {
  constexpr int NW = NT_TILE / WAVE;
  __shared__ int sh[NQ][NW + 1];
  const int w = threadIdx.x / WAVE;
  uint64_t m[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    m[q] = ballot(p[q]);
    if (lane_id() == 0) sh[q][w] = __popcll(m[q]);
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    const int q = threadIdx.x;
    int tot = 0;
#pragma unroll
    for (int x = 0; x < NW; ++x) tot += sh[q][x];
    sh[q][NW] = tot ? atomicAdd(ctr[q], tot) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    int base = sh[q][NW];
#pragma unroll
    for (int x = 0; x < NW; ++x)
      if (x < w) base += sh[q][x];
    pos[q] = p[q] ? base + rank_below(m[q]) : -1;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- OPEN tiers
// OPEN is split by a threshold T on F1: the near tier (F1 < T) is scanned by
// every pop; the far tier (F1 >= T) is only touched when the near tier runs
// low (refill, below) or grows too large (spill, in k_open_scatter).  Every far
// entry has a larger F1 than every near entry, so a pop from the near tier is
// still an exact lexicographic prefix of all of OPEN.
//
// The per-slot decision of a tiled kernel is taken by its last workgroup to
// finish (an atomic count of finished workgroups; all of them take part).
__device__ __forceinline__ bool last_block(int32_t* counter) {
  __shared__ bool is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(counter, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (is_last) __threadfence();
  return is_last;
}

// Refill, part 1: histogram of the live far entries over F1 - T; the last
// workgroup picks the refill threshold r_T so that the near tier grows back
// to about NEAR_TARGET * B entries (or takes the whole far tier).
__global__ __launch_bounds__(NT_TILE) void k_far_hist(Slot* slots, int32_t* hist) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN || !S.refill) return;
  __shared__ int32_t h[NB];
  __shared__ int tmp[NT_TILE / WAVE];
  for (int i = threadIdx.x; i < NB; i += NT_TILE) h[i] = 0;
  __syncthreads();
  const int n = S.far_n, T = S.T;
  const int32_t* F1 = pick(S.far_f1, S.far_sel);
  const int32_t* LB = pick(S.far_lab, S.far_sel);
  for (int i = blockIdx.x * NT_TILE + threadIdx.x; i < n; i += gridDim.x * NT_TILE)
    if (S.Lstate[LB[i]] == L_OPEN) atomicAdd(&h[min(F1[i] - T, NB - 1)], 1);
  __syncthreads();
  int32_t* gh = hist + (size_t)blockIdx.y * NB;
  for (int i = threadIdx.x; i < NB; i += NT_TILE)
    if (h[i]) atomicAdd(&gh[i], h[i]);
  if (!last_block(&Sp->blocks_a)) return;
  constexpr int PER = NB / NT_TILE;
  int loc[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    loc[j] = gh[threadIdx.x * PER + j];
    gh[threadIdx.x * PER + j] = 0;
    sum += loc[j];
  }
  int total;
  int ex = block_exscan<NT_TILE>(sum, &total, tmp);
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    ex += loc[j];
    h[threadIdx.x * PER + j] = ex;  // inclusive
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int target = max(S.B, NEAR_TARGET * S.B - S.open_n);
    int r_all = 0, r_T = T;
    if (total <= target || h[NB - 2] == 0) {
      r_all = 1;
    } else {
      int lo_i = 0, hi_i = NB - 1;
      while (lo_i < hi_i) {
        const int mid = (lo_i + hi_i) >> 1;
        if (h[mid] >= target) hi_i = mid; else lo_i = mid + 1;
      }
      r_T = T + min(lo_i + 1, NB - 1);
    }
    Sp->st[ST_FAR_SCAN] += n;
    Sp->r_all = r_all;
    Sp->r_T = r_T;
    Sp->r_moved = 0;
    Sp->r_keep = 0;
    Sp->lo_refill = INT32_MAX;
    Sp->blocks_a = 0;
  }
}

// Refill, part 2: live far entries below r_T join the near tier, the rest is
// compacted into the other far buffer (dead entries vanish); the last
// workgroup publishes the new tier sizes and threshold.
__global__ __launch_bounds__(NT_TILE) void k_far_move(Slot* slots) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN || !S.refill) return;
  const int n = S.far_n, base = S.open_n, r_T = S.r_T, r_all = S.r_all;
  const int32_t* F1 = pick(S.far_f1, S.far_sel);
  const int32_t* LB = pick(S.far_lab, S.far_sel);
  int32_t* KF = pick(S.far_f1, S.far_sel ^ 1);
  int32_t* KL = pick(S.far_lab, S.far_sel ^ 1);
  int32_t* NF = pick(S.open_f1, S.open_sel);
  int32_t* NLb = pick(S.open_lab, S.open_sel);
  int mn = INT32_MAX;
  for (int b0 = blockIdx.x * NT_TILE; b0 < n; b0 += gridDim.x * NT_TILE) {
    const int i = b0 + threadIdx.x;
    int f = 0, lab = 0;
    bool live = false;
    if (i < n) {
      f = F1[i];
      lab = LB[i];
      live = S.Lstate[lab] == L_OPEN;
    }
    const bool move = live && (r_all || f < r_T);
    const bool keep = live && !move;
    int32_t* const ctr[2] = {&Sp->r_moved, &Sp->r_keep};
    const bool fl[2] = {move, keep};
    int pos[2];
    block_append<2>(ctr, fl, pos);
    int p = pos[0];
    if (move && base + p < S.open_cap) {
      NF[base + p] = f;
      NLb[base + p] = lab;
      mn = min(mn, f);
    }
    p = pos[1];
    if (keep && p < S.open_cap) {
      KF[p] = f;
      KL[p] = lab;
    }
  }
  mn = wave_min(mn);
  if (lane_id() == 0 && mn != INT32_MAX) atomicMin(&Sp->lo_refill, mn);
  if (!last_block(&Sp->blocks_b)) return;
  if (threadIdx.x == 0) {
    const int moved = Sp->r_moved, kept = Sp->r_keep;
    Sp->open_n = base + moved;
    Sp->far_n = kept;
    Sp->far_sel = S.far_sel ^ 1;
    if (r_all) {
      Sp->t_all = 1;
      Sp->T = INT32_MAX;
    } else {
      Sp->T = r_T;
    }
    if (moved > 0) Sp->lo = base > 0 ? min(S.lo, Sp->lo_refill) : Sp->lo_refill;
    if (base + moved > S.open_cap || kept > S.open_cap) {
      Sp->status = S_OVERFLOW;
      Sp->err_line = __LINE__;
    }
    Sp->refill = 0;
    Sp->blocks_b = 0;
  }
}

// ---------------------------------------------------------------- pop
// Histogram of live near entries over F1 (bin = F1 - lo, width 1, last bin = overflow).
__global__ __launch_bounds__(NT_TILE) void k_open_hist(Slot* slots, int32_t* hist) {
  const Slot S = slots[blockIdx.y];
  if (S.status != S_RUN) return;
  const int n = S.open_n;
  if ((int)(blockIdx.x * NT_TILE) >= n) return;
  __shared__ int32_t h[NB];
  for (int i = threadIdx.x; i < NB; i += NT_TILE) h[i] = 0;
  __syncthreads();
  const int32_t* F1 = pick(S.open_f1, S.open_sel);
  const int32_t* LB = pick(S.open_lab, S.open_sel);
  const int lo = S.lo;
  constexpr int HU = 4;  // entries per thread in flight
  const int stride = gridDim.x * NT_TILE;
  for (int i0 = blockIdx.x * NT_TILE + threadIdx.x; i0 < n; i0 += HU * stride) {
    int lab[HU], f[HU];
#pragma unroll
    for (int u = 0; u < HU; ++u) {
      const int i = i0 + u * stride;
      lab[u] = i < n ? LB[i] : -1;
      f[u] = i < n ? F1[i] : 0;
    }
    bool live[HU];
#pragma unroll
    for (int u = 0; u < HU; ++u) live[u] = lab[u] >= 0 && S.Lstate[lab[u]] == L_OPEN;
#pragma unroll
    for (int u = 0; u < HU; ++u)
      if (live[u]) atomicAdd(&h[min(max(f[u] - lo, 0), NB - 1)], 1);
  }
  __syncthreads();
  int32_t* gh = hist + (size_t)blockIdx.y * NB;
  for (int i = threadIdx.x; i < NB; i += NT_TILE)
    if (h[i]) atomicAdd(&gh[i], h[i]);
}

// Pick the threshold bin: bins below t_star are popped whole; r_tie entries of
// bin t_star are then selected exactly by k_batch_finalize (tie_mode).
__global__ __launch_bounds__(NT_SLOT) void k_open_threshold(Slot* slots, int32_t* hist) {
  Slot* Sp = &slots[blockIdx.x];
  if (Sp->status != S_RUN) return;
  const int B = Sp->B;
  __shared__ int32_t cum[NB];
  __shared__ int tmp[NT_SLOT / WAVE];
  int32_t* gh = hist + (size_t)blockIdx.x * NB;
  constexpr int PER = NB / NT_SLOT;
  int loc[PER], s = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    loc[j] = gh[threadIdx.x * PER + j];
    s += loc[j];
  }
  int total;
  int ex = block_exscan<NT_SLOT>(s, &total, tmp);
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    ex += loc[j];
    cum[threadIdx.x * PER + j] = ex;  // inclusive
    gh[threadIdx.x * PER + j] = 0;    // reset for the next step
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int t_star = NB, r = 0, mode = 0;
    if (total > B) {
      int lo_i = 0, hi_i = NB - 1;  // first bin with cum >= B
      while (lo_i < hi_i) {
        const int mid = (lo_i + hi_i) >> 1;
        if (cum[mid] >= B) hi_i = mid; else lo_i = mid + 1;
      }
      const int t = lo_i;
      const int below = t > 0 ? cum[t - 1] : 0;
      const int inbin = cum[t] - below;
      r = B - below;
      if (r == inbin) {
        t_star = t + 1;  // the threshold bin is popped whole
        r = 0;
      } else {
        t_star = t;  // r of its entries are selected exactly in k_batch_finalize
        mode = 1;
      }
    }
    // spill: a near tier above NEAR_HIGH * B live entries keeps its lowest
    // NEAR_TARGET * B (whole F1 values); the rest moves to the far tier
    if (total > NEAR_HIGH * B) {
      const int keep = NEAR_TARGET * B;
      int lo_i = 0, hi_i = NB - 1;
      while (lo_i < hi_i) {
        const int mid = (lo_i + hi_i) >> 1;
        if (cum[mid] >= keep) hi_i = mid; else lo_i = mid + 1;
      }
      if (lo_i < NB - 2) {
        Sp->T = Sp->lo + lo_i + 1;
        Sp->t_all = 0;
      }
    }
    Sp->st[ST_NEAR_SCAN] += Sp->open_n;
    Sp->t_star = t_star;
    Sp->r_tie = r;
    Sp->tie_mode = mode;
    Sp->batch_n = 0;
    Sp->tie_n = 0;
    Sp->keep_n = 0;
    Sp->lo_next = INT32_MAX;
  }
}

// Route every live OPEN entry: popped (bin < t_star), tie (bin == t_star in
// tie mode) or kept (into the other OPEN buffer).  Dead entries vanish here.
__global__ __launch_bounds__(NT_TILE) void k_open_scatter(Slot* slots) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  const int n = S.open_n;
  const int sel = S.open_sel, lo = S.lo, t_star = S.t_star, mode = S.tie_mode;
  const int32_t* F1 = pick(S.open_f1, sel);
  const int32_t* LB = pick(S.open_lab, sel);
  int32_t* KF = pick(S.open_f1, sel ^ 1);
  int32_t* KL = pick(S.open_lab, sel ^ 1);
  int32_t* FF = pick(S.far_f1, S.far_sel);
  int32_t* FL = pick(S.far_lab, S.far_sel);
  const int stride = gridDim.x * NT_TILE;
  int kmin = INT32_MAX;
  for (int base = blockIdx.x * NT_TILE; base < n; base += stride) {
    const int i = base + threadIdx.x;
    const bool valid = i < n;
    int lab = 0, f = 0;
    bool live = false;
    if (valid) {
      lab = LB[i];
      f = F1[i];
      live = S.Lstate[lab] == L_OPEN;
    }
    const int b = min(max(f - lo, 0), NB - 1);
    const bool to_batch = live && b < t_star;
    const bool to_tie = live && mode && b == t_star;
    const bool to_keep = live && !to_batch && !to_tie;
    const bool to_far = to_keep && !S.t_all && f >= S.T;  // spilled this step
    const bool to_near = to_keep && !to_far;
    int32_t* const ctr[4] = {&Sp->batch_n, &Sp->tie_n, &Sp->keep_n, &Sp->far_n};
    const bool fl[4] = {to_batch, to_tie, to_near, to_far};
    int pos[4];
    block_append<4>(ctr, fl, pos);
    int p = pos[0];
    if (to_batch && p < S.batch_cap) S.batch[p] = lab;
    p = pos[1];
    if (to_tie && p < S.tie_cap) {
      S.tie_f1[p] = f;
      S.tie_lab[p] = lab;
      S.tie_st[p] = 0;
      const int v = S.Lnode[lab];
      for (int k = 1; k < S.d; ++k)
        S.tie_key[(size_t)(k - 1) * S.tie_cap + p] = S.Lg[(size_t)k * S.pool_cap + lab] +
                                                     S.h[(size_t)k * S.hn + v];
      // last key word: the node (unique with F in lexicographic order); the
      // label id in generation order, where the key does not hold F1
      S.tie_key[(size_t)(S.d - 1) * S.tie_cap + p] = S.pop_fifo ? lab : v;
    }
    p = pos[2];
    if (to_near && p < S.open_cap) {
      KF[p] = f;
      KL[p] = lab;
      kmin = min(kmin, f);
    }
    p = pos[3];
    if (to_far && p < S.open_cap) {
      FF[p] = f;
      FL[p] = lab;
    }
  }
  kmin = wave_min(kmin);
  if (lane_id() == 0 && kmin != INT32_MAX) atomicMin(&Sp->lo_next, kmin);
}

// Word w of the full key of tie entry i: F_{w+1} for w < d, the node for w = d
// (words 1..d were gathered into tie_key when the entry joined the tie set).
__device__ __forceinline__ int key_word(const Slot& S, int i, int w) {
  return w == 0 ? S.tie_f1[i] : S.tie_key[(size_t)(w - 1) * S.tie_cap + i];
}


// Exact selection inside the tie bin (one workgroup per slot); the batch is
// assembled and split by k_split_count and k_split_scan.
template <int DM>
__global__ __launch_bounds__(NT_SLOT) void k_batch_finalize(Slot* slots, GraphDev G) {
  Slot* Sp = &slots[blockIdx.x];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  __shared__ int32_t lds[10240];
  __shared__ int tmp[NT_SLOT / WAVE];
  __shared__ int sh_a, sh_b, sh_c;
  const int d = S.d;
  int nb = S.batch_n, keep_n = S.keep_n;
  const uint64_t c0 = wall_clock64();
  if (S.tie_mode) {
    // ---- threshold bin: take exactly the r_tie lexicographically smallest of
    // its entries by (F_1..F_d, node).  While more than TIECAP remain
    // undecided, one radix level on the current key word decides every entry
    // outside the bin that holds the r-th smallest; the last <= TIECAP entries
    // are ordered in LDS.  (F, node) is unique among live labels, so this ends.
    const int n = min(S.tie_n, S.tie_cap);
    int need = S.r_tie;
    int32_t* TS = S.tie_st;  // 0 undecided (set by the scatter), 1 taken, 2 not taken
    // an inner bin holds a single F1 value: refinement starts at F2
    int und = n, word = (S.t_star > 0 && S.t_star < NB - 1) ? 1 : 0, levels = 0;
    int32_t* hist = lds;        // NB ints
    int32_t* kc = lds + NB;     // the current key word of each entry, when they fit
    constexpr int KC = 10240 - NB;
    const bool cache = n <= KC;
    while (und > TIECAP && need > 0 && need < und) {
      // one level: histogram of the undecided entries' current key word over
      // NB - 1 bins of width 2^shift spanning [min, max]; entries outside the
      // bin holding the need-th smallest are decided
      ++levels;
      if (threadIdx.x == 0) {
        sh_a = INT32_MAX;
        sh_c = INT32_MIN;
      }
      __syncthreads();
      // passes over the tie set: TU entries per thread with their loads issued
      // together (state and key word are independent loads)
      constexpr int TU = 4;
      int mn = INT32_MAX, mx = INT32_MIN;
      for (int base = threadIdx.x; base < n; base += TU * NT_SLOT) {
        int ts[TU], x[TU];
#pragma unroll
        for (int u = 0; u < TU; ++u) {
          const int i = base + u * NT_SLOT;
          ts[u] = i < n ? TS[i] : 3;
          x[u] = i < n ? key_word(S, i, word) : 0;
        }
#pragma unroll
        for (int u = 0; u < TU; ++u)
          if (ts[u] == 0) {
            if (cache) kc[base + u * NT_SLOT] = x[u];
            mn = min(mn, x[u]);
            mx = max(mx, x[u]);
          }
      }
      mn = wave_min(mn);
      mx = -wave_min(-mx);
      if (lane_id() == 0) {
        atomicMin(&sh_a, mn);
        atomicMax(&sh_c, mx);
      }
      for (int i = threadIdx.x; i < NB; i += NT_SLOT) hist[i] = 0;
      __syncthreads();
      const int m = sh_a;
      int shift = 0;
      while ((((int64_t)sh_c - m) >> shift) >= NB - 1) ++shift;
      for (int base = threadIdx.x; base < n; base += TU * NT_SLOT) {
        int ts[TU], x[TU];
#pragma unroll
        for (int u = 0; u < TU; ++u) {
          const int i = base + u * NT_SLOT;
          ts[u] = i < n ? TS[i] : 3;
          x[u] = i < n ? (cache ? kc[i] : key_word(S, i, word)) : 0;
        }
#pragma unroll
        for (int u = 0; u < TU; ++u)
          if (ts[u] == 0) atomicAdd(&hist[(int)(((int64_t)x[u] - m) >> shift)], 1);
      }
      __syncthreads();
      constexpr int PER = NB / NT_SLOT;
      int loc[PER], sum = 0;
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        loc[j] = hist[threadIdx.x * PER + j];
        sum += loc[j];
      }
      int tot;
      int ex = block_exscan<NT_SLOT>(sum, &tot, tmp);
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        ex += loc[j];
        hist[threadIdx.x * PER + j] = ex;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int lo_i = 0, hi_i = NB - 1;
        while (lo_i < hi_i) {
          const int mid = (lo_i + hi_i) >> 1;
          if (hist[mid] >= need) hi_i = mid; else lo_i = mid + 1;
        }
        sh_b = lo_i;
      }
      __syncthreads();
      const int bstar = sh_b;
      const int below = bstar > 0 ? hist[bstar - 1] : 0;
      const int inb = hist[bstar] - below;
      for (int base = threadIdx.x; base < n; base += TU * NT_SLOT) {
        int ts[TU], x[TU];
#pragma unroll
        for (int u = 0; u < TU; ++u) {
          const int i = base + u * NT_SLOT;
          ts[u] = i < n ? TS[i] : 3;
          x[u] = i < n ? (cache ? kc[i] : key_word(S, i, word)) : 0;
        }
#pragma unroll
        for (int u = 0; u < TU; ++u)
          if (ts[u] == 0) {
            const int b = (int)(((int64_t)x[u] - m) >> shift);
            if (b < bstar) TS[base + u * NT_SLOT] = 1;
            else if (b > bstar) TS[base + u * NT_SLOT] = 2;
          }
      }
      need -= below;
      und = inb;
      if (shift == 0) ++word;  // the undecided now share this word's value
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      Sp->st[ST_TIE] += n;
      Sp->st[ST_T0 + 4] += levels;
      Sp->st[ST_T0 + 5] += 1;
    }
    if (need == 0 || need >= und) {
      const int fill = need == 0 ? 2 : 1;
      for (int i = threadIdx.x; i < n; i += NT_SLOT)
        if (TS[i] == 0) TS[i] = fill;
      __syncthreads();
    } else {
      // the undecided (<= TIECAP): the rank of each one by full key decides it;
      // keys are packed as int4 words (padding words are equal for everyone)
      constexpr int KW = (DM + 1 + 3) / 4;
      int4* K4 = reinterpret_cast<int4*>(lds);          // TIECAP x KW words
      int32_t* idx = lds + 4 * KW * TIECAP;              // positions into the tie arrays
      if (threadIdx.x == 0) sh_a = 0;
      __syncthreads();
      for (int base = 0; base < n; base += NT_SLOT) {
        const int i = base + threadIdx.x;
        const int p = lds_append(&sh_a, i < n && TS[i] == 0);
        if (p >= 0 && p < TIECAP) idx[p] = i;
      }
      __syncthreads();
      const int cnt = min(sh_a, TIECAP);
      if (threadIdx.x < cnt) {
        const int i = threadIdx.x;
        int32_t key[KW * 4];
#pragma unroll
        for (int k = 0; k < KW * 4; ++k) key[k] = k <= d ? key_word(S, idx[i], k) : 0;
#pragma unroll
        for (int w = 0; w < KW; ++w)
          K4[i * KW + w] = make_int4(key[4 * w], key[4 * w + 1], key[4 * w + 2], key[4 * w + 3]);
      }
      __syncthreads();
      if (threadIdx.x < cnt) {
        const int i = threadIdx.x;
        int4 mine[KW];
#pragma unroll
        for (int w = 0; w < KW; ++w) mine[w] = K4[i * KW + w];
        int rank = 0;  // keys are distinct: (F, node) is unique among live labels
        for (int j = 0; j < cnt; ++j) {
          int less = 0, decided = 0;
#pragma unroll
          for (int w = 0; w < KW; ++w) {
            const int4 o = K4[j * KW + w];
            less |= !decided & (o.x < mine[w].x);
            decided |= o.x != mine[w].x;
            less |= !decided & (o.y < mine[w].y);
            decided |= o.y != mine[w].y;
            less |= !decided & (o.z < mine[w].z);
            decided |= o.z != mine[w].z;
            less |= !decided & (o.w < mine[w].w);
            decided |= o.w != mine[w].w;
          }
          rank += less;
        }
        TS[idx[i]] = rank < need ? 1 : 2;
      }
      __syncthreads();
    }
  }
  // taken tie entries join the batch and the others go back to OPEN in the
  // batch split (k_split_count, k_split_scan), which also splits the batch
  if (nb > S.batch_cap || nb > BATCH_MAX) {
    if (threadIdx.x == 0) {
      Sp->status = S_OVERFLOW;
      Sp->err_line = __LINE__;
    }
    return;
  }
  if (threadIdx.x == 0) {
    Sp->st[ST_T0 + 0] += wall_clock64() - c0;
    Sp->pop_nb = nb;
    Sp->pop_keep = S.keep_n;
    Sp->ngroups = 0;
    Sp->accept_n = 0;
  }
}

// Second half of the pop, over SPLIT_TILE-item tiles of the directly popped
// labels (batch[0, pop_nb)) followed by the tie entries: a taken tie entry
// joins the batch, a tie entry not taken goes back to the near tier of OPEN,
// and every batch label is split into goal labels (goal_lab, their goal-step
// flags cleared) and regular labels (reg, with the exclusive prefix of their
// out-degrees in reg_off).  k_split_count stores each tile's counts;
// k_split_scan starts each tile after the tiles before it and writes its items
// in order.  Item i of a tile is loaded by thread i % NT_TILE (U per thread).
enum { SPLIT_NONE = 0, SPLIT_GOAL = 1, SPLIT_REG = 2, SPLIT_BACK = 3 };

template <int U>
__device__ __forceinline__ void split_items(const Slot& S, const GraphDev& G, int t, int nb0,
                                            int items, int (&lab)[U], int (&kind)[U],
                                            int (&deg)[U], int (&f1)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = t * SPLIT_TILE + u * NT_TILE + threadIdx.x;
    lab[u] = -1;
    kind[u] = SPLIT_NONE;
    deg[u] = 0;
    f1[u] = 0;
    if (i < nb0) {
      lab[u] = S.batch[i];
      kind[u] = SPLIT_REG;  // goal or regular: decided by the node below
    } else if (i < items) {
      const int j = i - nb0, st = S.tie_st[j];
      if (st == 1) {
        lab[u] = S.tie_lab[j];
        kind[u] = SPLIT_REG;
      } else if (st == 2) {
        lab[u] = S.tie_lab[j];
        f1[u] = S.tie_f1[j];
        kind[u] = SPLIT_BACK;
      }
    }
  }
  int v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) v[u] = kind[u] == SPLIT_REG ? S.Lnode[lab[u]] : 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (kind[u] != SPLIT_REG) continue;
    if (v[u] == S.goal) kind[u] = SPLIT_GOAL;
    else deg[u] = (int)(G.row_ptr[v[u] + 1] - G.row_ptr[v[u]]);
  }
}

__device__ __forceinline__ int split_items_total(const Slot& S) {
  return S.pop_nb + (S.tie_mode ? min(S.tie_n, S.tie_cap) : 0);
}

__global__ __launch_bounds__(NT_TILE) void k_split_count(Slot* slots, GraphDev G) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  constexpr int U = SPLIT_TILE / NT_TILE;
  __shared__ int red[SPLIT_WORDS][GP_WAVES];
  const int wave = threadIdx.x / WAVE, lane = lane_id();
  const int nb0 = S.pop_nb, items = split_items_total(S);
  const int nt = (items + SPLIT_TILE - 1) / SPLIT_TILE;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    int lab[U], kind[U], deg[U], f1[U];
    split_items<U>(S, G, t, nb0, items, lab, kind, deg, f1);
    int c[SPLIT_WORDS] = {0, 0, 0, 0, INT32_MAX};
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[0] += kind[u] == SPLIT_GOAL;
      c[1] += kind[u] == SPLIT_REG;
      c[2] += deg[u];
      c[3] += kind[u] == SPLIT_BACK;
      if (kind[u] == SPLIT_BACK) c[4] = min(c[4], f1[u]);
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) c[w] = wave_sum(c[w]);
    c[4] = wave_min(c[4]);
    if (lane == 0)
#pragma unroll
      for (int w = 0; w < SPLIT_WORDS; ++w) red[w][wave] = c[w];
    __syncthreads();
    if (threadIdx.x < SPLIT_WORDS) {
      const int w = threadIdx.x;
      int a = w == 4 ? INT32_MAX : 0;
#pragma unroll
      for (int x = 0; x < GP_WAVES; ++x) a = w == 4 ? min(a, red[w][x]) : a + red[w][x];
      S.split_tile[(size_t)SPLIT_WORDS * t + w] = a;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(NT_TILE) void k_split_scan(Slot* slots, GraphDev G) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  constexpr int U = SPLIT_TILE / NT_TILE;
  __shared__ int red[SPLIT_WORDS][GP_WAVES];
  __shared__ int cw[4][U][GP_WAVES];  // per (kind, chunk, wave): goal, regular, degree sum, back
  __shared__ int sh_goal0;             // first goal-list position of the eager goal labels
  const int wave = threadIdx.x / WAVE, lane = lane_id();
  const int nb0 = S.pop_nb, keep0 = S.pop_keep, items = split_items_total(S);
  const int nt = (items + SPLIT_TILE - 1) / SPLIT_TILE;
  const int32_t* TT = S.split_tile;
  if (blockIdx.x == 0) {  // totals (no other workgroup reads the fields written here)
    int c[SPLIT_WORDS] = {0, 0, 0, 0, INT32_MAX};
    for (int x = threadIdx.x; x < nt; x += NT_TILE) {
#pragma unroll
      for (int w = 0; w < 4; ++w) c[w] += TT[(size_t)SPLIT_WORDS * x + w];
      c[4] = min(c[4], TT[(size_t)SPLIT_WORDS * x + 4]);
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) c[w] = wave_sum(c[w]);
    c[4] = wave_min(c[4]);
    if (lane == 0)
#pragma unroll
      for (int w = 0; w < SPLIT_WORDS; ++w) red[w][wave] = c[w];
    __syncthreads();
    if (threadIdx.x == 0) {
      int a[SPLIT_WORDS] = {0, 0, 0, 0, INT32_MAX};
#pragma unroll
      for (int x = 0; x < GP_WAVES; ++x) {
#pragma unroll
        for (int w = 0; w < 4; ++w) a[w] += red[w][x];
        a[4] = min(a[4], red[4][x]);
      }
      const int nb = a[0] + a[1], keep_n = keep0 + a[3];
      // eager mode: the goal labels accepted last step join the popped ones
      // (copied below; those the goal-front filter removed since enter as
      // rejected, counted as labels dropped at their pop)
      const int eager_n = S.pgoal_n;
      const int ng = a[0] + eager_n;
      sh_goal0 = a[0];
      Sp->pgoal_n = 0;
      Sp->goal_n = ng;
      Sp->reg_n = a[1];
      Sp->cand_n = a[2];
      Sp->batch_n = nb;
      Sp->keep_n = keep_n;
      if (a[1] <= S.batch_cap) S.reg_off[a[1]] = a[2];
      if (a[4] != INT32_MAX) atomicMin(&Sp->lo_next, a[4]);
      Sp->st[ST_POPS] += nb + eager_n;
      Sp->st[ST_GOAL_POPS] += ng;
      if (nb > S.batch_cap || a[2] > S.cand_cap || ng > S.cand_cap || keep_n > S.open_cap) {
        Sp->status = S_OVERFLOW;
        Sp->err_line = __LINE__;
        sh_goal0 = -1;
      } else if (nb == 0 && S.far_n == 0 && ng == 0) {
        Sp->status = S_DONE;  // no live label left in OPEN, no goal label waiting
      }
    }
    __syncthreads();
    const int g0 = sh_goal0;
    if (g0 >= 0)
      for (int j = threadIdx.x; j < S.pgoal_n; j += NT_TILE) {
        const int lab = S.pgoal[j];
        S.goal_lab[g0 + j] = lab;
        S.c_rej[g0 + j] = S.Lstate[lab] == L_DEAD ? GF_REJECTED : 0;
      }
  }
  int32_t* KF = pick(S.open_f1, S.open_sel ^ 1);
  int32_t* KL = pick(S.open_lab, S.open_sel ^ 1);
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    int lab[U], kind[U], deg[U], f1[U];
    split_items<U>(S, G, t, nb0, items, lab, kind, deg, f1);
    int b[4] = {0, 0, 0, 0};  // the tiles before this one
    for (int x = threadIdx.x; x < t; x += NT_TILE)
#pragma unroll
      for (int w = 0; w < 4; ++w) b[w] += TT[(size_t)SPLIT_WORDS * x + w];
#pragma unroll
    for (int w = 0; w < 4; ++w) b[w] = wave_sum(b[w]);
    uint64_t mg[U], mr[U], mk[U];
    int incl[U];  // inclusive prefix of the out-degrees over the wave, per chunk
#pragma unroll
    for (int u = 0; u < U; ++u) {
      mg[u] = ballot(kind[u] == SPLIT_GOAL);
      mr[u] = ballot(kind[u] == SPLIT_REG);
      mk[u] = ballot(kind[u] == SPLIT_BACK);
      int x = deg[u];
#pragma unroll
      for (int o = 1; o < WAVE; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
      }
      incl[u] = x;
    }
    if (lane == WAVE - 1) {
#pragma unroll
      for (int w = 0; w < 4; ++w) red[w][wave] = b[w];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        cw[0][u][wave] = __popcll(mg[u]);
        cw[1][u][wave] = __popcll(mr[u]);
        cw[2][u][wave] = incl[u];
        cw[3][u][wave] = __popcll(mk[u]);
      }
    }
    __syncthreads();
    int o[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      o[w] = 0;
#pragma unroll
      for (int x = 0; x < GP_WAVES; ++x) o[w] += red[w][x];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int p[4];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        p[w] = o[w];
#pragma unroll
        for (int x = 0; x < GP_WAVES; ++x) {
          if (x < wave) p[w] += cw[w][u][x];
          o[w] += cw[w][u][x];
        }
      }
      if (kind[u] == SPLIT_GOAL) {
        const int pg = p[0] + rank_below(mg[u]);
        if (pg < S.batch_cap) S.goal_lab[pg] = lab[u];
        if (pg < S.cand_cap) S.c_rej[pg] = 0;  // goal-step flag of this goal label
      } else if (kind[u] == SPLIT_REG) {
        const int pr = p[1] + rank_below(mr[u]);
        if (pr < S.batch_cap) {
          S.reg[pr] = lab[u];
          S.reg_off[pr] = p[2] + incl[u] - deg[u];
          S.reg_kill[pr] = 0;
        }
      } else if (kind[u] == SPLIT_BACK) {
        const int pk = keep0 + p[3] + rank_below(mk[u]);
        if (pk < S.open_cap) {
          KF[pk] = f1[u];
          KL[pk] = lab[u];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- goal-front tests
// A vector F is dropped when some goal-front entry p has p <= F in every
// objective.  Front chunks are staged in LDS as int4 words: components k >= d
// hold 0 (in the tested vectors too) and rows past the chunk hold INT32_MAX in
// every component k < d, so every test runs over whole words with no bounds
// or objective-count checks.  p <= F in every component exactly when the OR
// of the differences F_k - p_k has a clear sign bit: costs lie in
// [0, INT32_MAX), so no difference overflows.  A chunk dominates F when the
// AND over its rows of those ORs has a clear sign bit (one subtract per
// component, one OR and one AND per row; components at or beyond the
// compile-time bound DM are skipped).
template <int DM>
struct FrontChunk {
  static constexpr int NW = (DM + 3) / 4;
  int4 w[PCH][NW];
};

__device__ __forceinline__ int comp(const int4& v, int c) {
  return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}

// OR over components k < DM of (q_k - r_k): sign bit clear <=> r <= q everywhere.
template <int DM>
__device__ __forceinline__ int or_diff(const int4 (&r)[FrontChunk<DM>::NW],
                                       const int4 (&q)[FrontChunk<DM>::NW]) {
  int o = 0;
#pragma unroll
  for (int k = 0; k < DM; ++k) o |= comp(q[k >> 2], k & 3) - comp(r[k >> 2], k & 3);
  return o;
}

template <int DM>
__device__ __forceinline__ void stage_chunk(FrontChunk<DM>& ch, const int32_t* Pg, int Pc, int p0,
                                            int npt, int d) {
  constexpr int NW = FrontChunk<DM>::NW;
  for (int r = threadIdx.x; r < PCH; r += blockDim.x) {
    int32_t v[NW * 4];
#pragma unroll
    for (int k = 0; k < NW * 4; ++k)
      v[k] = k < d ? (r < npt ? Pg[(size_t)k * Pc + p0 + r] : INT32_MAX) : 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) ch.w[r][w] = make_int4(v[4 * w], v[4 * w + 1], v[4 * w + 2], v[4 * w + 3]);
  }
}

template <int DM>
__device__ __forceinline__ bool chunk_dominates(const FrontChunk<DM>& ch, const int4 (&F)[FrontChunk<DM>::NW]) {
  int acc = -1;
#pragma unroll 8
  for (int q = 0; q < PCH; ++q) acc &= or_diff<DM>(ch.w[q], F);
  return acc >= 0;
}

// ---------------------------------------------------------------- goal step
// P <- minimal(P ∪ G) for the goal labels G popped this step (Prune(P, l) and
// NotDominated(l, P) of Algorithm 1, for the whole batch of goal labels):
//  * a goal label is rejected if an entry of P is <= it (dominated or equal),
//    or another goal label of the step is <= it (equal vectors: the smaller
//    label id stays);
//  * an entry of P is removed if a goal label is strictly below it.
// Removal writes INT32_MAX into every plane of the entry (a tombstone: no cost
// reaches INT32_MAX, so it dominates nothing and is never matched); the front
// is compacted once half of its entries are tombstones.  P is kept unordered;
// the result is sorted when it is read out.
//
// k_goal_pairs: work items are (goal tile, chunk) pairs, the chunk being a
// chunk of P or a tile of the step's goal labels, both staged in LDS.  A
// tombstone written while another item reads the entry changes no outcome:
// the goal label that removed it is itself <= every goal label the entry was
// <= (and no entry of P is <= it, P being an antichain).
template <int DM>
__device__ __forceinline__ void pack_query(const int32_t (&x)[FrontChunk<DM>::NW * 4],
                                           int4 (&Q)[FrontChunk<DM>::NW]) {
#pragma unroll
  for (int w = 0; w < FrontChunk<DM>::NW; ++w)
    Q[w] = make_int4(x[4 * w], x[4 * w + 1], x[4 * w + 2], x[4 * w + 3]);
}

template <int DM>
__device__ __forceinline__ void le_ne(const int4 (&r)[FrontChunk<DM>::NW], const int4 (&Q)[FrontChunk<DM>::NW],
                                      int& le, int& ne) {
  int x = 0;
#pragma unroll
  for (int k = 0; k < DM; ++k) x |= comp(Q[k >> 2], k & 3) ^ comp(r[k >> 2], k & 3);
  le = or_diff<DM>(r, Q) >= 0;
  ne = x != 0;
}

template <int DM>
__global__ __launch_bounds__(NT_TILE) void k_goal_pairs(Slot* slots) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  const int ng = S.goal_n, np = S.P_n;
  if (ng == 0) return;
  constexpr int NW = FrontChunk<DM>::NW;
  const int ngt = (ng + PCH - 1) / PCH, npc = (np + PCH - 1) / PCH;
  const int per = npc + ngt;  // per goal tile: the chunks of P, then the goal tiles
  const int items = ngt * per;
  if ((int)blockIdx.x >= items) return;
  __shared__ FrontChunk<DM> other;   // chunk of P or tile of goal labels
  __shared__ FrontChunk<DM> mine;    // this item's goal tile
  __shared__ int32_t olab[PCH];
  const int d = S.d, pc = S.pool_cap, Pc = S.P_cap;
  int32_t* Pg = pick(S.Pg, S.P_sel);
  int32_t* gflag = S.c_rej;  // per goal label: rejected (zeroed at the pop)
  const int t = threadIdx.x;
  int64_t pairs = 0;
  int dead = 0;
  for (int it = blockIdx.x; it < items; it += gridDim.x) {
    const int gt = it / per, oc = it - gt * per;
    const int t0 = gt * PCH, nt = min(PCH, ng - t0);
    int32_t x[NW * 4];
    int mylab = -1;
    if (t < nt) {
      mylab = S.goal_lab[t0 + t];
#pragma unroll
      for (int k = 0; k < NW * 4; ++k) x[k] = k < d ? S.Lg[(size_t)k * pc + mylab] : 0;
    } else {
#pragma unroll
      for (int k = 0; k < NW * 4; ++k) x[k] = k < d ? INT32_MAX : 0;
    }
    int4 G[NW];
    pack_query<DM>(x, G);
    __syncthreads();  // the previous item is done with the LDS tiles
    bool rej = false, rej_eps = false;
    if (oc < npc) {
      const int p0 = oc * PCH, npt = min(PCH, np - p0);
#pragma unroll
      for (int w = 0; w < NW; ++w) mine.w[t][w] = G[w];
      stage_chunk<DM>(other, Pg, Pc, p0, npt, d);
      __syncthreads();
      if (t < nt) {
        // NotDominated(l, P); in approximate mode also by (1 + eps)-dominance
        rej = chunk_dominates<DM>(other, G);
        if (S.eps_ppm && !rej) {
          int32_t xe[NW * 4];
#pragma unroll
          for (int k = 0; k < NW * 4; ++k) xe[k] = eps_relax(x[k], S.eps_ppm);
          int4 Ge[NW];
          pack_query<DM>(xe, Ge);
          rej_eps = chunk_dominates<DM>(other, Ge);
        }
      }
      if (t < npt && other.w[t][0].x != INT32_MAX) {
        int4 Q[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) Q[w] = other.w[t][w];
        int hit = 0;
#pragma unroll 4
        for (int r = 0; r < PCH; ++r) {
          int4 R[NW];
#pragma unroll
          for (int w = 0; w < NW; ++w) R[w] = mine.w[r][w];
          int le, ne;
          le_ne<DM>(R, Q, le, ne);
          hit |= le & ne;
          // approximate mode: a goal label that removes an entry is kept even
          // if the front covers it within 1 + eps (it replaces what it removes)
          if (S.eps_ppm && (le & ne)) atomicOr(&gflag[t0 + r], GF_PRUNER);
        }
        if (hit && atomicExch(&Pg[p0 + t], INT32_MAX) != INT32_MAX) {
          for (int k = 1; k < d; ++k) Pg[(size_t)k * Pc + p0 + t] = INT32_MAX;
          ++dead;
        }
      }
      pairs += (int64_t)nt * npt;
    } else {
      const int u0 = (oc - npc) * PCH, nu = min(PCH, ng - u0);
      if (t < nu) {
        const int lb = S.goal_lab[u0 + t];
        olab[t] = lb;
        int32_t y[NW * 4];
#pragma unroll
        for (int k = 0; k < NW * 4; ++k) y[k] = k < d ? S.Lg[(size_t)k * pc + lb] : 0;
#pragma unroll
        for (int w = 0; w < NW; ++w)
          other.w[t][w] = make_int4(y[4 * w], y[4 * w + 1], y[4 * w + 2], y[4 * w + 3]);
      }
      __syncthreads();
      if (t < nt) {
        for (int r = 0; r < nu; ++r) {
          int4 R[NW];
#pragma unroll
          for (int w = 0; w < NW; ++w) R[w] = other.w[r][w];
          int le, ne;
          le_ne<DM>(R, G, le, ne);
          const int lb = olab[r];
          rej = rej | (le && lb != mylab && (ne || lb < mylab));
        }
      }
      pairs += (int64_t)nt * nu;
    }
    if (rej) atomicOr(&gflag[t0 + t], GF_REJECTED);
    if (rej_eps) atomicOr(&gflag[t0 + t], GF_EPS_COVERED);
  }
  // pairs are block-uniform; tombstones are counted per thread
  const int64_t dsum = wave_sum64(dead);
  if (lane_id() == 0 && dsum) atomicAdd(&Sp->P_dead, (int)dsum);
  if (t == 0 && pairs) atomicAdd((unsigned long long*)&Sp->st[ST_PPAIRS], (unsigned long long)pairs);
}

// Append the accepted goal labels to P (in batch order) and compact P once
// a quarter of its entries are tombstones (stable, into the other buffer).
template <int DM>
__global__ __launch_bounds__(NT_SLOT) void k_goal_merge(Slot* slots) {
  Slot* Sp = &slots[blockIdx.x];
  const Slot S = *Sp;
  if (S.status != S_RUN || S.goal_n == 0) return;
  __shared__ int tmp[NT_SLOT / WAVE];
  const int d = S.d, pc = S.pool_cap, Pc = S.P_cap;
  const int ng = S.goal_n, np = S.P_n;
  int32_t* Pg = pick(S.Pg, S.P_sel);
  int32_t* Pl = pick(S.Plab, S.P_sel);
  int32_t* Ps = pick(S.Pseq, S.P_sel);
  if (np + ng > Pc) {
    if (threadIdx.x == 0) {
      Sp->status = S_OVERFLOW;
      Sp->err_line = __LINE__;
    }
    return;
  }
  int na = 0;
  for (int base = 0; base < ng; base += NT_SLOT) {
    const int i = base + threadIdx.x;
    const int f = i < ng ? S.c_rej[i] : GF_REJECTED;
    const int a = !(f & GF_REJECTED) && (!(f & GF_EPS_COVERED) || (f & GF_PRUNER)) ? 1 : 0;
    int tot;
    const int pos = block_exscan<NT_SLOT>(a, &tot, tmp);
    if (a) {
      const int lab = S.goal_lab[i];
      FOR_K(k) Pg[(size_t)k * Pc + np + na + pos] = S.Lg[(size_t)k * pc + lab];
      Pl[np + na + pos] = lab;
      Ps[np + na + pos] = S.P_seq + na + pos;
    }
    na += tot;
  }
  const int n1 = np + na, dead = S.P_dead;
  int live = n1, sel = S.P_sel;
  if (dead > 0 && 4 * dead >= n1) {
    __syncthreads();  // appended entries visible to the whole workgroup
    int32_t* Qg = pick(S.Pg, S.P_sel ^ 1);
    int32_t* Ql = pick(S.Plab, S.P_sel ^ 1);
    int32_t* Qs = pick(S.Pseq, S.P_sel ^ 1);
    int carry = 0;
    for (int base = 0; base < n1; base += NT_SLOT) {
      const int i = base + threadIdx.x;
      const int a = (i < n1 && Pg[i] != INT32_MAX) ? 1 : 0;
      int tot;
      const int pos = block_exscan<NT_SLOT>(a, &tot, tmp);
      if (a) {
        FOR_K(k) Qg[(size_t)k * Pc + carry + pos] = Pg[(size_t)k * Pc + i];
        Ql[carry + pos] = Pl[i];
        Qs[carry + pos] = Ps[i];
      }
      carry += tot;
    }
    live = carry;
    sel ^= 1;
  }
  if (threadIdx.x == 0) {
    Sp->P_n = live;
    Sp->P_sel = sel;
    Sp->P_seq = S.P_seq + na;
    if (live != n1) Sp->P_dead = 0;
    Sp->st[ST_PREAD] += (int64_t)np * ((ng + PCH - 1) / PCH);
    // goal labels the front already covers were not processed (lazy PruneOPEN)
    Sp->st[ST_POPS] -= ng - na;
    Sp->st[ST_KILLED] += ng - na;
  }
}

// A tile of labels, L per thread (F packed as int4 words), against the front
// chunks c0 .. c1-1, each staged in LDS in turn (each row read from LDS serves
// all of a thread's tests); stops early once every label of the tile is
// dominated, and sets dom[] for this thread's labels.  Work items are
// (label tile, run of chunks) pairs with runs sized so that the items about
// fill the grid: a label's F is formed once per run.
template <int DM, int L>
__device__ void tile_vs_frontL(FrontChunk<DM>& ch, const int32_t* Pg, int Pc, int np, int d,
                               int c0, int c1, const bool (&have)[L],
                               const int4 (&F)[L][FrontChunk<DM>::NW], bool (&dom)[L],
                               int64_t& examined) {
  for (int c = c0; c < c1; ++c) {
    const int p0 = c * PCH;
    __syncthreads();
    stage_chunk<DM>(ch, Pg, Pc, p0, min(PCH, np - p0), d);
    __syncthreads();
    int nopen = 0;
#pragma unroll
    for (int h = 0; h < L; ++h) nopen += (have[h] && !dom[h]) ? 1 : 0;
    // pairs examined: every still-undecided label of this thread against the
    // chunk's entries (removed entries included: they are compared too)
    examined += (int64_t)nopen * min(PCH, np - p0);
    if (nopen) {
      int a[L];
#pragma unroll
      for (int h = 0; h < L; ++h) a[h] = -1;
#pragma unroll 8
      for (int q = 0; q < PCH; ++q)
#pragma unroll
        for (int h = 0; h < L; ++h) a[h] &= or_diff<DM>(ch.w[q], F[h]);
#pragma unroll
      for (int h = 0; h < L; ++h) dom[h] = dom[h] || a[h] >= 0;
    }
    bool done = true;
#pragma unroll
    for (int h = 0; h < L; ++h) done = done && (!have[h] || dom[h]);
    if (__syncthreads_and(done)) break;
  }
}

template <int DM>
__device__ void tile_vs_front2(FrontChunk<DM>& ch, const int32_t* Pg, int Pc, int np, int d,
                               int c0, int c1, bool have0, bool have1,
                               const int4 (&F0)[FrontChunk<DM>::NW],
                               const int4 (&F1)[FrontChunk<DM>::NW], bool& dom0, bool& dom1,
                               int64_t& examined) {
  const bool have[2] = {have0, have1};
  int4 F[2][FrontChunk<DM>::NW];
#pragma unroll
  for (int w = 0; w < FrontChunk<DM>::NW; ++w) {
    F[0][w] = F0[w];
    F[1][w] = F1[w];
  }
  bool dom[2] = {dom0, dom1};
  tile_vs_frontL<DM, 2>(ch, Pg, Pc, np, d, c0, c1, have, F, dom, examined);
  dom0 = dom[0];
  dom1 = dom[1];
}

__device__ __forceinline__ int chunks_per_item(int nlt, int npc) {
  return max(1, (nlt * npc + (int)gridDim.x - 1) / (int)gridDim.x);
}

// The paper's PruneOPEN drops every open label whose F the goal front
// dominates (Algorithm 1); here it is applied lazily to the
// popped regular labels (weak dominance), after this step's goal labels were
// merged into the front.  A dropped label is not expanded.  A label was tested
// against the whole front when it was inserted (k_pfilter), so only the
// entries appended since then (a suffix of P, found by the append numbers)
// can dominate it now.  Work items are (label tile, run of front chunks).
template <int DM>
__global__ __launch_bounds__(NT_TILE) void k_popcheck(Slot* slots, GraphDev G) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  const int R = S.reg_n, np = S.P_n;
  if (R == 0 || np == 0) return;
  constexpr int LT = 2 * NT_TILE;  // labels per tile: two per thread
  const int nlt = (R + LT - 1) / LT, npc = (np + PCH - 1) / PCH;
  const int cpi = chunks_per_item(nlt, npc), ngrp = (npc + cpi - 1) / cpi;
  const int ntiles = nlt * ngrp;
  if ((int)blockIdx.x >= ntiles) return;
  constexpr int NW = FrontChunk<DM>::NW;
  __shared__ FrontChunk<DM> ch;
  __shared__ int sh_seq, sh_first;
  const int d = S.d, pc = S.pool_cap, Pc = S.P_cap, n = G.n;
  const int32_t* Pg = pick(S.Pg, S.P_sel);
  const int32_t* Ps = pick(S.Pseq, S.P_sel);
  int killed = 0;
  int64_t examined = 0;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int lt = t / ngrp, gi = t - lt * ngrp;
    int ii[2], lab[2] = {0, 0};
    bool have[2], dom[2] = {false, false}, gone[2] = {false, false};
    int4 F[2][NW];
    __syncthreads();  // the previous item is done with sh_first
    if (threadIdx.x == 0) sh_seq = INT32_MAX;
    __syncthreads();
    int seq = INT32_MAX;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      ii[h] = lt * LT + h * NT_TILE + threadIdx.x;
      have[h] = ii[h] < R && !S.reg_kill[ii[h]];
      int32_t f[NW * 4];
#pragma unroll
      for (int k = 0; k < NW * 4; ++k) f[k] = 0;
      if (have[h]) {
        lab[h] = S.reg[ii[h]];
        // pipelined steps: the previous step's goal-front filter, which ran
        // beside this step's pop, may have removed the label after the pop
        // took it; every other popped label has been tested by that filter
        // up to its Lpseq mark (the filter finished before this kernel)
        gone[h] = S.pipelined && S.Lstate[lab[h]] == L_DEAD;
        have[h] = !gone[h];
      }
      if (have[h]) {
        seq = min(seq, S.Lpseq[lab[h]]);
        const int v = S.Lnode[lab[h]];
#pragma unroll
        for (int k = 0; k < NW * 4; ++k)
          f[k] = k < d ? eps_relax(S.Lg[(size_t)k * pc + lab[h]] + S.h[(size_t)k * n + v],
                                   S.eps_ppm)
                       : 0;
      }
#pragma unroll
      for (int w = 0; w < NW; ++w) F[h][w] = make_int4(f[4 * w], f[4 * w + 1], f[4 * w + 2], f[4 * w + 3]);
    }
    seq = wave_min(seq);
    if (lane_id() == 0) atomicMin(&sh_seq, seq);
    __syncthreads();
    if (threadIdx.x == 0) {  // first entry appended at or after the tile's earliest mark
      int lo_i = 0, hi_i = np;
      while (lo_i < hi_i) {
        const int mid = (lo_i + hi_i) >> 1;
        if (Ps[mid] < sh_seq) lo_i = mid + 1; else hi_i = mid;
      }
      sh_first = lo_i;
    }
    __syncthreads();
    const int c0 = max(gi * cpi, sh_first / PCH), c1 = min(npc, (gi + 1) * cpi);
    if (c0 < c1)
      tile_vs_front2<DM>(ch, Pg, Pc, np, d, c0, c1, have[0], have[1], F[0], F[1], dom[0], dom[1],
                         examined);
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (((have[h] && dom[h]) || gone[h]) && atomicExch(&S.reg_kill[ii[h]], 1) == 0) {
        S.Lstate[lab[h]] = L_DEAD;
        ++killed;
      }
  }
  const int64_t k64 = wave_sum64(killed);
  if (lane_id() == 0 && k64) {
    atomicAdd((unsigned long long*)&Sp->st[ST_KILLED], (unsigned long long)k64);
    atomicAdd((unsigned long long*)&Sp->st[ST_POPS], (unsigned long long)(-k64));
  }
  const int64_t e64 = wave_sum64(examined);
  if (lane_id() == 0 && e64) atomicAdd((unsigned long long*)&Sp->st[ST_PPAIRS], (unsigned long long)e64);
}

// ---------------------------------------------------------------- expand
// One thread per candidate (flat index over the regular labels' out-arcs):
// g' = g + c(e), F' = g' + h(v') (Algorithm 1, expansion).  A target that
// cannot reach the goal is dropped at once.
template <int DM>
__global__ __launch_bounds__(NT_TILE) void k_expand(Slot* slots, GraphDev G) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  const int M = S.cand_n;
  const int d = S.d, pc = S.pool_cap, cc = S.cand_cap, n = G.n;
  const int reg_n = S.reg_n;
  int64_t ncand = 0;
  for (int f = blockIdx.x * NT_TILE + threadIdx.x; f < M; f += gridDim.x * NT_TILE) {
    int lo_i = 0, hi_i = reg_n - 1;  // regular label owning flat index f
    while (lo_i < hi_i) {
      const int mid = (lo_i + hi_i + 1) >> 1;
      if (S.reg_off[mid] <= f) lo_i = mid; else hi_i = mid - 1;
    }
    S.c_rej[f] = 0;
    S.c_acc[f] = 0;
    if (S.reg_kill[lo_i]) {  // dropped at pop: nothing to expand
      S.c_keep[f] = 0;
      continue;
    }
    const int lab = S.reg[lo_i];
    const int u = S.Lnode[lab];
    const int e = G.row_ptr[u] + (f - S.reg_off[lo_i]);
    const int v = G.col[e];
    bool alive = true;
    FOR_K(k) {
      if (S.h[(size_t)k * n + v] == UNREACH) alive = false;
      S.c_g[(size_t)k * cc + f] = S.Lg[(size_t)k * pc + lab] + G.cost[(size_t)k * G.m + e];
    }
    S.c_node[f] = v;
    S.c_par[f] = lab;
    S.c_arc[f] = e;
    S.c_keep[f] = alive ? 1 : 0;
    ncand++;
  }
  ncand = wave_sum64(ncand);
  if (lane_id() == 0 && ncand)
    atomicAdd((unsigned long long*)&Sp->st[ST_CANDS], (unsigned long long)ncand);
}

// ---------------------------------------------------------------- goal-front filter
// NotDominated(F', P) of Algorithm 1 for the labels inserted this step (pool
// ids n_labels .. n_labels + accept_n - 1): a label whose F is weakly
// dominated by a goal-front entry is marked dead, so OPEN drops it at its
// next scan and it is never expanded, and its frontier entry is marked
// removed.  The test runs after the frontier test instead of before it: it
// then covers only the candidates that survived (a small fraction), and what
// such a candidate did in this step's frontier test is harmless: every label
// it rejected or pruned has a g no better than its own, so the goal front
// dominates that label's F as well.  Weak dominance: a completion of F = p
// cannot improve on p.  Work items are (label tile, front chunk) pairs so that
// a large front spreads over the whole chip; a label tile holds four labels
// per thread, so each front row read from LDS serves four tests.
template <int DM>
__global__ __launch_bounds__(NT_TILE) void k_pfilter(Slot* slots, GraphDev G) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  // the labels of this step's insertion, or of the previous step's when the
  // filter runs beside the next pop (the pop resets accept_n meanwhile)
  const int R = S.pipelined ? S.pf_n : S.accept_n, np = S.P_n;
  const int base = S.pipelined ? S.pf_base : S.n_labels;
  if (R == 0 || np == 0) return;
  constexpr int LPT = 4;           // labels per thread
  constexpr int LT = LPT * NT_TILE;  // labels per tile
  const int nlt = (R + LT - 1) / LT, npc = (np + PCH - 1) / PCH;
  const int cpi = chunks_per_item(nlt, npc), ngrp = (npc + cpi - 1) / cpi;
  const int ntiles = nlt * ngrp;
  if ((int)blockIdx.x >= ntiles) return;
  constexpr int NW = FrontChunk<DM>::NW;
  __shared__ FrontChunk<DM> ch;
  const int d = S.d, pc = S.pool_cap, Pc = S.P_cap, n = G.n;
  const int32_t* Pg = pick(S.Pg, S.P_sel);
  int64_t examined = 0;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int lt = t / ngrp, gi = t - lt * ngrp;
    int ii[LPT];
    bool have[LPT], dom[LPT];
    int4 F[LPT][NW];
#pragma unroll
    for (int h = 0; h < LPT; ++h) {
      dom[h] = false;
      ii[h] = lt * LT + h * NT_TILE + threadIdx.x;
      const int id = base + ii[h];
      have[h] = ii[h] < R && S.Lstate[id] != L_DEAD;
      int32_t x[NW * 4];
#pragma unroll
      for (int k = 0; k < NW * 4; ++k) x[k] = 0;
      if (have[h]) {
        const int v = S.Lnode[id];
#pragma unroll
        for (int k = 0; k < NW * 4; ++k)
          x[k] = k < d ? eps_relax(S.Lg[(size_t)k * pc + id] + S.h[(size_t)k * n + v], S.eps_ppm)
                       : 0;
      }
#pragma unroll
      for (int w = 0; w < NW; ++w) F[h][w] = make_int4(x[4 * w], x[4 * w + 1], x[4 * w + 2], x[4 * w + 3]);
    }
    tile_vs_frontL<DM, LPT>(ch, Pg, Pc, np, d, gi * cpi, min(npc, (gi + 1) * cpi), have, F, dom,
                            examined);
#pragma unroll
    for (int h = 0; h < LPT; ++h)
      if (have[h] && dom[h]) {
        S.Lstate[base + ii[h]] = L_DEAD;
        S.fw[S.c_fslot[S.order[ii[h]]]] = FW_REMOVED;  // leaves its node's frontier
      }
  }
  const int64_t e64 = wave_sum64(examined);
  if (lane_id() == 0 && e64) atomicAdd((unsigned long long*)&Sp->st[ST_PPAIRS], (unsigned long long)e64);
}

// ---------------------------------------------------------------- group by target node
__global__ __launch_bounds__(NT_TILE) void k_group_count(Slot* slots) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  const int M = S.cand_n;
  for (int f = blockIdx.x * NT_TILE + threadIdx.x; f < M; f += gridDim.x * NT_TILE) {
    int v = 0, r = -1;
    if (S.c_keep[f]) {
      v = S.c_node[f];
      r = atomicAdd(&S.grp_cnt[v], 1);
      S.c_rank[f] = r;
    }
    // a node's first candidate opens its group: one group-count atomic per wave
    const uint64_t m = ballot(r == 0);
    if (m) {
      const int leader = __ffsll((long long)m) - 1;
      int gb = 0;
      if (lane_id() == leader) gb = atomicAdd(&Sp->ngroups, __popcll(m));
      gb = __shfl(gb, leader);
      if (r == 0) {
        const int gid = gb + rank_below(m);
        S.grp_node[gid] = v;
        S.grp_id[v] = gid;
      }
    }
  }
}

// Group offsets, and the split of groups into small (one wave, one pass) and
// big (pair tiles across waves): a group is big when it has more than one
// candidate tile or its candidate x (frontier + candidates) work is large.
__global__ __launch_bounds__(NT_SLOT) void k_group_offsets(Slot* slots) {
  Slot* Sp = &slots[blockIdx.x];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  __shared__ int4 tmp4[NT_SLOT / WAVE];
  const int ng = S.ngroups, cc = S.cand_cap;
  int carry = 0, ns = 0, nb = 0, nt[NPASS] = {};
  for (int base = 0; base < ng; base += NT_SLOT) {
    const int i = base + threadIdx.x;
    int sz = 0, cnt = 0;
    if (i < ng) {
      const int v = S.grp_node[i];
      sz = S.grp_cnt[v];
      cnt = S.node[v].count;
    }
    const bool big = i < ng && (sz > WAVE || (int64_t)sz * (cnt + sz) > S.big_work);
    const bool small = i < ng && !big;
    const int nct = (sz + WAVE - 1) / WAVE, nft = (cnt + BT_ENTRIES - 1) / BT_ENTRIES;
    // pair tiles per pass: pass 0 takes the candidate tiles against each
    // other and the first frontier tiles; later passes the following ones
    int tp[NPASS];
#pragma unroll
    for (int p = 0; p < NPASS; ++p)
      tp[p] = big ? (min(nft, pass_lo(p + 1)) - min(nft, pass_lo(p))) * nct + (p ? 0 : nct * nct) : 0;
    int4 tot4;
    const int4 pre = block_exscan4<NT_SLOT>(make_int4(sz, small ? 1 : 0, big ? 1 : 0, tp[0]),
                                            &tot4, tmp4);
    const int ex = pre.x, ps = pre.y, pb = pre.z;
    const int tot = tot4.x, ts = tot4.y, tb = tot4.z;
    static_assert(NPASS <= 4, "one scan for the later passes");
    int4 totp;
    const int4 prep = block_exscan4<NT_SLOT>(
        make_int4(NPASS > 1 ? tp[NPASS > 1 ? 1 : 0] : 0, NPASS > 2 ? tp[NPASS > 2 ? 2 : 0] : 0,
                  NPASS > 3 ? tp[NPASS > 3 ? 3 : 0] : 0, 0),
        &totp, tmp4);
    const int pt[4] = {pre.w, prep.x, prep.y, prep.z};
    const int ttot[4] = {tot4.w, totp.x, totp.y, totp.z};
    if (i < ng) S.grp_off[i] = carry + ex;
    if (small) S.small_list[ns + ps] = i;
    if (big) {
      S.big_list[nb + pb] = i;
#pragma unroll
      for (int p = 0; p < NPASS; ++p) S.big_toff[(size_t)p * (cc + 1) + nb + pb] = nt[p] + pt[p];
    }
    carry += tot;
    ns += ts;
    nb += tb;
#pragma unroll
    for (int p = 0; p < NPASS; ++p) nt[p] += ttot[p];
  }
  if (threadIdx.x == 0) {
    int all = 0;
#pragma unroll
    for (int p = 0; p < NPASS; ++p) {
      S.big_toff[(size_t)p * (cc + 1) + nb] = nt[p];
      Sp->big_tiles_pass[p] = nt[p];
      all += nt[p];
    }
    Sp->st[ST_T0 + 6] += nb;
    Sp->st[ST_T0 + 7] += all;
    Sp->nsmall = ns;
    Sp->nbig = nb;
    Sp->big_tiles = all;
    Sp->st[ST_GROUPS] += ng;
  }
}

__global__ __launch_bounds__(NT_TILE) void k_group_scatter(Slot* slots) {
  const Slot S = slots[blockIdx.y];
  if (S.status != S_RUN) return;
  const int M = S.cand_n;
  for (int f = blockIdx.x * NT_TILE + threadIdx.x; f < M; f += gridDim.x * NT_TILE) {
    if (!S.c_keep[f]) continue;
    const int gid = S.grp_id[S.c_node[f]];
    S.order[S.grp_off[gid] + S.c_rank[f]] = f;
  }
}

// OPEN key of a label generated in this step: its F1 in lexicographic order;
// in generation order the step number (labels of earlier steps first; the
// start label has key 0).  Either way keys never fall below the smallest key
// left in OPEN, which the bucket structure of the tiers relies on.
__device__ __forceinline__ int open_key(const Slot& S, int f1) {
  return S.pop_fifo ? (int)S.st[ST_STEPS] + 1 : f1;
}

// OPEN tier an accepted candidate joins, by its key: 1 near (key < T), 2 far.
__device__ __forceinline__ int open_tier(const Slot& S, int f1) {
  const int key = open_key(S, f1);
  return (S.t_all || key < S.T) ? 1 : 2;
}

// Take a new frontier block when `need` entries do not fit the node's block.
// Returns false (and marks the slot) when the slot's frontier region is exhausted.
__device__ __forceinline__ bool frontier_dest(Slot* Sp, const Slot& S, const NodeRec& nr, int need,
                                              int d, int64_t* doff, int* dcap) {
  *doff = nr.off;
  *dcap = nr.cap;
  if (need <= nr.cap) return true;
  int nc = MINCAP;
  while (nc < need) nc <<= 1;
  const int64_t words = (int64_t)nc * (d + 1);
  int64_t pos = 0;
  if (lane_id() == 0)
    pos = (int64_t)atomicAdd((unsigned long long*)&Sp->fw_top, (unsigned long long)words);
  pos = __shfl(pos, 0);
  if (pos + words > S.fw_cap) {
    if (lane_id() == 0) {
      Sp->status = S_OVERFLOW;
      Sp->err_line = __LINE__;
    }
    return false;
  }
  *doff = pos;
  *dcap = nc;
  return true;
}

// ---------------------------------------------------------------- frontier check (small groups)
// One wave per group (all candidates of this step with the same target node v,
// candidate i held by lane i, k <= 64):
//  A. candidates against each other: c_i is dropped if some c_j <= c_i in every
//     objective and (c_j != c_i or c_j's arc id is smaller; two distinct
//     candidates with equal vectors always differ in their arc, because the
//     labels popped at one node have distinct vectors);
//  B. survivors against the live frontier of v, U entries per lane per pass
//     (the next pass is loaded before the current one is compared); each
//     surviving candidate is broadcast from its lane: it is rejected if an entry
//     weakly dominates it (dominated or duplicate: Duplicate and NotDominated); an
//     entry is pruned if a candidate strictly dominates it (Prune; a
//     rejected candidate can dominate no live entry because the frontier is an
//     antichain, so no test on rejection is needed); pruned entries are marked
//     dead in the pool and the block is compacted as it is streamed;
//  C. accepted candidates are appended (a larger block is taken when needed).
// Rejections live in a wave-uniform 64-bit mask; all compares are branch-free.
constexpr int U = 4;  // frontier entries per lane per pass


// For candidate c and frontier entry e (components k >= d are 0 on both
// sides; costs lie in [0, INT32_MAX), so no difference overflows):
//   dmin = min_k (c_k - e_k), dmax = max_k (c_k - e_k);
//   e <= c in every component            <=>  dmin >= 0  (e rejects c)
//   c <= e everywhere and c != e         <=>  dmax <= 0 and dmin < 0
//                                        <=>  sign bit of ((dmax - 1) & dmin)  (c prunes e)
// Plain integer arithmetic (min3/max3, no per-component compares or masks).
// An absent entry is given INT32_MAX in every component k < d: then dmin < 0,
// so it rejects nothing, and its prune flag is masked out by its owner.
template <int DM>
__device__ __forceinline__ void diff_range(const int32_t (&c)[DM], const int32_t (&e)[DM], int& dmin,
                                           int& dmax) {
  dmin = c[0] - e[0];
  dmax = dmin;
#pragma unroll
  for (int k = 1; k < DM; ++k) {
    const int t = c[k] - e[k];
    dmin = min(dmin, t);
    dmax = max(dmax, t);
  }
}

template <int DM>
__device__ __forceinline__ void load_entries(const int32_t* fw, const NodeRec& nr, int d, int base,
                                             int32_t (&sv)[U][DM], int32_t (&lab)[U]) {
  const int lane = lane_id();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = base + u * WAVE + lane;
    const bool has = e < nr.count;
#pragma unroll
    for (int k = 0; k < DM; ++k) sv[u][k] = (has && k < d) ? fw[nr.off + (int64_t)k * nr.cap + e] : 0;
    lab[u] = has ? fw[nr.off + (int64_t)d * nr.cap + e] : 0;
  }
}

template <int DM>
__global__ __launch_bounds__(NT_TILE) void k_group_process(Slot* slots) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  const int nsmall = S.nsmall;
  const int wave = threadIdx.x / WAVE, lane = lane_id();
  const int d = S.d, cc = S.cand_cap;
  int32_t* fw = S.fw;
  int64_t gpairs = 0, fpairs = 0, fbytes = 0, pruned = 0;
  __shared__ int4 cstage[GP_WAVES][WAVE][FrontChunk<DM>::NW];  // per wave: its group's candidates
  __shared__ int astage[GP_WAVES][WAVE];                          // and their arcs
  for (int si = blockIdx.x * GP_WAVES + wave; si < nsmall; si += gridDim.x * GP_WAVES) {
    const int gid = S.small_list[si];
    const int v = S.grp_node[gid];
    const int k = S.grp_cnt[v];  // <= WAVE for small groups
    const int32_t* ord = S.order + S.grp_off[gid];
    const bool have = lane < k;
    const int fi = have ? ord[lane] : 0;
    const int ai = have ? S.c_arc[fi] : 0;
    int32_t ci[DM];
#pragma unroll
    for (int kk = 0; kk < DM; ++kk) ci[kk] = (have && kk < d) ? S.c_g[(size_t)kk * cc + fi] : 0;
    const NodeRec nr = S.node[v];
    const int cnt = nr.count;
    // first frontier pass in flight while the candidates are resolved
    int32_t sv[U][DM], slab[U];
    load_entries<DM>(fw, nr, d, 0, sv, slab);
    // the group's candidates go through LDS: one broadcast read per candidate
    // on the LDS pipe instead of DM lane reads on the vector ALU
    constexpr int NW = FrontChunk<DM>::NW;
    {
      int32_t x[NW * 4];
#pragma unroll
      for (int q = 0; q < NW * 4; ++q) x[q] = q < DM ? ci[q] : 0;
#pragma unroll
      for (int w = 0; w < NW; ++w)
        cstage[wave][lane][w] = make_int4(x[4 * w], x[4 * w + 1], x[4 * w + 2], x[4 * w + 3]);
      astage[wave][lane] = ai;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // read across lanes below
    // ---- A. intra-group resolution
    bool rej = false;
    if (k > 1) {
      gpairs += (int64_t)k * (k - 1);
      for (int jj = 0; jj < k; ++jj) {
        int4 cw[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) cw[w] = cstage[wave][jj][w];
        bool le = true, eq = true;
#pragma unroll
        for (int kk = 0; kk < DM; ++kk) {
          const int b = comp(cw[kk >> 2], kk & 3);
          le = le & (b <= ci[kk]);
          eq = eq & (b == ci[kk]);
        }
        const int aj = astage[wave][jj];
        rej = rej | (jj != lane && le && (!eq || aj < ai));
      }
    }
    const uint64_t surv = ballot(have && !rej);
    const int ks = __popcll(surv);
    // ---- B. frontier check + prune + compaction
    int64_t doff;
    int dcap;
    if (!frontier_dest(Sp, S, nr, cnt + ks, d, &doff, &dcap)) break;
    const bool moved = doff != nr.off;
    uint64_t rejm = 0;  // surviving candidates rejected by the frontier
    int cursor = 0, nlive = 0;
    for (int t = 0; t < cnt; t += U * WAVE) {
      int32_t cv[U][DM], clab[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int kk = 0; kk < DM; ++kk) cv[u][kk] = sv[u][kk];
        clab[u] = slab[u];
      }
      if (t + U * WAVE < cnt) load_entries<DM>(fw, nr, d, t + U * WAVE, sv, slab);
      bool present[U], prune[U];
      int32_t ev[U][DM];  // compare values: absent entries get INT32_MAX (k < d)
      int pacc[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        present[u] = t + u * WAVE + lane < cnt && clab[u] != FW_REMOVED;
#pragma unroll
        for (int kk = 0; kk < DM; ++kk) ev[u][kk] = present[u] ? cv[u][kk] : (kk < d ? INT32_MAX : 0);
        pacc[u] = 0;
      }
      for (uint64_t m = surv & ~rejm; m; m &= m - 1) {
        const int jj = __ffsll((long long)m) - 1;
        int4 cw[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) cw[w] = cstage[wave][jj][w];
        int32_t c[DM];
#pragma unroll
        for (int kk = 0; kk < DM; ++kk) c[kk] = comp(cw[kk >> 2], kk & 3);
        int allneg = -1;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          int dmin, dmax;
          diff_range<DM>(c, ev[u], dmin, dmax);
          allneg &= dmin;
          pacc[u] |= (dmax - 1) & dmin;
        }
        if (ballot(allneg >= 0)) rejm |= 1ull << jj;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) prune[u] = present[u] && pacc[u] < 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int tb = t + u * WAVE;
        if (tb >= cnt) break;
        const bool has = tb + lane < cnt;
        if (prune[u]) S.Lstate[clab[u]] = L_DEAD;
        const uint64_t hm = ballot(has);
        const uint64_t am = ballot(has && clab[u] != FW_REMOVED && !prune[u]);
        pruned += __popcll(ballot(prune[u]));
        nlive += __popcll(ballot(has && clab[u] != FW_REMOVED));
        if (moved || cursor != tb || am != hm) {
          if (has && clab[u] != FW_REMOVED && !prune[u]) {
            const int64_t w = doff + cursor + rank_below(am);
#pragma unroll
            for (int kk = 0; kk < DM; ++kk)
              if (kk < d) fw[w + (int64_t)kk * dcap] = cv[u][kk];
            fw[w + (int64_t)d * dcap] = clab[u];
          }
        }
        cursor += __popcll(am);
      }
    }
    fpairs += (int64_t)ks * nlive;
    fbytes += (int64_t)nlive * 4 * d;
    // ---- C. append the accepted candidates
    const uint64_t accm = surv & ~rejm;
    const bool acc = (accm >> lane) & 1ull;
    if (acc) {
      const int64_t w = doff + cursor + rank_below(accm);
#pragma unroll
      for (int kk = 0; kk < DM; ++kk)
        if (kk < d) fw[w + (int64_t)kk * dcap] = ci[kk];
      fw[w + (int64_t)d * dcap] = -1;
      S.c_fslot[fi] = w + (int64_t)d * dcap;
      S.c_acc[fi] = open_tier(S, ci[0] + S.h[v]);
    }
    cursor += __popcll(accm);
    if (lane == 0) {
      NodeRec out;
      out.off = doff;
      out.cap = dcap;
      out.count = cursor;
      S.node[v] = out;
      S.grp_cnt[v] = 0;
      S.grp_id[v] = -1;
    }
  }
  // the per-group totals are wave-uniform: lane 0 publishes them
  if (lane == 0) {
    if (gpairs) atomicAdd((unsigned long long*)&Sp->st[ST_GPAIRS], (unsigned long long)gpairs);
    if (fpairs) atomicAdd((unsigned long long*)&Sp->st[ST_FPAIRS], (unsigned long long)fpairs);
    if (gpairs + fpairs)
      atomicAdd((unsigned long long*)&Sp->st[ST_PAIRS_WAVE], (unsigned long long)(gpairs + fpairs));
    if (fbytes) {
      atomicAdd((unsigned long long*)&Sp->st[ST_FBYTES], (unsigned long long)fbytes);
      atomicAdd((unsigned long long*)&Sp->st[ST_FBYTES_WAVE], (unsigned long long)fbytes);
    }
    if (pruned) atomicAdd((unsigned long long*)&Sp->st[ST_PRUNED], (unsigned long long)pruned);
  }
}

// ---------------------------------------------------------------- big groups
// Pair tiles of the big groups, one wave per tile, both operands in lanes:
//   A-tiles (candidate tile I x candidate tile J, 64 x 64): a candidate of I is
//     rejected if a candidate of J weakly dominates it (ties: the smaller arc
//     id stays);
//   B-tiles (frontier tile T of 256 entries, 4 per lane, x candidate tile J
//     of 64): a candidate is rejected if an entry of T weakly dominates it; an
//     entry is pruned if a candidate strictly dominates it.  Any candidate may
//     prune: the minimal candidates below a pruning one are accepted (the live
//     frontier is an antichain), so the outcome equals pruning by accepted
//     candidates only.
// Rejections are idempotent stores; a prune sets PRUNED_BIT in the entry's
// label-id slot with an atomic OR, and the first setter marks the label dead.
template <int DM>
__global__ __launch_bounds__(NT_TILE) void k_group_pairs(Slot* slots, int pass) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  const int total = Sp->big_tiles_pass[pass], nbig = S.nbig;
  const int32_t* toff = S.big_toff + (size_t)pass * (S.cand_cap + 1);
  const int lvl0 = pass_lo(pass);
  const int wave = threadIdx.x / WAVE, lane = lane_id();
  const int d = S.d, cc = S.cand_cap;
  int32_t* fw = S.fw;
  int64_t pruned = 0;
  __shared__ int4 cstage[GP_WAVES][WAVE][FrontChunk<DM>::NW];  // per wave: its candidate tile
  __shared__ int2 fstage[GP_WAVES][WAVE];                         // and their ids and arcs
  for (int tt = blockIdx.x * GP_WAVES + wave; tt < total; tt += gridDim.x * GP_WAVES) {
    int lo_i = 0, hi_i = nbig - 1;  // big group owning tile tt
    while (lo_i < hi_i) {
      const int mid = (lo_i + hi_i + 1) >> 1;
      if (toff[mid] <= tt) lo_i = mid; else hi_i = mid - 1;
    }
    const int gid = S.big_list[lo_i];
    const int local = tt - toff[lo_i];
    const int v = S.grp_node[gid];
    const int k = S.grp_cnt[v];
    const int32_t* ord = S.order + S.grp_off[gid];
    const int nct = (k + WAVE - 1) / WAVE;
    // pass 0: A-tiles first; then frontier tiles from the pass's first level
    const bool is_a = !pass && local < nct * nct;
    const int rest = is_a ? local : (pass ? local : local - nct * nct) + lvl0 * nct;
    const int I = rest / nct, J = rest % nct;
    // candidate tile J, one candidate per lane
    const int j = J * WAVE + lane;
    const bool hj = j < k;
    const int fj = hj ? ord[j] : 0;
    const int aj = hj ? S.c_arc[fj] : 0;
    int32_t cj[DM];
#pragma unroll
    for (int kk = 0; kk < DM; ++kk) cj[kk] = (hj && kk < d) ? S.c_g[(size_t)kk * cc + fj] : 0;
    const int nj = __builtin_amdgcn_readfirstlane(min(WAVE, k - J * WAVE));  // wave-uniform
    // the wave's candidates go through LDS: one broadcast read per candidate
    // on the LDS pipe instead of DM lane reads on the vector ALU
    constexpr int NW = FrontChunk<DM>::NW;
    {
      int32_t x[NW * 4];
#pragma unroll
      for (int q = 0; q < NW * 4; ++q) x[q] = q < DM ? cj[q] : 0;
#pragma unroll
      for (int w = 0; w < NW; ++w)
        cstage[wave][lane][w] = make_int4(x[4 * w], x[4 * w + 1], x[4 * w + 2], x[4 * w + 3]);
      fstage[wave][lane] = make_int2(fj, aj);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // read across lanes below
    if (is_a) {
      const int i = I * WAVE + lane;
      const bool hi = i < k;
      const int fi = hi ? ord[i] : 0;
      const int ai = hi ? S.c_arc[fi] : 0;
      int32_t ci[DM];
#pragma unroll
      for (int kk = 0; kk < DM; ++kk) ci[kk] = (hi && kk < d) ? S.c_g[(size_t)kk * cc + fi] : 0;
      bool rej = false;
      for (int jj = 0; jj < nj; ++jj) {
        int4 cw[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) cw[w] = cstage[wave][jj][w];
        bool le = true, eq = true;
#pragma unroll
        for (int kk = 0; kk < DM; ++kk) {
          const int b = comp(cw[kk >> 2], kk & 3);
          le = le & (b <= ci[kk]);
          eq = eq & (b == ci[kk]);
        }
        const int2 fa = fstage[wave][jj];
        rej = rej | (fa.x != fi && le && (!eq || fa.y < ai));
      }
      if (hi && rej) S.c_rej[fi] = 1;
    } else {
      // frontier tile I: BT_U entries per lane
      const NodeRec nr = S.node[v];
      int32_t sv[BT_U][DM];
      bool has[BT_U], prune[BT_U];
#pragma unroll
      for (int u = 0; u < BT_U; ++u) {
        const int e = I * BT_ENTRIES + u * WAVE + lane;
        has[u] = e < nr.count && fw[nr.off + (int64_t)d * nr.cap + e] != FW_REMOVED;
#pragma unroll
        for (int kk = 0; kk < DM; ++kk)
          sv[u][kk] = kk < d ? (has[u] ? fw[nr.off + (int64_t)kk * nr.cap + e] : INT32_MAX) : 0;
      }
      uint64_t rejm = 0;
      int pacc[BT_U];
#pragma unroll
      for (int u = 0; u < BT_U; ++u) pacc[u] = 0;
      // a candidate already rejected (by the first pass, or by another tile)
      // can prune no live entry (the frontier is an antichain, and a candidate
      // below it prunes the same entries), so its row is skipped
      const uint64_t live = ballot(hj && !S.c_rej[fj]);
      for (uint64_t m = live; m; m &= m - 1) {
        const int jj = __ffsll((long long)m) - 1;
        int4 cw[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) cw[w] = cstage[wave][jj][w];
        int32_t c[DM];
#pragma unroll
        for (int kk = 0; kk < DM; ++kk) c[kk] = comp(cw[kk >> 2], kk & 3);
        int allneg = -1;
#pragma unroll
        for (int u = 0; u < BT_U; ++u) {
          int dmin, dmax;
          diff_range<DM>(c, sv[u], dmin, dmax);
          allneg &= dmin;
          pacc[u] |= (dmax - 1) & dmin;
        }
        if (ballot(allneg >= 0)) rejm |= 1ull << jj;
      }
#pragma unroll
      for (int u = 0; u < BT_U; ++u) prune[u] = has[u] && pacc[u] < 0;
      if ((rejm >> lane) & 1ull) S.c_rej[fj] = 1;
#pragma unroll
      for (int u = 0; u < BT_U; ++u) {
        if (prune[u]) {
          const int e = I * BT_ENTRIES + u * WAVE + lane;
          const int old = atomicOr(&fw[nr.off + (int64_t)d * nr.cap + e], PRUNED_BIT);
          if (old >= 0) {
            S.Lstate[old] = L_DEAD;
            pruned++;
          }
        }
      }
    }
  }
  pruned = wave_sum64(pruned);
  if (lane == 0 && pruned)
    atomicAdd((unsigned long long*)&Sp->st[ST_PRUNED], (unsigned long long)pruned);
}

// Finish a big group (one wave): compact the frontier without its pruned and
// removed entries, append the accepted candidates, reset the node's group
// scratch.
template <int DM>
__global__ __launch_bounds__(NT_TILE) void k_group_finish(Slot* slots) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  const int nbig = S.nbig;
  const int wave = threadIdx.x / WAVE, lane = lane_id();
  const int d = S.d, cc = S.cand_cap;
  int32_t* fw = S.fw;
  int64_t gpairs = 0, fpairs = 0, fbytes = 0;
  __shared__ int32_t hole_list[GP_WAVES][HOLECAP];  // per wave: hole positions of its group
  for (int bi = blockIdx.x * GP_WAVES + wave; bi < nbig; bi += gridDim.x * GP_WAVES) {
    const int gid = S.big_list[bi];
    const int v = S.grp_node[gid];
    const int k = S.grp_cnt[v];
    const int32_t* ord = S.order + S.grp_off[gid];
    const NodeRec nr = S.node[v];
    const int cnt = nr.count;
    gpairs += (int64_t)k * (k - 1);
    int64_t doff;
    int dcap;
    if (!frontier_dest(Sp, S, nr, cnt + k, d, &doff, &dcap)) break;
    const bool moved = doff != nr.off;
    int cursor = 0, nlive = 0;  // nlive: entries the pair tiles compared
    constexpr int FU = 16;      // label ids per lane in flight
    // A frontier is a set, so a block that stays in place is compacted by
    // moving the kept entries behind the new end K = cnt - holes into the
    // holes before K (pass 1 lists the holes in LDS, pass 2 walks the tail
    // [K, cnt), which is only `holes` entries long).  A block that moves, or
    // one with more holes than the list holds, is rewritten in order.
    bool ordered = moved, counted = false;
    if (!moved) {
      int32_t* hl = hole_list[wave];
      int nh = 0;
      constexpr int HU = 16;  // label ids per lane in flight in the hole scan
      for (int t0 = 0; t0 < cnt; t0 += HU * WAVE) {
        int slab[HU];
#pragma unroll
        for (int u = 0; u < HU; ++u) {
          const int e = t0 + u * WAVE + lane;
          slab[u] = e < cnt ? fw[nr.off + (int64_t)d * nr.cap + e] : 0;
        }
#pragma unroll
        for (int u = 0; u < HU; ++u) {
          const int e = t0 + u * WAVE + lane;
          const bool has = e < cnt;
          nlive += __popcll(ballot(has && slab[u] != FW_REMOVED));
          const bool hole = has && slab[u] < 0;
          const uint64_t m = ballot(hole);
          if (hole) {
            const int r = nh + rank_below(m);
            if (r < HOLECAP) hl[r] = e;
          }
          nh += __popcll(m);
        }
      }
      counted = true;
      if (nh > HOLECAP) {
        ordered = true;
      } else {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the list is read across lanes
        const int K = cnt - nh;
        int r = 0;
        for (int t = K; t < cnt; t += WAVE) {
          const int e = t + lane;
          const int id = e < cnt ? fw[nr.off + (int64_t)d * nr.cap + e] : -1;
          const bool keep = id >= 0;
          const uint64_t m = ballot(keep);
          if (keep) {
            const int dst = hl[r + rank_below(m)];  // a hole before K
            int32_t sv[DM];
            FOR_K(kk) sv[kk] = fw[nr.off + (int64_t)kk * nr.cap + e];
            FOR_K(kk) fw[nr.off + (int64_t)kk * nr.cap + dst] = sv[kk];
            fw[nr.off + (int64_t)d * nr.cap + dst] = id;
          }
          r += __popcll(m);
        }
        cursor = K;
      }
    }
    if (ordered) {
      // label ids FU x 64 at a time; the vectors are read only where the block
      // has to be rewritten (it moved, or entries before were dropped).  Every
      // entry's destination lies at or before its own position, so within one
      // block of ids all rewritten vectors of RU sub-chunks are loaded before
      // any of them is stored (one memory round trip instead of RU).
      constexpr int RU = DM <= 3 ? 16 : (DM <= 6 ? 8 : 4);  // rewritten sub-chunks in flight
      for (int t0 = 0; t0 < cnt; t0 += FU * WAVE) {
        int slab[FU];
#pragma unroll
        for (int u = 0; u < FU; ++u) {
          const int e = t0 + u * WAVE + lane;
          slab[u] = e < cnt ? fw[nr.off + (int64_t)d * nr.cap + e] : 0;
        }
        uint64_t am[FU];
        int cur[FU];
        uint32_t rw = 0;  // sub-chunks to rewrite (wave-uniform)
#pragma unroll
        for (int u = 0; u < FU; ++u) {
          const int t = t0 + u * WAVE;
          const int e = t + lane;
          const bool has = e < cnt;
          if (!counted) nlive += __popcll(ballot(has && slab[u] != FW_REMOVED));
          const uint64_t hm = ballot(has);
          am[u] = ballot(has && slab[u] >= 0);
          cur[u] = cursor;
          if (hm && (moved || cursor != t || am[u] != hm)) rw |= 1u << u;
          cursor += __popcll(am[u]);
        }
        if (!rw) continue;
#pragma unroll
        for (int u0 = 0; u0 < FU; u0 += RU) {
          int32_t sv[RU][DM];
#pragma unroll
          for (int u = 0; u < RU; ++u) {
            const int uu = u0 + u;
            if (((rw >> uu) & 1) && ((am[uu] >> lane) & 1)) {
              const int e = t0 + uu * WAVE + lane;
              FOR_K(kk) sv[u][kk] = fw[nr.off + (int64_t)kk * nr.cap + e];
            }
          }
#pragma unroll
          for (int u = 0; u < RU; ++u) {
            const int uu = u0 + u;
            if (((rw >> uu) & 1) && ((am[uu] >> lane) & 1)) {
              const int64_t w = doff + cur[uu] + rank_below(am[uu]);
              FOR_K(kk) fw[w + (int64_t)kk * dcap] = sv[u][kk];
              fw[w + (int64_t)d * dcap] = slab[uu];
            }
          }
        }
      }
    }
    fpairs += (int64_t)k * nlive;
    fbytes += (int64_t)nlive * 4 * d;
    const int hv = S.h[v];
    constexpr int CU = 4;  // candidates per lane in flight
    for (int c0 = 0; c0 < k; c0 += CU * WAVE) {
      int fjs[CU];
      bool accs[CU];
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        const int j = c0 + u * WAVE + lane;
        fjs[u] = j < k ? ord[j] : -1;
      }
#pragma unroll
      for (int u = 0; u < CU; ++u) accs[u] = fjs[u] >= 0 && !S.c_rej[fjs[u]];
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        const uint64_t m = ballot(accs[u]);
        if (accs[u]) {
          const int fj = fjs[u];
          const int64_t w = doff + cursor + rank_below(m);
          FOR_K(kk) fw[w + (int64_t)kk * dcap] = S.c_g[(size_t)kk * cc + fj];
          fw[w + (int64_t)d * dcap] = -1;
          S.c_fslot[fj] = w + (int64_t)d * dcap;
          S.c_acc[fj] = open_tier(S, S.c_g[fj] + hv);
        }
        cursor += __popcll(m);
      }
    }
    if (lane == 0) {
      NodeRec out;
      out.off = doff;
      out.cap = dcap;
      out.count = cursor;
      S.node[v] = out;
      S.grp_cnt[v] = 0;
      S.grp_id[v] = -1;
    }
  }
  if (lane == 0) {
    if (gpairs) atomicAdd((unsigned long long*)&Sp->st[ST_GPAIRS], (unsigned long long)gpairs);
    if (fpairs) atomicAdd((unsigned long long*)&Sp->st[ST_FPAIRS], (unsigned long long)fpairs);
    if (fbytes) atomicAdd((unsigned long long*)&Sp->st[ST_FBYTES], (unsigned long long)fbytes);
  }
}

// ---------------------------------------------------------------- insert
// Ranks of the accepted candidates in flat order: c_rank = rank among all
// accepted (label id offset), c_rej = rank within the OPEN tier it joins
// (c_acc: 0 rejected, 1 near, 2 far).  Two grid-wide passes over tiles of
// ACC_TILE candidates: k_accept_count stores each tile's near and far counts;
// k_accept_scan starts each tile after the counts of the tiles before it and
// numbers the tile's accepted candidates in index order.
__global__ __launch_bounds__(NT_TILE) void k_accept_count(Slot* slots) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  constexpr int U = ACC_TILE / NT_TILE;
  __shared__ int wn[GP_WAVES], wf[GP_WAVES];
  const int M = S.cand_n, nt = (M + ACC_TILE - 1) / ACC_TILE;
  const int wave = threadIdx.x / WAVE, lane = lane_id();
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    int a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = t * ACC_TILE + u * NT_TILE + threadIdx.x;
      a[u] = i < M ? S.c_acc[i] : 0;
    }
    int cn = 0, cf = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cn += __popcll(ballot(a[u] == 1));
      cf += __popcll(ballot(a[u] == 2));
    }
    if (lane == 0) {
      wn[wave] = cn;
      wf[wave] = cf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int n = 0, f = 0;
#pragma unroll
      for (int w = 0; w < GP_WAVES; ++w) {
        n += wn[w];
        f += wf[w];
      }
      S.acc_tile[2 * t] = n;
      S.acc_tile[2 * t + 1] = f;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(NT_TILE) void k_accept_scan(Slot* slots) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  constexpr int U = ACC_TILE / NT_TILE;
  __shared__ int red[4][GP_WAVES];
  __shared__ int cwn[U][GP_WAVES], cwf[U][GP_WAVES];
  const int M = S.cand_n, nt = (M + ACC_TILE - 1) / ACC_TILE;
  const int wave = threadIdx.x / WAVE, lane = lane_id();
  if (blockIdx.x == 0) {  // totals and the capacity check
    int tn = 0, tf = 0;
    for (int x = threadIdx.x; x < nt; x += NT_TILE) {
      tn += S.acc_tile[2 * x];
      tf += S.acc_tile[2 * x + 1];
    }
    tn = wave_sum(tn);
    tf = wave_sum(tf);
    if (lane == 0) {
      red[2][wave] = tn;
      red[3][wave] = tf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      tn = tf = 0;
#pragma unroll
      for (int w = 0; w < GP_WAVES; ++w) {
        tn += red[2][w];
        tf += red[3][w];
      }
      Sp->accept_n = tn + tf;
      Sp->accept_near = tn;
      Sp->accept_far = tf;
      if (S.n_labels + tn + tf > S.pool_cap || S.keep_n + tn > S.open_cap ||
          S.far_n + tf > S.open_cap) {
        Sp->status = S_OVERFLOW;
        Sp->err_line = __LINE__;
      }
    }
    __syncthreads();
  }
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    int a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = t * ACC_TILE + u * NT_TILE + threadIdx.x;
      a[u] = i < M ? S.c_acc[i] : 0;
    }
    int bn = 0, bf = 0;  // accepted in the tiles before this one
    for (int x = threadIdx.x; x < t; x += NT_TILE) {
      bn += S.acc_tile[2 * x];
      bf += S.acc_tile[2 * x + 1];
    }
    bn = wave_sum(bn);
    bf = wave_sum(bf);
    uint64_t mn[U], mf[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      mn[u] = ballot(a[u] == 1);
      mf[u] = ballot(a[u] == 2);
    }
    if (lane == 0) {
      red[0][wave] = bn;
      red[1][wave] = bf;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        cwn[u][wave] = __popcll(mn[u]);
        cwf[u][wave] = __popcll(mf[u]);
      }
    }
    __syncthreads();
    // chunk u of the tile is candidates t*ACC_TILE + u*NT_TILE + [0, NT_TILE),
    // wave w holds 64 of them: its base is every chunk before u plus the
    // waves before w in chunk u
    int on = 0, of = 0;
#pragma unroll
    for (int w = 0; w < GP_WAVES; ++w) {
      on += red[0][w];
      of += red[1][w];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int pn = on, pf = of;
#pragma unroll
      for (int w = 0; w < GP_WAVES; ++w) {
        if (w < wave) {
          pn += cwn[u][w];
          pf += cwf[u][w];
        }
        on += cwn[u][w];
        of += cwf[u][w];
      }
      if (a[u]) {
        const int i = t * ACC_TILE + u * NT_TILE + threadIdx.x;
        const int rn = pn + rank_below(mn[u]), rf = pf + rank_below(mf[u]);
        S.c_rank[i] = rn + rf;
        S.c_rej[i] = a[u] == 1 ? rn : rf;
        S.order[rn + rf] = i;  // accepted candidates by label id (grouping is done)
      }
    }
    __syncthreads();
  }
}

template <int DM>
__global__ __launch_bounds__(NT_TILE) void k_insert(Slot* slots, GraphDev G) {
  Slot* Sp = &slots[blockIdx.y];
  const Slot S = *Sp;
  if (S.status != S_RUN) return;
  const int M = S.cand_n;
  const int d = S.d, pc = S.pool_cap, cc = S.cand_cap;
  const int base_id = S.n_labels, keep = S.keep_n, far = S.far_n;
  int32_t* KF = pick(S.open_f1, S.open_sel ^ 1);
  int32_t* KL = pick(S.open_lab, S.open_sel ^ 1);
  int32_t* FF = pick(S.far_f1, S.far_sel);
  int32_t* FL = pick(S.far_lab, S.far_sel);
  int mn = INT32_MAX;
  for (int f = blockIdx.x * NT_TILE + threadIdx.x; f < M; f += gridDim.x * NT_TILE) {
    if (!S.c_acc[f]) continue;
    const int r = S.c_rank[f];
    const int id = base_id + r;
    const int v = S.c_node[f];
    S.Lnode[id] = v;
    S.Lpar[id] = S.c_par[f];
    S.Larc[id] = S.c_arc[f];
    // eager mode: a label at the goal goes to the next step's goal step and is
    // never popped (closed at once, its OPEN entry vanishes at the next pop)
    const bool eager = S.eager_goal && v == S.goal;
    S.Lstate[id] = eager ? L_CLOSED : L_OPEN;
    if (eager) S.pgoal[atomicAdd(&Sp->pgoal_n, 1)] = id;
    S.Lpseq[id] = S.P_seq;  // k_pfilter tests it against every entry appended so far
    FOR_K(k) S.Lg[(size_t)k * pc + id] = S.c_g[(size_t)k * cc + f];
    S.fw[S.c_fslot[f]] = id;
    const int f1 = open_key(S, S.c_g[f] + S.h[v]);
    const int q = S.c_rej[f];  // rank within its tier
    if (S.c_acc[f] == 1) {
      KF[keep + q] = f1;
      KL[keep + q] = id;
      mn = min(mn, f1);
    } else {
      FF[far + q] = f1;
      FL[far + q] = id;
    }
  }
  mn = wave_min(mn);
  if (lane_id() == 0 && mn != INT32_MAX) atomicMin(&Sp->lo_next, mn);
}

__global__ void k_step_end(Slot* slots, int nslots) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  Slot* S = &slots[s];
  if (S->status != S_RUN) return;
  S->pf_base = S->n_labels;
  S->pf_n = S->accept_n;
  S->n_labels += S->accept_n;
  S->st[ST_INSERTED] += S->accept_n;
  S->open_n = S->keep_n + S->accept_near;
  S->far_n += S->accept_far;
  S->open_sel ^= 1;
  if (S->open_n > 0) S->lo = S->lo_next;
  S->st[ST_STEPS] += 1;
  S->refill = !S->t_all && S->far_n > 0 && S->open_n < NEAR_LOW * S->B;
  if (S->open_n == 0 && S->far_n == 0 && S->pgoal_n == 0) S->status = S_DONE;
}

// ---------------------------------------------------------------- launchers
const char* const kStepKernelNames[kStepKernels] = {
    "k_far_hist",      "k_far_move",      "k_open_hist",     "k_open_threshold", "k_open_scatter",
    "k_batch_finalize", "k_split_count",  "k_split_scan",    "k_goal_pairs",   "k_goal_merge",    "k_popcheck",       "k_expand",
    "k_group_count",   "k_group_offsets", "k_group_scatter", "k_group_process",  "k_group_pairs",
    "k_group_pairs2",  "k_group_finish",  "k_accept_count",  "k_accept_scan",    "k_insert",
    "k_pfilter",       "k_step_end"};

template <int DM>
static void launch_step_dm(const StepArgs& a, hipStream_t st, hipEvent_t* ev, uint32_t mask) {
  const dim3 tiled(a.gx, a.nslots), per(a.nslots);
  const dim3 cand(a.gc, a.nslots);                    // per-candidate loops
  const dim3 refill(std::min(a.gx, 256), a.nslots);   // far-tier kernels: idle on most steps
  // OPEN scans: several entries per thread, so that the per-workgroup appends
  // (one atomic per counter and workgroup) stay few
  const dim3 scan(std::min(a.gx, 256), a.nslots);
  // kernel i on stream s, bracketed by events when profiled
  auto run = [&](int i, hipStream_t s, auto&& launch) {
    const bool timed = ev && ((mask >> i) & 1u);
    if (timed) hipEventRecord(ev[2 * i], s);
    launch(s);
    if (timed) hipEventRecord(ev[2 * i + 1], s);
  };
  auto pop = [&](hipStream_t s) {
    run(0, s, [&](hipStream_t q) { hipLaunchKernelGGL(k_far_hist, refill, dim3(NT_TILE), 0, q, a.slots, a.hist); });
    run(1, s, [&](hipStream_t q) { hipLaunchKernelGGL(k_far_move, refill, dim3(NT_TILE), 0, q, a.slots); });
    run(2, s, [&](hipStream_t q) { hipLaunchKernelGGL(k_open_hist, scan, dim3(NT_TILE), 0, q, a.slots, a.hist); });
    run(3, s, [&](hipStream_t q) { hipLaunchKernelGGL(k_open_threshold, per, dim3(NT_SLOT), 0, q, a.slots, a.hist); });
    run(4, s, [&](hipStream_t q) { hipLaunchKernelGGL(k_open_scatter, scan, dim3(NT_TILE), 0, q, a.slots); });
    run(5, s, [&](hipStream_t q) { hipLaunchKernelGGL(k_batch_finalize<DM>, per, dim3(NT_SLOT), 0, q, a.slots, a.G); });
    run(6, s, [&](hipStream_t q) { hipLaunchKernelGGL(k_split_count, tiled, dim3(NT_TILE), 0, q, a.slots, a.G); });
    run(7, s, [&](hipStream_t q) { hipLaunchKernelGGL(k_split_scan, tiled, dim3(NT_TILE), 0, q, a.slots, a.G); });
  };
  auto pfilter = [&](hipStream_t s) {
    run(20 + NPASS, s, [&](hipStream_t q) { hipLaunchKernelGGL(k_pfilter<DM>, tiled, dim3(NT_TILE), 0, q, a.slots, a.G); });
  };
  if (!a.pipelined) {
    pop(st);
  } else if (ev || !a.st2) {
    pfilter(st);
    pop(st);
  } else {
    // the previous step's filter beside this step's pop: they touch disjoint
    // state (the filter reads the goal front, the previous step's candidates
    // and pf_base/pf_n; the pop rewrites OPEN and the batch); label states
    // are read by the pop and set dead by the filter, and a label popped
    // before the filter marks it is caught by the pop-time goal-front check
    hipEventRecord(a.fork, st);
    hipStreamWaitEvent(a.st2, a.fork, 0);
    pop(a.st2);
    pfilter(st);
    hipEventRecord(a.join, a.st2);
    hipStreamWaitEvent(st, a.join, 0);
  }
  run(8, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_goal_pairs<DM>, tiled, dim3(NT_TILE), 0, q, a.slots); });
  run(9, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_goal_merge<DM>, per, dim3(NT_SLOT), 0, q, a.slots); });
  run(10, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_popcheck<DM>, tiled, dim3(NT_TILE), 0, q, a.slots, a.G); });
  run(11, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_expand<DM>, cand, dim3(NT_TILE), 0, q, a.slots, a.G); });
  run(12, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_group_count, cand, dim3(NT_TILE), 0, q, a.slots); });
  run(13, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_group_offsets, per, dim3(NT_SLOT), 0, q, a.slots); });
  run(14, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_group_scatter, cand, dim3(NT_TILE), 0, q, a.slots); });
  run(15, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_group_process<DM>, tiled, dim3(NT_TILE), 0, q, a.slots); });
  for (int p = 0; p < NPASS; ++p)
    run(16 + p, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_group_pairs<DM>, tiled, dim3(NT_TILE), 0, q, a.slots, p); });
  run(16 + NPASS, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_group_finish<DM>, tiled, dim3(NT_TILE), 0, q, a.slots); });
  run(17 + NPASS, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_accept_count, cand, dim3(NT_TILE), 0, q, a.slots); });
  run(18 + NPASS, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_accept_scan, cand, dim3(NT_TILE), 0, q, a.slots); });
  run(19 + NPASS, st, [&](hipStream_t q) { hipLaunchKernelGGL(k_insert<DM>, cand, dim3(NT_TILE), 0, q, a.slots, a.G); });
  if (!a.pipelined) pfilter(st);
  run(21 + NPASS, st, [&](hipStream_t q) {
    hipLaunchKernelGGL(k_step_end, dim3((a.nslots + 63) / 64), dim3(64), 0, q, a.slots, a.nslots);
  });
  if (ev) hipEventRecord(ev[2 * kStepKernels], st);
}

int dm_for(int d) {
  if (d <= 2) return 2;
  if (d <= 3) return 3;
  if (d <= 4) return 4;
  if (d <= 5) return 5;
  if (d <= 6) return 6;
  if (d <= 8) return 8;
  return 12;
}

void launch_step(const StepArgs& a, hipStream_t st, hipEvent_t* ev, uint32_t mask) {
  switch (a.dm) {
    case 2: launch_step_dm<2>(a, st, ev, mask); break;
    case 3: launch_step_dm<3>(a, st, ev, mask); break;
    case 4: launch_step_dm<4>(a, st, ev, mask); break;
    case 5: launch_step_dm<5>(a, st, ev, mask); break;
    case 6: launch_step_dm<6>(a, st, ev, mask); break;
    case 8: launch_step_dm<8>(a, st, ev, mask); break;
    default: launch_step_dm<12>(a, st, ev, mask); break;
  }
}

}  // namespace mos
