// Shared definitions of the GPU search: slot descriptors, graph view, device helpers.
//
// A "slot" is one query resident on the device.  All search state of a slot
// lives in one contiguous reservation of the engine's device arena; the host
// carves it into the regions below when the query is admitted and stores typed
// pointers in the Slot descriptor.  Every step kernel takes the whole slot
// table (blockIdx.y = slot for the tiled kernels), so one launch advances
// every resident query.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mos {

constexpr int MAXD = 12;          // objectives supported by the kernels
constexpr int NB = 4096;          // OPEN histogram bins: exact F1 values lo..lo+NB-2, then overflow
constexpr int ACC_TILE = 2048;    // candidates per tile of the accepted-candidate numbering
constexpr int SPLIT_TILE = 2048;  // items (popped labels, tie entries) per tile of the batch split
constexpr int SPLIT_WORDS = 5;    // per split tile: goal, regular, out-degree sum, back to OPEN, min F1
constexpr int TIECAP = 256;       // tie sets up to this size are ranked in LDS; larger ones
                                  // are first narrowed by exact radix refinement
constexpr int MINCAP = 8;         // smallest frontier block, in entries
constexpr int BATCH_MAX = 32768;  // largest popped batch
// Pair tiles of large groups run in NPASS launches: pass p covers frontier
// tiles [pass_lo(p), pass_lo(p + 1)) of every group (pass 0 also the tiles of
// candidates against candidates); a later pass skips candidates an earlier
// one rejected.
constexpr int NPASS = 2;
__host__ __device__ constexpr int pass_lo(int p) { return p <= 0 ? 0 : (p == 1 ? 1 : 1 << 30); }
// near-tier sizing, in multiples of B: refill below LOW, refill up to TARGET,
// spill to far above HIGH (keeping TARGET)
constexpr int NEAR_LOW = 4, NEAR_TARGET = 16, NEAR_HIGH = 48;
constexpr int32_t UNREACH = INT32_MAX;  // heuristic of a node that cannot reach the goal
constexpr int WAVE = 64;
constexpr int64_t BIG_WORK = 4096;  // pair checks above which a group is split across waves
constexpr int32_t PRUNED_BIT = (int32_t)0x80000000;  // marks a pruned entry in a label-id slot
// label-id slot of a frontier entry whose label the goal front dominated after
// it was inserted: the entry takes part in no test and goes at the next
// compaction of its block (PRUNED_BIT | label cannot produce this value)
constexpr int32_t FW_REMOVED = -2;

enum SlotStatus : int32_t {
  S_IDLE = 0,
  S_RUN = 1,
  S_DONE = 2,
  S_OVERFLOW = 3,  // a capacity of the reservation was exceeded
  S_SOLO = 4,      // running: the query's steps run in one workgroup of its own
  S_SOLO_QUIT = 5, // left the one-workgroup step: to be run by the multi-kernel step
};

enum LabelState : uint8_t { L_OPEN = 0, L_CLOSED = 1, L_DEAD = 2 };

// Per-slot statistics counters (int64 each).
enum Stat {
  ST_POPS = 0,
  ST_GOAL_POPS,
  ST_CANDS,
  ST_PPAIRS,
  ST_GPAIRS,
  ST_FPAIRS,
  ST_INSERTED,
  ST_PRUNED,
  ST_STEPS,
  ST_FBYTES,
  ST_GROUPS,
  ST_KILLED,
  ST_FBYTES_WAVE,  // frontier bytes of the groups checked in one pass by one wave
  ST_PAIRS_WAVE,   // candidate pairs (frontier + same group) of those groups
  ST_NEAR_SCAN,    // near-tier OPEN entries scanned by pops
  ST_FAR_SCAN,     // far-tier OPEN entries scanned by refills
  ST_TIE,          // entries of threshold bins refined by full key
  ST_PREAD,        // goal-front entries read by goal merges
  ST_T0 = 24,      // ST_T0..ST_T0+7: phase timers and diagnostics
  NSTAT = 32
};

// Frontier record of one node: the node's live labels are entries [0, count)
// of a block of `cap` entries at word offset `off` of the slot's frontier
// region; the block holds d int32 planes (objective k at off + k*cap) followed
// by a plane of pool label ids.
struct NodeRec {
  int64_t off;
  int32_t cap;
  int32_t count;
};

struct GraphDev {
  int32_t n, m, D, maxdeg;
  int32_t csum[MAXD];      // sum of each objective over all arcs (bounds every simple path)
  const int32_t* row_ptr;  // n+1
  const int32_t* col;      // m
  const int32_t* cost;     // D planes of m: cost[k*m + e]
  const int32_t* rrow;     // reverse CSR: arcs entering v are rrow[v]..rrow[v+1]-1
  const int32_t* rsrc;     //   source node of each entering arc
  const int32_t* rarc;     //   forward arc id of each entering arc
};

struct Slot {
  // ---------------- set at admission
  int32_t status;
  int32_t start, goal, d;
  int32_t B, batch_cap, cand_cap, tie_cap;
  int32_t pool_cap, open_cap, P_cap, query_id;
  int32_t heur_factor;  // heuristic radius as a multiple of h(start); 0 = exact everywhere
  int32_t heur_bounded; // set when the radius cut the reverse search (h is then a lower bound outside it)
  int64_t fw_cap;  // words of the frontier region
  int32_t hn;        // nodes of the graph (stride of the heuristic planes)
  int32_t pop_fifo;  // OPEN order: 0 = lexicographic by F (exact top-B); 1 = by the
                     // step that generated the label (oldest generation first), a
                     // relaxed order: the OPEN key is the generating step, not F1
  int32_t eps_ppm;   // 0 = exact; else tests against the goal front use
                     // (1 + eps_ppm / 10^6)-dominance (approximate front)
  int32_t eager_goal;  // 1: labels accepted at the goal join the goal front in the
                       // next step's goal step instead of waiting in OPEN to be popped
  int32_t pipelined;   // 1: the goal-front filter of a step's new labels runs at the
                       // start of the next step, beside its pop (pf_base, pf_n)
  int32_t solo;        // 1: the query's steps run in one workgroup of its own (S_SOLO)

  int32_t* h;          // d planes of n: heuristic
  NodeRec* node;       // n
  int32_t* grp_cnt;    // n: candidates of this step per node (0 outside a step)
  int32_t* grp_id;     // n: group id of the node in this step (-1 outside)
  int32_t* Lnode;      // pool_cap: node of each label
  int32_t* Lpar;       //   parent label (-1 for the start label)
  int32_t* Larc;       //   arc that created the label (-1 for the start label)
  int32_t* Lg;         //   d planes of pool_cap: g vectors
  uint8_t* Lstate;     //   LabelState
  int32_t* open_f1[2]; // open_cap each: near tier of OPEN (F1 < T): F1 of the entry
  int32_t* open_lab[2];//   label id of the entry
  int32_t* far_f1[2];  // open_cap each: far tier of OPEN (F1 >= T)
  int32_t* far_lab[2];
  int32_t* Pg[2];      // d planes of P_cap each: goal front (unordered; a removed
                       //   entry holds INT32_MAX in every plane until compaction)
  int32_t* Plab[2];    //   label id of each goal-front entry
  int32_t* Pseq[2];    //   append number of each entry (increasing along P)
  int32_t* Lpseq;      // pool_cap: goal-front appends already tested against the label
  int32_t* batch;      // batch_cap: popped labels
  int32_t* reg;        // batch_cap: popped regular labels (ascending label id)
  int32_t* reg_off;    // batch_cap+1: exclusive prefix of their out-degrees
  int32_t* reg_kill;   // batch_cap: popped regular label found dominated by the goal front
  int32_t* goal_lab;   // batch_cap + cand_cap: goal labels of this step's goal step
                       //   (popped ones, then the eager ones of the previous step)
  int32_t* pgoal;      // cand_cap: eager mode, labels accepted at the goal this step
  int32_t* tie_f1;     // tie_cap (= open_cap): entries of the threshold F1 bin
  int32_t* tie_lab;    // tie_cap
  int32_t* tie_st;     // tie_cap: refinement state of each tie entry
  int32_t* tie_key;    // d planes of tie_cap: F_2..F_d and the node of each tie entry
  int32_t* split_tile; // SPLIT_WORDS per SPLIT_TILE items of the batch split
  int32_t* c_node;     // cand_cap: candidate target node
  int32_t* c_par;      //   parent label
  int32_t* c_arc;      //   arc
  int32_t* c_g;        //   d planes of cand_cap
  int32_t* c_keep;     //   survived the goal-front filter
  int32_t* c_rank;     //   rank within its group, later rank among accepted
  int32_t* c_rej;      //   rejected inside its group or by the frontier
  int32_t* c_acc;      //   accepted (inserted)
  int64_t* c_fslot;    //   word offset of the frontier label-id slot it was given
  int32_t* acc_tile;   // 2 per ACC_TILE candidates: near and far accepted in the tile
  int32_t* order;      // cand_cap: candidates grouped by node
  int32_t* grp_node;   // cand_cap: node of each group
  int32_t* grp_off;    // cand_cap: first position of each group in `order`
  int32_t* small_list; // cand_cap: groups handled by one wave in one pass
  int32_t* big_list;   // cand_cap: groups split into pair tiles across waves
  int32_t* big_toff;   // NPASS planes of cand_cap+1: per pass of the pair tiles, the
                       //   exclusive prefix of the big groups' tiles in that pass
  int32_t* fw;         // frontier words

  // ---------------- dynamic (device-updated)
  int32_t n_labels, open_n, open_sel, P_n;
  int32_t P_sel, lo, lo_next, P_dead;  // P_dead: removed entries among the first P_n
  int32_t P_seq, pgoal_n;               // P_seq: goal-front entries appended so far;
                                        // pgoal_n: entries of pgoal
  int64_t fw_top;
  int32_t t_star, r_tie, tie_mode, big_work;  // big_work: set at admission
  int32_t batch_n, goal_n, reg_n, cand_n;
  int32_t ngroups, tie_n, keep_n, accept_n;
  int32_t nsmall, nbig, big_tiles, err_line;
  int32_t big_tiles_pass[4];  // pair tiles of each pass (NPASS <= 4)
  // two-tier OPEN: near holds F1 < T (all of OPEN while t_all), far holds F1 >= T
  int32_t far_n, far_sel, T, t_all;
  int32_t refill, r_T, r_all, r_moved;  // refill of near from far, decided per step
  int32_t r_keep, lo_refill, blocks_a, blocks_b;
  int32_t spill_T, spill_on, accept_near, accept_far;
  int32_t pop_nb, pop_keep;      // set by k_batch_finalize: direct pops, near-tier length
  int32_t pf_base, pf_n;         // set by k_step_end: the labels the step inserted, for a
                                 // goal-front filter that runs after it (pipelined)

  int64_t st[NSTAT];
};

// ------------------------------------------------------------ device helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Make LDS writes of this wave visible to its other lanes before they read.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Element i (0 or 1) of a two-entry member array, as a select: a runtime
// index into a member array would force a local copy of the descriptor into
// scratch memory.
template <class T>
__device__ __forceinline__ T pick(const T (&a)[2], int i) {
  return i ? a[1] : a[0];
}

__device__ __forceinline__ int rank_below(uint64_t m) {
  return __popcll(m & ((1ull << lane_id()) - 1ull));
}

// Wave-aggregated append: every active lane calls it; lanes with p get
// consecutive positions from *ctr (one atomic per wave).  Returns -1 for !p.
__device__ __forceinline__ int agg_append(int32_t* ctr, bool p) {
  uint64_t m = ballot(p);
  if (m == 0) return -1;
  int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane_id() == leader) base = atomicAdd(ctr, __popcll(m));
  base = __shfl(base, leader);
  return p ? base + rank_below(m) : -1;
}

__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// x scaled by 1 + eps_ppm / 10^6 and rounded down, so that for an integer p,
// p <= eps_relax(x) exactly when p <= (1 + eps) x.  Kept below INT32_MAX, the
// value of removed goal-front entries, which must never pass a test.
__device__ __forceinline__ int32_t eps_relax(int32_t x, int32_t eps_ppm) {
  if (eps_ppm == 0 || x == INT32_MAX) return x;
  const int64_t r = (int64_t)x + ((int64_t)x * eps_ppm) / 1000000;
  return (int32_t)(r < INT32_MAX - 1 ? r : INT32_MAX - 1);
}

// a <= b in every one of the d components (weak dominance, equality included).
__device__ __forceinline__ bool weak_le(const int32_t* a, const int32_t* b, int d) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < MAXD; ++k)
    if (k < d) ok = ok && (a[k] <= b[k]);
  return ok;
}

}  // namespace mos
