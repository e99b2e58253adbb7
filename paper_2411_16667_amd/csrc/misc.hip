// Per-query set-up and tear-down kernels: heuristic, slot initialisation, result paths.
//
// Heuristic (paper, Section 4: an admissible heuristic computed by
// single-source shortest paths for each objective): h_k(v) is the exact
// shortest v -> goal distance under objective k, found by label-correcting
// relaxation over the reversed arcs from the goal.  Each round relaxes the
// arcs entering the nodes improved in the previous round; a round stamp per
// node keeps every worklist duplicate-free.  All (query, objective) instances
// of an admission wave run in the same launches: one workgroup each, handing
// an instance over to grid-wide rounds when its worklist grows wide.
#include "kernels.h"

namespace mos {

constexpr int NT_H = 256;

// job j: slot slot_of[j]; instance (j, k) uses scratch hs + (j*MAXD + k) * 3n:
//   [0, n) worklist A, [n, 2n) worklist B, [2n, 3n) round stamps;
// counts at cnt + (j*MAXD + k) * 3 (three rotating counters).
__global__ void k_heur_init(Slot* slots, const int32_t* slot_of, GraphDev G, int32_t* hs,
                            int32_t* cnt) {
  const int j = blockIdx.z, k = blockIdx.y;
  Slot* S = &slots[slot_of[j]];
  const bool used = k < S->d;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // every counter of the job is initialised: the host polls all MAXD of them
    int32_t* c = cnt + ((size_t)j * MAXD + k) * 3;
    c[0] = used ? 1 : 0;
    c[1] = 0;
    c[2] = 0;
  }
  if (!used) return;
  const int n = G.n;
  int32_t* h = S->h + (size_t)k * n;
  int32_t* base = hs + ((size_t)j * MAXD + k) * 3 * n;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    h[v] = (v == S->goal) ? 0 : UNREACH;
    base[2 * n + v] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) base[0] = S->goal;
}

__global__ void k_heur_round(Slot* slots, const int32_t* slot_of, GraphDev G, int32_t* hs,
                             int32_t* cnt, int r) {
  const int j = blockIdx.z, k = blockIdx.y;
  Slot* S = &slots[slot_of[j]];
  if (k >= S->d) return;
  const int n = G.n;
  int32_t* h = S->h + (size_t)k * n;
  int32_t* base = hs + ((size_t)j * MAXD + k) * 3 * n;
  const int32_t* cur = base + (size_t)(r & 1) * n;
  int32_t* nxt = base + (size_t)((r + 1) & 1) * n;
  int32_t* stamp = base + 2 * (size_t)n;
  int32_t* c = cnt + ((size_t)j * MAXD + k) * 3;
  const int ncur = c[r % 3];
  int32_t* ncnt = &c[(r + 1) % 3];
  if (blockIdx.x == 0 && threadIdx.x == 0) c[(r + 2) % 3] = 0;
  const int32_t* cost = G.cost + (size_t)k * G.m;
  // radius: only nodes within heur_factor * h(start) are propagated further
  // (h(start) only decreases, so the cut never grows)
  const int h0 = h[S->start];
  const int64_t cut = (S->heur_factor > 0 && h0 != UNREACH) ? (int64_t)S->heur_factor * h0
                                                            : INT64_MAX;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncur; i += gridDim.x * blockDim.x) {
    const int v = cur[i];
    const int dv = h[v];
    for (int p = G.rrow[v]; p < G.rrow[v + 1]; ++p) {
      const int u = G.rsrc[p];
      const int nd = dv + cost[G.rarc[p]];
      if (nd < h[u]) {
        const int old = atomicMin(&h[u], nd);
        if (nd < old && nd <= cut && atomicMax(&stamp[u], r + 1) < r + 1) {
          const int pos = atomicAdd(ncnt, 1);
          nxt[pos] = u;
        }
      }
    }
  }
}

// Persistent form of the same search: one workgroup runs the rounds of one
// (query, objective) instance, the worklist lengths in LDS and a workgroup
// barrier between rounds, so a round costs no launch and no host poll.  The
// rounds, relaxations and stamps are those of k_heur_round; the lengths are
// read after a barrier, so every thread leaves the loop together.  On exit the
// instance's counters say where it stopped:
//   finished          c = {0, 0, 0}
//   handed over       c = {r + 1, 0, len}: at an even round r the worklist (in
//                     list A) held len > limit nodes; the grid-wide rounds
//                     carry on from there
//   no convergence    c[1] = 1 (after 4n + 64 rounds; the host fails it)
constexpr int NT_HP = 1024;
__global__ __launch_bounds__(NT_HP) void k_heur_persistent(Slot* slots, const int32_t* slot_of,
                                                          GraphDev G, int32_t* hs, int32_t* cnt,
                                                          int limit) {
  const int j = blockIdx.z, k = blockIdx.y;
  Slot* S = &slots[slot_of[j]];
  if (k >= S->d) return;
  const int n = G.n;
  int32_t* h = S->h + (size_t)k * n;
  int32_t* base = hs + ((size_t)j * MAXD + k) * 3 * n;
  int32_t* stamp = base + 2 * (size_t)n;
  int32_t* c = cnt + ((size_t)j * MAXD + k) * 3;
  const int32_t* cost = G.cost + (size_t)k * G.m;
  __shared__ int len[2];  // worklist lengths: list r & 1 is this round's, the other the next's
  if (threadIdx.x == 0) {
    len[0] = 1;  // k_heur_init put the goal in list 0
    len[1] = 0;
  }
  __syncthreads();
  for (int r = 0;; ++r) {
    const int ncur = len[r & 1];
    if (ncur == 0) {
      if (threadIdx.x == 0) c[0] = c[2] = 0;
      break;
    }
    if (ncur > limit && !(r & 1)) {
      if (threadIdx.x == 0) {
        c[0] = r + 1;
        c[2] = ncur;
      }
      break;
    }
    if (r > 4 * n + 64) {
      if (threadIdx.x == 0) c[1] = 1;
      break;
    }
    const int32_t* cur = base + (size_t)(r & 1) * n;
    int32_t* nxt = base + (size_t)((r + 1) & 1) * n;
    const int h0 = h[S->start];
    const int64_t cut = (S->heur_factor > 0 && h0 != UNREACH) ? (int64_t)S->heur_factor * h0
                                                              : INT64_MAX;
    for (int i = threadIdx.x; i < ncur; i += NT_HP) {
      const int v = cur[i];
      const int dv = h[v];
      for (int p = G.rrow[v]; p < G.rrow[v + 1]; ++p) {
        const int u = G.rsrc[p];
        const int nd = dv + cost[G.rarc[p]];
        if (nd < h[u]) {
          const int old = atomicMin(&h[u], nd);
          if (nd < old && nd <= cut && atomicMax(&stamp[u], r + 1) < r + 1)
            nxt[atomicAdd(&len[(r + 1) & 1], 1)] = u;
        }
      }
    }
    __syncthreads();  // the round is done and every thread has read len[r & 1]
    if (threadIdx.x == 0) len[r & 1] = 0;
    __syncthreads();
  }
}

// After the reverse search: with a radius cut R = heur_factor * h(start) below
// the largest possible distance (the objective's total over all arcs), every
// node with distance <= R holds its exact distance (its whole shortest path
// lies within R and was propagated) and every other node has distance > R,
// so it gets R + 1: an admissible lower bound.  Inside the cut the heuristic
// stays consistent; across it, F may decrease along an arc, which the search
// tolerates (its result does not depend on the pop order).
__global__ void k_heur_clamp(Slot* slots, const int32_t* slot_of, GraphDev G) {
  const int j = blockIdx.z, k = blockIdx.y;
  Slot* S = &slots[slot_of[j]];
  if (k >= S->d) return;
  const int n = G.n;
  int32_t* h = S->h + (size_t)k * n;
  const int hs = h[S->start];
  if (S->heur_factor <= 0 || hs == UNREACH) return;
  const int64_t cut = (int64_t)S->heur_factor * hs;
  if (cut >= G.csum[k]) return;  // no reachable distance exceeds the cut: exact
  const int lb = (int)cut + 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) S->heur_bounded = 1;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    if (h[v] > cut) h[v] = lb;
}

// Reset the per-node structures of a slot and seed the start label
// (the start of Algorithm 1).  A start that cannot reach the goal finishes the
// query at once with an empty front.
__global__ void k_slot_init(Slot* slots, int s, GraphDev G) {
  Slot* S = &slots[s];
  const int n = G.n;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    NodeRec z;
    z.off = 0;
    z.cap = 0;
    z.count = 0;
    S->node[v] = z;
    S->grp_cnt[v] = 0;
    S->grp_id[v] = -1;
  }
}

__global__ void k_slot_seed(Slot* slots, int s, GraphDev G) {
  Slot* S = &slots[s];
  const int d = S->d, st = S->start, n = G.n;
  bool reach = true;
  for (int k = 0; k < d; ++k) reach = reach && S->h[(size_t)k * n + st] != UNREACH;
  S->P_n = 0;
  S->P_sel = 0;
  S->P_dead = 0;
  S->P_seq = 0;
  S->lo_next = INT32_MAX;
  if (!reach) {
    S->n_labels = 0;
    S->open_n = 0;
    S->status = S_DONE;
    return;
  }
  S->Lnode[0] = st;
  S->Lpar[0] = -1;
  S->Larc[0] = -1;
  S->Lstate[0] = L_OPEN;
  S->Lpseq[0] = 0;
  for (int k = 0; k < d; ++k) S->Lg[(size_t)k * S->pool_cap] = 0;
  S->n_labels = 1;
  S->pf_base = 1;  // no label of a previous step waits for its goal-front filter
  S->pf_n = 0;
  NodeRec r;
  r.off = 0;
  r.cap = MINCAP;
  r.count = 1;
  for (int k = 0; k < d; ++k) S->fw[(size_t)k * MINCAP] = 0;
  S->fw[(size_t)d * MINCAP] = 0;
  S->node[st] = r;
  S->fw_top = (int64_t)MINCAP * (d + 1);
  const int32_t key0 = S->pop_fifo ? 0 : S->h[st];  // the start label's OPEN key
  S->open_f1[0][0] = key0;
  S->open_lab[0][0] = 0;
  S->open_n = 1;
  S->open_sel = 0;
  S->far_n = 0;
  S->far_sel = 0;
  S->t_all = 1;  // OPEN starts as one near tier; spills create the far tier
  S->T = INT32_MAX;
  S->refill = 0;
  S->blocks_a = 0;
  S->blocks_b = 0;
  S->lo = key0;
  S->st[ST_INSERTED] = 1;
  S->status = S->solo ? S_SOLO : S_RUN;
}

// Witness paths (paper, Section 3: parent pointers allow path reconstruction)
// of the goal labels labs[0 .. np): lengths, then arc ids written backwards
// from the end of each path's range.
__global__ void k_path_len(const Slot* slots, int s, const int32_t* labs, int np, int32_t* len) {
  const Slot* S = &slots[s];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
    int c = 0;
    for (int x = labs[i]; S->Lpar[x] >= 0; x = S->Lpar[x]) ++c;
    len[i] = c;
  }
}

__global__ void k_path_write(const Slot* slots, int s, const int32_t* labs, int np,
                             const int64_t* off, int32_t* arcs) {
  const Slot* S = &slots[s];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
    int64_t pos = off[i + 1];
    for (int x = labs[i]; S->Lpar[x] >= 0; x = S->Lpar[x]) arcs[--pos] = S->Larc[x];
  }
}

// Smallest F1 over the OPEN entries of slot s (both tiers; entries of labels
// that died since they were queued are included, which can only lower it),
// INT32_MAX when OPEN is empty.  Every label still to be processed has an F1
// at least this large, and a goal label's F is its cost, so the goal front's
// vectors whose first objective lies below it are final.  One workgroup.
__global__ void k_open_min(const Slot* slots, int s, int32_t* out) {
  const Slot* S = &slots[s];
  __shared__ int32_t red[1024 / WAVE];
  int32_t m = INT32_MAX;
  // F1 = g_1 + h_1 from the label itself (the tiers' key is F1 only in
  // lexicographic order)
  const int32_t* nl = pick(S->open_lab, S->open_sel);
  const int32_t* fl = pick(S->far_lab, S->far_sel);
  for (int i = threadIdx.x; i < S->open_n + S->far_n; i += blockDim.x) {
    const int lab = i < S->open_n ? nl[i] : fl[i - S->open_n];
    m = min(m, S->Lg[lab] + S->h[S->Lnode[lab]]);
  }
  m = wave_min(m);
  if (lane_id() == 0) red[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)blockDim.x / WAVE; ++w) m = min(m, red[w]);
    *out = min(m, red[0]);
  }
}

// ---------------------------------------------------------------- launchers
void launch_heur_init(Slot* slots, const int32_t* slot_of, int njobs, const GraphDev& G,
                      int32_t* hs, int32_t* cnt, hipStream_t st) {
  const int gx = std::min(1024, (G.n + NT_H - 1) / NT_H);
  hipLaunchKernelGGL(k_heur_init, dim3(gx, MAXD, njobs), dim3(NT_H), 0, st, slots, slot_of, G, hs,
                     cnt);
}

void launch_heur_round(Slot* slots, const int32_t* slot_of, int njobs, const GraphDev& G,
                       int32_t* hs, int32_t* cnt, int r, int gx, hipStream_t st) {
  // objectives beyond the graph's D belong to no query
  hipLaunchKernelGGL(k_heur_round, dim3(gx, G.D, njobs), dim3(NT_H), 0, st, slots, slot_of, G,
                     hs, cnt, r);
}

void launch_heur_clamp(Slot* slots, const int32_t* slot_of, int njobs, const GraphDev& G,
                       hipStream_t st) {
  const int gx = std::min(1024, (G.n + NT_H - 1) / NT_H);
  hipLaunchKernelGGL(k_heur_clamp, dim3(gx, MAXD, njobs), dim3(NT_H), 0, st, slots, slot_of, G);
}

void launch_slot_init(Slot* slots, int s, const GraphDev& G, hipStream_t st) {
  const int gx = std::min(2048, (G.n + 255) / 256);
  hipLaunchKernelGGL(k_slot_init, dim3(gx), dim3(256), 0, st, slots, s, G);
  hipLaunchKernelGGL(k_slot_seed, dim3(1), dim3(1), 0, st, slots, s, G);
}

int run_heuristic(Slot* slots, const int32_t* slot_of, int njobs, const GraphDev& G, int32_t* hs,
                  int32_t* cnt, int32_t* cnt_host, hipStream_t st) {
  launch_heur_init(slots, slot_of, njobs, G, hs, cnt, st);
  if (hipGetLastError() != hipSuccess) return -1;
  // Every instance starts in its own workgroup.  One whose worklist outgrows
  // a few wavefronts' worth is handed to the grid-wide rounds, which spread a
  // wide front over many CUs; on a small graph with enough instances to fill
  // the chip, every instance instead runs to the end in its workgroup (its
  // arrays stay cache-resident and the round launches would dominate).
  const size_t nc = (size_t)njobs * MAXD * 3;
  const bool whole = (int64_t)njobs * G.D >= 16 && G.n <= (1 << 18);
  const int limit = whole ? INT32_MAX : 256;
  hipLaunchKernelGGL(k_heur_persistent, dim3(1, G.D, njobs), dim3(NT_HP), 0, st, slots, slot_of,
                     G, hs, cnt, limit);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(cnt_host, cnt, nc * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return -1;
  int r0 = -1;  // the latest hand-over round (even, so every list is list A)
  for (size_t i = 0; i < nc; i += 3) {
    if (cnt_host[i + 1]) return -2;
    if (cnt_host[i] > 0) r0 = std::max(r0, cnt_host[i] - 1);
  }
  if (r0 >= 0) {
    // the grid-wide rounds resume at round r0 for all handed-over instances:
    // the count of round r0 sits in counter r0 % 3, the other two are zero;
    // the stamps left behind are all <= r0, so no node is kept out of a list
    int maxlen = 0;
    for (size_t i = 0; i < nc; i += 3) {
      const int32_t len = cnt_host[i] > 0 ? cnt_host[i + 2] : 0;
      cnt_host[i] = cnt_host[i + 1] = cnt_host[i + 2] = 0;
      cnt_host[i + r0 % 3] = len;
      maxlen = std::max(maxlen, len);
    }
    if (hipMemcpyAsync(cnt, cnt_host, nc * 4, hipMemcpyHostToDevice, st) != hipSuccess) return -1;
    // workgroups per instance: one worklist node per thread for four times the
    // longest worklist the host last saw (a round's grid-stride loop covers
    // any length; the size only sets the parallelism until the next look)
    const int gmax = std::max(1, std::min(512, (G.n / 8 + 255) / 256));
    const auto gx_for = [&](int64_t len) {
      return (int)std::max<int64_t>(1, std::min<int64_t>(gmax, (4 * len + NT_H - 1) / NT_H));
    };
    int gx = gx_for(maxlen);
    for (int r = r0;; ++r) {
      launch_heur_round(slots, slot_of, njobs, G, hs, cnt, r, gx, st);
      if ((r & 7) == 7) {
        if (hipMemcpyAsync(cnt_host, cnt, nc * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
          return -1;
        // after round r the worklist of round r + 1 is in counter (r + 1) % 3
        maxlen = 0;
        for (size_t i = (r + 1) % 3; i < nc; i += 3) maxlen = std::max(maxlen, cnt_host[i]);
        if (maxlen == 0) break;
        gx = gx_for(maxlen);
      }
      if (r > 4 * G.n + 64) return -2;
    }
  }
  launch_heur_clamp(slots, slot_of, njobs, G, st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

void launch_open_min(const Slot* slots, int s, int32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_open_min, dim3(1), dim3(1024), 0, st, slots, s, out);
}

void launch_path_len(const Slot* slots, int s, const int32_t* labs, int np, int32_t* len,
                     hipStream_t st) {
  const int gx = std::max(1, std::min(1024, (np + 255) / 256));
  hipLaunchKernelGGL(k_path_len, dim3(gx), dim3(256), 0, st, slots, s, labs, np, len);
}

void launch_path_write(const Slot* slots, int s, const int32_t* labs, int np, const int64_t* off,
                       int32_t* arcs, hipStream_t st) {
  const int gx = std::max(1, std::min(1024, (np + 255) / 256));
  hipLaunchKernelGGL(k_path_write, dim3(gx), dim3(256), 0, st, slots, s, labs, np, off, arcs);
}

}  // namespace mos
