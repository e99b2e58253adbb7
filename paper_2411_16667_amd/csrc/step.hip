// The batched label step on gfx950: one pass of the search over every resident query.
//
// A step follows the paper's Algorithm 1 body (NAMOA*), applied to a batch of
// labels popped in lexicographic order as Algorithm 2 (OPMOS) does:
//   pop     k_open_hist, k_open_threshold, k_open_scatter, k_batch_finalize
//           (the B lexicographically smallest live OPEN labels; labels pruned
//           since they were queued are skipped lazily, Section 5.1)
//   goal    k_goal_merge   (Algorithm 1 lines 11-13: P <- minimal(P + goal labels))
//   expand  k_expand       (lines 15-17: g' = g + c, F' = g' + h; lines 19/29:
//                           drop F' that the goal front weakly dominates)
//   group   k_group_count, k_group_offsets, k_group_scatter (candidates by target node)
//   check   k_group_process (candidates of one node against each other and
//           against the node's frontier: lines 22-28, fused in one read of the
//           frontier, which is compacted and extended in the same pass)
//   insert  k_accept_scan, k_insert, k_step_end (lines 20-21 / 30-31)
//
// All arithmetic is exact int32.  Tiled kernels run on a (gx, slots) grid and
// grid-stride over the slot's items; per-slot kernels run one 1024-thread
// workgroup per slot.
#include "kernels.h"

namespace mos {

constexpr int NT_SLOT = 1024;  // threads of the one-workgroup-per-slot kernels
constexpr int NT_TILE = 256;   // threads of the tiled kernels
constexpr int GP_WAVES = NT_TILE / WAVE;

// Exclusive scan of one value per thread across a workgroup of NT threads.
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

// Exclusive scan of flags[0..n) into out[0..n) by one workgroup; returns the total.
template <int NT>
__device__ int block_scan_array(const int32_t* in, int32_t* out, int n, int* tmp) {
  int carry = 0;
  for (int base = 0; base < n; base += NT) {
    int i = base + threadIdx.x;
    int v = i < n ? in[i] : 0;
    int tot;
    int ex = block_exscan<NT>(v, &tot, tmp);
    if (i < n) out[i] = carry + ex;
    carry += tot;
  }
  return carry;
}

// ---------------------------------------------------------------- pop
// Histogram of live OPEN entries over F1 (bin = F1 - lo, width 1, last bin = overflow).
__global__ __launch_bounds__(NT_TILE) void k_open_hist(Slot* slots, int32_t* hist) {
  Slot* S = &slots[blockIdx.y];
  if (S->status != S_RUN) return;
  const int n = S->open_n;
  if ((int)(blockIdx.x * NT_TILE) >= n) return;
  __shared__ int32_t h[NB];
  for (int i = threadIdx.x; i < NB; i += NT_TILE) h[i] = 0;
  __syncthreads();
  const int sel = S->open_sel, lo = S->lo;
  const int32_t* F1 = S->open_f1[sel];
  const int32_t* LB = S->open_lab[sel];
  const uint8_t* st = S->Lstate;
  int mn = INT32_MAX;
  for (int i = blockIdx.x * NT_TILE + threadIdx.x; i < n; i += gridDim.x * NT_TILE) {
    if (st[LB[i]] == L_OPEN) {
      int f = F1[i];
      int b = min(max(f - lo, 0), NB - 1);
      atomicAdd(&h[b], 1);
      mn = min(mn, f);
    }
  }
  mn = wave_min(mn);
  if (lane_id() == 0 && mn != INT32_MAX) atomicMin(&S->cur_min, mn);
  __syncthreads();
  int32_t* gh = hist + (size_t)blockIdx.y * NB;
  for (int i = threadIdx.x; i < NB; i += NT_TILE)
    if (h[i]) atomicAdd(&gh[i], h[i]);
}

// Pick the threshold bin: bins below t_star are popped whole; r_tie entries of
// bin t_star are taken in exact lexicographic order (tie_mode).
__global__ __launch_bounds__(NT_SLOT) void k_open_threshold(Slot* slots, int32_t* hist) {
  Slot* S = &slots[blockIdx.x];
  if (S->status != S_RUN) return;
  __shared__ int32_t cum[NB];
  __shared__ int tmp[NT_SLOT / WAVE];
  int32_t* gh = hist + (size_t)blockIdx.x * NB;
  constexpr int PER = NB / NT_SLOT;
  int loc[PER], s = 0;
  for (int j = 0; j < PER; ++j) {
    loc[j] = gh[threadIdx.x * PER + j];
    s += loc[j];
  }
  int total;
  int ex = block_exscan<NT_SLOT>(s, &total, tmp);
  for (int j = 0; j < PER; ++j) {
    ex += loc[j];
    cum[threadIdx.x * PER + j] = ex;  // inclusive
    gh[threadIdx.x * PER + j] = 0;    // reset for the next step
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int B = S->B;
    int t_star = NB, r = 0, mode = 0, rebase = 0;
    if (total > B) {
      int lo_i = 0, hi_i = NB - 1;  // first bin with cum >= B
      while (lo_i < hi_i) {
        int mid = (lo_i + hi_i) >> 1;
        if (cum[mid] >= B) hi_i = mid; else lo_i = mid + 1;
      }
      int t = lo_i;
      int below = t > 0 ? cum[t - 1] : 0;
      int inbin = cum[t] - below;
      r = B - below;
      if (r == inbin) {
        t_star = t + 1; r = 0;
      } else if (inbin <= TIECAP && inbin <= S->tie_cap) {
        t_star = t; mode = 1;
      } else if (below > 0) {
        t_star = t; r = 0;  // pop the bins below only: still an exact lexicographic prefix
      } else if (t < NB - 1 && inbin <= S->batch_cap) {
        t_star = t + 1; r = 0;  // the whole lowest F1 value: an exact prefix, larger than B
      } else if (t == NB - 1) {
        t_star = 0; r = 0; rebase = 1;  // every live entry lies far above lo: re-anchor, pop nothing
      } else {
        S->status = S_TIE;
        S->err_line = __LINE__;
      }
    }
    S->t_star = t_star;
    S->r_tie = r;
    S->tie_mode = mode;
    S->rebase = rebase;
    S->batch_n = 0;
    S->tie_n = 0;
    S->keep_n = 0;
    S->lo_next = INT32_MAX;
  }
}

// Route every live OPEN entry: popped (bin < t_star), tie (bin == t_star in
// tie mode) or kept (into the other OPEN buffer).  Dead entries vanish here.
__global__ __launch_bounds__(NT_TILE) void k_open_scatter(Slot* slots) {
  Slot* S = &slots[blockIdx.y];
  if (S->status != S_RUN) return;
  const int n = S->open_n;
  const int sel = S->open_sel, lo = S->lo, t_star = S->t_star, mode = S->tie_mode;
  const int32_t* F1 = S->open_f1[sel];
  const int32_t* LB = S->open_lab[sel];
  int32_t* KF = S->open_f1[sel ^ 1];
  int32_t* KL = S->open_lab[sel ^ 1];
  const uint8_t* st = S->Lstate;
  const int bcap = S->batch_cap, tcap = S->tie_cap, ocap = S->open_cap;
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
      live = st[lab] == L_OPEN;
    }
    const int b = min(max(f - lo, 0), NB - 1);
    const bool to_batch = live && b < t_star;
    const bool to_tie = live && mode && b == t_star;
    const bool to_keep = live && !to_batch && !to_tie;
    int p = agg_append(&S->batch_n, to_batch);
    if (to_batch && p < bcap) S->batch[p] = lab;
    p = agg_append(&S->tie_n, to_tie);
    if (to_tie && p < tcap) {
      S->tie_f1[p] = f;
      S->tie_lab[p] = lab;
    }
    p = agg_append(&S->keep_n, to_keep);
    if (to_keep && p < ocap) {
      KF[p] = f;
      KL[p] = lab;
      kmin = min(kmin, f);
    }
  }
  kmin = wave_min(kmin);
  if (lane_id() == 0 && kmin != INT32_MAX) atomicMin(&S->lo_next, kmin);
}

// Lexicographic key of a label: F_1..F_d, then node.
__device__ __forceinline__ void label_key(const Slot* S, const GraphDev& G, int lab, int32_t* key) {
  const int d = S->d;
  const int v = S->Lnode[lab];
  const int pc = S->pool_cap;
  for (int k = 0; k < d; ++k) key[k] = S->Lg[(size_t)k * pc + lab] + S->h[(size_t)k * G.n + v];
  key[d] = v;
}

// Finish the pop: exact selection inside the tie bin, canonical batch order
// (ascending label id), goal/regular split, out-degree prefix of the regular labels.
__global__ __launch_bounds__(NT_SLOT) void k_batch_finalize(Slot* slots, GraphDev G) {
  Slot* S = &slots[blockIdx.x];
  if (S->status != S_RUN) return;
  __shared__ int32_t lds[10240];
  __shared__ int tmp[NT_SLOT / WAVE];
  __shared__ int sh_base;
  const int d = S->d;
  if (S->tie_mode) {
    // ---- tie bin: order by (F_1..F_d, node), take the first r_tie
    const int n = min(S->tie_n, TIECAP);
    int n2 = 1;
    while (n2 < n) n2 <<= 1;
    int32_t* K = lds;               // (d+1) planes of TIECAP
    int32_t* idx = lds + 9 * TIECAP;
    for (int i = threadIdx.x; i < n2; i += NT_SLOT) {
      int32_t key[MAXD + 1];
      if (i < n) {
        label_key(S, G, S->tie_lab[i], key);
      } else {
        for (int k = 0; k <= d; ++k) key[k] = INT32_MAX;
      }
      for (int k = 0; k <= d; ++k) K[k * TIECAP + i] = key[k];
      idx[i] = i;
    }
    __syncthreads();
    for (int kk = 2; kk <= n2; kk <<= 1) {
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < n2; i += NT_SLOT) {
          int ixj = i ^ j;
          if (ixj > i) {
            int a = idx[i], b = idx[ixj];
            // lexicographic less(b, a)
            int c = 0;
            for (int k = 0; k <= d && c == 0; ++k) {
              int ka = K[k * TIECAP + a], kb = K[k * TIECAP + b];
              c = (kb < ka) ? 1 : (kb > ka ? -1 : 0);
            }
            bool b_less = c == 1;
            bool asc = (i & kk) == 0;
            if (asc ? b_less : (c == -1)) {
              idx[i] = b;
              idx[ixj] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    const int r = S->r_tie;
    const int nb0 = S->batch_n;
    int32_t* KF = S->open_f1[S->open_sel ^ 1];
    int32_t* KL = S->open_lab[S->open_sel ^ 1];
    int kmin = INT32_MAX;
    for (int i = threadIdx.x; i < n; i += NT_SLOT) {
      int e = idx[i];
      if (i < r) {
        int p = nb0 + i;
        if (p < S->batch_cap) S->batch[p] = S->tie_lab[e];
      } else {
        int p = S->keep_n + (i - r);
        if (p < S->open_cap) {
          KF[p] = S->tie_f1[e];
          KL[p] = S->tie_lab[e];
        }
        kmin = min(kmin, S->tie_f1[e]);
      }
    }
    kmin = wave_min(kmin);
    if (lane_id() == 0 && kmin != INT32_MAX) atomicMin(&S->lo_next, kmin);
    __syncthreads();
    if (threadIdx.x == 0) {
      S->batch_n = nb0 + min(r, n);
      S->keep_n += max(n - r, 0);
    }
    __syncthreads();
  }
  // ---- canonical batch order: ascending label id
  int nb = S->batch_n;
  if (nb > S->batch_cap || nb > BATCH_SORT || S->keep_n > S->open_cap) {
    if (threadIdx.x == 0) {
      S->status = S_OVERFLOW;
      S->err_line = __LINE__;
    }
    return;
  }
  int n2 = 1;
  while (n2 < nb) n2 <<= 1;
  int32_t* V = lds;
  for (int i = threadIdx.x; i < n2; i += NT_SLOT) V[i] = i < nb ? S->batch[i] : INT32_MAX;
  __syncthreads();
  for (int kk = 2; kk <= n2; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += NT_SLOT) {
        int ixj = i ^ j;
        if (ixj > i) {
          int a = V[i], b = V[ixj];
          bool asc = (i & kk) == 0;
          if (asc ? (b < a) : (a < b)) {
            V[i] = b;
            V[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  // ---- split into goal and regular labels (stable), mark them closed
  const int goal = S->goal;
  int goal_total = 0, reg_total = 0, deg_carry = 0;
  for (int base = 0; base < nb; base += NT_SLOT) {
    int i = base + threadIdx.x;
    bool valid = i < nb;
    int lab = valid ? V[i] : 0;
    int v = valid ? S->Lnode[lab] : 0;
    bool isg = valid && v == goal;
    bool isr = valid && !isg;
    int deg = isr ? (G.row_ptr[v + 1] - G.row_ptr[v]) : 0;
    if (valid) S->Lstate[lab] = L_CLOSED;
    int tg, tr, td;
    int pg = block_exscan<NT_SLOT>(isg ? 1 : 0, &tg, tmp);
    int pr = block_exscan<NT_SLOT>(isr ? 1 : 0, &tr, tmp);
    int pd = block_exscan<NT_SLOT>(deg, &td, tmp);
    if (isg) S->goal_lab[goal_total + pg] = lab;
    if (isr) {
      S->reg[reg_total + pr] = lab;
      S->reg_off[reg_total + pr] = deg_carry + pd;
    }
    goal_total += tg;
    reg_total += tr;
    deg_carry += td;
  }
  if (threadIdx.x == 0) {
    S->reg_off[reg_total] = deg_carry;
    S->goal_n = goal_total;
    S->reg_n = reg_total;
    S->cand_n = deg_carry;
    S->ngroups = 0;
    S->accept_n = 0;
    S->st[ST_POPS] += nb;
    S->st[ST_GOAL_POPS] += goal_total;
    if (deg_carry > S->cand_cap) {
      S->status = S_OVERFLOW;
      S->err_line = __LINE__;
    } else if (nb == 0 && !S->rebase) {
      S->status = S_DONE;  // no live label left in OPEN
    }
  }
}

// ---------------------------------------------------------------- goal step
// P <- minimal(P ∪ G) for the goal labels G popped this step (Algorithm 1
// lines 11-13).  A goal label is dropped if an old P entry weakly dominates it
// or another goal label dominates it (equal vectors: the smaller label id
// stays); an old entry is dropped if some goal label strictly dominates it.
// The new front is written lexicographically sorted into the other buffer.
__global__ __launch_bounds__(NT_SLOT) void k_goal_merge(Slot* slots) {
  Slot* S = &slots[blockIdx.x];
  if (S->status != S_RUN || S->goal_n == 0) return;
  constexpr int GT = 256;  // goal labels per pass
  __shared__ int32_t gv[MAXD][GT];
  __shared__ int32_t glab[GT];
  __shared__ int32_t gacc[GT];
  __shared__ int tmp[NT_SLOT / WAVE];
  const int d = S->d, pc = S->pool_cap, Pc = S->P_cap;
  const int ng = S->goal_n;
  const int np = S->P_n;
  const int32_t* Pg = S->Pg[S->P_sel];
  const int32_t* Pl = S->Plab[S->P_sel];
  int32_t* Qg = S->Pg[S->P_sel ^ 1];
  int32_t* Ql = S->Plab[S->P_sel ^ 1];
  // Scratch: prune flags of old P entries and their survivor prefix; the
  // accepted goal labels are collected in `batch` (free after the pop).
  int32_t* pflag = S->pscr;
  int32_t* sprefix = S->pscr + (Pc + 1);
  int32_t* acc_lab = S->batch;
  if (np + ng > Pc) {
    if (threadIdx.x == 0) {
      S->status = S_OVERFLOW;
      S->err_line = __LINE__;
    }
    return;
  }
  for (int i = threadIdx.x; i < np; i += NT_SLOT) pflag[i] = 0;
  int na = 0;
  int64_t pairs = 0;
  for (int t0 = 0; t0 < ng; t0 += GT) {
    const int nt = min(GT, ng - t0);
    __syncthreads();
    if (threadIdx.x < nt) {
      int lab = S->goal_lab[t0 + threadIdx.x];
      glab[threadIdx.x] = lab;
      for (int k = 0; k < d; ++k) gv[k][threadIdx.x] = S->Lg[(size_t)k * pc + lab];
      gacc[threadIdx.x] = 1;
    }
    __syncthreads();
    // old P entries: pruned if a goal label of this tile strictly dominates them;
    // goal labels rejected if an old entry weakly dominates them.
    for (int i = threadIdx.x; i < np; i += NT_SLOT) {
      int32_t p[MAXD];
      for (int k = 0; k < d; ++k) p[k] = Pg[(size_t)k * Pc + i];
      bool pruned = false;
      for (int j = 0; j < nt; ++j) {
        bool le = true, gl = true, anylt = false;
        for (int k = 0; k < d; ++k) {
          int gk = gv[k][j];
          le = le && (p[k] <= gk);
          gl = gl && (gk <= p[k]);
          anylt = anylt || (gk < p[k]);
        }
        if (le) gacc[j] = 0;  // benign race: every writer stores 0
        if (gl && anylt) pruned = true;
      }
      if (pruned) pflag[i] = 1;
    }
    __syncthreads();
    // goal labels against every goal label (all tiles)
    if (threadIdx.x < nt && gacc[threadIdx.x]) {
      const int me = threadIdx.x;
      int32_t a[MAXD];
      for (int k = 0; k < d; ++k) a[k] = gv[k][me];
      const int mylab = glab[me];
      bool rej = false;
      for (int j = 0; j < ng && !rej; ++j) {
        const int lb = S->goal_lab[j];
        if (lb == mylab) continue;
        bool le = true, eq = true;
        for (int k = 0; k < d; ++k) {
          int bk = S->Lg[(size_t)k * pc + lb];
          le = le && (bk <= a[k]);
          eq = eq && (bk == a[k]);
        }
        if (le && (!eq || lb < mylab)) rej = true;
      }
      if (rej) gacc[me] = 0;
    }
    __syncthreads();
    // append the accepted goal labels of this tile to acc_lab (ascending label id)
    int v = (threadIdx.x < nt) ? gacc[threadIdx.x] : 0;
    int tot;
    int pos = block_exscan<NT_SLOT>(v, &tot, tmp);
    if (v) acc_lab[na + pos] = glab[threadIdx.x];
    na += tot;
    pairs += (int64_t)nt * np + (int64_t)nt * ng;
  }
  __syncthreads();
  // survivors of old P: exclusive prefix (stored in the batch scratch `reg_off`? no: reuse c_rank)
  int carry = 0;
  for (int base = 0; base < np; base += NT_SLOT) {
    int i = base + threadIdx.x;
    int alive = (i < np && !pflag[i]) ? 1 : 0;
    int tot;
    int ex = block_exscan<NT_SLOT>(alive, &tot, tmp);
    if (i < np) sprefix[i] = carry + ex;
    carry += tot;
  }
  const int nsurv = carry;
  __syncthreads();
  if (threadIdx.x == 0) sprefix[np] = nsurv;
  __syncthreads();
  // output positions: old survivor i -> sprefix[i] + #(accepted goal vectors < it)
  //                   accepted goal j -> #(old survivors < it) + #(accepted goal vectors < it)
  // (vectors are pairwise distinct across the two lists after the filtering above)
  auto lexless = [&](const int32_t* a, const int32_t* b) {
    for (int k = 0; k < d; ++k)
      if (a[k] != b[k]) return a[k] < b[k];
    return false;
  };
  // Write old survivors into the other buffer.
  for (int base = 0; base < np; base += NT_SLOT) {
    int i = base + threadIdx.x;
    bool alive = i < np && !pflag[i];
    int32_t p[MAXD];
    int lab = 0, outpos = 0;
    if (alive) {
      for (int k = 0; k < d; ++k) p[k] = Pg[(size_t)k * Pc + i];
      lab = Pl[i];
      int c = 0;
      for (int j = 0; j < na; ++j) {
        int32_t q[MAXD];
        const int lb = acc_lab[j];
        for (int k = 0; k < d; ++k) q[k] = S->Lg[(size_t)k * pc + lb];
        if (lexless(q, p)) ++c;
      }
      outpos = sprefix[i] + c;
    }
    if (alive) {
      for (int k = 0; k < d; ++k) Qg[(size_t)k * Pc + outpos] = p[k];
      Ql[outpos] = lab;
    }
  }
  // accepted goal labels
  for (int j = threadIdx.x; j < na; j += NT_SLOT) {
    const int lb = acc_lab[j];
    int32_t q[MAXD];
    for (int k = 0; k < d; ++k) q[k] = S->Lg[(size_t)k * pc + lb];
    // #old survivors lexicographically below q: binary search in old P, then sprefix
    int lo_i = 0, hi_i = np;
    while (lo_i < hi_i) {
      int mid = (lo_i + hi_i) >> 1;
      int32_t p[MAXD];
      for (int k = 0; k < d; ++k) p[k] = Pg[(size_t)k * Pc + mid];
      if (lexless(p, q)) lo_i = mid + 1; else hi_i = mid;
    }
    int c = 0;
    for (int i = 0; i < na; ++i) {
      if (i == j) continue;
      const int lb2 = acc_lab[i];
      int32_t r[MAXD];
      for (int k = 0; k < d; ++k) r[k] = S->Lg[(size_t)k * pc + lb2];
      if (lexless(r, q)) ++c;
    }
    int outpos = sprefix[lo_i] + c;
    for (int k = 0; k < d; ++k) Qg[(size_t)k * Pc + outpos] = q[k];
    Ql[outpos] = lb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    S->P_n = nsurv + na;
    S->P_sel ^= 1;
    S->st[ST_PPAIRS] += pairs;
  }
}

// ---------------------------------------------------------------- expand + P filter
__global__ __launch_bounds__(NT_TILE) void k_expand(Slot* slots, GraphDev G) {
  Slot* S = &slots[blockIdx.y];
  if (S->status != S_RUN) return;
  const int M = S->cand_n;
  if ((int)(blockIdx.x * NT_TILE) >= M) return;
  constexpr int PT = NT_TILE;
  __shared__ int32_t ps[MAXD][PT];
  const int d = S->d, pc = S->pool_cap, cc = S->cand_cap, n = G.n;
  const int reg_n = S->reg_n;
  const int np = S->P_n;
  const int32_t* Pg = S->Pg[S->P_sel];
  const int Pc = S->P_cap;
  int64_t ncand = 0, npairs = 0;
  for (int base = blockIdx.x * NT_TILE; base < M; base += gridDim.x * NT_TILE) {
    const int f = base + threadIdx.x;
    const bool valid = f < M;
    bool alive = false;
    int32_t g[MAXD], F[MAXD];
    int v = 0, lab = 0, e = 0;
    if (valid) {
      // regular label owning flat index f: last j with reg_off[j] <= f
      int lo_i = 0, hi_i = reg_n - 1;
      while (lo_i < hi_i) {
        int mid = (lo_i + hi_i + 1) >> 1;
        if (S->reg_off[mid] <= f) lo_i = mid; else hi_i = mid - 1;
      }
      lab = S->reg[lo_i];
      const int u = S->Lnode[lab];
      e = G.row_ptr[u] + (f - S->reg_off[lo_i]);
      v = G.col[e];
      alive = true;
      for (int k = 0; k < d; ++k) {
        int hk = S->h[(size_t)k * n + v];
        if (hk == UNREACH) alive = false;
        g[k] = S->Lg[(size_t)k * pc + lab] + G.cost[(size_t)k * G.m + e];
        F[k] = g[k] + (hk == UNREACH ? 0 : hk);
      }
      ncand++;
      if (alive) npairs += np;
    }
    // goal-front filter: drop F' weakly dominated by some P entry
    for (int p0 = 0; p0 < np; p0 += PT) {
      const int npt = min(PT, np - p0);
      __syncthreads();
      if ((int)threadIdx.x < npt)
        for (int k = 0; k < d; ++k) ps[k][threadIdx.x] = Pg[(size_t)k * Pc + p0 + threadIdx.x];
      __syncthreads();
      if (alive) {
        for (int q = 0; q < npt; ++q) {
          bool le = true;
          for (int k = 0; k < d; ++k) le = le && (ps[k][q] <= F[k]);
          if (le) {
            alive = false;
            break;
          }
        }
      }
    }
    if (valid) {
      S->c_node[f] = v;
      S->c_par[f] = lab;
      S->c_arc[f] = e;
      for (int k = 0; k < d; ++k) S->c_g[(size_t)k * cc + f] = g[k];
      S->c_keep[f] = alive ? 1 : 0;
      S->c_rej[f] = 0;
      S->c_acc[f] = 0;
    }
  }
  ncand = wave_sum64(ncand);
  npairs = wave_sum64(npairs);
  if (lane_id() == 0) {
    if (ncand) atomicAdd((unsigned long long*)&S->st[ST_CANDS], (unsigned long long)ncand);
    if (npairs) atomicAdd((unsigned long long*)&S->st[ST_PPAIRS], (unsigned long long)npairs);
  }
}

// ---------------------------------------------------------------- group by target node
__global__ __launch_bounds__(NT_TILE) void k_group_count(Slot* slots) {
  Slot* S = &slots[blockIdx.y];
  if (S->status != S_RUN) return;
  const int M = S->cand_n;
  for (int f = blockIdx.x * NT_TILE + threadIdx.x; f < M; f += gridDim.x * NT_TILE) {
    if (!S->c_keep[f]) continue;
    const int v = S->c_node[f];
    const int r = atomicAdd(&S->grp_cnt[v], 1);
    S->c_rank[f] = r;
    if (r == 0) {
      const int gid = atomicAdd(&S->ngroups, 1);
      S->grp_node[gid] = v;
      S->grp_id[v] = gid;
    }
  }
}

__global__ __launch_bounds__(NT_SLOT) void k_group_offsets(Slot* slots) {
  Slot* S = &slots[blockIdx.x];
  if (S->status != S_RUN) return;
  __shared__ int tmp[NT_SLOT / WAVE];
  const int ng = S->ngroups;
  int carry = 0;
  for (int base = 0; base < ng; base += NT_SLOT) {
    int i = base + threadIdx.x;
    int sz = i < ng ? S->grp_cnt[S->grp_node[i]] : 0;
    int tot;
    int ex = block_exscan<NT_SLOT>(sz, &tot, tmp);
    if (i < ng) S->grp_off[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) S->st[ST_GROUPS] += ng;
}

__global__ __launch_bounds__(NT_TILE) void k_group_scatter(Slot* slots) {
  Slot* S = &slots[blockIdx.y];
  if (S->status != S_RUN) return;
  const int M = S->cand_n;
  for (int f = blockIdx.x * NT_TILE + threadIdx.x; f < M; f += gridDim.x * NT_TILE) {
    if (!S->c_keep[f]) continue;
    const int gid = S->grp_id[S->c_node[f]];
    S->order[S->grp_off[gid] + S->c_rank[f]] = f;
  }
}

// ---------------------------------------------------------------- frontier check
// One wave per group (all candidates of this step with the same target node v):
//  A. candidates against each other: c_i is dropped if some c_j <= c_i in every
//     objective and (c_j != c_i or j precedes i in flat order);
//  B. survivors against the live frontier of v, 64 frontier entries per lane
//     tile, every entry loaded once: a candidate is rejected if an entry
//     weakly dominates it (dominated or duplicate, Algorithm 1 lines 22-25);
//     an entry is pruned if a survivor strictly dominates it (lines 26-28; a
//     rejected candidate can dominate no live entry because the frontier is an
//     antichain); pruned entries are marked dead in the pool and the block is
//     compacted as it is streamed;
//  C. accepted candidates are appended (a larger block is taken when needed).
__global__ __launch_bounds__(NT_TILE) void k_group_process(Slot* slots) {
  Slot* S = &slots[blockIdx.y];
  if (S->status != S_RUN) return;
  const int ngroups = S->ngroups;
  const int wave = threadIdx.x / WAVE, lane = lane_id();
  __shared__ int32_t cg_all[GP_WAVES][MAXD][WAVE];
  __shared__ int32_t cf_all[GP_WAVES][WAVE];
  __shared__ int32_t cr_all[GP_WAVES][WAVE];
  int32_t(*cg)[WAVE] = cg_all[wave];
  int32_t* cf = cf_all[wave];
  int32_t* cr = cr_all[wave];
  const int d = S->d, cc = S->cand_cap;
  int32_t* fw = S->fw;
  int64_t gpairs = 0, fpairs = 0, fbytes = 0, pruned = 0;
  for (int gid = blockIdx.x * GP_WAVES + wave; gid < ngroups; gid += gridDim.x * GP_WAVES) {
    const int v = S->grp_node[gid];
    const int off = S->grp_off[gid];
    const int k = S->grp_cnt[v];
    int32_t* ord = S->order + off;
    // ---- A. intra-group resolution
    int ks = k;
    if (k > 1) {
      gpairs += (int64_t)k * (k - 1);
      for (int it = 0; it < k; it += WAVE) {
        const int i = it + lane;
        const bool have = i < k;
        const int fi = have ? ord[i] : 0;
        int32_t ci[MAXD];
        for (int kk = 0; kk < d; ++kk) ci[kk] = have ? S->c_g[(size_t)kk * cc + fi] : 0;
        bool rej = false;
        for (int jt = 0; jt < k; jt += WAVE) {
          const int j = jt + lane;
          wave_sync();
          if (j < k) {
            const int fj = ord[j];
            cf[lane] = fj;
            for (int kk = 0; kk < d; ++kk) cg[kk][lane] = S->c_g[(size_t)kk * cc + fj];
          }
          wave_sync();
          const int nj = min(WAVE, k - jt);
          if (have && !rej) {
            for (int jj = 0; jj < nj; ++jj) {
              if (jt + jj == i) continue;
              bool le = true, eq = true;
              for (int kk = 0; kk < d; ++kk) {
                const int b = cg[kk][jj];
                le = le && (b <= ci[kk]);
                eq = eq && (b == ci[kk]);
              }
              if (le && (!eq || cf[jj] < fi)) {
                rej = true;
                break;
              }
            }
          }
        }
        if (have && rej) S->c_rej[fi] = 1;
      }
      __threadfence_block();
      // compact survivors to the front of the group's order list (in place)
      int cur = 0;
      for (int it = 0; it < k; it += WAVE) {
        const int i = it + lane;
        const bool have = i < k;
        const int fi = have ? ord[i] : 0;
        const bool surv = have && !S->c_rej[fi];
        const uint64_t m = ballot(surv);
        wave_sync();
        if (surv) ord[cur + rank_below(m)] = fi;
        cur += __popcll(m);
      }
      ks = cur;
      __threadfence_block();
    }
    // ---- B. frontier check + prune + compaction
    const NodeRec nr = S->node[v];
    const int cnt = nr.count;
    int64_t doff = nr.off;
    int dcap = nr.cap;
    if (cnt + ks > nr.cap) {
      int nc = MINCAP;
      while (nc < cnt + ks) nc <<= 1;
      const int64_t words = (int64_t)nc * (d + 1);
      int64_t pos = 0;
      if (lane == 0) pos = (int64_t)atomicAdd((unsigned long long*)&S->fw_top, (unsigned long long)words);
      pos = __shfl(pos, 0);
      if (pos + words > S->fw_cap) {
        if (lane == 0) {
          S->status = S_OVERFLOW;
          S->err_line = __LINE__;
        }
        break;
      }
      doff = pos;
      dcap = nc;
    }
    const bool moved = doff != nr.off;
    fpairs += (int64_t)ks * cnt;
    fbytes += (int64_t)cnt * 4 * d;
    int cursor = 0;
    for (int t = 0; t < cnt; t += WAVE) {
      const int e = t + lane;
      const bool has = e < cnt;
      int32_t sv[MAXD];
      for (int kk = 0; kk < d; ++kk) sv[kk] = has ? fw[nr.off + (int64_t)kk * nr.cap + e] : 0;
      const int slab = has ? fw[nr.off + (int64_t)d * nr.cap + e] : 0;
      bool prune = false;
      for (int ct = 0; ct < ks; ct += WAVE) {
        const int j = ct + lane;
        wave_sync();
        if (j < ks) {
          const int fj = ord[j];
          cf[lane] = fj;
          cr[lane] = S->c_rej[fj];
          for (int kk = 0; kk < d; ++kk) cg[kk][lane] = S->c_g[(size_t)kk * cc + fj];
        }
        wave_sync();
        const int nj = min(WAVE, ks - ct);
        for (int jj = 0; jj < nj; ++jj) {
          if (cr[jj]) continue;  // uniform across the wave
          bool le = has, ge = has, lt = false;
          for (int kk = 0; kk < d; ++kk) {
            const int c = cg[kk][jj];
            le = le && (sv[kk] <= c);
            ge = ge && (c <= sv[kk]);
            lt = lt || (c < sv[kk]);
          }
          if (ballot(le)) {
            if (lane == 0) cr[jj] = 1;
            wave_sync();
          } else if (ge && lt) {
            prune = true;
          }
        }
        wave_sync();
        if (j < ks && cr[lane]) S->c_rej[cf[lane]] = 1;
      }
      if (prune) S->Lstate[slab] = L_DEAD;
      const uint64_t hm = ballot(has);
      const uint64_t am = ballot(has && !prune);
      pruned += __popcll(hm & ~am);
      if (moved || cursor != t || am != hm) {
        if (has && !prune) {
          const int64_t w = doff + cursor + rank_below(am);
          for (int kk = 0; kk < d; ++kk) fw[w + (int64_t)kk * dcap] = sv[kk];
          fw[w + (int64_t)d * dcap] = slab;
        }
      }
      cursor += __popcll(am);
    }
    __threadfence_block();
    // ---- C. append the accepted candidates
    for (int ct = 0; ct < ks; ct += WAVE) {
      const int j = ct + lane;
      const bool have = j < ks;
      const int fj = have ? ord[j] : 0;
      const bool acc = have && !S->c_rej[fj];
      const uint64_t m = ballot(acc);
      if (acc) {
        const int64_t w = doff + cursor + rank_below(m);
        for (int kk = 0; kk < d; ++kk) fw[w + (int64_t)kk * dcap] = S->c_g[(size_t)kk * cc + fj];
        fw[w + (int64_t)d * dcap] = -1;
        S->c_fslot[fj] = w + (int64_t)d * dcap;
        S->c_acc[fj] = 1;
      }
      cursor += __popcll(m);
    }
    if (lane == 0) {
      NodeRec out;
      out.off = doff;
      out.cap = dcap;
      out.count = cursor;
      S->node[v] = out;
      S->grp_cnt[v] = 0;
      S->grp_id[v] = -1;
    }
  }
  // the per-group totals are wave-uniform: lane 0 publishes them
  if (lane == 0) {
    if (gpairs) atomicAdd((unsigned long long*)&S->st[ST_GPAIRS], (unsigned long long)gpairs);
    if (fpairs) atomicAdd((unsigned long long*)&S->st[ST_FPAIRS], (unsigned long long)fpairs);
    if (fbytes) atomicAdd((unsigned long long*)&S->st[ST_FBYTES], (unsigned long long)fbytes);
    if (pruned) atomicAdd((unsigned long long*)&S->st[ST_PRUNED], (unsigned long long)pruned);
  }
}

// ---------------------------------------------------------------- insert
__global__ __launch_bounds__(NT_SLOT) void k_accept_scan(Slot* slots) {
  Slot* S = &slots[blockIdx.x];
  if (S->status != S_RUN) return;
  __shared__ int tmp[NT_SLOT / WAVE];
  const int M = S->cand_n;
  const int total = block_scan_array<NT_SLOT>(S->c_acc, S->c_rank, M, tmp);
  if (threadIdx.x == 0) {
    S->accept_n = total;
    if (S->n_labels + total > S->pool_cap || S->keep_n + total > S->open_cap) {
      S->status = S_OVERFLOW;
      S->err_line = __LINE__;
    }
  }
}

__global__ __launch_bounds__(NT_TILE) void k_insert(Slot* slots, GraphDev G) {
  Slot* S = &slots[blockIdx.y];
  if (S->status != S_RUN) return;
  const int M = S->cand_n;
  const int d = S->d, pc = S->pool_cap, cc = S->cand_cap;
  const int base_id = S->n_labels, keep = S->keep_n;
  int32_t* KF = S->open_f1[S->open_sel ^ 1];
  int32_t* KL = S->open_lab[S->open_sel ^ 1];
  int mn = INT32_MAX;
  for (int f = blockIdx.x * NT_TILE + threadIdx.x; f < M; f += gridDim.x * NT_TILE) {
    if (!S->c_acc[f]) continue;
    const int r = S->c_rank[f];
    const int id = base_id + r;
    const int v = S->c_node[f];
    S->Lnode[id] = v;
    S->Lpar[id] = S->c_par[f];
    S->Larc[id] = S->c_arc[f];
    S->Lstate[id] = L_OPEN;
    for (int k = 0; k < d; ++k) S->Lg[(size_t)k * pc + id] = S->c_g[(size_t)k * cc + f];
    S->fw[S->c_fslot[f]] = id;
    const int f1 = S->c_g[f] + S->h[v];
    KF[keep + r] = f1;
    KL[keep + r] = id;
    mn = min(mn, f1);
  }
  mn = wave_min(mn);
  if (lane_id() == 0 && mn != INT32_MAX) atomicMin(&S->lo_next, mn);
}

__global__ void k_step_end(Slot* slots, int nslots) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  Slot* S = &slots[s];
  if (S->status != S_RUN) return;
  S->n_labels += S->accept_n;
  S->st[ST_INSERTED] += S->accept_n;
  S->open_n = S->keep_n + S->accept_n;
  S->open_sel ^= 1;
  if (S->rebase) S->lo = S->cur_min;
  else if (S->open_n > 0) S->lo = S->lo_next;
  S->cur_min = INT32_MAX;
  S->st[ST_STEPS] += 1;
  if (S->open_n == 0) S->status = S_DONE;
}

// ---------------------------------------------------------------- launchers
void launch_step(const StepArgs& a, hipStream_t st) {
  const dim3 tiled(a.gx, a.nslots), per(a.nslots);
  hipLaunchKernelGGL(k_open_hist, tiled, dim3(NT_TILE), 0, st, a.slots, a.hist);
  hipLaunchKernelGGL(k_open_threshold, per, dim3(NT_SLOT), 0, st, a.slots, a.hist);
  hipLaunchKernelGGL(k_open_scatter, tiled, dim3(NT_TILE), 0, st, a.slots);
  hipLaunchKernelGGL(k_batch_finalize, per, dim3(NT_SLOT), 0, st, a.slots, a.G);
  hipLaunchKernelGGL(k_goal_merge, per, dim3(NT_SLOT), 0, st, a.slots);
  hipLaunchKernelGGL(k_expand, tiled, dim3(NT_TILE), 0, st, a.slots, a.G);
  hipLaunchKernelGGL(k_group_count, tiled, dim3(NT_TILE), 0, st, a.slots);
  hipLaunchKernelGGL(k_group_offsets, per, dim3(NT_SLOT), 0, st, a.slots);
  hipLaunchKernelGGL(k_group_scatter, tiled, dim3(NT_TILE), 0, st, a.slots);
  hipLaunchKernelGGL(k_group_process, tiled, dim3(NT_TILE), 0, st, a.slots);
  hipLaunchKernelGGL(k_accept_scan, per, dim3(NT_SLOT), 0, st, a.slots);
  hipLaunchKernelGGL(k_insert, tiled, dim3(NT_TILE), 0, st, a.slots, a.G);
  hipLaunchKernelGGL(k_step_end, dim3((a.nslots + 63) / 64), dim3(64), 0, st, a.slots, a.nslots);
}

}  // namespace mos
