// Per-query persistent step: one workgroup owns one resident query and runs
// its label steps back to back, up to a step count per launch, with workgroup
// barriers between the phases of a step and no launch per phase or per step.
// It serves short queries, whose steps are too small to fill the chip and
// would otherwise pay the fixed cost of the multi-kernel step (one launch per
// phase) on every step.
//
// The search is the same method (paper, Algorithm 1 with the batched
// extraction of Section 5: pop a batch, expand, test each candidate against
// the labels of its node and the other candidates, prune, insert), kept in the
// query's own slot (pool, frontier blocks, OPEN buffers, goal front), with
// these choices, all of which leave the front unchanged:
//   * the batch is every live OPEN label with F1 below a threshold, the
//     largest that keeps the batch within its width (a histogram of F1 over
//     OPEN, refined inside the first bin when that bin alone is too wide);
//     when more labels share the smallest F1 than a batch holds, it is those
//     of them whose node id lies below a second threshold;
//   * the goal front is the frontier of the goal node: a candidate at the goal
//     is tested and inserted like any other and prunes the entries it
//     dominates, so the front stays an antichain and no goal label waits in
//     OPEN (the eager form of the goal step);
//   * a popped label is dropped when the goal front weakly dominates its F
//     (g + h; h is admissible), and a candidate whose node cannot reach the
//     goal is dropped;
//   * among candidates of one node, one is rejected by another that weakly
//     dominates it (equal vectors: the smaller arc id stays), or by a label of
//     the node that weakly dominates it; an accepted candidate removes the
//     node's labels it dominates.
// No decision depends on label ids or on the order of items in a buffer, so
// the result (costs and witness paths) does not depend on timing.
//
// A query whose step outgrows what one workgroup holds (one node with more
// labels of the smallest F1 than the batch width, or an out-degree too large
// for the candidate arrays) leaves with S_SOLO_QUIT and is run again by the
// multi-kernel step.
//
// Measured against the multi-kernel step, this form is slower on every
// workload tried (short ship-grid queries, batched or alone, and the served
// road-like workload): one compute unit per query cannot keep up with a step
// of hundreds of labels and thousands of candidates, and the multi-kernel
// step already shares its fixed launch cost among all resident queries and
// widens the batch of the last ones.  It stays an option, off by default.
#include "kernels.h"

namespace mos {

constexpr int SO_NT = 1024;
constexpr int SO_WAVES = SO_NT / WAVE;
constexpr int SO_BINS = 2048;   // F1 histogram bins of the batch threshold
constexpr int SO_CANDS = 8192;   // largest candidate set of one step

#define SFOR_K(k) _Pragma("unroll") for (int k = 0; k < DM; ++k) if (k < d)

// Exclusive scan of one value per thread of the workgroup; *total receives
// the sum.  Every thread calls it (it holds workgroup barriers).
__device__ __forceinline__ int so_exscan(int v, int* wsum, int* total) {
  int x = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane_id() >= o) x += y;
  }
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane_id() == WAVE - 1) wsum[w] = x;
  __syncthreads();
  int before = 0, all = 0;
  for (int u = 0; u < SO_WAVES; ++u) {
    const int s = wsum[u];
    before += u < w ? s : 0;
    all += s;
  }
  *total = all;
  return before + x - v;
}

__device__ __forceinline__ int wave_max_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// After the workgroup filled hist[SO_BINS]: the last bin whose running count
// stays within cap (SO_BINS - 1 when all do, -1 when the first bin alone
// exceeds it); *first gets the first non-empty bin.  Every thread calls it
// (it holds workgroup barriers).
__device__ __forceinline__ int so_pick(const int* hist, int cap, int* s_out, int* first) {
  __syncthreads();
  if (threadIdx.x < WAVE) {
    constexpr int PER = SO_BINS / WAVE;
    const int ln = lane_id();
    int c = 0;
    for (int q = 0; q < PER; ++q) c += hist[ln * PER + q];
    int x = c;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (ln >= o) x += y;
    }
    const uint64_t over = ballot(x > cap);
    int bstar = SO_BINS - 1;
    if (over) {
      const int L = __ffsll((long long)over) - 1;
      int res = -1;
      if (ln == L) {
        int cum = x - c;
        for (int q = 0; q < PER; ++q) {
          cum += hist[L * PER + q];
          if (cum > cap) break;
          res = L * PER + q;
        }
      }
      bstar = __shfl(res, L);
    }
    const uint64_t nz = ballot(c > 0);
    int fb = SO_BINS;
    if (nz) {
      const int L0 = __ffsll((long long)nz) - 1;
      int r0 = 0;
      if (ln == L0)
        for (int q = PER - 1; q >= 0; --q)
          if (hist[L0 * PER + q] > 0) r0 = L0 * PER + q;
      fb = __shfl(r0, L0);
    }
    if (ln == 0) {
      s_out[0] = bstar;
      s_out[1] = fb;
    }
  }
  __syncthreads();
  const int r = s_out[0];
  *first = s_out[1];
  __syncthreads();  // every thread has read them before they are written again
  return r;
}

enum SoloFlag : int { SO_RUN = 0, SO_OVERFLOW = 2, SO_QUIT = 3 };

template <int DM>
__global__ __launch_bounds__(SO_NT) void k_solo(Slot* slots, GraphDev G, int max_steps) {
  Slot* Sp = &slots[blockIdx.x];
  if (Sp->status != S_SOLO) return;

  __shared__ int hist[SO_BINS];
  __shared__ uint8_t acc8[SO_CANDS];  // large groups: survivor flag per grouped candidate position
  __shared__ int wsum[SO_WAVES];
  __shared__ int s_open_n, s_sel, s_keep, s_nb, s_nvalid, s_nlab, s_flag, s_ng, s_ni;
  __shared__ int s_pick[2];
  __shared__ int s_fmin, s_fmax, s_nmin, s_nmax;
  __shared__ int s_pops, s_killed, s_cands, s_ins, s_pruned, s_steps;
  __shared__ unsigned long long s_fwtop;

  const int d = Sp->d, n = G.n, m = G.m, goal = Sp->goal;
  const int pool_cap = Sp->pool_cap, open_cap = Sp->open_cap, cand_cap = Sp->cand_cap;
  const int64_t fw_cap = Sp->fw_cap;
  const int32_t* h = Sp->h;
  NodeRec* node = Sp->node;
  int32_t* Lnode = Sp->Lnode;
  int32_t* Lpar = Sp->Lpar;
  int32_t* Larc = Sp->Larc;
  int32_t* Lg = Sp->Lg;
  uint8_t* Lstate = Sp->Lstate;
  int32_t* fw = Sp->fw;
  int32_t* batch = Sp->batch;
  int32_t* c_par = Sp->c_par;
  int32_t* c_arc = Sp->c_arc;
  int32_t* c_g = Sp->c_g;
  int32_t* grp_off = Sp->small_list;  // cand_cap + 1 entries: group starts and the end
  int32_t* items = Sp->big_list;      // frontier-test work items: group * 128 + chunk
  int32_t* order = Sp->order;         // candidates grouped by node
  int32_t* grp_node = Sp->grp_node;
  int32_t* grp_cnt = Sp->grp_cnt;     // n: candidates of this step per node
  int32_t* grp_id = Sp->grp_id;       // n: group of the node in this step
  int32_t* c_node = Sp->c_node;
  int32_t* c_rank = Sp->c_rank;
  const int maxdeg = max(1, G.maxdeg);
  // batch width: one popped label per thread, and every candidate of the step
  // within the grouping limit and the slot's candidate arrays
  const int bcap = min(min(min(Sp->B, Sp->batch_cap), SO_NT), min(SO_CANDS, cand_cap) / maxdeg);
  const int ln = lane_id(), wv = threadIdx.x / WAVE;

  if (threadIdx.x == 0) {
    s_open_n = Sp->open_n;
    s_sel = Sp->open_sel;
    s_nlab = Sp->n_labels;
    s_fwtop = (unsigned long long)Sp->fw_top;
    s_flag = bcap >= 1 ? SO_RUN : SO_QUIT;
    s_fmin = INT32_MAX;
    s_fmax = INT32_MIN;
    s_pops = s_killed = s_cands = s_ins = s_pruned = s_steps = 0;
  }
  __syncthreads();
  {
    // F1 range of OPEN at launch start (kept up to date by the steps after)
    const int32_t* cf = pick(Sp->open_f1, s_sel);
    const int on = s_open_n;
    int lo = INT32_MAX, hi = INT32_MIN;
    for (int i = threadIdx.x; i < on; i += SO_NT) {
      lo = min(lo, cf[i]);
      hi = max(hi, cf[i]);
    }
    lo = wave_min(lo);
    hi = wave_max_i(hi);
    if (ln == 0) {
      atomicMin(&s_fmin, lo);
      atomicMax(&s_fmax, hi);
    }
  }

  for (int step = 0; step < max_steps; ++step) {
    __syncthreads();
    const int on = s_open_n;
    if (s_flag != SO_RUN || on == 0) break;
    const int sel = s_sel;
    const int32_t* cf = pick(Sp->open_f1, sel);
    const int32_t* cl = pick(Sp->open_lab, sel);
    int32_t* nf = pick(Sp->open_f1, sel ^ 1);
    int32_t* nl = pick(Sp->open_lab, sel ^ 1);

    // ---- 1. batch threshold: the largest F1 bound that keeps the batch
    // within bcap labels (dead entries counted too, so the bound is safe).
    // When more labels share the smallest F1 than a batch holds, those of
    // them whose node id lies below a second bound are taken.
    const int64_t lo = s_fmin;
    int64_t range = (int64_t)s_fmax - lo + 1;
    int64_t thr = lo;
    bool tie = false;  // more labels share the smallest F1 than a batch holds
    int tnode = 0;     // then the ones of them with node < tnode are popped
    bool quit = false;
    int fb = 0;
    for (;;) {
      const int64_t W = (range + SO_BINS - 1) / SO_BINS;
      for (int b = threadIdx.x; b < SO_BINS; b += SO_NT) hist[b] = 0;
      __syncthreads();
      for (int i = threadIdx.x; i < on; i += SO_NT) {
        const int64_t df = (int64_t)cf[i] - lo;
        if (df >= 0 && df < range) atomicAdd(&hist[(int)(df / W)], 1);
      }
      // bin 0 holds the smallest F1, so a bound past it pops something
      const int bstar = so_pick(hist, bcap, s_pick, &fb);
      if (bstar >= 0) {
        // bins past the refined range count nothing: the bound stays inside it
        thr = lo + min(range, (int64_t)(bstar + 1) * W);
        break;
      }
      if (W == 1) {
        tie = true;
        break;
      }
      range = W;  // refine inside the first bin
    }
    if (tie) {
      // the labels of F1 == lo by node id: refine into the first non-empty
      // bin until a bound takes at least one of them and at most bcap
      int64_t nlo = 0, nrange = n;
      for (;;) {
        const int64_t W = (nrange + SO_BINS - 1) / SO_BINS;
        for (int b = threadIdx.x; b < SO_BINS; b += SO_NT) hist[b] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < on; i += SO_NT) {
          if (cf[i] != lo) continue;
          const int64_t dn = (int64_t)Lnode[cl[i]] - nlo;
          if (dn >= 0 && dn < nrange) atomicAdd(&hist[(int)(dn / W)], 1);
        }
        const int bstar = so_pick(hist, bcap, s_pick, &fb);
        if (bstar >= fb) {
          tnode = (int)(nlo + min(nrange, (int64_t)(bstar + 1) * W));
          break;
        }
        if (W == 1) {
          quit = true;  // one node holds more labels of the smallest F1 than a batch
          break;
        }
        nlo += (int64_t)fb * W;  // the first non-empty bin holds more than bcap
        nrange = W;
      }
    }
    if (quit) {
      if (threadIdx.x == 0) s_flag = SO_QUIT;
      break;
    }

    // ---- 2. pop: labels below the threshold go to the batch, the rest to
    // the other OPEN buffer; dead entries are dropped
    if (threadIdx.x == 0) {
      s_nb = 0;
      s_keep = 0;
      s_nvalid = 0;
      s_ng = 0;
      s_nmin = INT32_MAX;
      s_nmax = INT32_MIN;
    }
    __syncthreads();
    int kmin = INT32_MAX, kmax = INT32_MIN;
    for (int i = threadIdx.x; i < on; i += SO_NT) {
      const int32_t f = cf[i];
      const int32_t lab = cl[i];
      const bool live = Lstate[lab] != L_DEAD;
      const bool pop = live && ((int64_t)f < thr || (tie && f == lo && Lnode[lab] < tnode));
      const bool keep = live && !pop;
      const int pb = agg_append(&s_nb, pop);
      if (pop) batch[pb] = lab;
      const int pk = agg_append(&s_keep, keep);
      if (keep) {
        nf[pk] = f;
        nl[pk] = lab;
        kmin = min(kmin, f);
        kmax = max(kmax, f);
      }
    }
    __syncthreads();

    // ---- 3. the goal front's test of the popped labels
    const int nb = s_nb;
    const NodeRec gr = node[goal];
    const bool act = (int)threadIdx.x < nb;
    int lab = -1, v = -1;
    int32_t g[DM], F[DM];
#pragma unroll
    for (int k = 0; k < DM; ++k) g[k] = F[k] = 0;
    if (act) {
      lab = batch[threadIdx.x];
      v = Lnode[lab];
      SFOR_K(k) {
        g[k] = Lg[(size_t)k * pool_cap + lab];
        F[k] = g[k] + h[(size_t)k * n + v];
      }
    }
    const bool at_goal = act && v == goal;  // only the start label can be popped there
    // the wave's labels against the goal node's labels, 64 of those at a
    // time in lanes (the next 64 in flight), each label's F read back from
    // registers
    bool dom = false;
    {
      uint64_t todo = ballot(act && !at_goal), domm = 0;
      int32_t e[DM], en[DM];
#pragma unroll
      for (int k = 0; k < DM; ++k) e[k] = en[k] = 0;
      if (ln < gr.count) SFOR_K(k) e[k] = fw[gr.off + (int64_t)k * gr.cap + ln];
      for (int q0 = 0; q0 < gr.count && todo; q0 += WAVE) {
        const int qn = q0 + WAVE + ln;
        if (qn < gr.count) SFOR_K(k) en[k] = fw[gr.off + (int64_t)k * gr.cap + qn];
        const bool qon = q0 + ln < gr.count;
        for (uint64_t mm = todo; mm; mm &= mm - 1) {
          const int j = __ffsll((long long)mm) - 1;
          bool le = qon;
          SFOR_K(k) le = le && e[k] <= __builtin_amdgcn_readlane(F[k], j);
          if (ballot(le)) {
            todo &= ~(1ull << j);
            domm |= 1ull << j;
          }
        }
#pragma unroll
        for (int k = 0; k < DM; ++k) e[k] = en[k];
      }
      dom = (domm >> ln) & 1ull;
    }
    const bool expand = act && !at_goal && !dom;
    if (act) Lstate[lab] = dom ? L_DEAD : L_CLOSED;
    {
      const int kc = __popcll(ballot(act && dom)), pc = __popcll(ballot(act));
      if (ln == 0 && pc) {
        atomicAdd(&s_killed, kc);
        atomicAdd(&s_pops, pc);
      }
    }

    // ---- 4. expansion, and grouping by target node: a counting sort with
    // the slot's per-node counters (zero outside a step)
    int rb = 0, deg = 0;
    if (expand) {
      rb = G.row_ptr[v];
      deg = G.row_ptr[v + 1] - rb;
    }
    int nc = 0;
    const int coff = so_exscan(deg, wsum, &nc);  // nc <= bcap * maxdeg <= SO_CANDS
    int nvalid_t = 0;
    for (int q = 0; q < deg; ++q) {
      const int j = coff + q, e = rb + q, w = G.col[e];
      bool reach = true;
      SFOR_K(k) {
        c_g[(size_t)k * cand_cap + j] = g[k] + G.cost[(size_t)k * m + e];
        reach = reach && h[(size_t)k * n + w] != UNREACH;
      }
      c_par[j] = lab;
      c_arc[j] = e;
      c_node[j] = reach ? w : -1;
      if (reach) {
        const int rk = atomicAdd(&grp_cnt[w], 1);
        c_rank[j] = rk;
        if (rk == 0) {
          const int gid = atomicAdd(&s_ng, 1);
          grp_node[gid] = w;
          grp_id[w] = gid;
        }
        ++nvalid_t;
      }
    }
    if (nvalid_t) atomicAdd(&s_nvalid, nvalid_t);
    __syncthreads();
    const int nv = s_nvalid, ng = s_ng;
    // group offsets (positions in `order`) and the frontier-test work items
    // (one per 64 candidates of a group), a block of groups per thread
    {
      const int ch = (ng + SO_NT - 1) / SO_NT;
      const int g0 = min(ng, (int)threadIdx.x * ch), g1 = min(ng, g0 + ch);
      int csum = 0, isum = 0;
      for (int gq = g0; gq < g1; ++gq) {
        const int k = grp_cnt[grp_node[gq]];
        csum += k;
        isum += k > WAVE ? (k + WAVE - 1) / WAVE : 0;
      }
      int ctot = 0, itot = 0;
      int co = so_exscan(csum, wsum, &ctot);
      int io = so_exscan(isum, wsum, &itot);
      for (int gq = g0; gq < g1; ++gq) {
        const int k = grp_cnt[grp_node[gq]];
        grp_off[gq] = co;
        co += k;
        if (k > WAVE)
          for (int i = 0; i < (k + WAVE - 1) / WAVE; ++i) items[io++] = gq * 128 + i;
      }
      if (threadIdx.x == 0) {
        grp_off[ng] = nv;
        s_ni = itot;
        s_cands += nv;
      }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nc; j += SO_NT) {
      const int w = c_node[j];
      if (w >= 0) order[grp_off[grp_id[w]] + c_rank[j]] = j;
    }
    __syncthreads();

    // ---- 5. groups of more than 64 candidates: the labels of the node
    // against each candidate, 64 candidates per work item over all waves (a
    // lane holds one candidate; the wave loads the node's labels 64 at a time,
    // the next 64 in flight, and every lane reads them back from registers)
    const int ni = s_ni;
    for (int it = wv; it < ni; it += SO_WAVES) {
      const int code = items[it];
      const int gq = code >> 7, c = grp_off[gq] + (code & 127) * WAVE + ln;
      const bool on = c < grp_off[gq + 1];
      const NodeRec r = node[grp_node[gq]];
      const int32_t* eb = fw + r.off;
      int32_t cg[DM], e[DM], en[DM];
#pragma unroll
      for (int k = 0; k < DM; ++k) cg[k] = e[k] = en[k] = 0;
      if (on) {
        const int cid = order[c];
        SFOR_K(k) cg[k] = c_g[(size_t)k * cand_cap + cid];
      }
      bool rej = !on;
      if (ln < r.count) SFOR_K(k) e[k] = eb[(int64_t)k * r.cap + ln];
      for (int q0 = 0; q0 < r.count && ballot(!rej); q0 += WAVE) {
        const int qn = q0 + WAVE + ln;
        if (qn < r.count) SFOR_K(k) en[k] = eb[(int64_t)k * r.cap + qn];
        const int tn = min(WAVE, r.count - q0);
        for (int j = 0; j < tn; ++j) {
          bool le = true;
          SFOR_K(k) le = le && __builtin_amdgcn_readlane(e[k], j) <= cg[k];
          rej = rej || le;
        }
#pragma unroll
        for (int k = 0; k < DM; ++k) e[k] = en[k];
      }
      if (on) acc8[c] = rej ? 0 : 1;
    }
    __syncthreads();

    // ---- 6. one wave per group: decide, prune, insert.  A wave reads the
    // descriptors of its next 64 groups at once (one per lane).
    int w_ins = 0, w_pruned = 0;
    for (int gb = wv; gb < ng; gb += SO_WAVES * WAVE) {
      const int gl = gb + ln * SO_WAVES;
      int d_beg = 0, d_end = 0, d_v = 0, d_cnt = 0, d_cap = 0, d_lo = 0, d_hi = 0;
      if (gl < ng) {
        d_beg = grp_off[gl];
        d_end = grp_off[gl + 1];
        d_v = grp_node[gl];
        const NodeRec r = node[d_v];
        d_cnt = r.count;
        d_cap = r.cap;
        d_lo = (int)(uint32_t)((uint64_t)r.off & 0xffffffffull);
        d_hi = (int)(uint32_t)((uint64_t)r.off >> 32);
      }
      const int nloc = min(WAVE, (ng - gb + SO_WAVES - 1) / SO_WAVES);
      for (int gi2 = 0; gi2 < nloc; ++gi2) {
        const int beg = __builtin_amdgcn_readlane(d_beg, gi2);
        const int end = __builtin_amdgcn_readlane(d_end, gi2);
        const int vv = __builtin_amdgcn_readlane(d_v, gi2);
        const int rcount = __builtin_amdgcn_readlane(d_cnt, gi2);
        const int rcap = __builtin_amdgcn_readlane(d_cap, gi2);
        const int64_t roff = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(d_hi, gi2) << 32) |
                                       (uint32_t)__builtin_amdgcn_readlane(d_lo, gi2));
        const int kg = end - beg;
        int32_t* eb = fw + roff;
        if (ln == 0) {
          grp_cnt[vv] = 0;  // the node's counters back to their idle values
          grp_id[vv] = -1;
        }
        // candidates of a small group stay in lanes 0 .. kg-1
        int cid = 0, carc = 0;
        int32_t cg[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k) cg[k] = 0;
        uint64_t acc = 0;  // small group: accepted candidates (lanes)
        int nacc = 0;
        if (kg <= WAVE) {
          if (ln < kg) {
            cid = order[beg + ln];
            carc = c_arc[cid];
            SFOR_K(k) cg[k] = c_g[(size_t)k * cand_cap + cid];
          }
          // (a) the node's labels, one per lane, against each live candidate
          uint64_t alive = kg == WAVE ? ~0ull : ((1ull << kg) - 1ull);
          int32_t e[DM], en[DM];
#pragma unroll
          for (int k = 0; k < DM; ++k) e[k] = en[k] = 0;
          if (ln < rcount) SFOR_K(k) e[k] = eb[(int64_t)k * rcap + ln];
          for (int q0 = 0; q0 < rcount && alive; q0 += WAVE) {
            const int qn = q0 + WAVE + ln;
            if (qn < rcount) SFOR_K(k) en[k] = eb[(int64_t)k * rcap + qn];
            const bool qon = q0 + ln < rcount;
            for (uint64_t mm = alive; mm; mm &= mm - 1) {
              const int j = __ffsll((long long)mm) - 1;
              bool le = qon;
              SFOR_K(k) le = le && e[k] <= __builtin_amdgcn_readlane(cg[k], j);
              if (ballot(le)) alive &= ~(1ull << j);
            }
#pragma unroll
            for (int k = 0; k < DM; ++k) e[k] = en[k];
          }
          // (b) survivors against each other (equal vectors: the smaller arc
          // stays); a candidate rejected by the node's labels rejects nothing
          // those labels do not
          bool rej = !((alive >> ln) & 1ull);
          for (uint64_t mm = alive; mm; mm &= mm - 1) {
            const int j = __ffsll((long long)mm) - 1;
            bool le = true, eq = true;
            SFOR_K(k) {
              const int32_t o = __builtin_amdgcn_readlane(cg[k], j);
              le = le && o <= cg[k];
              eq = eq && o == cg[k];
            }
            const int oa = __builtin_amdgcn_readlane(carc, j);
            rej = rej || (j != ln && le && (!eq || oa < carc));
          }
          acc = ballot(!rej);
          nacc = __popcll(acc);
        } else {
          // large group: step 5 left the survivors of the node's labels in
          // acc8; survivors against each other, 64 at a time.  Clearing a
          // rejected one at once is safe: whatever it would reject, the
          // survivor that rejected it (or the first of that chain, which
          // stays) rejects too.
          for (int a0 = beg; a0 < end; a0 += WAVE) {
            const int c = a0 + ln;
            const bool sa = c < end && acc8[c];
            if (ballot(sa) == 0) continue;
            int ac = 0;
            int32_t ag[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k) ag[k] = 0;
            if (sa) {
              const int id2 = order[c];
              ac = c_arc[id2];
              SFOR_K(k) ag[k] = c_g[(size_t)k * cand_cap + id2];
            }
            bool rej = !sa;
            for (int b0 = beg; b0 < end && ballot(!rej); b0 += WAVE) {
              const int t = b0 + ln;
              const bool sb = t < end && acc8[t];
              const uint64_t mb = ballot(sb);
              if (mb == 0) continue;
              int oarc = 0;
              int32_t og[DM];
#pragma unroll
              for (int k = 0; k < DM; ++k) og[k] = 0;
              if (sb) {
                const int oid = order[t];
                oarc = c_arc[oid];
                SFOR_K(k) og[k] = c_g[(size_t)k * cand_cap + oid];
              }
              for (uint64_t mm = mb; mm; mm &= mm - 1) {
                const int j = __ffsll((long long)mm) - 1;
                bool le = true, eq = true;
                SFOR_K(k) {
                  const int32_t o = __builtin_amdgcn_readlane(og[k], j);
                  le = le && o <= ag[k];
                  eq = eq && o == ag[k];
                }
                const int oa = __builtin_amdgcn_readlane(oarc, j);
                rej = rej || (b0 + j != c && le && (!eq || oa < ac));
              }
            }
            if (sa && rej) acc8[c] = 0;
            nacc += __popcll(ballot(sa && !rej));
            wave_sync();
          }
        }
        if (nacc == 0) continue;
        // (c) the node's labels that an accepted candidate dominates leave its
        // block; the others move down in place (each wave of entries is read
        // before any of it is written)
        int live = 0;
        for (int q0 = 0; q0 < rcount; q0 += WAVE) {
          const int q = q0 + ln;
          const bool on = q < rcount;
          int32_t e[DM];
#pragma unroll
          for (int k = 0; k < DM; ++k) e[k] = 0;
          int elab = 0;
          if (on) {
            SFOR_K(k) e[k] = eb[(int64_t)k * rcap + q];
            elab = eb[(int64_t)d * rcap + q];
          }
          bool dead = false;
          if (kg <= WAVE) {
            for (uint64_t mm = acc; mm; mm &= mm - 1) {
              const int j = __ffsll((long long)mm) - 1;
              bool le = true;
              SFOR_K(k) le = le && __builtin_amdgcn_readlane(cg[k], j) <= e[k];
              dead = dead || le;
            }
          } else {
            for (int t0 = beg; t0 < end; t0 += WAVE) {
              const int t = t0 + ln;
              const bool at = t < end && acc8[t];
              const uint64_t am = ballot(at);
              if (am == 0) continue;
              int32_t og[DM];
#pragma unroll
              for (int k = 0; k < DM; ++k) og[k] = 0;
              if (at) {
                const int oid = order[t];
                SFOR_K(k) og[k] = c_g[(size_t)k * cand_cap + oid];
              }
              for (uint64_t mm = am; mm; mm &= mm - 1) {
                const int j = __ffsll((long long)mm) - 1;
                bool le = true;
                SFOR_K(k) le = le && __builtin_amdgcn_readlane(og[k], j) <= e[k];
                dead = dead || le;
              }
            }
          }
          dead = dead && on;
          if (dead) Lstate[elab] = L_DEAD;
          const uint64_t lm = ballot(on && !dead);
          if (on && !dead) {
            const int p = live + rank_below(lm);
            SFOR_K(k) eb[(int64_t)k * rcap + p] = e[k];
            eb[(int64_t)d * rcap + p] = elab;
          }
          live += __popcll(lm);
          w_pruned += __popcll(ballot(dead));
        }
        // (d) insert: a larger block when the accepted ones do not fit
        const int need = live + nacc;
        int64_t off = roff;
        int cap = rcap;
        bool ok = true;
        if (need > cap) {
          int cap2 = max(cap, MINCAP);
          while (cap2 < need) cap2 <<= 1;
          const int64_t words = (int64_t)cap2 * (d + 1);
          unsigned long long o2 = 0;
          if (ln == 0) o2 = atomicAdd(&s_fwtop, (unsigned long long)words);
          const int lo32 = __shfl((int)(uint32_t)(o2 & 0xffffffffull), 0);
          const int hi32 = __shfl((int)(uint32_t)(o2 >> 32), 0);
          const int64_t noff = (int64_t)(((uint64_t)(uint32_t)hi32 << 32) | (uint32_t)lo32);
          if (noff + words > fw_cap) {
            ok = false;
          } else {
            for (int q = ln; q < live; q += WAVE) {
              SFOR_K(k) fw[noff + (int64_t)k * cap2 + q] = eb[(int64_t)k * rcap + q];
              fw[noff + (int64_t)d * cap2 + q] = eb[(int64_t)d * rcap + q];
            }
            off = noff;
            cap = cap2;
          }
        }
        int base = 0;
        if (ln == 0 && ok) base = atomicAdd(&s_nlab, nacc);
        base = __shfl(base, 0);
        if (ok && base + nacc > pool_cap) ok = false;
        if (!ok) {
          if (ln == 0) s_flag = SO_OVERFLOW;
          continue;
        }
        const int nchunks = kg <= WAVE ? 1 : (kg + WAVE - 1) / WAVE;
        int rank = 0;
        for (int ci = 0; ci < nchunks; ++ci) {
          const int c = beg + ci * WAVE + ln;
          bool a;
          if (kg <= WAVE) {
            a = (acc >> ln) & 1ull;
          } else {
            a = c < end && acc8[c];
            if (a) {
              cid = order[c];
              carc = c_arc[cid];
              SFOR_K(k) cg[k] = c_g[(size_t)k * cand_cap + cid];
            }
          }
          const uint64_t am = ballot(a);
          const bool to_open = a && vv != goal;
          const int pk = agg_append(&s_keep, to_open);
          if (a) {
            const int id = base + rank + rank_below(am);
            const int p = live + rank + rank_below(am);
            Lnode[id] = vv;
            Lpar[id] = c_par[cid];
            Larc[id] = carc;
            SFOR_K(k) Lg[(size_t)k * pool_cap + id] = cg[k];
            Lstate[id] = vv == goal ? L_CLOSED : L_OPEN;
            SFOR_K(k) fw[off + (int64_t)k * cap + p] = cg[k];
            fw[off + (int64_t)d * cap + p] = id;
            if (to_open) {
              if (pk < open_cap) {
                const int32_t f1 = cg[0] + h[vv];
                nf[pk] = f1;
                nl[pk] = id;
                kmin = min(kmin, f1);
                kmax = max(kmax, f1);
              } else {
                s_flag = SO_OVERFLOW;
              }
            }
          }
          rank += __popcll(am);
        }
        if (ln == 0) {
          NodeRec nr;
          nr.off = off;
          nr.cap = cap;
          nr.count = need;
          node[vv] = nr;
        }
        w_ins += nacc;
      }
    }
    kmin = wave_min(kmin);
    kmax = wave_max_i(kmax);
    if (ln == 0) {
      atomicMin(&s_nmin, kmin);
      atomicMax(&s_nmax, kmax);
      if (w_ins) atomicAdd(&s_ins, w_ins);
      if (w_pruned) atomicAdd(&s_pruned, w_pruned);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_open_n = min(s_keep, open_cap);
      s_sel = sel ^ 1;
      s_fmin = s_nmin;
      s_fmax = s_nmax;
      s_steps++;
    }
  }
  __syncthreads();

  // ---- leave: state back to the slot; a finished query's front into P
  const int flag = s_flag;
  const bool done = flag == SO_RUN && s_open_n == 0;
  const NodeRec gr = node[goal];
  const bool p_over = done && gr.count > Sp->P_cap;
  if (done && !p_over) {
    int32_t* Pg0 = Sp->Pg[0];
    int32_t* Pl0 = Sp->Plab[0];
    const int pc = Sp->P_cap;
    for (int q = threadIdx.x; q < gr.count; q += SO_NT) {
      SFOR_K(k) Pg0[(size_t)k * pc + q] = fw[gr.off + (int64_t)k * gr.cap + q];
      Pl0[q] = fw[gr.off + (int64_t)d * gr.cap + q];
    }
  }
  if (threadIdx.x == 0) {
    Sp->open_n = s_open_n;
    Sp->open_sel = s_sel;
    Sp->n_labels = min(s_nlab, pool_cap);
    Sp->fw_top = (int64_t)s_fwtop;
    Sp->st[ST_POPS] += s_pops;
    Sp->st[ST_KILLED] += s_killed;
    Sp->st[ST_CANDS] += s_cands;
    Sp->st[ST_INSERTED] += s_ins;
    Sp->st[ST_PRUNED] += s_pruned;
    Sp->st[ST_STEPS] += s_steps;
    if (flag == SO_OVERFLOW || p_over) {
      Sp->status = S_OVERFLOW;
    } else if (flag == SO_QUIT) {
      Sp->status = S_SOLO_QUIT;
    } else if (done) {
      Sp->P_n = gr.count;
      Sp->P_sel = 0;
      Sp->P_dead = 0;
      Sp->status = S_DONE;
    }
  }
}

void launch_solo(Slot* slots, int nslots, const GraphDev& G, int dm, int max_steps,
                 hipStream_t st) {
  const dim3 grid(nslots), block(SO_NT);
  switch (dm) {
    case 2: hipLaunchKernelGGL(k_solo<2>, grid, block, 0, st, slots, G, max_steps); break;
    case 3: hipLaunchKernelGGL(k_solo<3>, grid, block, 0, st, slots, G, max_steps); break;
    case 4: hipLaunchKernelGGL(k_solo<4>, grid, block, 0, st, slots, G, max_steps); break;
    case 5: hipLaunchKernelGGL(k_solo<5>, grid, block, 0, st, slots, G, max_steps); break;
    case 6: hipLaunchKernelGGL(k_solo<6>, grid, block, 0, st, slots, G, max_steps); break;
    case 8: hipLaunchKernelGGL(k_solo<8>, grid, block, 0, st, slots, G, max_steps); break;
    default: hipLaunchKernelGGL(k_solo<12>, grid, block, 0, st, slots, G, max_steps); break;
  }
}

}  // namespace mos
