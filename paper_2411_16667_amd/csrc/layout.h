// Layout of one query's search state inside a device reservation (the host
// plans the sizes and carves typed pointers into the Slot descriptor).
#pragma once

#include <algorithm>

#include "mos_core.h"

namespace mos {

struct Layout {
  int32_t B, batch_cap, cand_cap, tie_cap, pool_cap, open_cap, P_cap;
  int64_t fw_cap;
  int64_t bytes;
};

inline int64_t al(int64_t x) { return (x + 255) & ~int64_t(255); }

// per-tile counts of the batch split: SPLIT_WORDS ints per SPLIT_TILE items
// (direct pops and tie entries)
inline int64_t split_tile_bytes(int64_t batch_cap, int64_t tie_cap) {
  return 4 * (int64_t)SPLIT_WORDS * ((batch_cap + tie_cap) / SPLIT_TILE + 2);
}

inline int64_t fixed_bytes(int64_t n, int d, int batch_cap, int cand_cap, int tie_cap) {
  int64_t b = 0;
  b += al(4 * d * n) + al(16 * n) + 2 * al(4 * n);                   // h, node, grp
  b += 3 * al(4 * (int64_t)batch_cap) + al(4 * ((int64_t)batch_cap + 1));  // batch, reg, kill, reg_off
  b += al(4 * ((int64_t)batch_cap + cand_cap)) + al(4 * (int64_t)cand_cap);  // goal list, pending goals
  b += 12 * al(4 * ((int64_t)cand_cap + 1)) + al(4 * (int64_t)NPASS * ((int64_t)cand_cap + 1));
  b += al(4 * (int64_t)d * cand_cap) + al(8 * (int64_t)cand_cap);
  b += al(8 * ((int64_t)cand_cap / ACC_TILE + 2));  // per-tile accept counts
  return b + 64 * 256;
}

// Split a reservation of `budget` bytes: fixed per-query regions, then label
// pool, OPEN (double buffered), goal front (double buffered) and frontier
// words in proportion to the pool size.
inline bool plan_slot_layout(int64_t n, int maxdeg, int d, int B, int64_t budget,
                             int64_t label_limit, Layout* L) {
  L->B = B;
  L->batch_cap = std::min(2 * B, BATCH_MAX);
  L->cand_cap = L->batch_cap * std::max(1, maxdeg);
  L->tie_cap = TIECAP;
  const int64_t fixed = fixed_bytes(n, d, L->batch_cap, L->cand_cap, 0);
  if (budget <= fixed) return false;
  // bytes per pooled label: pool (node, parent, arc, g, state, tested mark) + OPEN 2x(F1,
  // lab) + tie set (F1, lab, state, d key words, split tile share) + frontier 3*(d+1)
  // words + goal front share
  const double per = (16.0 + 4.0 * d + 1.0) + 32.0 + 12.0 + 4.0 * d +
                     4.0 * SPLIT_WORDS / SPLIT_TILE + 12.0 * (d + 1) + (8.0 * (d + 2) + 8.0) / 8.0;
  int64_t pool = (int64_t)((double)(budget - fixed - 48 * 256) / per);
  pool = std::min<int64_t>(pool, (int64_t)1 << 30);
  if (label_limit > 0) pool = std::min<int64_t>(pool, label_limit);
  if (pool < 16) return false;
  L->pool_cap = (int32_t)pool;
  L->open_cap = (int32_t)pool;
  L->tie_cap = (int32_t)pool;
  L->P_cap = (int32_t)std::max<int64_t>(std::min<int64_t>(pool, 1024), pool / 8);
  L->fw_cap = 3 * (int64_t)(d + 1) * pool + (int64_t)MINCAP * (d + 1);
  int64_t b = fixed;
  b += 3 * al(4 * pool) + al(4 * (int64_t)d * pool) + al(pool);  // pool
  b += 8 * al(4 * pool);                                          // OPEN near + far tiers
  b += 3 * al(4 * pool) + al(4 * (int64_t)d * pool);             // tie set and its keys
  b += al(split_tile_bytes(L->batch_cap, (int32_t)pool));         // batch split tiles
  b += 2 * (al(4 * (int64_t)d * L->P_cap) + 2 * al(4 * (int64_t)L->P_cap)) + al(4 * pool);
  b += al(4 * L->fw_cap);
  L->bytes = al(b);
  return L->bytes <= budget;
}

// Carve the reservation at `base` into the regions of a Slot; false if the
// regions would overrun the planned size.
inline bool carve_slot(Slot& s, char* base, const Layout& L, int64_t n, int d) {
  char* p = base;
  auto take = [&](int64_t bytes) {
    char* r = p;
    p += al(bytes);
    return r;
  };
  s.h = (int32_t*)take(4 * d * n);
  s.node = (NodeRec*)take(16 * n);
  s.grp_cnt = (int32_t*)take(4 * n);
  s.grp_id = (int32_t*)take(4 * n);
  s.batch = (int32_t*)take(4 * (int64_t)L.batch_cap);
  s.reg = (int32_t*)take(4 * (int64_t)L.batch_cap);
  s.goal_lab = (int32_t*)take(4 * ((int64_t)L.batch_cap + L.cand_cap));
  s.pgoal = (int32_t*)take(4 * (int64_t)L.cand_cap);
  s.reg_off = (int32_t*)take(4 * ((int64_t)L.batch_cap + 1));
  s.reg_kill = (int32_t*)take(4 * (int64_t)L.batch_cap);
  const int64_t cc = L.cand_cap;
  s.c_node = (int32_t*)take(4 * cc);
  s.c_par = (int32_t*)take(4 * cc);
  s.c_arc = (int32_t*)take(4 * cc);
  s.c_keep = (int32_t*)take(4 * cc);
  s.c_rank = (int32_t*)take(4 * cc);
  s.c_rej = (int32_t*)take(4 * cc);
  s.c_acc = (int32_t*)take(4 * cc);
  s.order = (int32_t*)take(4 * cc);
  s.grp_node = (int32_t*)take(4 * cc);
  s.grp_off = (int32_t*)take(4 * cc);
  s.small_list = (int32_t*)take(4 * (cc + 1));
  s.big_list = (int32_t*)take(4 * (cc + 1));
  s.big_toff = (int32_t*)take(4 * (int64_t)NPASS * (cc + 1));
  s.c_g = (int32_t*)take(4 * (int64_t)d * cc);
  s.c_fslot = (int64_t*)take(8 * cc);
  s.acc_tile = (int32_t*)take(8 * (cc / ACC_TILE + 2));
  const int64_t pc = L.pool_cap;
  s.Lnode = (int32_t*)take(4 * pc);
  s.Lpar = (int32_t*)take(4 * pc);
  s.Larc = (int32_t*)take(4 * pc);
  s.Lg = (int32_t*)take(4 * (int64_t)d * pc);
  s.Lpseq = (int32_t*)take(4 * pc);
  s.Lstate = (uint8_t*)take(pc);
  for (int b = 0; b < 2; ++b) {
    s.open_f1[b] = (int32_t*)take(4 * (int64_t)L.open_cap);
    s.open_lab[b] = (int32_t*)take(4 * (int64_t)L.open_cap);
    s.far_f1[b] = (int32_t*)take(4 * (int64_t)L.open_cap);
    s.far_lab[b] = (int32_t*)take(4 * (int64_t)L.open_cap);
  }
  s.tie_f1 = (int32_t*)take(4 * (int64_t)L.tie_cap);
  s.tie_lab = (int32_t*)take(4 * (int64_t)L.tie_cap);
  s.tie_st = (int32_t*)take(4 * (int64_t)L.tie_cap);
  s.tie_key = (int32_t*)take(4 * (int64_t)d * L.tie_cap);
  s.split_tile = (int32_t*)take(split_tile_bytes(L.batch_cap, L.tie_cap));
  for (int b = 0; b < 2; ++b) {
    s.Pg[b] = (int32_t*)take(4 * (int64_t)d * L.P_cap);
    s.Plab[b] = (int32_t*)take(4 * (int64_t)L.P_cap);
    s.Pseq[b] = (int32_t*)take(4 * (int64_t)L.P_cap);
  }
  s.fw = (int32_t*)take(4 * L.fw_cap);
  return p - base <= L.bytes;
}

}  // namespace mos
