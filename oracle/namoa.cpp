// CPU oracle for the exact multi-objective shortest-path search.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark do.  It shares no code with the GPU path.
//
// What it computes (paper, Section 3, "Background and Complexity of MOS"):
// given a graph whose edges carry non-negative cost vectors of length d, a
// start node and a goal node, the cost-unique set of Pareto-optimal
// (non-dominated) start->goal path costs, with one witness path per cost.
//
// How: sequential NAMOA* exactly as Algorithm 1 of the paper lays it out
// (OPEN ordered lexicographically by F = g + h; per-node open/closed label
// sets G_OP / G_CL; goal front P; procedures NotDominated, Prune, PruneOPEN,
// Duplicate and Visited as defined right after Algorithm 1), with the
// heuristic h_k(v) = exact shortest distance from v to the goal under
// objective k alone (Section 4: admissible heuristic computed with SSSP per
// objective), obtained by binary-heap Dijkstra on the reversed arcs.
//
// Readings where the paper is silent or ambiguous:
//  * Dominance is strict (<= everywhere, < somewhere), Section 3; a separate
//    Duplicate test handles equal vectors.  Goal insertion also rejects an
//    equal vector so that P stays cost-unique.
//  * The P tests (NotDominated(F, P) and PruneOPEN) are strict by default; the
//    flag ORACLE_WEAK_P switches them to weak dominance (<= everywhere), which
//    gives the same cost set.
//  * The PruneOPEN relation printed as "F(l) >= F(l*)" is read as "l*'s F is
//    dominated by l's cost".
//  * OPEN ties are broken by (node, label id) after F; equal F at one node
//    means equal g, i.e. a duplicate, so the tie-break never decides a result.
//  * Visited(v') is read as "the frontier of v' is currently empty".
//  * A candidate whose node cannot reach the goal (infinite heuristic in any
//    objective) has no completion and is discarded.
//  * ORACLE_LAZY_PRUNEOPEN replaces the eager full scan of OPEN by a check of
//    each label against P when it is popped (the lazy delete of Algorithm 2,
//    applied to P-dominance); the cost set is unchanged.
//  * Approximate mode (eps_ppm > 0, Sections 2 and 8 name epsilon-dominance as
//    the way to trade exactness for work): every test against the goal front
//    P -- NotDominated(F, P) of a candidate, PruneOPEN, and NotDominated(l, P)
//    of a goal label -- uses epsilon-dominance, p <= (1 + eps) x in every
//    component with eps = eps_ppm / 10^6, while Prune(P, l) and every test
//    against a node's own labels stay exact.  Every label is then dropped only
//    when a vector already in P (or one that later replaces it, which is
//    smaller still) lies within a factor 1 + eps of every cost it could reach,
//    so the final P covers the exact front within that factor.
//
// Arithmetic is int64; every cost sum is asserted to stay below 2^31.

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <queue>
#include <set>
#include <stdexcept>
#include <vector>

typedef long long i64;
static const i64 INF = INT64_MAX;
static const i64 LIM = (i64(1) << 31);

enum {
  ORACLE_ZERO_H = 1,          // h == 0 (Martin-like search)
  ORACLE_WEAK_P = 2,          // weak dominance for the P tests
  ORACLE_LAZY_PRUNEOPEN = 4,  // P check at pop instead of the eager OPEN scan
};

enum { ORACLE_OK = 0, ORACLE_BAD_INPUT = 1, ORACLE_LABEL_LIMIT = 2, ORACLE_TIME_LIMIT = 3 };

// ---------------------------------------------------------------- Dijkstra
// Plain Dijkstra from `src` over arcs (row_ptr, col) with int64 weights w.
// dist[v] = INT64_MAX when v is unreachable.
extern "C" int oracle_dijkstra(int n, const i64* row_ptr, const int* col, const i64* w,
                               int src, i64* dist) {
  if (n <= 0 || src < 0 || src >= n) return ORACLE_BAD_INPUT;
  for (int v = 0; v < n; ++v) dist[v] = INF;
  typedef std::pair<i64, int> QE;
  std::priority_queue<QE, std::vector<QE>, std::greater<QE>> pq;
  dist[src] = 0;
  pq.push(QE(0, src));
  while (!pq.empty()) {
    QE top = pq.top();
    pq.pop();
    int u = top.second;
    if (top.first != dist[u]) continue;
    for (i64 e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      i64 nd = top.first + w[e];
      int v = col[e];
      if (nd < dist[v]) {
        dist[v] = nd;
        pq.push(QE(nd, v));
      }
    }
  }
  return ORACLE_OK;
}

struct Csr {
  int n;
  i64 m;
  int D;
  const i64* row_ptr;
  const int* col;
  const int* cost;  // arc-major: cost[e * D + k]
};

// Reverse-arc CSR: for every arc e = (u -> v), an arc v -> u carrying index e.
static void reverse_csr(const Csr& g, std::vector<i64>& rptr, std::vector<int>& rcol,
                        std::vector<i64>& rarc) {
  rptr.assign(g.n + 1, 0);
  for (i64 e = 0; e < g.m; ++e) rptr[g.col[e] + 1]++;
  for (int v = 0; v < g.n; ++v) rptr[v + 1] += rptr[v];
  std::vector<i64> fill(rptr.begin(), rptr.end() - 1);
  rcol.assign(g.m, 0);
  rarc.assign(g.m, 0);
  for (int u = 0; u < g.n; ++u)
    for (i64 e = g.row_ptr[u]; e < g.row_ptr[u + 1]; ++e) {
      i64 p = fill[g.col[e]]++;
      rcol[p] = u;
      rarc[p] = e;
    }
}

// h[k * n + v] = shortest v -> goal distance under objective k (INT64_MAX if none).
extern "C" int oracle_heuristic(int n, i64 m, int D, const i64* row_ptr, const int* col,
                                const int* cost, int goal, int d, i64* h) {
  if (n <= 0 || d <= 0 || d > D || goal < 0 || goal >= n) return ORACLE_BAD_INPUT;
  Csr g{n, m, D, row_ptr, col, cost};
  std::vector<i64> rptr, rarc;
  std::vector<int> rcol;
  reverse_csr(g, rptr, rcol, rarc);
  std::vector<i64> w(m);
  for (int k = 0; k < d; ++k) {
    for (i64 p = 0; p < m; ++p) w[p] = cost[rarc[p] * D + k];
    oracle_dijkstra(n, rptr.data(), rcol.data(), w.data(), goal, h + (i64)k * n);
  }
  return ORACLE_OK;
}

// ------------------------------------------------------------------ NAMOA*
struct Result {
  int status = ORACLE_OK;
  int d = 0;
  std::vector<i64> costs;               // size * d, lexicographically ascending
  std::vector<std::vector<int>> paths;  // arc ids per front entry
  // counters (paper Section 6: label extractions, candidate labels, solutions)
  i64 pops = 0;          // labels extracted from OPEN and processed
  i64 goal_pops = 0;     // of which at the goal
  i64 candidates = 0;    // candidate labels l' generated (arcs followed)
  i64 unreachable = 0;   // candidates discarded for an infinite heuristic
  i64 frontier_pairs = 0;// (candidate, alpha(v') label) pairs examined
  i64 p_pairs = 0;       // (vector, P label) pairs examined
  i64 open_pairs = 0;    // (goal label, OPEN label) pairs of PruneOPEN
  i64 inserted = 0;      // labels inserted into OPEN
  i64 pruned = 0;        // frontier labels removed by Prune
  i64 killed = 0;        // OPEN labels removed by PruneOPEN (eager or lazy)
  i64 max_open = 0;      // largest OPEN size seen
  i64 max_alpha = 0;     // largest |alpha(v)| seen
  double search_seconds = 0;
  // A search stopped early (time or extraction limit) still reports its goal
  // front so far, and the F of the smallest label left in OPEN: with OPEN in
  // lexicographic order and a consistent heuristic, the front so far is
  // exactly the part of the final front lexicographically below that F.
  bool stopped_open = false;
  std::vector<i64> open_min;  // d values when stopped_open
};

namespace {

struct Search {
  const Csr& g;
  int s, t, d, flags;
  i64 label_limit;
  double time_limit;
  std::vector<i64> h;  // d * n

  // label store
  std::vector<int> lv, lpar, larc;
  std::vector<i64> lg;  // label * d + k

  i64 F(int l, int k) const { return lg[(i64)l * d + k] + h[(i64)k * g.n + lv[l]]; }

  struct Cmp {
    const Search* S;
    bool operator()(int a, int b) const {
      for (int k = 0; k < S->d; ++k) {
        i64 fa = S->F(a, k), fb = S->F(b, k);
        if (fa != fb) return fa < fb;
      }
      if (S->lv[a] != S->lv[b]) return S->lv[a] < S->lv[b];
      return a < b;
    }
  };

  i64 pop_limit = 0;  // extractions before an early stop (0 = none)
  i64 eps_ppm = 0;    // approximate mode: P tests by (1 + eps_ppm / 10^6)-dominance

  Search(const Csr& g_, int s_, int t_, int d_, int f_, i64 lim, double tl)
      : g(g_), s(s_), t(t_), d(d_), flags(f_), label_limit(lim), time_limit(tl) {}

  // a dominates b (strict): a <= b everywhere, a < b somewhere.
  bool dominates(const i64* a, const i64* b) const {
    bool less = false;
    for (int k = 0; k < d; ++k) {
      if (a[k] > b[k]) return false;
      if (a[k] < b[k]) less = true;
    }
    return less;
  }
  bool weakly_dominates(const i64* a, const i64* b) const {
    for (int k = 0; k < d; ++k)
      if (a[k] > b[k]) return false;
    return true;
  }
  bool equal(const i64* a, const i64* b) const {
    for (int k = 0; k < d; ++k)
      if (a[k] != b[k]) return false;
    return true;
  }
  // p <= (1 + eps) x in every component (exact integer arithmetic)
  bool eps_dominates(const i64* p, const i64* x) const {
    for (int k = 0; k < d; ++k)
      if (p[k] * 1000000 > x[k] * (1000000 + eps_ppm)) return false;
    return true;
  }
  // The P relation: strict dominance, or weak dominance under ORACLE_WEAK_P,
  // or epsilon-dominance in approximate mode.
  bool p_rel(const i64* p, const i64* x) const {
    if (eps_ppm > 0) return eps_dominates(p, x);
    return (flags & ORACLE_WEAK_P) ? weakly_dominates(p, x) : dominates(p, x);
  }

  int new_label(int v, const i64* gv, int parent, int arc) {
    int id = (int)lv.size();
    lv.push_back(v);
    lpar.push_back(parent);
    larc.push_back(arc);
    for (int k = 0; k < d; ++k) {
      if (gv[k] >= LIM) throw std::overflow_error("cost above 2^31");
      lg.push_back(gv[k]);
    }
    return id;
  }

  static void remove_from(std::vector<int>& S, int l) {
    for (size_t i = 0; i < S.size(); ++i)
      if (S[i] == l) {
        S[i] = S.back();
        S.pop_back();
        return;
      }
  }

  void run(Result& R) {
    const int n = g.n;
    h.assign((size_t)d * n, 0);
    if (!(flags & ORACLE_ZERO_H))
      oracle_heuristic(n, g.m, g.D, g.row_ptr, g.col, g.cost, t, d, h.data());
    auto reachable = [&](int v) {
      for (int k = 0; k < d; ++k)
        if (h[(i64)k * n + v] == INF) return false;
      return true;
    };
    R.d = d;
    if (!reachable(s)) return;  // no s -> t path: empty front

    auto t0 = std::chrono::steady_clock::now();
    // Algorithm 1: empty OPEN, goal front and per-node label sets
    std::set<int, Cmp> OPEN(Cmp{this});
    std::vector<int> P;
    std::vector<std::vector<int>> Gop(n), Gcl(n);
    // the start label (g = 0) opens the search
    std::vector<i64> zero(d, 0), gp(d), Fp(d), Fl(d);
    int ls = new_label(s, zero.data(), -1, -1);
    OPEN.insert(ls);
    Gop[s].push_back(ls);
    R.inserted++;

    i64 iter = 0;
    while (!OPEN.empty()) {
      ++iter;
      bool stop = pop_limit > 0 && iter > pop_limit;
      if (!stop && (iter & 4095) == 0 && time_limit > 0)
        stop = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() >
               time_limit;
      if (stop) {
        R.status = ORACLE_TIME_LIMIT;
        // counters so far describe the searched prefix
        R.search_seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        R.stopped_open = true;
        for (int k = 0; k < d; ++k) R.open_min.push_back(F(*OPEN.begin(), k));
        break;
      }
      R.max_open = std::max<i64>(R.max_open, (i64)OPEN.size());
      int l = *OPEN.begin();  // lexicographically smallest open label
      OPEN.erase(OPEN.begin());
      int v = lv[l];
      // copy g(l): the label store may grow (and move) while l is expanded
      std::vector<i64> glv(lg.begin() + (i64)l * d, lg.begin() + (i64)(l + 1) * d);
      const i64* gl = glv.data();
      for (int k = 0; k < d; ++k) Fl[k] = F(l, k);
      if (flags & ORACLE_LAZY_PRUNEOPEN) {
        // Lazy PruneOPEN: a label heuristic-dominated by the goal front is
        // dropped from OPEN and G_OP when it reaches the top of OPEN.
        bool dead = false;
        for (int p : P) {
          R.p_pairs++;
          if (p_rel(&lg[(i64)p * d], Fl.data())) { dead = true; break; }
        }
        if (dead) {
          remove_from(Gop[v], l);
          R.killed++;
          continue;
        }
      }
      R.pops++;
      remove_from(Gop[v], l);  // the label moves from G_OP to G_CL
      Gcl[v].push_back(l);

      if (v == t) {  // a label at the goal updates the goal front
        R.goal_pops++;
        if (!(flags & ORACLE_LAZY_PRUNEOPEN)) {
          // PruneOPEN(l): full scan of OPEN
          std::vector<int> killed;
          for (int x : OPEN) {
            R.open_pairs++;
            i64 Fx[16];
            for (int k = 0; k < d; ++k) Fx[k] = F(x, k);
            if (p_rel(gl, Fx)) killed.push_back(x);
          }
          for (int x : killed) {
            OPEN.erase(x);
            remove_from(Gop[lv[x]], x);
            R.killed++;
          }
        }
        // Prune(P, l)
        std::vector<int> keep;
        for (int p : P) {
          R.p_pairs++;
          if (!dominates(gl, &lg[(i64)p * d])) keep.push_back(p);
        }
        P.swap(keep);
        // NotDominated(l, P) (cost-unique: an equal vector also blocks)
        bool ok = true;
        for (int p : P) {
          R.p_pairs++;
          const i64* pg = &lg[(i64)p * d];
          if (dominates(pg, gl) || equal(pg, gl) || (eps_ppm > 0 && eps_dominates(pg, gl))) {
            ok = false;
            break;
          }
        }
        if (ok) P.push_back(l);
        continue;
      }

      // expansion of l over its out-arcs
      for (i64 e = g.row_ptr[v]; e < g.row_ptr[v + 1]; ++e) {
        int w = g.col[e];
        R.candidates++;
        if (!reachable(w)) { R.unreachable++; continue; }
        for (int k = 0; k < d; ++k) {  // g' = g + c(e), F' = g' + h(v')
          gp[k] = gl[k] + g.cost[e * g.D + k];
          Fp[k] = gp[k] + h[(i64)k * n + w];
          if (gp[k] >= LIM || Fp[k] >= LIM) throw std::overflow_error("cost above 2^31");
        }
        std::vector<int>& op = Gop[w];
        std::vector<int>& cl = Gcl[w];
        i64 asz = (i64)op.size() + (i64)cl.size();
        R.max_alpha = std::max(R.max_alpha, asz);
        bool insert = false;
        if (asz == 0) {  // not Visited(v')
          insert = true;
        } else {
          R.frontier_pairs += asz;
          // Duplicate(l')
          bool dup = false;
          for (int x : op) if (equal(&lg[(i64)x * d], gp.data())) { dup = true; break; }
          if (!dup) for (int x : cl) if (equal(&lg[(i64)x * d], gp.data())) { dup = true; break; }
          if (dup) continue;
          // NotDominated(l', G_OP) and NotDominated(l', G_CL)
          bool domd = false;
          for (int x : op) if (dominates(&lg[(i64)x * d], gp.data())) { domd = true; break; }
          if (!domd) for (int x : cl) if (dominates(&lg[(i64)x * d], gp.data())) { domd = true; break; }
          if (domd) continue;
          // Prune(G_CL(v'), l')
          for (size_t i = 0; i < cl.size();) {
            if (dominates(gp.data(), &lg[(i64)cl[i] * d])) {
              cl[i] = cl.back(); cl.pop_back(); R.pruned++;
            } else ++i;
          }
          // Prune(G_OP(v'), l') and remove the pruned labels from OPEN
          for (size_t i = 0; i < op.size();) {
            if (dominates(gp.data(), &lg[(i64)op[i] * d])) {
              OPEN.erase(op[i]);
              op[i] = op.back(); op.pop_back(); R.pruned++;
            } else ++i;
          }
          insert = true;
        }
        if (insert) {
          // NotDominated(F(l'), P)
          bool ok = true;
          for (int p : P) {
            R.p_pairs++;
            if (p_rel(&lg[(i64)p * d], Fp.data())) { ok = false; break; }
          }
          if (!ok) continue;
          if (label_limit > 0 && (i64)lv.size() >= label_limit) {
            R.status = ORACLE_LABEL_LIMIT;
            return;
          }
          int nl = new_label(w, gp.data(), l, (int)e);  // into OPEN and G_OP(v')
          OPEN.insert(nl);
          Gop[w].push_back(nl);
          R.inserted++;
        }
      }
    }
    if (!R.stopped_open)
      R.search_seconds =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();

    // the result: P sorted lexicographically, with parent-chain paths
    std::sort(P.begin(), P.end(), [&](int a, int b) {
      for (int k = 0; k < d; ++k)
        if (lg[(i64)a * d + k] != lg[(i64)b * d + k]) return lg[(i64)a * d + k] < lg[(i64)b * d + k];
      return a < b;
    });
    for (int p : P) {
      for (int k = 0; k < d; ++k) R.costs.push_back(lg[(i64)p * d + k]);
      std::vector<int> path;
      for (int x = p; lpar[x] >= 0; x = lpar[x]) path.push_back(larc[x]);
      std::reverse(path.begin(), path.end());
      R.paths.push_back(path);
    }
  }
};

}  // namespace

extern "C" void* oracle_namoa_eps(int n, i64 m, int D, const i64* row_ptr, const int* col,
                                  const int* cost, int s, int t, int d, int flags, i64 label_limit,
                                  double time_limit, i64 pop_limit, i64 eps_ppm) {
  Result* R = new Result();
  if (n <= 0 || d <= 0 || d > D || d > 16 || s < 0 || s >= n || t < 0 || t >= n) {
    R->status = ORACLE_BAD_INPUT;
    return R;
  }
  for (i64 e = 0; e < m * D; ++e)
    if (cost[e] < 0) { R->status = ORACLE_BAD_INPUT; return R; }
  Csr g{n, m, D, row_ptr, col, cost};
  if (eps_ppm < 0 || eps_ppm > 1000000000) {
    R->status = ORACLE_BAD_INPUT;
    return R;
  }
  Search S(g, s, t, d, flags, label_limit, time_limit);
  S.pop_limit = pop_limit;
  S.eps_ppm = eps_ppm;
  try {
    S.run(*R);
  } catch (const std::overflow_error&) {
    R->status = ORACLE_BAD_INPUT;
  }
  return R;
}

extern "C" void* oracle_namoa_ex(int n, i64 m, int D, const i64* row_ptr, const int* col,
                                 const int* cost, int s, int t, int d, int flags, i64 label_limit,
                                 double time_limit, i64 pop_limit) {
  return oracle_namoa_eps(n, m, D, row_ptr, col, cost, s, t, d, flags, label_limit, time_limit,
                          pop_limit, 0);
}

extern "C" void* oracle_namoa(int n, i64 m, int D, const i64* row_ptr, const int* col,
                              const int* cost, int s, int t, int d, int flags, i64 label_limit,
                              double time_limit) {
  return oracle_namoa_ex(n, m, D, row_ptr, col, cost, s, t, d, flags, label_limit, time_limit, 0);
}

// After an early stop: 1 and the F of the smallest label left in OPEN; else 0.
extern "C" int oracle_open_min(void* r, i64* out) {
  Result* R = (Result*)r;
  if (!R->stopped_open) return 0;
  std::copy(R->open_min.begin(), R->open_min.end(), out);
  return 1;
}

extern "C" int oracle_status(void* r) { return ((Result*)r)->status; }
extern "C" i64 oracle_size(void* r) { return (i64)((Result*)r)->paths.size(); }
extern "C" void oracle_costs(void* r, i64* out) {
  Result* R = (Result*)r;
  std::copy(R->costs.begin(), R->costs.end(), out);
}
extern "C" i64 oracle_path_len(void* r, i64 i) { return (i64)((Result*)r)->paths[i].size(); }
extern "C" void oracle_path(void* r, i64 i, int* out) {
  const std::vector<int>& p = ((Result*)r)->paths[i];
  std::copy(p.begin(), p.end(), out);
}
// counters in the order of the Result fields, then search seconds (as double bits)
extern "C" void oracle_stats(void* r, i64* out, double* secs) {
  Result* R = (Result*)r;
  i64 v[] = {R->pops, R->goal_pops, R->candidates, R->unreachable, R->frontier_pairs,
             R->p_pairs, R->open_pairs, R->inserted, R->pruned, R->killed, R->max_open,
             R->max_alpha};
  std::memcpy(out, v, sizeof(v));
  *secs = R->search_seconds;
}
extern "C" void oracle_free(void* r) { delete (Result*)r; }
