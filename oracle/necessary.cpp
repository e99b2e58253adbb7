// Necessary conditions on an exact Pareto front that stay cheap on large graphs.
//
// TEST INFRASTRUCTURE ONLY, like namoa.cpp (built into the same library; it
// shares nothing with the GPU path).
//
// Paper, Section 3: the answer is the set of Pareto-optimal start->goal path
// costs.  Three families of its members can be computed without the search:
//  * the ideal point: component k of the front's componentwise minimum is the
//    single-objective shortest distance under objective k (plain Dijkstra,
//    oracle_dijkstra / oracle_heuristic in namoa.cpp);
//  * lexicographic extremes: for an order sigma of the objectives, the
//    sigma-lexicographically smallest front vector is the cost of the
//    sigma-lexicographically shortest path.  Arc costs are non-negative, so
//    lexicographic order on cost vectors is a total order that adding a
//    non-negative vector preserves, and Dijkstra's label-setting argument holds
//    with vector distances compared in that order (this file);
//  * supported points: for positive weights w, the smallest w . y over the
//    front is the shortest distance under the scalar arc cost w . c(e)
//    (oracle_dijkstra on the weighted costs).
// Any front that misses one of these points, or holds a vector below one of
// these minima, is wrong; a right front passes them all.
#include <cstddef>
#include <cstdint>
#include <queue>
#include <vector>

typedef long long i64;

// Lexicographic Dijkstra from s over the first d objectives of the arc-major
// cost array (cost[e * D + k]), objectives compared in the order
// perm[0], perm[1], ..., perm[d-1].  On return out[k] (k = 0..d-1, original
// objective order) is the cost vector of the perm-lexicographically smallest
// s -> t path.  Returns 1 when t is reachable, 0 when not, -1 on bad input.
extern "C" int oracle_lex_dijkstra(int n, i64 m, int D, const i64* row_ptr, const int* col,
                                   const int* cost, int s, int t, int d, const int* perm,
                                   i64* out) {
  if (n <= 0 || d <= 0 || d > D || s < 0 || s >= n || t < 0 || t >= n) return -1;
  for (int k = 0; k < d; ++k)
    if (perm[k] < 0 || perm[k] >= d) return -1;
  // dist[v * d + j] holds objective perm[j] of v's tentative distance, so that
  // comparing the rows as plain sequences is the lexicographic order.  Heap
  // items refer to a snapshot of the key taken when they were pushed (a flat
  // pool of d values per push).
  std::vector<i64> dist((size_t)n * d, 0);
  std::vector<char> reached(n, 0), done(n, 0);
  std::vector<i64> pool;
  auto less_key = [&](const i64* a, const i64* b) {
    for (int j = 0; j < d; ++j)
      if (a[j] != b[j]) return a[j] < b[j];
    return false;
  };
  struct Item {
    size_t key;  // offset into pool
    int v;
  };
  auto greater = [&](const Item& a, const Item& b) {
    const i64* ka = &pool[a.key];
    const i64* kb = &pool[b.key];
    if (less_key(kb, ka)) return true;
    if (less_key(ka, kb)) return false;
    return a.v > b.v;
  };
  std::priority_queue<Item, std::vector<Item>, decltype(greater)> pq(greater);
  reached[s] = 1;
  pool.assign(d, 0);
  pq.push(Item{0, s});
  std::vector<i64> nd(d);
  while (!pq.empty()) {
    const Item it = pq.top();
    pq.pop();
    const int u = it.v;
    if (done[u]) continue;
    done[u] = 1;
    if (u == t) break;
    const i64* ku = &dist[(size_t)u * d];
    for (i64 e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      const int v = col[e];
      if (done[v]) continue;
      for (int j = 0; j < d; ++j) nd[j] = ku[j] + cost[e * D + perm[j]];
      if (!reached[v] || less_key(nd.data(), &dist[(size_t)v * d])) {
        reached[v] = 1;
        for (int j = 0; j < d; ++j) dist[(size_t)v * d + j] = nd[j];
        const size_t off = pool.size();
        pool.insert(pool.end(), nd.begin(), nd.end());
        pq.push(Item{off, v});
      }
    }
  }
  if (!reached[t]) return 0;
  for (int j = 0; j < d; ++j) out[perm[j]] = dist[(size_t)t * d + j];
  return 1;
}

// Mutual non-dominance of a front given as n rows of d values in
// lexicographically ascending order: only an earlier row can weakly dominate
// a later one, so each row is tested against the rows before it.  Returns -1
// when no row is weakly dominated by (or equal to) another, else the index of
// the first such row; -2 when the rows are not in ascending order.
extern "C" i64 oracle_first_dominated(i64 n, int d, const i64* rows) {
  for (i64 i = 1; i < n; ++i) {
    const i64* a = rows + (size_t)(i - 1) * d;
    const i64* b = rows + (size_t)i * d;
    for (int k = 0; k < d; ++k) {
      if (a[k] != b[k]) {
        if (a[k] > b[k]) return -2;
        break;
      }
    }
  }
  for (i64 i = 0; i < n; ++i) {
    const i64* y = rows + (size_t)i * d;
    for (i64 j = 0; j < i; ++j) {
      const i64* x = rows + (size_t)j * d;
      bool le = true;
      for (int k = 0; k < d && le; ++k) le = x[k] <= y[k];
      if (le) return i;
    }
  }
  return -1;
}

// Epsilon-cover (Sections 2 and 8: an approximate front trades exactness for
// work).  `apx` covers `exact` within 1 + eps, eps = eps_ppm / 10^6, when every
// exact vector y has some a in apx with a <= (1 + eps) y in every component.
// Returns -1 when it does, else the index of the first exact vector no
// approximate vector covers.  Direct check of every pair.
extern "C" i64 oracle_first_uncovered(i64 n_exact, const i64* exact, i64 n_apx, const i64* apx,
                                      int d, i64 eps_ppm) {
  for (i64 i = 0; i < n_exact; ++i) {
    const i64* y = exact + (size_t)i * d;
    bool covered = false;
    for (i64 j = 0; j < n_apx && !covered; ++j) {
      const i64* a = apx + (size_t)j * d;
      bool ok = true;
      for (int k = 0; k < d && ok; ++k) ok = a[k] * 1000000 <= y[k] * (1000000 + eps_ppm);
      covered = ok;
    }
    if (!covered) return i;
  }
  return -1;
}
