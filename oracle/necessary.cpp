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
  // comparing the rows as plain sequences is the lexicographic order
  std::vector<i64> dist((size_t)n * d, 0);
  std::vector<char> reached(n, 0), done(n, 0);
  struct Item {
    std::vector<i64> key;
    int v;
  };
  struct Greater {
    bool operator()(const Item& a, const Item& b) const {
      if (a.key != b.key) return a.key > b.key;
      return a.v > b.v;
    }
  };
  std::priority_queue<Item, std::vector<Item>, Greater> pq;
  reached[s] = 1;
  pq.push(Item{std::vector<i64>(d, 0), s});
  std::vector<i64> nd(d);
  while (!pq.empty()) {
    Item it = pq.top();
    pq.pop();
    const int u = it.v;
    if (done[u]) continue;
    done[u] = 1;
    if (u == t) break;
    for (i64 e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      const int v = col[e];
      if (done[v]) continue;
      for (int j = 0; j < d; ++j) nd[j] = it.key[j] + cost[e * D + perm[j]];
      bool better = !reached[v];
      if (!better) {
        for (int j = 0; j < d; ++j) {
          const i64 cur = dist[(size_t)v * d + j];
          if (nd[j] != cur) {
            better = nd[j] < cur;
            break;
          }
        }
      }
      if (better) {
        reached[v] = 1;
        for (int j = 0; j < d; ++j) dist[(size_t)v * d + j] = nd[j];
        pq.push(Item{nd, v});
      }
    }
  }
  if (!reached[t]) return 0;
  for (int j = 0; j < d; ++j) out[perm[j]] = dist[(size_t)t * d + j];
  return 1;
}
