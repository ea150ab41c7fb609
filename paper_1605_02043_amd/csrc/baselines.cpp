// Edge-partition baselines the paper compares against (Section 3.3, other
// edge partition methods): the vertex-cut placements of PowerGraph (Gonzalez
// et al., OSDI 2012), random
// and greedy, here with the same hard capacity as the other orders
// (k = ceil(m / cap) parts of at most cap edges).
//
// Random: edges sorted by a counter-based hash of their id (SplitMix64, Steele,
// Lea and Flood, OOPSLA 2014), ties by id, then consecutive blocks of cap.
//
// Greedy, edges in ascending id, A(v) = parts already holding an edge of v,
// rem(v) = edges of v not yet placed, candidates = parts with fewer than cap
// edges:
//   A(u) and A(v) share a part       -> least loaded candidate of A(u) & A(v);
//   both non-empty, nothing shared   -> least loaded candidate of A(w), w the
//                                       endpoint with larger rem (ties: u);
//   only one endpoint placed         -> least loaded candidate of its A;
//   neither placed, or no candidate  -> least loaded candidate overall.
// "Least loaded" breaks ties by the smaller part id.  Tasks inside a part run
// in ascending edge id (the placement order).
#include <algorithm>
#include <cstdint>
#include <set>
#include <utility>
#include <vector>

#include "epk_internal.h"

namespace epk {

uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

void random_order(int64_t m, int32_t cap, std::vector<int32_t> &part, std::vector<int32_t> &task) {
  std::vector<std::pair<uint64_t, int32_t>> key(static_cast<size_t>(m));
  for (int64_t e = 0; e < m; ++e) key[e] = {splitmix64(uint64_t(e)), int32_t(e)};
  std::sort(key.begin(), key.end());
  part.assign(size_t(m), 0);
  task.assign(size_t(m), 0);
  for (int64_t i = 0; i < m; ++i) {
    task[i] = key[i].second;
    part[key[i].second] = int32_t(i / cap);
  }
}

void greedy_vertex_cut(int32_t n, int64_t m, const int32_t *uv, int32_t cap, std::vector<int32_t> &part,
                       std::vector<int32_t> &task) {
  const int64_t k = m ? (m + cap - 1) / cap : 0;
  std::vector<int64_t> load(static_cast<size_t>(k), 0);
  std::vector<int64_t> rem(static_cast<size_t>(n), 0);
  for (int64_t e = 0; e < m; ++e) {
    rem[uv[2 * e]]++;
    rem[uv[2 * e + 1]]++;
  }
  std::vector<std::vector<int32_t>> A(static_cast<size_t>(n));  // sorted
  std::set<std::pair<int64_t, int32_t>> open;                    // (load, part) with room
  for (int64_t p = 0; p < k; ++p) open.insert({0, int32_t(p)});
  auto least = [&](const std::vector<int32_t> &c) {
    int32_t best = -1;
    for (int32_t p : c)
      if (load[p] < cap && (best < 0 || load[p] < load[best] || (load[p] == load[best] && p < best))) best = p;
    return best;
  };
  std::vector<int32_t> both;
  part.assign(size_t(m), 0);
  for (int64_t e = 0; e < m; ++e) {
    const int32_t u = uv[2 * e], v = uv[2 * e + 1];
    const std::vector<int32_t> &Au = A[u], &Av = A[v];
    int32_t p = -1;
    if (!Au.empty() && !Av.empty()) {
      both.clear();
      std::set_intersection(Au.begin(), Au.end(), Av.begin(), Av.end(), std::back_inserter(both));
      if (!both.empty())
        p = least(both);
      else
        p = least(rem[v] > rem[u] ? Av : Au);
    } else if (!Au.empty()) {
      p = least(Au);
    } else if (!Av.empty()) {
      p = least(Av);
    }
    if (p < 0) p = open.begin()->second;
    part[e] = p;
    open.erase({load[p], p});
    if (++load[p] < cap) open.insert({load[p], p});
    for (int32_t w : {u, v}) {
      std::vector<int32_t> &a = A[w];
      auto it = std::lower_bound(a.begin(), a.end(), p);
      if (it == a.end() || *it != p) a.insert(it, p);
      rem[w]--;
    }
  }
  // tasks: parts in ascending id, edges in ascending id inside each part
  std::vector<int64_t> off(static_cast<size_t>(k) + 1, 0);
  for (int64_t e = 0; e < m; ++e) off[part[e] + 1]++;
  for (int64_t p = 0; p < k; ++p) off[p + 1] += off[p];
  task.assign(size_t(m), 0);
  for (int64_t e = 0; e < m; ++e) task[off[part[e]]++] = int32_t(e);
}

}  // namespace epk
