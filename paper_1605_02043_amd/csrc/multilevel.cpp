// Multilevel balanced vertex partition of the contracted clone-and-connect
// graph (Section 3.2: the paper runs METIS, a multilevel partitioner, on D').
//
// Nodes are the edges of the data-affinity graph (weight 1); link weights
// count the auxiliary edges of D' between two nodes.  Capacity: at most c
// edges per part, k = ceil(m / (c - c/20)) parts, growth target ceil(m / k).
//  1. coarsen by heavy-edge matching (ascending visit, heaviest unmatched
//     neighbour, ties smallest id, combined weight <= W) while the graph has
//     more than 16k nodes and a level removes at least 10% of them.
//     W = min(max(2, c/32), c/20 + 1): a coarse node weighs at most one more
//     than the room above the growth target T <= c - c/20, so a part below T
//     always fits the next node, every part grows to T and k*T >= m places
//     every node (c < 20 leaves no room: W = 1, nothing merges);
//  2. greedy growing on the coarsest graph, placement of any remainder on a
//     part with room (none is left by the rule above), refine, contiguity,
//     refine;
//  3. project to each finer level, refine, contiguity.
// refine: up to 8 passes; each node (ascending id) moves to the linked part
// with the largest positive gain (link weight to it minus to its own part;
// ties smallest part) when the target has room and its own part keeps >= 1.
// contiguity: pieces of all parts are found first; part by part, every piece
// but the heaviest (ties smallest member) moves, heaviest first, to the
// adjacent part it links to most (ties smallest id) if that part has room.
#include <algorithm>
#include <cstdint>
#include <queue>
#include <vector>

#include "epk_internal.h"

namespace epk {
namespace {

struct LGraph {
  int32_t n = 0;
  std::vector<int64_t> off;  // [n + 1]
  std::vector<int32_t> nb;   // neighbours, ascending inside a node
  std::vector<int32_t> lw;   // link weights
  std::vector<int32_t> w;    // node weights
};

// Finest level from the contracted links (4 slots per node, -1 if absent); a link's weight is the
// number of chain links between its two nodes, or the sum of their slot weights nbw.
LGraph finest(int64_t m, const std::vector<int32_t> &nbr, const std::vector<int32_t> *nbw) {
  LGraph G;
  G.n = int32_t(m);
  G.off.assign(size_t(m) + 1, 0);
  G.w.assign(size_t(m), 1);
  G.nb.reserve(size_t(4 * m));
  G.lw.reserve(size_t(4 * m));
  int64_t tmp[4];  // neighbour << 32 | slot weight, sorted by neighbour
  for (int64_t e = 0; e < m; ++e) {
    int c = 0;
    for (int j = 0; j < 4; ++j) {
      const int32_t x = nbr[4 * size_t(e) + j];
      if (x >= 0) tmp[c++] = (int64_t(x) << 32) | (nbw ? (*nbw)[4 * size_t(e) + j] : 1);
    }
    std::sort(tmp, tmp + c);
    for (int j = 0; j < c;) {
      int r = j;
      int32_t w = 0;
      while (r < c && (tmp[r] >> 32) == (tmp[j] >> 32)) w += int32_t(tmp[r++] & 0xffffffff);
      G.nb.push_back(int32_t(tmp[j] >> 32));
      G.lw.push_back(w);
      j = r;
    }
    G.off[e + 1] = int64_t(G.nb.size());
  }
  return G;
}

LGraph coarsen(const LGraph &G, int32_t maxw, std::vector<int32_t> &cmap) {
  const int32_t n = G.n;
  std::vector<int32_t> match(size_t(n), -1);
  cmap.assign(size_t(n), -1);
  int32_t nc = 0;
  for (int32_t u = 0; u < n; ++u) {
    if (match[u] >= 0) continue;
    int32_t best = -1, bw = 0;
    for (int64_t t = G.off[u]; t < G.off[u + 1]; ++t) {
      const int32_t v = G.nb[t], l = G.lw[t];
      if (v != u && match[v] < 0 && G.w[u] + G.w[v] <= maxw && (l > bw || (l == bw && v < best))) {
        best = v;
        bw = l;
      }
    }
    match[u] = best >= 0 ? best : u;
    cmap[u] = nc;
    if (best >= 0) {
      match[best] = u;
      cmap[best] = nc;
    }
    ++nc;
  }
  // members of each coarse node
  std::vector<int32_t> mem_off(size_t(nc) + 1, 0), mem(static_cast<size_t>(n));
  for (int32_t u = 0; u < n; ++u) mem_off[cmap[u] + 1]++;
  for (int32_t c = 0; c < nc; ++c) mem_off[c + 1] += mem_off[c];
  {
    std::vector<int32_t> cur(mem_off.begin(), mem_off.end() - 1);
    for (int32_t u = 0; u < n; ++u) mem[cur[cmap[u]]++] = u;
  }
  LGraph C;
  C.n = nc;
  C.off.assign(size_t(nc) + 1, 0);
  C.w.assign(size_t(nc), 0);
  std::vector<int32_t> acc(size_t(nc), 0), touched;
  std::vector<char> in(size_t(nc), 0);
  for (int32_t c = 0; c < nc; ++c) {
    touched.clear();
    for (int32_t i = mem_off[c]; i < mem_off[c + 1]; ++i) {
      const int32_t u = mem[i];
      C.w[c] += G.w[u];
      for (int64_t t = G.off[u]; t < G.off[u + 1]; ++t) {
        const int32_t cv = cmap[G.nb[t]];
        if (cv == c) continue;
        if (!in[cv]) {
          in[cv] = 1;
          touched.push_back(cv);
        }
        acc[cv] += G.lw[t];
      }
    }
    std::sort(touched.begin(), touched.end());
    for (int32_t cv : touched) {
      C.nb.push_back(cv);
      C.lw.push_back(acc[cv]);
      acc[cv] = 0;
      in[cv] = 0;
    }
    C.off[c + 1] = int64_t(C.nb.size());
  }
  return C;
}

// (value, id) max-heap: largest value first, smallest id on ties.
struct Entry {
  int32_t val, id;
};
struct EntryLess {
  bool operator()(const Entry &a, const Entry &b) const { return a.val != b.val ? a.val < b.val : a.id > b.id; }
};
using MaxHeap = std::priority_queue<Entry, std::vector<Entry>, EntryLess>;

int32_t pop_fitting(MaxHeap &h, const std::vector<int32_t> &val, const std::vector<int32_t> &part,
                    const std::vector<int32_t> &w, int64_t size, int32_t cap) {
  while (!h.empty()) {
    const Entry e = h.top();
    h.pop();
    if (part[e.id] == -1 && val[e.id] == e.val && size + w[e.id] <= cap) return e.id;
  }
  return -1;
}

std::vector<int32_t> grow(const LGraph &G, int32_t k, int64_t target, int32_t cap) {
  const int32_t n = G.n;
  std::vector<int32_t> part(size_t(n), -1), g(size_t(n), 0), t(size_t(n), 0), touched;
  MaxHeap th;
  int32_t smallest = 0;
  int64_t placed = 0;
  for (int32_t p = 0; p < k && placed < n; ++p) {
    int64_t size = 0;
    for (int32_t f : touched) g[f] = 0;
    touched.clear();
    MaxHeap gh;
    while (size < target) {
      int32_t e = pop_fitting(gh, g, part, G.w, size, cap);
      if (e < 0) e = pop_fitting(th, t, part, G.w, size, cap);
      if (e < 0) {
        while (smallest < n && part[smallest] != -1) ++smallest;
        if (smallest >= n || size + G.w[smallest] > cap) break;
        e = smallest;
      }
      part[e] = p;
      size += G.w[e];
      ++placed;
      for (int64_t q = G.off[e]; q < G.off[e + 1]; ++q) {
        const int32_t f = G.nb[q];
        if (part[f] != -1) continue;
        if (g[f] == 0) touched.push_back(f);
        g[f] += G.lw[q];
        gh.push({g[f], f});
        t[f] += G.lw[q];
        th.push({t[f], f});
      }
    }
  }
  std::vector<int64_t> sizes(size_t(k), 0);
  for (int32_t u = 0; u < n; ++u)
    if (part[u] >= 0) sizes[part[u]] += G.w[u];
  std::vector<int64_t> conn(size_t(k), 0);
  std::vector<int32_t> cl;
  for (int32_t u = 0; u < n; ++u) {
    if (part[u] != -1) continue;
    cl.clear();
    for (int64_t q = G.off[u]; q < G.off[u + 1]; ++q) {
      const int32_t pv = part[G.nb[q]];
      if (pv < 0 || sizes[pv] + G.w[u] > cap) continue;
      if (conn[pv] == 0) cl.push_back(pv);
      conn[pv] += G.lw[q];
    }
    int32_t best = -1;
    for (int32_t q : cl) {
      if (best < 0 || conn[q] > conn[best] || (conn[q] == conn[best] && q < best)) best = q;
    }
    for (int32_t q : cl) conn[q] = 0;
    if (best < 0) {
      for (int32_t q = 0; q < k; ++q)
        if (sizes[q] + G.w[u] <= cap && (best < 0 || sizes[q] < sizes[best])) best = q;
      if (best < 0) throw CapacityExceeded{};
    }
    part[u] = best;
    sizes[best] += G.w[u];
  }
  return part;
}

void refine(const LGraph &G, std::vector<int32_t> &part, int32_t k, int32_t cap) {
  const int32_t n = G.n;
  std::vector<int64_t> sizes(size_t(k), 0), conn(size_t(k), 0);
  for (int32_t u = 0; u < n; ++u) sizes[part[u]] += G.w[u];
  std::vector<int32_t> cl;
  std::vector<char> in(size_t(k), 0);
  for (int pass = 0; pass < 8; ++pass) {
    check_cancel();
    int64_t moved = 0;
    for (int32_t u = 0; u < n; ++u) {
      const int32_t a = part[u];
      cl.clear();
      for (int64_t q = G.off[u]; q < G.off[u + 1]; ++q) {
        const int32_t pv = part[G.nb[q]];
        if (!in[pv]) {
          in[pv] = 1;
          cl.push_back(pv);
        }
        conn[pv] += G.lw[q];
      }
      const int64_t own = in[a] ? conn[a] : 0;
      int32_t best = -1;
      int64_t bg = 0;
      for (int32_t b : cl) {
        if (b == a) continue;
        const int64_t gain = conn[b] - own;
        if (gain > 0 && (gain > bg || (gain == bg && b < best)) && sizes[b] + G.w[u] <= cap &&
            sizes[a] - G.w[u] >= 1) {
          best = b;
          bg = gain;
        }
      }
      for (int32_t b : cl) {
        conn[b] = 0;
        in[b] = 0;
      }
      if (best >= 0) {
        part[u] = best;
        sizes[a] -= G.w[u];
        sizes[best] += G.w[u];
        ++moved;
      }
    }
    if (moved == 0) break;
  }
}

void contiguity(const LGraph &G, std::vector<int32_t> &part, int32_t k, int32_t cap) {
  const int32_t n = G.n;
  std::vector<int64_t> sizes(size_t(k), 0);
  for (int32_t u = 0; u < n; ++u) sizes[part[u]] += G.w[u];
  // pieces of every part on the partition as it stands
  std::vector<char> seen(size_t(n), 0);
  std::vector<int32_t> piece_nodes, stack;
  piece_nodes.reserve(size_t(n));
  struct Piece {
    int64_t begin, end, weight;
    int32_t min_id, part;
  };
  std::vector<Piece> pieces;
  for (int32_t u = 0; u < n; ++u) {
    if (seen[u]) continue;
    seen[u] = 1;
    const int64_t b = int64_t(piece_nodes.size());
    int64_t wt = 0;
    stack.assign(1, u);
    piece_nodes.push_back(u);
    while (!stack.empty()) {
      const int32_t x = stack.back();
      stack.pop_back();
      wt += G.w[x];
      for (int64_t q = G.off[x]; q < G.off[x + 1]; ++q) {
        const int32_t v = G.nb[q];
        if (!seen[v] && part[v] == part[u]) {
          seen[v] = 1;
          stack.push_back(v);
          piece_nodes.push_back(v);
        }
      }
    }
    pieces.push_back({b, int64_t(piece_nodes.size()), wt, u, part[u]});  // u is the piece's smallest member
  }
  std::vector<int32_t> by_part_off(size_t(k) + 1, 0), by_part(pieces.size());
  for (const Piece &pc : pieces) by_part_off[pc.part + 1]++;
  for (int32_t p = 0; p < k; ++p) by_part_off[p + 1] += by_part_off[p];
  {
    std::vector<int32_t> cur(by_part_off.begin(), by_part_off.end() - 1);
    for (size_t i = 0; i < pieces.size(); ++i) by_part[cur[pieces[i].part]++] = int32_t(i);
  }
  std::vector<int64_t> conn(size_t(k), 0);
  std::vector<int32_t> cl, list;
  for (int32_t p = 0; p < k; ++p) {
    if (by_part_off[p + 1] - by_part_off[p] <= 1) continue;
    list.assign(by_part.begin() + by_part_off[p], by_part.begin() + by_part_off[p + 1]);
    std::sort(list.begin(), list.end(), [&](int32_t a, int32_t b) {
      return pieces[a].weight != pieces[b].weight ? pieces[a].weight > pieces[b].weight
                                                  : pieces[a].min_id < pieces[b].min_id;
    });
    for (size_t i = 1; i < list.size(); ++i) {
      const Piece &pc = pieces[list[i]];
      cl.clear();
      for (int64_t j = pc.begin; j < pc.end; ++j) {
        const int32_t x = piece_nodes[j];
        for (int64_t q = G.off[x]; q < G.off[x + 1]; ++q) {
          const int32_t pv = part[G.nb[q]];
          if (pv == p) continue;
          if (conn[pv] == 0) cl.push_back(pv);
          conn[pv] += G.lw[q];
        }
      }
      int32_t best = -1;
      for (int32_t q : cl)
        if (sizes[q] + pc.weight <= cap &&
            (best < 0 || conn[q] > conn[best] || (conn[q] == conn[best] && q < best)))
          best = q;
      for (int32_t q : cl) conn[q] = 0;
      if (best < 0) continue;
      for (int64_t j = pc.begin; j < pc.end; ++j) part[piece_nodes[j]] = best;
      sizes[p] -= pc.weight;
      sizes[best] += pc.weight;
    }
  }
}

}  // namespace

int32_t multilevel_max_node_weight(int32_t cap) { return std::min(std::max(2, cap / 32), cap / 20 + 1); }

int64_t multilevel_parts(int64_t m, int32_t cap) {
  if (m == 0) return 0;
  const int64_t t0 = cap - cap / 20;
  return (m + t0 - 1) / t0;
}

void multilevel(int64_t m, int32_t cap, const std::vector<int32_t> &nbr, const std::vector<int32_t> *nbw,
                std::vector<int32_t> &part, std::vector<int32_t> &task) {
  part.assign(size_t(m), 0);
  task.resize(size_t(m));
  if (m == 0) return;
  const int32_t k = int32_t(multilevel_parts(m, cap));
  const int64_t target = (m + k - 1) / k;
  const int32_t maxw = multilevel_max_node_weight(cap);
  std::vector<LGraph> levels;
  std::vector<std::vector<int32_t>> cmaps;
  levels.push_back(finest(m, nbr, nbw));
  while (int64_t(levels.back().n) > 16 * int64_t(k)) {
    check_cancel();
    std::vector<int32_t> cmap;
    LGraph C = coarsen(levels.back(), maxw, cmap);
    if (10 * int64_t(C.n) > 9 * int64_t(levels.back().n)) break;
    cmaps.push_back(std::move(cmap));
    levels.push_back(std::move(C));
  }
  std::vector<int32_t> p = grow(levels.back(), k, target, cap);
  refine(levels.back(), p, k, cap);
  contiguity(levels.back(), p, k, cap);
  refine(levels.back(), p, k, cap);
  for (int64_t l = int64_t(levels.size()) - 2; l >= 0; --l) {
    const std::vector<int32_t> &cmap = cmaps[size_t(l)];
    std::vector<int32_t> fp(size_t(levels[l].n));
    for (int32_t u = 0; u < levels[l].n; ++u) fp[u] = p[cmap[u]];
    p.swap(fp);
    levels.resize(size_t(l) + 1);  // the coarser graph is no longer needed
    refine(levels[l], p, k, cap);
    contiguity(levels[l], p, k, cap);
  }
  part = p;
  // task order: parts ascending, edge id inside a part (counting sort)
  std::vector<int64_t> off(size_t(k) + 1, 0);
  for (int64_t e = 0; e < m; ++e) off[part[e] + 1]++;
  for (int32_t q = 0; q < k; ++q) off[q + 1] += off[q];
  for (int64_t e = 0; e < m; ++e) task[off[part[e]]++] = int32_t(e);
}

}  // namespace epk
