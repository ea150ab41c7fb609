// Balanced edge partition through the clone-and-connect transform (Section 3.2).
//
// 1. Clone-and-connect (Definition 3): each vertex of degree d becomes d clones
//    chained into a path of d-1 auxiliary edges, clones ordered by ascending
//    edge id (the paper chains them "in index order").
// 2. Original edges carry a very large weight so they are never cut; here they
//    are contracted, so a node of the transformed graph is an edge of the input
//    and its links are the auxiliary edges at its two clones (at most four).
// 3. Balanced vertex partition of the contracted graph.  The paper uses METIS;
//    this library grows parts greedily: part p takes, one node at a time, the
//    unplaced node with the most links into p (ties: smallest id), else the one
//    with the most links to any placed node, else the smallest unplaced id.
//    Parts hold exactly `cap` nodes except the last (hard-capacity reading of
//    the balance constraint of Eq. 1).
// 4. Reconstruction (Definition 4) is the identity on contracted nodes.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <functional>
#include <new>
#include <queue>
#include <string>

#include "epk_internal.h"

namespace epk {

static thread_local std::string g_last_error;

int fail(int status, const std::string &msg) {
  g_last_error = msg;
  return status;
}
void clear_error() { g_last_error.clear(); }
const char *last_error() { return g_last_error.c_str(); }

int validate_graph(const epk_graph *g, int32_t kind) {
  if (!g) return fail(EPK_EINVAL, "graph is NULL");
  if (g->n_vertices < 0) return fail(EPK_EINVAL, "n_vertices < 0");
  if (g->n_edges < 0) return fail(EPK_EINVAL, "n_edges < 0");
  if (g->n_edges > 0 && !g->edge_uv) return fail(EPK_EINVAL, "edge_uv is NULL");
  if (g->n_edges >= (int64_t(1) << 31)) return fail(EPK_ERANGE, "n_edges must be < 2^31");
  const int32_t n = g->n_vertices;
  const bool spmv = kind == EPK_SPMV;
  if (spmv && (g->n_x < 0 || g->n_x > n)) return fail(EPK_EINVAL, "n_x out of [0, n_vertices]");
  for (int64_t e = 0; e < g->n_edges; ++e) {
    const int32_t u = g->edge_uv[2 * e], v = g->edge_uv[2 * e + 1];
    if (u < 0 || u >= n || v < 0 || v >= n)
      return fail(EPK_EINVAL, "edge " + std::to_string(e) + " has a vertex id out of range");
    if (u == v) return fail(EPK_EINVAL, "edge " + std::to_string(e) + " is a self-loop");
    if (spmv && !(u < g->n_x && v >= g->n_x))
      return fail(EPK_EINVAL, "SpMV edge " + std::to_string(e) + " must join an x vertex (first) to a y vertex");
  }
  if (kind == EPK_FLUX5 || kind == EPK_SPMV) {
    if (g->n_edges > 0 && !g->edge_geom) return fail(EPK_EINVAL, "edge_geom is NULL");
    if (kind == EPK_FLUX5 && g->geom_ncomp != 2 && g->geom_ncomp != 4)
      return fail(EPK_EINVAL, "FLUX5 needs geom_ncomp 2 (nx, ny) or 4 (nx, ny, nz, area)");
    if (spmv && g->geom_ncomp != 1) return fail(EPK_EINVAL, "SpMV needs geom_ncomp 1 (the weight)");
  }
  return EPK_OK;
}

void build_incidence(int32_t n, int64_t m, const int32_t *uv, Incidence &inc) {
  inc.off.assign(size_t(n) + 1, 0);
  for (int64_t e = 0; e < m; ++e) {
    inc.off[uv[2 * e] + 1]++;
    inc.off[uv[2 * e + 1] + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) inc.off[v + 1] += inc.off[v];
  inc.adj.resize(size_t(2 * m));
  std::vector<int64_t> cur(inc.off.begin(), inc.off.end() - 1);
  for (int64_t e = 0; e < m; ++e) {  // ascending e keeps every list sorted
    inc.adj[cur[uv[2 * e]]++] = int32_t(e);
    inc.adj[cur[uv[2 * e + 1]]++] = int32_t(e);
  }
}

void contracted_links(int64_t m, const int32_t *uv, const Incidence &inc, std::vector<int32_t> &nbr,
                      std::vector<int32_t> *nbw, int32_t n_x, const int32_t *class_weight) {
  nbr.assign(size_t(4 * m), -1);
  if (nbw) nbw->assign(size_t(4 * m), 0);
  // fill count per node; each chain link (a, b) adds b to a's list and a to b's, with the weight
  // of the chain's vertex class (x: vertices below n_x, y: the rest)
  std::vector<uint8_t> cnt(size_t(m), 0);
  const int64_t n = int64_t(inc.off.size()) - 1;
  for (int64_t v = 0; v < n; ++v) {
    const int32_t w = class_weight ? class_weight[v < n_x ? 0 : 1] : 1;
    for (int64_t t = inc.off[v]; t + 1 < inc.off[v + 1]; ++t) {
      const int32_t a = inc.adj[t], b = inc.adj[t + 1];
      if (nbw) {
        (*nbw)[4 * size_t(a) + cnt[a]] = w;
        (*nbw)[4 * size_t(b) + cnt[b]] = w;
      }
      nbr[4 * size_t(a) + cnt[a]++] = b;
      nbr[4 * size_t(b) + cnt[b]++] = a;
    }
  }
  (void)uv;
}

namespace {
// Min-heap on (255 - value) << 32 | id: pops the largest value, smallest id first.
using Heap = std::priority_queue<uint64_t, std::vector<uint64_t>, std::greater<uint64_t>>;
inline uint64_t key(uint32_t val, int32_t e) { return (uint64_t(255u - val) << 32) | uint32_t(e); }

// Pop the best valid entry of `h` (unplaced and carrying the node's current value > 0).
inline int32_t pop_best(Heap &h, const std::vector<uint8_t> &val, const std::vector<int32_t> &part) {
  while (!h.empty()) {
    const uint64_t k = h.top();
    h.pop();
    const int32_t e = int32_t(k & 0xffffffffu);
    const uint32_t v = 255u - uint32_t(k >> 32);
    if (part[e] == -1 && val[e] == v && v > 0) return e;
  }
  return -1;
}
}  // namespace

void greedy_growing(int64_t m, int32_t cap, const std::vector<int32_t> &nbr, std::vector<int32_t> &part,
                    std::vector<int32_t> &task) {
  part.assign(size_t(m), -1);
  task.clear();
  task.reserve(size_t(m));
  if (m == 0) return;
  const int64_t k = (m + cap - 1) / cap;
  std::vector<uint8_t> g(size_t(m), 0), t(size_t(m), 0);
  std::vector<int32_t> touched;
  Heap gh, th;
  int64_t smallest = 0;
  for (int64_t p = 0; p < k; ++p) {
    const int64_t size = std::min<int64_t>(cap, m - p * cap);
    for (int32_t f : touched) g[f] = 0;
    touched.clear();
    gh = Heap();
    for (int64_t s = 0; s < size; ++s) {
      int32_t e = pop_best(gh, g, part);
      if (e < 0) e = pop_best(th, t, part);
      if (e < 0) {
        while (part[smallest] != -1) ++smallest;
        e = int32_t(smallest);
      }
      part[e] = int32_t(p);
      task.push_back(e);
      for (int j = 0; j < 4; ++j) {
        const int32_t f = nbr[4 * size_t(e) + j];
        if (f < 0 || part[f] != -1) continue;
        if (g[f] == 0) touched.push_back(f);
        g[f]++;
        gh.push(key(g[f], f));
        t[f]++;
        th.push(key(t[f], f));
      }
    }
  }
}

void input_order(int64_t m, int32_t cap, std::vector<int32_t> &part, std::vector<int32_t> &task) {
  part.resize(size_t(m));
  task.resize(size_t(m));
  for (int64_t e = 0; e < m; ++e) {
    part[e] = int32_t(e / cap);
    task[e] = int32_t(e);
  }
}

// Definition 2 over the partition: loads, cost, replication; aux cut of the
// index-order transform; balance factor.
void partition_stats(int32_t n, int64_t m, const int32_t *uv, int64_t k, const std::vector<int32_t> &part,
                     const std::vector<int32_t> &task, const Incidence &inc, epk_stats &st) {
  std::vector<int32_t> stamp(size_t(n), -1), pv(size_t(n), 0);
  std::vector<int64_t> size(size_t(k), 0), nverts(size_t(k), 0);
  int64_t L = 0;
  for (int64_t pos = 0; pos < m; ++pos) {  // task order is part-major
    const int32_t e = task[pos];
    const int32_t p = part[e];
    size[p]++;
    for (int side = 0; side < 2; ++side) {
      const int32_t w = uv[2 * size_t(e) + side];
      if (stamp[w] != p) {
        stamp[w] = p;
        pv[w]++;
        nverts[p]++;
        L++;
      }
    }
  }
  int64_t max_pe = 0, max_pv = 0;
  for (int64_t p = 0; p < k; ++p) {
    max_pe = std::max(max_pe, size[p]);
    max_pv = std::max(max_pv, nverts[p]);
  }
  int64_t n_active = 0, R = 0, S = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (pv[v] >= 1) n_active++;
    if (pv[v] >= 2) {
      R++;
      S += pv[v];
    }
  }
  int64_t cut = 0;
  for (int32_t v = 0; v < n; ++v)
    for (int64_t t = inc.off[v]; t + 1 < inc.off[v + 1]; ++t)
      if (part[inc.adj[t]] != part[inc.adj[t + 1]]) cut++;
  st.n_parts = k;
  st.loads = L;
  st.cost = L - n_active;
  st.replicated = R;
  st.slots = S;
  st.aux_cut = cut;
  st.n_active = n_active;
  st.max_part_edges = max_pe;
  st.max_part_vertices = max_pv;
  st.balance = (m && k) ? double(max_pe) / (double(m) / double(k)) : 0.0;
}

static thread_local const std::atomic<bool> *tl_cancel = nullptr;
void set_cancel_flag(const std::atomic<bool> *flag) { tl_cancel = flag; }
void check_cancel() {
  if (tl_cancel && tl_cancel->load(std::memory_order_relaxed)) throw Cancelled{};
}

// The hub split: an edge whose class-y endpoint (the larger-degree one if both are in class y,
// ties to the smaller id) has degree above hub_degree is a hub edge.  The hub edges, sorted by
// (that endpoint, the other endpoint, edge id), fill parts 0 .. kh-1 in runs of cap; the other
// edges, in ascending id, form a graph of their own that the multilevel partition splits into
// parts kh, kh+1, ... .  Task order: the hub parts, then the multilevel task order.
static void hub_split(const epk_graph *g, int32_t cap, int32_t hub_degree, const int32_t *class_weight,
                      const Incidence &inc, std::vector<int32_t> &part, std::vector<int32_t> &task, int64_t &k) {
  const int64_t m = g->n_edges;
  const int32_t *uv = g->edge_uv;
  auto deg = [&](int32_t v) { return inc.off[v + 1] - inc.off[v]; };
  std::vector<int32_t> hub, rest;
  std::vector<int32_t> key(size_t(m), -1);
  for (int64_t e = 0; e < m; ++e) {
    const int32_t u = uv[2 * e], v = uv[2 * e + 1];
    const bool yu = u >= g->n_x, yv = v >= g->n_x;
    int32_t h = -1;
    if (yu && yv)
      h = (deg(u) > deg(v) || (deg(u) == deg(v) && u < v)) ? u : v;
    else if (yu)
      h = u;
    else if (yv)
      h = v;
    if (h >= 0 && deg(h) > hub_degree) {
      key[e] = h;
      hub.push_back(int32_t(e));
    } else {
      rest.push_back(int32_t(e));
    }
  }
  std::sort(hub.begin(), hub.end(), [&](int32_t a, int32_t b) {
    const int32_t oa = uv[2 * a] == key[a] ? uv[2 * a + 1] : uv[2 * a];
    const int32_t ob = uv[2 * b] == key[b] ? uv[2 * b + 1] : uv[2 * b];
    if (key[a] != key[b]) return key[a] < key[b];
    if (oa != ob) return oa < ob;
    return a < b;
  });
  const int64_t nh = int64_t(hub.size()), kh = (nh + cap - 1) / cap;
  part.assign(size_t(m), 0);
  task.resize(size_t(m));
  for (int64_t j = 0; j < nh; ++j) {
    part[hub[j]] = int32_t(j / cap);
    task[j] = hub[j];
  }
  k = kh;
  const int64_t mr = int64_t(rest.size());
  if (mr == 0) return;
  std::vector<int32_t> uv_r(size_t(2 * mr));
  for (int64_t j = 0; j < mr; ++j) {
    uv_r[2 * j] = uv[2 * int64_t(rest[j])];
    uv_r[2 * j + 1] = uv[2 * int64_t(rest[j]) + 1];
  }
  const epk_graph sub{g->n_vertices, g->n_x, mr, uv_r.data(), nullptr, 0};
  Incidence inc_r;
  build_incidence(sub.n_vertices, mr, sub.edge_uv, inc_r);
  std::vector<int32_t> nbr, nbw, part_r, task_r;
  const bool weighted = class_weight && (class_weight[0] != 1 || class_weight[1] != 1);
  contracted_links(mr, sub.edge_uv, inc_r, nbr, weighted ? &nbw : nullptr, g->n_x, class_weight);
  multilevel(mr, cap, nbr, weighted ? &nbw : nullptr, part_r, task_r);
  for (int64_t j = 0; j < mr; ++j) {
    part[rest[j]] = int32_t(kh + part_r[j]);
    task[nh + j] = rest[task_r[j]];
  }
  k = kh + multilevel_parts(mr, cap);
}

int run_partition(const epk_graph *g, int32_t cap, int32_t order, std::vector<int32_t> &part,
                  std::vector<int32_t> &task, epk_stats &st, Incidence *inc_out, const int32_t *class_weight,
                  int32_t hub_degree) {
  if (cap < 1) return fail(EPK_EINVAL, "capacity must be >= 1");
  if (order < EPK_ORDER_EP || order > EPK_ORDER_GREEDY) return fail(EPK_EINVAL, "unknown order");
  if (hub_degree < 0) return fail(EPK_EINVAL, "hub_degree must be >= 0");
  if (hub_degree > 0 && order != EPK_ORDER_EP) return fail(EPK_EINVAL, "the hub split applies to the EP order only");
  if (class_weight) {
    for (int c = 0; c < 2; ++c)
      if (class_weight[c] < 1 || class_weight[c] > kMaxClassWeight)
        return fail(EPK_EINVAL, "class weights must be 1..64");
    if (order != EPK_ORDER_EP && (class_weight[0] != 1 || class_weight[1] != 1))
      return fail(EPK_EINVAL, "class weights apply to the EP order only");
  }
  std::memset(&st, 0, sizeof(st));
  try {
    const auto t0 = std::chrono::steady_clock::now();
    Incidence inc;
    build_incidence(g->n_vertices, g->n_edges, g->edge_uv, inc);
    const int64_t m = g->n_edges;
    int64_t k = m ? (m + cap - 1) / cap : 0;
    if (order == EPK_ORDER_INPUT) {
      input_order(m, cap, part, task);
    } else if (order == EPK_ORDER_RANDOM) {
      random_order(m, cap, part, task);
    } else if (order == EPK_ORDER_GREEDY) {
      greedy_vertex_cut(g->n_vertices, m, g->edge_uv, cap, part, task);
    } else if (hub_degree > 0) {
      hub_split(g, cap, hub_degree, class_weight, inc, part, task, k);
    } else {
      std::vector<int32_t> nbr, nbw;
      const bool weighted = class_weight && (class_weight[0] != 1 || class_weight[1] != 1);
      contracted_links(m, g->edge_uv, inc, nbr, weighted ? &nbw : nullptr, g->n_x, class_weight);
      if (order == EPK_ORDER_GGP) {
        greedy_growing(m, cap, nbr, part, task);
      } else {
        k = multilevel_parts(m, cap);
        multilevel(m, cap, nbr, weighted ? &nbw : nullptr, part, task);
      }
    }
    const auto t1 = std::chrono::steady_clock::now();
    partition_stats(g->n_vertices, m, g->edge_uv, k, part, task, inc, st);
    st.partition_seconds = std::chrono::duration<double>(t1 - t0).count();
    // every part holds at most cap edges (Eq. 1's balance as a hard capacity)
    if (st.max_part_edges > cap) return fail(EPK_ERANGE, "a part holds more edges than the capacity");
    if (inc_out) *inc_out = std::move(inc);
  } catch (const std::bad_alloc &) {
    return fail(EPK_ENOMEM, "host allocation failed while partitioning");
  } catch (const Cancelled &) {
    return fail(EPK_ECANCELED, "partition cancelled");
  } catch (const CapacityExceeded &) {
    return fail(EPK_ERANGE, "a part would hold more edges than the capacity");
  }
  return EPK_OK;
}

int given_partition(const epk_graph *g, int64_t k, const int32_t *part_in, const int32_t *task_in,
                    std::vector<int32_t> &part, std::vector<int32_t> &task, epk_stats &st, Incidence *inc_out) {
  const int64_t m = g->n_edges;
  if (m > 0 && !part_in) return fail(EPK_EINVAL, "part_of_edge is NULL");
  if (k < 0 || (m > 0 && k < 1) || k > (int64_t(1) << 31) - 1) return fail(EPK_EINVAL, "n_parts out of range");
  std::memset(&st, 0, sizeof(st));
  try {
    const auto t0 = std::chrono::steady_clock::now();
    part.assign(part_in, part_in + m);
    for (int64_t e = 0; e < m; ++e)
      if (part[e] < 0 || part[e] >= k) return fail(EPK_EINVAL, "part_of_edge entry outside [0, n_parts)");
    task.resize(size_t(m));
    if (task_in) {
      // a permutation of the edges listing the parts in ascending order
      std::vector<char> seen(size_t(m), 0);
      for (int64_t j = 0; j < m; ++j) {
        const int32_t e = task_in[j];
        if (e < 0 || e >= m || seen[e]) return fail(EPK_EINVAL, "task_order is not a permutation of the edges");
        seen[e] = 1;
        if (j > 0 && part[e] < part[task_in[j - 1]]) return fail(EPK_EINVAL, "task_order does not list parts in ascending order");
        task[j] = e;
      }
    } else {  // parts ascending, edge id inside a part
      std::vector<int64_t> off(size_t(k) + 1, 0);
      for (int64_t e = 0; e < m; ++e) off[part[e] + 1]++;
      for (int64_t q = 0; q < k; ++q) off[q + 1] += off[q];
      for (int64_t e = 0; e < m; ++e) task[off[part[e]]++] = int32_t(e);
    }
    Incidence inc;
    build_incidence(g->n_vertices, m, g->edge_uv, inc);
    const auto t1 = std::chrono::steady_clock::now();
    partition_stats(g->n_vertices, m, g->edge_uv, k, part, task, inc, st);
    st.partition_seconds = std::chrono::duration<double>(t1 - t0).count();
    if (inc_out) *inc_out = std::move(inc);
  } catch (const std::bad_alloc &) {
    return fail(EPK_ENOMEM, "host allocation failed while reading the partition");
  }
  return EPK_OK;
}

}  // namespace epk

extern "C" {

int epk_partition(const epk_graph *g, int32_t capacity, int32_t order, int32_t *part_of_edge,
                  int32_t *task_order, epk_stats *stats) {
  return epk_partition_weighted(g, capacity, order, nullptr, part_of_edge, task_order, stats);
}

int epk_partition_weighted(const epk_graph *g, int32_t capacity, int32_t order, const int32_t *class_weight,
                           int32_t *part_of_edge, int32_t *task_order, epk_stats *stats) {
  epk::clear_error();
  int s = epk::validate_graph(g, -1);
  if (s) return s;
  if (g->n_edges > 0 && !part_of_edge) return epk::fail(EPK_EINVAL, "part_of_edge is NULL");
  std::vector<int32_t> part, task;
  epk_stats st;
  s = epk::run_partition(g, capacity, order, part, task, st, nullptr, class_weight);
  if (s) return s;
  if (g->n_edges > 0) {
    std::memcpy(part_of_edge, part.data(), sizeof(int32_t) * size_t(g->n_edges));
    if (task_order) std::memcpy(task_order, task.data(), sizeof(int32_t) * size_t(g->n_edges));
  }
  if (stats) *stats = st;
  return EPK_OK;
}

int epk_partition_hub(const epk_graph *g, int32_t capacity, const int32_t *class_weight, int32_t hub_degree,
                      int32_t *part_of_edge, int32_t *task_order, epk_stats *stats) {
  epk::clear_error();
  int s = epk::validate_graph(g, -1);
  if (s) return s;
  if (g->n_edges > 0 && !part_of_edge) return epk::fail(EPK_EINVAL, "part_of_edge is NULL");
  if (hub_degree < 1) return epk::fail(EPK_EINVAL, "hub_degree must be >= 1");
  std::vector<int32_t> part, task;
  epk_stats st;
  s = epk::run_partition(g, capacity, EPK_ORDER_EP, part, task, st, nullptr, class_weight, hub_degree);
  if (s) return s;
  if (g->n_edges > 0) {
    std::memcpy(part_of_edge, part.data(), sizeof(int32_t) * size_t(g->n_edges));
    if (task_order) std::memcpy(task_order, task.data(), sizeof(int32_t) * size_t(g->n_edges));
  }
  if (stats) *stats = st;
  return EPK_OK;
}

const char *epk_last_error(void) { return epk::last_error(); }
const char *epk_version(void) { return "epk 0.1 (gfx950)"; }

}  // extern "C"
