// Adaptive overhead control (the paper's EP-adapt, Section 4.2 and the
// overhead discussion of Section 5): the edge partition is computed on a
// background CPU thread while the application keeps running in its default
// order; the caller polls, takes the partitioned plan once it is ready and
// keeps whichever order times faster.  A reuse pre-check skips the partition
// when the default order already loads almost every vertex once: no order can
// load fewer than n_active vertex copies, so 1 - n_active / L_input bounds the
// fraction of loads any partition can save.  Destroying an unfinished handle
// cancels the partition at its next coarsening level or refinement pass.
#include <atomic>
#include <chrono>
#include <cstring>
#include <new>
#include <system_error>
#include <thread>
#include <vector>

#include "epk_internal.h"

struct epk_adaptive {
  std::vector<int32_t> uv;
  std::vector<float> geom;
  epk_graph g{};
  int32_t cap = 0, kind = 0;
  std::atomic<bool> cancel{false};
  std::atomic<int32_t> state{0};  // 0 running, 1 ready, 2 skipped, 3 failed or cancelled
  std::thread worker;
  epk_plan *plan = nullptr;
  int status = 0;
  double saving = 0, seconds = 0;
};

namespace epk {

// Upper bound on the saved fraction of vertex loads: 1 - n_active / L_input,
// L_input = sum over blocks of cap consecutive edges of their distinct vertices.
double reuse_bound(const epk_graph *g, int32_t cap) {
  const int64_t m = g->n_edges;
  if (m == 0) return 0.0;
  std::vector<int64_t> stamp(size_t(g->n_vertices), -1);
  std::vector<uint8_t> active(size_t(g->n_vertices), 0);
  int64_t loads = 0, n_active = 0;
  for (int64_t e = 0; e < m; ++e) {
    const int64_t blk = e / cap;
    for (int s = 0; s < 2; ++s) {
      const int32_t v = g->edge_uv[2 * e + s];
      if (stamp[v] != blk) {
        stamp[v] = blk;
        ++loads;
      }
      if (!active[v]) {
        active[v] = 1;
        ++n_active;
      }
    }
  }
  return 1.0 - double(n_active) / double(loads);
}

}  // namespace epk

extern "C" {

int epk_adaptive_start(const epk_graph *g, int32_t capacity, int32_t kind, double min_saving, epk_adaptive **out) {
  epk::clear_error();
  if (!out) return epk::fail(EPK_EINVAL, "out is NULL");
  *out = nullptr;
  int s = epk::validate_graph(g, kind);
  if (s) return s;
  if (capacity < 1) return epk::fail(EPK_EINVAL, "capacity must be >= 1");
  epk_adaptive *a = nullptr;
  try {
    a = new epk_adaptive();
    a->uv.assign(g->edge_uv, g->edge_uv + 2 * g->n_edges);
    a->geom.assign(g->edge_geom, g->edge_geom + size_t(g->n_edges) * size_t(g->geom_ncomp));
    a->g = *g;
    a->g.edge_uv = a->uv.data();
    a->g.edge_geom = a->geom.data();
    a->cap = capacity;
    a->kind = kind;
    a->saving = epk::reuse_bound(&a->g, capacity);
    if (a->saving < min_saving) {
      a->state = 2;
    } else {
      a->worker = std::thread([a]() {
        epk::set_cancel_flag(&a->cancel);
        const auto t0 = std::chrono::steady_clock::now();
        int st = 0;
        epk_plan *P = epk::plan_build(&a->g, a->cap, EPK_ORDER_EP, a->kind, &st);
        a->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        a->plan = P;
        a->status = P ? EPK_OK : st;
        epk::set_cancel_flag(nullptr);
        a->state.store(P ? 1 : 3);
      });
    }
  } catch (const std::bad_alloc &) {
    delete a;
    return epk::fail(EPK_ENOMEM, "host allocation failed");
  } catch (const std::system_error &) {
    delete a;
    return epk::fail(EPK_ENOMEM, "could not start the partition thread");
  }
  *out = a;
  return EPK_OK;
}

int epk_adaptive_poll(epk_adaptive *a, int32_t *state, double *saving_bound, double *seconds) {
  epk::clear_error();
  if (!a) return epk::fail(EPK_EINVAL, "handle is NULL");
  const int32_t st = a->state.load();
  if (state) *state = st;
  if (saving_bound) *saving_bound = a->saving;
  if (seconds) *seconds = st == 1 || st == 3 ? a->seconds : 0.0;
  return EPK_OK;
}

int epk_adaptive_take(epk_adaptive *a, int32_t wait, epk_plan **plan) {
  epk::clear_error();
  if (!a || !plan) return epk::fail(EPK_EINVAL, "NULL argument");
  *plan = nullptr;
  if (wait && a->worker.joinable()) a->worker.join();
  const int32_t st = a->state.load();
  if (st == 0) return epk::fail(EPK_ESTATE, "the partition is still running");
  if (st == 2) return epk::fail(EPK_ESTATE, "the reuse pre-check skipped the partition");
  if (st == 3) return epk::fail(a->status ? a->status : EPK_ESTATE, "the partition failed or was cancelled");
  if (!a->plan) return epk::fail(EPK_ESTATE, "the plan was already taken");
  if (a->worker.joinable()) a->worker.join();
  *plan = a->plan;
  a->plan = nullptr;
  return EPK_OK;
}

void epk_adaptive_destroy(epk_adaptive *a) {
  if (!a) return;
  a->cancel.store(true);
  if (a->worker.joinable()) a->worker.join();
  if (a->plan) epk_plan_destroy(a->plan);
  delete a;
}

}  // extern "C"
