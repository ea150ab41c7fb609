// Plan: partition + data packing along the task order + the device image.
//
// Packing (Section 4.1, cpack): walk the tasks part by part and, inside a
// part, in placement order; for each edge take u then v; the first touch of a
// vertex gives it the next packed id of its class (SpMV: x and y are packed
// apart, x into [0, n_x), y into [n_x, n)).  Untouched vertices follow in
// ascending original id.  Hence every part OWNS a contiguous packed range
// (the vertices it touches first) and reads its other, FOREIGN, vertices
// from ranges owned by earlier parts.
//
// Per part the kernels see the local vertex list "owned range, then foreign
// ids ascending"; a vertex's local index is its position in that list.
// FLUX5 parts also carry a local incidence list (for each local vertex, the
// (local edge, side) pairs in edge order) so that per-vertex sums run in a
// fixed order.  SpMV parts keep their edges sorted by local y.
//
// Partials of replicated vertices: the owner writes its partial into the
// output itself; every other part writes its partial to the workspace slot
// (part-major, one per foreign entry; there are exactly C of them), and a
// reduction adds the slots of each vertex in ascending part order.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <numeric>

#include "epk_internal.h"

namespace epk {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Must match the LDS carve-up of flux_fwd_part / flux_bwd_part.
int64_t flux_fwd_lds(int64_t max_u, int64_t max_nf, int64_t cap, bool sidx) {
  const int64_t nlo = (max_u + 3) & ~int64_t(1);
  const int64_t b = 4 * (5 * max_u + 5 * cap) + 2 * (2 * cap + nlo) + (sidx ? 4 * max_nf : 0);
  return (b + 15) & ~int64_t(15);
}
int64_t flux_bwd_lds(int64_t max_u, int64_t max_nf, int64_t cap, bool sidx) {
  const int64_t nlo = (max_u + 3) & ~int64_t(1);
  const int64_t b = 4 * (10 * max_u + 10 * cap) + 2 * (2 * cap + nlo) + (sidx ? 4 * max_nf : 0);
  return (b + 15) & ~int64_t(15);
}
// Mirror of the device carve-up of the pipelined kernels: two state buffers
// (two more for the adjoint's gradients), q_new sums, one (two) edge value
// buffer(s), two id buffers, two incidence lists and two offset lists, and
// two slot-index buffers for the vertex-major workspace.  (These kernels write
// a part's sums from LDS one iteration later, so that the stores overlap the
// next part's compute instead of the next wait.)
int64_t flux_pipe_lds(int64_t max_u, int64_t max_nf, int64_t cap, bool bwd, bool qnew, bool sidx) {
  const int64_t su = 5 * max_u, sf = 5 * cap, nlo = (max_u + 3) & ~int64_t(1);
  const int64_t b = 4 * ((bwd ? 4 : 2) * su + (qnew ? su : 0) + (bwd ? 2 : 1) * sf) + 4 * 2 * max_nf +
                    2 * (4 * cap + 2 * nlo) + (sidx ? 4 * 2 * max_nf : 0);
  return (b + 15) & ~int64_t(15);
}
// Mirror of the cache-only kernels' LDS: per-edge values (two arrays for the
// adjoint), foreign ids, incidence lists and offsets, slot indices.
int64_t flux_cached_lds(int64_t max_u, int64_t max_nf, int64_t cap, bool bwd, bool sidx) {
  const int64_t nlo = (max_u + 3) & ~int64_t(1);
  const int64_t b = 4 * (bwd ? 10 : 5) * cap + 4 * max_nf + 2 * (2 * cap + nlo) + (sidx ? 4 * max_nf : 0);
  return (b + 15) & ~int64_t(15);
}

std::vector<int32_t> reduction_records(const std::vector<int32_t> &rvid, const std::vector<int32_t> &roff,
                                       const std::vector<int32_t> &rslot) {
  std::vector<int32_t> rec(rvid.size() * 4, -1);
  for (size_t v = 0; v < rvid.size(); ++v) {
    rec[4 * v] = rvid[v];
    const int32_t n = roff[v + 1] - roff[v];
    if (n > kRecSlots) continue;
    for (int32_t t = 0; t < n; ++t) rec[4 * v + 1 + t] = rslot[size_t(roff[v] + t)];
  }
  return rec;
}

// LDS of every FLUX5 kernel of a plan for its workspace layout (the slot
// indices take LDS only in the vertex-major layout).
void set_flux_lds(epk_plan *P) {
  const int64_t u = P->max_u, f = P->max_nf, c = P->cap;
  const bool sx = P->vmajor;
  P->lds_fwd = flux_fwd_lds(u, f, c, sx);
  P->lds_fwd_qn = P->lds_fwd;  // the sums (and q_new) leave from registers
  P->lds_bwd = flux_bwd_lds(u, f, c, sx);
  P->lds_pipe_fwd = flux_pipe_lds(u, f, c, false, false, sx);
  P->lds_pipe_fwd_qn = flux_pipe_lds(u, f, c, false, true, sx);
  P->lds_pipe_bwd = flux_pipe_lds(u, f, c, true, false, sx);
  P->lds_cached_fwd = flux_cached_lds(u, f, c, false, sx);
  P->lds_cached_bwd = flux_cached_lds(u, f, c, true, sx);
}
// SpMV adjoint: y gradients, x values, per-edge values, x incidence lists and
// offsets, x slot indices.
int64_t spmv_adj_lds(int64_t max_ux, int64_t max_uy, int64_t cap) {
  const int64_t nlo = (max_ux + 3) & ~int64_t(1), ncap = (cap + 1) & ~int64_t(1);
  const int64_t b = 4 * (max_uy + max_ux + cap) + 2 * (ncap + nlo) + 4 * max_ux;
  return (b + 15) & ~int64_t(15);
}
int64_t spmv_lds(int64_t max_ux, int64_t max_uy, int64_t wg, int64_t max_nf) {
  const int64_t b = 4 * (max_ux + 2 * max_uy + max_nf) + 8 * (wg / 64);
  return (b + 15) & ~int64_t(15);
}

// The automatic workspace layout.  FLUX5: vertex-major when the reduction
// gathers many partials per replicated vertex (more than four).  SpMV (4-byte
// partials): vertex-major while the part kernel's scattered partial writes
// stay few (at most one per eight edges), since the reduction then reads each
// vertex's partials as one run; part-major when most edges leave a partial.
bool auto_vmajor(const epk_plan *p) {
  if (p->kind == EPK_SPMV) return 8 * p->n_slots <= p->m;
  return p->n_slots > 4 * p->R;
}

// Algorithmic bytes of one launch under the plan's workspace layout:
// which = 0 forward part kernel, 1 adjoint part kernel, 2 reduction.  The
// vertex-major layout adds the slot-index reads to the part kernels; the
// part-major reduction reads a record per replicated vertex instead of its
// id and offsets, and the slot lists only for vertices with more slots than
// a record holds.
int64_t plan_bytes(const epk_plan *p, int which) {
  const int64_t ids = 4 * p->n_slots;
  if (which == 0) return p->bytes_fwd_kernel + (p->vmajor ? ids : 0);
  if (which == 1) return p->kind == EPK_FLUX5 ? p->bytes_bwd_kernel + (p->vmajor ? ids : 0) : 0;
  return p->vmajor ? p->bytes_reduce : p->bytes_reduce + p->rec_delta;
}

namespace {

template <typename T>
void put(std::vector<uint8_t> &img, size_t off, const std::vector<T> &v) {
  if (!v.empty()) std::memcpy(img.data() + off, v.data(), v.size() * sizeof(T));
}

struct Build {
  // inputs
  const epk_graph *g;
  int32_t cap, kind;
  // partition
  std::vector<int32_t> part, task;
  epk_stats st;
  Incidence inc;
  // packing
  std::vector<int32_t> o2p, perm, first_part;
  std::vector<int32_t> own_start;  // [(k+1) * ncls]
};

}  // namespace

epk_plan *plan_build(const epk_graph *g, int32_t cap, int32_t order, int32_t kind, int *status, int64_t given_k,
                     const int32_t *given_part, const int32_t *given_task, const int32_t *class_weight,
                     int32_t hub_degree) {
  *status = EPK_OK;
  if (kind != EPK_FLUX5 && kind != EPK_SPMV) {
    *status = fail(EPK_EINVAL, "unknown kind");
    return nullptr;
  }
  if ((*status = validate_graph(g, kind))) return nullptr;
  if (cap < 1) {
    *status = fail(EPK_EINVAL, "capacity must be >= 1");
    return nullptr;
  }
  if (kind == EPK_SPMV && cap > 1024) {
    *status = fail(EPK_ERANGE, "SpMV capacity must be <= 1024 (one edge per thread)");
    return nullptr;
  }
  if (2 * int64_t(cap) > 65535) {
    *status = fail(EPK_ERANGE, "capacity too large for 16-bit local indices");
    return nullptr;
  }
  epk_plan *P = nullptr;
  try {
    P = new epk_plan();
    P->n = g->n_vertices;
    P->n_x = kind == EPK_SPMV ? g->n_x : 0;
    P->kind = kind;
    P->order = order;
    P->cap = cap;
    P->geom_ncomp = g->geom_ncomp;
    P->ncls = kind == EPK_SPMV ? 2 : 1;
    P->m = g->n_edges;
    // SpMV: four edges per lane; FLUX5: one edge per lane up to 256 lanes
    P->wg = kind == EPK_SPMV ? std::max(64, (((cap + 3) / 4 + 63) / 64) * 64)
                             : std::min(256, std::max(64, ((cap + 63) / 64) * 64));
    Incidence inc;
    int s = order >= 0 ? run_partition(g, cap, order, P->part, P->task, P->stats, &inc, class_weight, hub_degree)
                       : given_partition(g, given_k, given_part, given_task, P->part, P->task, P->stats, &inc);
    if (s) {
      delete P;
      *status = s;
      return nullptr;
    }
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t m = P->m;
    const int32_t n = P->n;
    const int32_t ncls = P->ncls;
    const int64_t k = P->stats.n_parts;
    P->k = k;
    const int32_t *uv = g->edge_uv;
    // parts are contiguous in the task order; poff[p] is part p's first task
    std::vector<int64_t> poff(size_t(k) + 1, 0);
    for (int64_t e = 0; e < m; ++e) poff[P->part[e] + 1]++;
    for (int64_t q = 0; q < k; ++q) poff[q + 1] += poff[q];
    // A part's records fill a block of cap slots (part p's at p * cap): a part
    // above the capacity would overwrite its neighbour's block.
    for (int64_t q = 0; q < k; ++q)
      if (poff[q + 1] - poff[q] > cap) {
        delete P;
        *status = fail(EPK_ERANGE, "a part holds more edges than the capacity");
        return nullptr;
      }
    auto cls = [&](int32_t w) { return (kind == EPK_SPMV && w >= P->n_x) ? 1 : 0; };

    // ---- first-touch packing, per part ordered by the next part that touches
    // the vertex (none first), then by first touch
    std::vector<int32_t> o2p(size_t(n), -1), first_part(size_t(n), -1), second_part(size_t(n), -1);
    std::vector<int32_t> touch;  // vertices in first-touch order (part-major)
    touch.reserve(size_t(n));
    std::vector<int64_t> touch_begin(size_t(k) + 1, 0);
    for (int64_t p = 0, pos = 0; p < k; ++p) {
      touch_begin[p] = int64_t(touch.size());
      const int64_t ne = poff[p + 1] - poff[p];
      for (int64_t j = 0; j < ne; ++j, ++pos) {
        const int32_t e = P->task[pos];
        for (int side = 0; side < 2; ++side) {
          const int32_t w = uv[2 * size_t(e) + side];
          if (first_part[w] < 0) {
            first_part[w] = int32_t(p);
            touch.push_back(w);
          } else if (second_part[w] < 0 && first_part[w] != int32_t(p)) {
            second_part[w] = int32_t(p);
          }
        }
      }
    }
    touch_begin[k] = int64_t(touch.size());
    std::vector<int32_t> own_start(size_t((k + 1) * ncls), 0);
    int32_t nxt[2] = {0, P->n_x};
    for (int64_t p = 0; p < k; ++p) {
      for (int c = 0; c < ncls; ++c) own_start[p * ncls + c] = nxt[c];
      auto b = touch.begin() + touch_begin[p], e = touch.begin() + touch_begin[p + 1];
      std::stable_sort(b, e, [&](int32_t x, int32_t y) { return second_part[x] < second_part[y]; });
      for (auto it = b; it != e; ++it) o2p[*it] = nxt[cls(*it)]++;
    }
    for (int c = 0; c < ncls; ++c) own_start[k * ncls + c] = nxt[c];
    const int32_t active[2] = {nxt[0], nxt[1]};
    for (int32_t w = 0; w < n; ++w)
      if (o2p[w] < 0) o2p[w] = nxt[cls(w)]++;
    P->perm.assign(size_t(n), 0);
    for (int32_t w = 0; w < n; ++w) P->perm[o2p[w]] = w;

    // ---- per-part vertex lists, local ids, kernel edge order
    P->own_begin.assign(size_t(k * ncls), 0);
    P->own_count.assign(size_t(k * ncls), 0);
    P->foreign_off.assign(size_t(k * ncls + 1), 0);
    P->foreign_ids.clear();
    P->foreign_ids.reserve(size_t(P->stats.cost));
    std::vector<int32_t> stamp(size_t(n), -1), loc(size_t(n), 0);
    // Edge records sit at a fixed stride: part p's at [p cap, p cap + ne), the
    // rest of its block zero.  A kernel then knows where a part's edges are
    // before its header has arrived.
    const int64_t me = k * int64_t(cap);
    if (me >= (int64_t(1) << 31)) {
      delete P;
      *status = fail(EPK_ERANGE, "parts x capacity must be < 2^31 (32-bit edge offsets)");
      return nullptr;
    }
    P->me = me;
    std::vector<uint32_t> eloc(static_cast<size_t>(me));
    // 3D flux geometry (n, a) is stored as the area vector A = a n: 3 floats per edge
    const int gstore = (kind == EPK_FLUX5 && g->geom_ncomp == 4) ? 3 : g->geom_ncomp;
    std::vector<float> geomk(size_t(me) * size_t(gstore));
    std::vector<int32_t> hdr(size_t(k) * kHdrInts, 0);
    std::vector<uint16_t> incl, loff;
    if (kind == EPK_FLUX5) {
      incl.resize(size_t(2 * me));
      loff.reserve(size_t(P->stats.loads + k));
    }
    std::vector<int32_t> fid;  // device foreign-id list (FLUX5: all; SpMV: x only)
    fid.reserve(size_t(P->stats.cost));
    std::vector<int32_t> red_foreign;  // packed ids of the reduced class's foreign entries, part-major
    int64_t max_u[2] = {0, 0}, max_nf = 0;
    std::vector<int32_t> fl[2];
    std::vector<int32_t> cnt, cur;
    std::vector<int64_t> order_idx;
    // SpMV adjoint: per part, the kernel-order edges of each local x (ascending)
    std::vector<uint16_t> xinc, xlo;
    std::vector<int32_t> xlofs;
    std::vector<int32_t> eid;  // SpMV adjoint: original edge id of each kernel-order edge
    if (kind == EPK_SPMV) {
      xinc.resize(size_t(2 * me));  // a part's list starts at 2 e0, an even index
      xlofs.reserve(size_t(k));
      eid.resize(size_t(me));
    }
    int64_t lofs = 0;
    int64_t fdev = 0;           // running x/all foreign offset in fid
    int64_t fred = 0;           // running foreign offset of the reduced class (slot base)
    for (int64_t p = 0, pos = 0; p < k; ++p) {
      const int64_t e0 = poff[p];
      const int64_t ne = poff[p + 1] - e0;
      fl[0].clear();
      fl[1].clear();
      for (int64_t j = 0; j < ne; ++j) {
        const int32_t e = P->task[pos + j];
        for (int side = 0; side < 2; ++side) {
          const int32_t w = uv[2 * size_t(e) + side];
          if (stamp[w] == int32_t(p)) continue;
          stamp[w] = int32_t(p);
          if (first_part[w] != int32_t(p)) fl[cls(w)].push_back(o2p[w]);
        }
      }
      int32_t own0[2], nown[2], nf[2];
      for (int c = 0; c < ncls; ++c) {
        own0[c] = own_start[p * ncls + c];
        nown[c] = own_start[(p + 1) * ncls + c] - own0[c];
        std::sort(fl[c].begin(), fl[c].end());
        nf[c] = int32_t(fl[c].size());
        for (int32_t i = 0; i < nf[c]; ++i) loc[P->perm[fl[c][i]]] = nown[c] + i;
        P->own_begin[p * ncls + c] = own0[c];
        P->own_count[p * ncls + c] = nown[c];
        P->foreign_off[p * ncls + c + 1] = P->foreign_off[p * ncls + c] + nf[c];
        P->foreign_ids.insert(P->foreign_ids.end(), fl[c].begin(), fl[c].end());
        const int64_t U = int64_t(nown[c]) + nf[c];
        if (U > 65535) {
          delete P;
          *status = fail(EPK_ERANGE, "a part touches more than 65535 vertices");
          return nullptr;
        }
        max_u[c] = std::max(max_u[c], U);
        max_nf = std::max<int64_t>(max_nf, nf[c]);
      }
      auto local = [&](int32_t w) -> uint32_t {
        const int c = cls(w);
        return first_part[w] == int32_t(p) ? uint32_t(o2p[w] - own0[c]) : uint32_t(loc[w]);
      };
      int32_t *h = &hdr[size_t(p) * kHdrInts];
      if (kind == EPK_FLUX5) {
        const int64_t e0 = p * int64_t(cap);  // the part's record block
        const int32_t U = nown[0] + nf[0];
        cnt.assign(size_t(U) + 1, 0);
        for (int64_t j = 0; j < ne; ++j) {
          const int32_t e = P->task[pos + j];
          const uint32_t lu = local(uv[2 * size_t(e)]), lv = local(uv[2 * size_t(e) + 1]);
          eloc[e0 + j] = lu | (lv << 16);
          const float *ge = &g->edge_geom[size_t(e) * g->geom_ncomp];
          float *gk = &geomk[size_t(e0 + j) * gstore];
          if (gstore == 3)
            for (int c = 0; c < 3; ++c) gk[c] = ge[c] * ge[3];
          else
            std::memcpy(gk, ge, sizeof(float) * gstore);
          cnt[lu + 1]++;
          cnt[lv + 1]++;
        }
        for (int32_t i = 0; i < U; ++i) cnt[i + 1] += cnt[i];
        for (int32_t i = 0; i <= U; ++i) loff.push_back(uint16_t(cnt[i]));
        if ((U + 1) & 1) loff.push_back(0);  // blocks start at even indices: staged as whole dwords
        cur.assign(cnt.begin(), cnt.end() - 1);
        for (int64_t j = 0; j < ne; ++j) {  // ascending local edge: fixed summation order
          const uint32_t w = eloc[e0 + j];
          incl[2 * e0 + cur[w & 0xffff]++] = uint16_t((j << 1) | 0);
          incl[2 * e0 + cur[w >> 16]++] = uint16_t((j << 1) | 1);
        }
        h[0] = int32_t(e0);
        h[1] = int32_t(ne);
        h[2] = own0[0];
        h[3] = nown[0];
        h[4] = int32_t(fdev);
        h[5] = nf[0];
        h[6] = int32_t(lofs);
        h[7] = U;
        lofs += (U + 2) & ~1;
        fid.insert(fid.end(), fl[0].begin(), fl[0].end());
        fdev += nf[0];
        red_foreign.insert(red_foreign.end(), fl[0].begin(), fl[0].end());
        fred += nf[0];
      } else {
        const int64_t e0 = p * int64_t(cap);  // the part's record block
        // edges of the part sorted by local y (stable in task order)
        order_idx.resize(size_t(ne));
        std::vector<uint32_t> ly(static_cast<size_t>(ne)), lx(static_cast<size_t>(ne));
        for (int64_t j = 0; j < ne; ++j) {
          const int32_t e = P->task[pos + j];
          lx[j] = local(uv[2 * size_t(e)]);
          ly[j] = local(uv[2 * size_t(e) + 1]);
          order_idx[j] = j;
        }
        std::stable_sort(order_idx.begin(), order_idx.end(), [&](int64_t a, int64_t b) { return ly[a] < ly[b]; });
        for (int64_t jj = 0; jj < ne; ++jj) {
          const int64_t j = order_idx[jj];
          const int32_t e = P->task[pos + j];
          eloc[e0 + jj] = lx[j] | (ly[j] << 16);
          geomk[size_t(e0 + jj)] = g->edge_geom[size_t(e)];
          eid[e0 + jj] = e;
        }
        {
          const int32_t Ux = nown[0] + nf[0];
          std::vector<int32_t> c(size_t(Ux) + 1, 0);
          for (int64_t jj = 0; jj < ne; ++jj) c[(eloc[e0 + jj] & 0xffffu) + 1]++;
          for (int32_t i = 0; i < Ux; ++i) c[i + 1] += c[i];
          xlofs.push_back(int32_t(xlo.size()));
          for (int32_t i = 0; i <= Ux; ++i) xlo.push_back(uint16_t(c[i]));
          if ((Ux + 1) & 1) xlo.push_back(0);  // lists start at even indices: staged as whole dwords
          for (int64_t jj = 0; jj < ne; ++jj) xinc[2 * e0 + c[eloc[e0 + jj] & 0xffffu]++] = uint16_t(jj);
        }
        h[0] = own0[0];
        h[1] = nown[0];
        h[2] = int32_t(fdev);
        h[3] = nf[0];
        h[4] = own0[1] - P->n_x;
        h[5] = nown[1];
        h[6] = int32_t(fred);
        h[7] = nf[1];
        fid.insert(fid.end(), fl[0].begin(), fl[0].end());
        fdev += nf[0];
        for (int32_t v : fl[1]) red_foreign.push_back(v - P->n_x);
        fred += nf[1];
      }
      pos += ne;
    }
    P->max_u = max_u[0];
    P->max_uy = max_u[1];
    P->max_nf = max_nf;
    // every part's foreign ids again (SpMV: its foreign x), in a block of max_nf
    // at p max_nf (padding -1 is never used), so a part's ids are found from its
    // index alone
    std::vector<int32_t> pfid(size_t(k * max_nf), -1);
    for (int64_t p = 0; p < k; ++p) {
      const int32_t *h = &hdr[size_t(p) * kHdrInts];
      const int32_t f0 = kind == EPK_FLUX5 ? h[4] : h[2], nf = kind == EPK_FLUX5 ? h[5] : h[3];
      std::copy(fid.begin() + f0, fid.begin() + f0 + nf, pfid.begin() + p * max_nf);
    }

    // ---- reduction tables: for each replicated vertex of the reduced class,
    // its slots (non-owner parts) in ascending part order.  Two workspace
    // layouts: part-major (a part writes its foreign partials as one block;
    // rslot lists, vertex by vertex, where the reduction finds them) and
    // vertex-major (a vertex's slots side by side; sidx gives each part's
    // entries their slot).  Both tables are in the image; the layout in use
    // is chosen per plan (epk_plan_set_slot_layout).
    const int32_t nred = kind == EPK_SPMV ? n - P->n_x : n;
    std::vector<int32_t> scount(size_t(nred), 0);
    for (int32_t v : red_foreign) scount[v]++;
    std::vector<int32_t> rvid, roff(1, 0), sidx(red_foreign.size()), rslot(red_foreign.size()), heavy;
    std::vector<int32_t> start(size_t(nred), 0);
    for (int32_t v = 0; v < nred; ++v) {
      if (scount[v] == 0) continue;
      start[v] = roff.back();
      if (scount[v] > kHeavySlots) heavy.push_back(int32_t(rvid.size()));
      rvid.push_back(v);
      roff.push_back(roff.back() + scount[v]);
    }
    std::fill(scount.begin(), scount.end(), 0);
    for (size_t s = 0; s < red_foreign.size(); ++s) {  // part-major walk: ascending part order
      const int32_t v = red_foreign[s];
      sidx[s] = start[v] + scount[v]++;
      rslot[sidx[s]] = int32_t(s);
    }
    P->R = int64_t(rvid.size());
    P->n_slots = int64_t(red_foreign.size());
    P->vmajor = auto_vmajor(P);
    P->n_heavy = int64_t(heavy.size());
    P->n_out = nred;
    P->n_active_out = kind == EPK_SPMV ? active[1] - P->n_x : active[0];

    // ---- SpMV adjoint: the same tables for the x class (its foreign entries are fid)
    std::vector<int32_t> xrvid, xroff(1, 0), xsidx, xrslot, xheavy;
    if (kind == EPK_SPMV) {
      std::vector<int32_t> xc(size_t(P->n_x), 0), xs(size_t(P->n_x), 0);
      for (int32_t v : fid) xc[v]++;
      for (int32_t v = 0; v < P->n_x; ++v) {
        if (xc[v] == 0) continue;
        xs[v] = xroff.back();
        if (xc[v] > kHeavySlots) xheavy.push_back(int32_t(xrvid.size()));
        xrvid.push_back(v);
        xroff.push_back(xroff.back() + xc[v]);
      }
      std::fill(xc.begin(), xc.end(), 0);
      xsidx.resize(fid.size());
      xrslot.resize(fid.size());
      for (size_t q = 0; q < fid.size(); ++q) {
        xsidx[q] = xs[fid[q]] + xc[fid[q]]++;
        xrslot[xsidx[q]] = int32_t(q);
      }
      P->xR = int64_t(xrvid.size());
      P->xn_heavy = int64_t(xheavy.size());
      P->xn_active = active[0];
      P->xn_slots = int64_t(fid.size());
      P->xvmajor = P->xn_slots > 4 * P->xR;
    }

    // ---- single-launch reduction (FLUX5, part-major): the workgroup that completes the last
    // partial of a part's replicated vertices sums them.  Part p signals itself (if it owns
    // replicated vertices) and the owner of each of its foreign vertices; a part's target is the
    // number of parts that signal it.  The library's packing puts a part's replicated owned
    // vertices at the end of its owned range, so its owner partials are a known suffix.
    std::vector<int32_t> nfy_off, nfy_flat, rsuf;
    if (kind == EPK_FLUX5 && k > 0) {
      std::vector<int32_t> rbeg(size_t(k) + 1, 0), owner(size_t(n), -1), target(size_t(k), 0);
      std::vector<std::vector<int32_t>> sig(static_cast<size_t>(k));
      bool ok = P->n_heavy == 0 && int64_t(n) * 20 < (int64_t(1) << 31) &&
                int64_t(red_foreign.size()) * 20 < (int64_t(1) << 31);
      rsuf.assign(size_t(k), 0);
      for (int64_t q = 0; q < k; ++q) {
        const int32_t o0 = P->own_begin[q], no = P->own_count[q];
        for (int32_t i = 0; i < no; ++i) owner[o0 + i] = int32_t(q);
        rbeg[q] = int32_t(std::lower_bound(rvid.begin(), rvid.end(), o0) - rvid.begin());
        const int32_t re = int32_t(std::lower_bound(rvid.begin(), rvid.end(), o0 + no) - rvid.begin());
        const int32_t nrep = re - rbeg[q];
        rsuf[q] = no - nrep;
        for (int32_t j = 0; j < nrep && ok; ++j) ok = rvid[rbeg[q] + j] == o0 + rsuf[q] + j;
        if (nrep > 0) sig[q].push_back(int32_t(q));
      }
      rbeg[k] = int32_t(rvid.size());
      for (int64_t p2 = 0; p2 < k && ok; ++p2) {
        const int32_t *h = &hdr[size_t(p2) * kHdrInts];
        for (int32_t f = 0; f < h[5]; ++f) sig[p2].push_back(owner[fid[size_t(h[4] + f)]]);
        std::sort(sig[p2].begin(), sig[p2].end());
        sig[p2].erase(std::unique(sig[p2].begin(), sig[p2].end()), sig[p2].end());
        for (int32_t q : sig[p2]) ok = ok && q >= 0 && q <= p2;  // owners come first in the task order
        if (ok) for (int32_t q : sig[p2]) target[q]++;
        P->n_signals += int64_t(sig[p2].size());
        P->max_nfy = std::max<int64_t>(P->max_nfy, int64_t(sig[p2].size()));
      }
      ok = ok && P->max_nfy <= kMaxSignals;
      P->fused_ok = ok;
      P->fused = false;  // measured slower than the reduction launch on gfx950: opt-in
      if (ok) {
        nfy_off.assign(size_t(k) + 1, 0);
        for (int64_t p2 = 0; p2 < k; ++p2) {
          nfy_off[p2 + 1] = nfy_off[p2] + int32_t(sig[p2].size());
          for (int32_t q : sig[p2]) {
            nfy_flat.push_back(q);
            nfy_flat.push_back(target[q]);
            nfy_flat.push_back(rbeg[q]);
            nfy_flat.push_back(rbeg[q + 1]);
          }
        }
      } else {
        rsuf.clear();
        P->max_nfy = 0;
        P->n_signals = 0;
      }
    }

    // ---- device image
    ImageLayout &L = P->lay;
    size_t off = 0;
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off = align256(off + bytes);
      return o;
    };
    std::vector<int32_t> eoff(poff.begin(), poff.end());
    L.eoff = take(eoff.size() * 4);
    L.hdr = take(hdr.size() * 4);
    L.eloc = take(eloc.size() * 4);
    L.geom = take(geomk.size() * 4);
    L.inc = take(incl.size() * 2);
    L.loff = take(loff.size() * 2);
    L.fid = take(fid.size() * 4);
    L.pfid = take(pfid.size() * 4);
    L.rvid = take(rvid.size() * 4);
    L.roff = take(roff.size() * 4);
    L.sidx = take(sidx.size() * 4);
    L.rslot = take(rslot.size() * 4);
    const std::vector<int32_t> rrec = reduction_records(rvid, roff, rslot);
    L.rrec = take(rrec.size() * 4);
    {
      // part-major reduction: a 16-byte record replaces the id (4) and the
      // offsets (4 (R + 1)); vertices with more slots also read offsets and list
      int64_t extra = 0;
      for (size_t v = 0; v < rvid.size(); ++v) {
        const int64_t ns = roff[v + 1] - roff[v];
        if (ns > kRecSlots) extra += 8 + 4 * ns;
      }
      P->rec_delta = 16 * int64_t(rvid.size()) + extra - 4 * int64_t(rvid.size()) - 4 * (int64_t(rvid.size()) + 1);
    }
    L.xinc = take(xinc.size() * 2);
    L.xlo = take(xlo.size() * 2);
    L.xlofs = take(xlofs.size() * 4);
    L.rfid = take(kind == EPK_SPMV ? red_foreign.size() * 4 : 0);
    L.eid = take(eid.size() * 4);
    L.xrvid = take(xrvid.size() * 4);
    L.xroff = take(xroff.size() * 4);
    L.xsidx = take(xsidx.size() * 4);
    L.xrslot = take(xrslot.size() * 4);
    L.xheavy = take(xheavy.size() * 4);
    L.heavy = take(heavy.size() * 4);
    L.nfy_off = take(nfy_off.size() * 4);
    L.nfy = take(nfy_flat.size() * 4);
    L.rsuf = take(rsuf.size() * 4);
    L.cnt = take(rsuf.empty() ? 0 : size_t(k) * 4 * kCntStride);  // zero in the image
    L.total = std::max<size_t>(off, 256);
    P->image.assign(L.total, 0);
    put(P->image, L.eoff, eoff);
    put(P->image, L.hdr, hdr);
    put(P->image, L.eloc, eloc);
    put(P->image, L.geom, geomk);
    put(P->image, L.inc, incl);
    put(P->image, L.loff, loff);
    P->n_loff = int64_t(loff.size());
    put(P->image, L.fid, fid);
    put(P->image, L.pfid, pfid);
    put(P->image, L.rvid, rvid);
    put(P->image, L.roff, roff);
    put(P->image, L.sidx, sidx);
    put(P->image, L.rslot, rslot);
    put(P->image, L.rrec, rrec);
    if (kind == EPK_SPMV) {
      put(P->image, L.xinc, xinc);
      put(P->image, L.xlo, xlo);
      put(P->image, L.xlofs, xlofs);
      put(P->image, L.rfid, red_foreign);
      put(P->image, L.eid, eid);
      put(P->image, L.xrvid, xrvid);
      put(P->image, L.xroff, xroff);
      put(P->image, L.xsidx, xsidx);
      put(P->image, L.xrslot, xrslot);
      put(P->image, L.xheavy, xheavy);
    }
    put(P->image, L.heavy, heavy);
    put(P->image, L.nfy_off, nfy_off);
    put(P->image, L.nfy, nfy_flat);
    put(P->image, L.rsuf, rsuf);
    const int nc = kind == EPK_SPMV ? 1 : 5;
    // the SpMV adjoint's x partials share the workspace (one launch pair at a time)
    P->ws_bytes = align256(std::max<size_t>(std::max(red_foreign.size() * nc, size_t(P->xn_slots)) * 4, 4));

    // ---- LDS and algorithmic bytes
    const int64_t C = P->stats.cost, Lds = P->stats.loads, R = P->R;
    const int64_t Cred = int64_t(red_foreign.size());
    if (kind == EPK_FLUX5) {
      set_flux_lds(P);
      const int64_t G = gstore, na = P->n_active_out;
      const int64_t meta = 32 * k + 4 * m + 4 * G * m + 4 * m + 2 * int64_t(loff.size()) + 4 * C;
      P->bytes_fwd_kernel = meta + 20 * Lds + 20 * na + 20 * C;
      P->bytes_bwd_kernel = meta + 40 * Lds + 20 * na + 20 * C;
      P->bytes_reduce = 4 * R + 4 * (R + 1) + 20 * Cred + 40 * R + 20 * (nred - na);
      P->bytes_reduce_qnew = P->bytes_reduce + 40 * R + 40 * (nred - na);
    } else {
      P->lds_fwd = spmv_lds(P->max_u, P->max_uy, P->wg, P->max_nf);
      P->lds_bwd = spmv_adj_lds(P->max_u, P->max_uy, cap);
      // x loads = owned x + foreign x over all parts
      int64_t Lxs = 0, Cx = 0;
      for (int64_t p = 0; p < k; ++p) {
        Lxs += P->own_count[p * 2] + (P->foreign_off[p * 2 + 1] - P->foreign_off[p * 2]);
        Cx += P->foreign_off[p * 2 + 1] - P->foreign_off[p * 2];
      }
      const int64_t na = P->n_active_out;
      P->bytes_fwd_kernel = 32 * k + 4 * m + 4 * m + 4 * Cx + 4 * Lxs + 4 * na + 4 * Cred;
      P->bytes_bwd_kernel = 0;
      P->bytes_reduce = 4 * R + 4 * (R + 1) + 4 * Cred + 8 * R + 4 * (nred - na);
      P->bytes_reduce_qnew = P->bytes_reduce;
    }
    if (P->lds_fwd > kMaxLdsBytes || P->lds_fwd_qn > kMaxLdsBytes || P->lds_bwd > kMaxLdsBytes) {
      delete P;
      *status = fail(EPK_ERANGE, "capacity needs more LDS than a workgroup may use");
      return nullptr;
    }
    const auto t1 = std::chrono::steady_clock::now();
    P->stats.plan_seconds = std::chrono::duration<double>(t1 - t0).count();
    return P;
  } catch (const std::bad_alloc &) {
    delete P;
    *status = fail(EPK_ENOMEM, "host allocation failed while building the plan");
    return nullptr;
  }
}

}  // namespace epk

extern "C" {

int epk_plan_create(const epk_graph *g, int32_t capacity, int32_t order, int32_t kind, epk_plan **out) {
  epk::clear_error();
  if (!out) return epk::fail(EPK_EINVAL, "out is NULL");
  *out = nullptr;
  int s = EPK_OK;
  epk_plan *p = epk::plan_build(g, capacity, order, kind, &s);
  if (!p) return s ? s : epk::fail(EPK_EINVAL, "plan build failed");
  *out = p;
  return EPK_OK;
}

int epk_plan_create_weighted(const epk_graph *g, int32_t capacity, int32_t order, int32_t kind,
                             const int32_t *class_weight, epk_plan **out) {
  epk::clear_error();
  if (!out) return epk::fail(EPK_EINVAL, "out is NULL");
  *out = nullptr;
  int s = EPK_OK;
  epk_plan *p = epk::plan_build(g, capacity, order, kind, &s, 0, nullptr, nullptr, class_weight);
  if (!p) return s ? s : epk::fail(EPK_EINVAL, "plan build failed");
  *out = p;
  return EPK_OK;
}

int epk_plan_create_hub(const epk_graph *g, int32_t capacity, int32_t kind, const int32_t *class_weight,
                        int32_t hub_degree, epk_plan **out) {
  epk::clear_error();
  if (!out) return epk::fail(EPK_EINVAL, "out is NULL");
  *out = nullptr;
  if (hub_degree < 1) return epk::fail(EPK_EINVAL, "hub_degree must be >= 1");
  int s = EPK_OK;
  epk_plan *p = epk::plan_build(g, capacity, EPK_ORDER_EP, kind, &s, 0, nullptr, nullptr, class_weight, hub_degree);
  if (!p) return s ? s : epk::fail(EPK_EINVAL, "plan build failed");
  *out = p;
  return EPK_OK;
}

int epk_plan_create_partitioned(const epk_graph *g, int32_t capacity, int64_t n_parts, const int32_t *part_of_edge,
                                const int32_t *task_order, int32_t kind, epk_plan **out) {
  epk::clear_error();
  if (!out) return epk::fail(EPK_EINVAL, "out is NULL");
  *out = nullptr;
  int s = EPK_OK;
  epk_plan *p = epk::plan_build(g, capacity, -1, kind, &s, n_parts, part_of_edge, task_order);
  if (!p) return s ? s : epk::fail(EPK_EINVAL, "plan build failed");
  *out = p;
  return EPK_OK;
}

int epk_plan_device_bytes(const epk_plan *p, size_t *image_bytes, size_t *workspace_bytes) {
  epk::clear_error();
  if (!p) return epk::fail(EPK_EINVAL, "plan is NULL");
  if (image_bytes) *image_bytes = p->lay.total;
  if (workspace_bytes) *workspace_bytes = p->ws_bytes;
  return EPK_OK;
}

int epk_plan_vertex_perm(const epk_plan *p, int32_t *packed_to_orig) {
  epk::clear_error();
  if (!p || (!packed_to_orig && p->n > 0)) return epk::fail(EPK_EINVAL, "NULL argument");
  if (p->n) std::memcpy(packed_to_orig, p->perm.data(), sizeof(int32_t) * size_t(p->n));
  return EPK_OK;
}

int epk_plan_part_of_edge(const epk_plan *p, int32_t *part_of_edge, int32_t *task_order) {
  epk::clear_error();
  if (!p) return epk::fail(EPK_EINVAL, "plan is NULL");
  if (p->m) {
    if (part_of_edge) std::memcpy(part_of_edge, p->part.data(), sizeof(int32_t) * size_t(p->m));
    if (task_order) std::memcpy(task_order, p->task.data(), sizeof(int32_t) * size_t(p->m));
  }
  return EPK_OK;
}

int epk_plan_layout(const epk_plan *p, int32_t *own_begin, int32_t *own_count, int64_t *foreign_offset,
                    int32_t *foreign_ids) {
  epk::clear_error();
  if (!p) return epk::fail(EPK_EINVAL, "plan is NULL");
  const size_t kc = size_t(p->k) * size_t(p->ncls);
  if (own_begin && kc) std::memcpy(own_begin, p->own_begin.data(), sizeof(int32_t) * kc);
  if (own_count && kc) std::memcpy(own_count, p->own_count.data(), sizeof(int32_t) * kc);
  if (foreign_offset) std::memcpy(foreign_offset, p->foreign_off.data(), sizeof(int64_t) * (kc + 1));
  if (foreign_ids && !p->foreign_ids.empty())
    std::memcpy(foreign_ids, p->foreign_ids.data(), sizeof(int32_t) * p->foreign_ids.size());
  return EPK_OK;
}

int epk_plan_stats(const epk_plan *p, epk_stats *s) {
  epk::clear_error();
  if (!p || !s) return epk::fail(EPK_EINVAL, "NULL argument");
  *s = p->stats;
  return EPK_OK;
}

int epk_plan_info(const epk_plan *p, int64_t *info, int32_t n_info) {
  epk::clear_error();
  if (!p || !info) return epk::fail(EPK_EINVAL, "NULL argument");
  const int64_t bf = epk::plan_bytes(p, 0), bb = epk::plan_bytes(p, 1), br = epk::plan_bytes(p, 2);
  // the single launch moves the reduction's bytes plus its signals (a 16-byte record read and a
  // 4-byte counter read and written per signal)
  const bool fu = epk::fused_in_use(p);
  const int64_t sig = 24 * p->n_signals;
  const int64_t v[17] = {p->k,
                         p->lds_fwd,
                         p->lds_bwd,
                         p->wg,
                         p->ncls,
                         bf + br + (fu ? sig : 0),
                         p->kind == EPK_FLUX5 ? bb + br + (fu ? sig : 0) : 0,
                         fu ? bf + br + sig : bf,
                         fu ? bb + br + sig : bb,
                         p->max_nf,
                         p->pipe,
                         p->pipe ? p->grid_pipe_fwd : 0,
                         p->pipe ? p->grid_pipe_bwd : 0,
                         p->lds_pipe_bwd,
                         p->vmajor ? 1 : 0,
                         p->staging,
                         fu ? 1 : 0};
  for (int32_t i = 0; i < n_info && i < 17; ++i) info[i] = v[i];
  return EPK_OK;
}

int epk_plan_set_fused(epk_plan *p, int32_t on) {
  epk::clear_error();
  if (!p) return epk::fail(EPK_EINVAL, "plan is NULL");
  if (on != 0 && on != 1) return epk::fail(EPK_EINVAL, "on must be 0 or 1");
  if (on && !p->fused_ok) return epk::fail(EPK_ESTATE, "this plan cannot sum its replicated vertices in one launch");
  p->fused = on == 1;
  return EPK_OK;
}

int epk_plan_set_launch(epk_plan *p, int32_t wg, int32_t xcd_swizzle) {
  epk::clear_error();
  if (!p) return epk::fail(EPK_EINVAL, "plan is NULL");
  if (wg != 0) {
    if (wg < 64 || wg > 1024 || wg % 64) return epk::fail(EPK_EINVAL, "workgroup must be 64..1024, multiple of 64");
    if (p->kind == EPK_SPMV && 4 * wg < p->cap) return epk::fail(EPK_EINVAL, "SpMV needs capacity <= 4 * workgroup");
    if (p->kind == EPK_FLUX5 && p->cap > 8 * wg) return epk::fail(EPK_EINVAL, "FLUX5 needs capacity <= 8 * workgroup");
  }
  if (xcd_swizzle < -1 || xcd_swizzle > 1) return epk::fail(EPK_EINVAL, "xcd_swizzle must be -1, 0 or 1");
  if (wg != 0) {
    p->wg = wg;
    if (p->kind == EPK_SPMV) p->lds_fwd = epk::spmv_lds(p->max_u, p->max_uy, wg, p->max_nf);
  }
  if (xcd_swizzle >= 0) p->swizzle = xcd_swizzle;
  p->pipe = 0;  // the pipelined grid depends on both: set it again
  return EPK_OK;
}

int epk_plan_set_staging(epk_plan *p, int32_t staged) {
  epk::clear_error();
  if (!p) return epk::fail(EPK_EINVAL, "plan is NULL");
  if (staged != 0 && staged != 1) return epk::fail(EPK_EINVAL, "staged must be 0 or 1");
  if (p->kind != EPK_FLUX5) return epk::fail(EPK_EINVAL, "the cache-only kernels are for FLUX5 plans");
  if (!staged && (p->lds_cached_fwd > epk::kMaxLdsBytes || p->lds_cached_bwd > epk::kMaxLdsBytes))
    return epk::fail(EPK_ERANGE, "capacity needs more LDS than a workgroup may use");
  p->staging = staged;
  if (!staged) p->pipe = 0;  // the pipelined launch stages states
  return EPK_OK;
}

int epk_plan_set_slot_layout(epk_plan *p, int32_t layout) {
  epk::clear_error();
  if (!p) return epk::fail(EPK_EINVAL, "plan is NULL");
  if (layout < -1 || layout > 1) return epk::fail(EPK_EINVAL, "layout must be -1, 0 or 1");
  const bool before = p->vmajor;
  p->vmajor = layout < 0 ? epk::auto_vmajor(p) : layout == 1;
  if (p->kind == EPK_FLUX5 && p->vmajor != before) {
    // the slot indices take LDS in the vertex-major layout: resize, and keep
    // the old layout if the kernels in use would no longer fit
    epk::set_flux_lds(p);
    const int64_t M = epk::kMaxLdsBytes;
    const bool over = p->lds_fwd > M || p->lds_fwd_qn > M || p->lds_bwd > M ||
                      (!p->staging && (p->lds_cached_fwd > M || p->lds_cached_bwd > M)) ||
                      (p->pipe && (p->lds_pipe_fwd_qn > M || p->lds_pipe_bwd > M));
    if (over) {
      p->vmajor = before;
      epk::set_flux_lds(p);
      return epk::fail(EPK_ERANGE, "the vertex-major layout's slot indices do not fit in LDS");
    }
    if (p->pipe) return epk_plan_set_pipeline(p, p->pipe);  // grids follow the LDS size
  }
  return EPK_OK;
}

void epk_plan_destroy(epk_plan *p) { delete p; }

}  // extern "C"
