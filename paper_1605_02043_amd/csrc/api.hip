// Device-side C ABI of libepk: upload, forward, adjoint, SpMV, permutation,
// batched persistent launch and capacity autotuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "epk_internal.h"
#include "kernels.h"

namespace epk {

template <typename T>
static const T *dptr(void *base, size_t off) {
  return reinterpret_cast<const T *>(static_cast<uint8_t *>(base) + off);
}

DevPlan dev_plan(const epk_plan *p) {
  DevPlan P{};
  void *b = p->d_image;
  const ImageLayout &L = p->lay;
  P.hdr = dptr<int32_t>(b, L.hdr);
  P.eoff = dptr<int32_t>(b, L.eoff);
  P.eloc = dptr<uint32_t>(b, L.eloc);
  P.geom = dptr<float>(b, L.geom);
  P.inc = dptr<uint16_t>(b, L.inc);
  P.loff = dptr<uint16_t>(b, L.loff);
  P.fid = dptr<int32_t>(b, L.fid);
  P.pfid = dptr<int32_t>(b, L.pfid);
  P.rvid = dptr<int32_t>(b, L.rvid);
  P.roff = dptr<int32_t>(b, L.roff);
  P.sidx = p->vmajor ? dptr<int32_t>(b, L.sidx) : nullptr;
  P.rslot = p->vmajor ? nullptr : dptr<int32_t>(b, L.rslot);
  P.rrec = p->vmajor ? nullptr : dptr<int32_t>(b, L.rrec);
  P.heavy = dptr<int32_t>(b, L.heavy);
  P.iso = nullptr;
  if (p->kind == EPK_SPMV) {
    P.xinc = dptr<uint16_t>(b, L.xinc);
    P.xlo = dptr<uint16_t>(b, L.xlo);
    P.xlofs = dptr<int32_t>(b, L.xlofs);
    P.rfid = dptr<int32_t>(b, L.rfid);
    P.eid = dptr<int32_t>(b, L.eid);
    P.xsidx = p->xvmajor ? dptr<int32_t>(b, L.xsidx) : nullptr;
  }
  P.m = p->me;
  P.k = int32_t(p->k);
  P.cap = p->cap;
  P.geom_ncomp = p->geom_ncomp;
  P.n = int32_t(p->n_out);
  P.n_active = int32_t(p->n_active_out);
  P.R = int32_t(p->R);
  P.n_heavy = int32_t(p->n_heavy);
  P.max_u = int32_t(p->max_u);
  P.max_uy = int32_t(p->max_uy);
  P.max_nf = int32_t(p->max_nf);
  P.n_iso = 0;
  P.n_slots = int32_t(p->n_slots);
  if (p->fused_ok) {
    P.nfy_off = dptr<int32_t>(b, L.nfy_off);
    P.nfy = dptr<int32_t>(b, L.nfy);
    P.rsuf = dptr<int32_t>(b, L.rsuf);
    P.cnt = reinterpret_cast<int32_t *>(static_cast<uint8_t *>(b) + L.cnt);
    P.max_nfy = int32_t(p->max_nfy);
  }
  return P;
}

DevPlan dev_plan_xreduce(const epk_plan *p) {
  DevPlan P = dev_plan(p);
  void *b = p->d_image;
  const ImageLayout &L = p->lay;
  P.rvid = dptr<int32_t>(b, L.xrvid);
  P.roff = dptr<int32_t>(b, L.xroff);
  P.sidx = p->xvmajor ? dptr<int32_t>(b, L.xsidx) : nullptr;
  P.rslot = p->xvmajor ? nullptr : dptr<int32_t>(b, L.xrslot);
  P.rrec = nullptr;  // the x class reduces through its slot lists
  P.heavy = dptr<int32_t>(b, L.xheavy);
  P.R = int32_t(p->xR);
  P.n_heavy = int32_t(p->xn_heavy);
  P.n = p->n_x;
  P.n_active = int32_t(p->xn_active);
  return P;
}

DevPlan dev_batch(const epk_batch *bt) {
  DevPlan P{};
  void *b = bt->d_image;
  const ImageLayout &L = bt->lay;
  P.hdr = dptr<int32_t>(b, L.hdr);
  P.eoff = dptr<int32_t>(b, L.eoff);
  P.eloc = dptr<uint32_t>(b, L.eloc);
  P.geom = dptr<float>(b, L.geom);
  P.inc = dptr<uint16_t>(b, L.inc);
  P.loff = dptr<uint16_t>(b, L.loff);
  P.fid = dptr<int32_t>(b, L.fid);
  P.rvid = dptr<int32_t>(b, L.rvid);
  P.roff = dptr<int32_t>(b, L.roff);
  P.sidx = bt->vmajor ? dptr<int32_t>(b, L.sidx) : nullptr;
  P.rslot = bt->vmajor ? nullptr : dptr<int32_t>(b, L.rslot);
  P.rrec = bt->vmajor ? nullptr : dptr<int32_t>(b, L.rrec);
  P.heavy = dptr<int32_t>(b, L.heavy);
  P.iso = dptr<int32_t>(b, L.iso);
  P.m = bt->me;
  P.k = int32_t(bt->k);
  P.cap = int32_t(bt->max_cap);
  P.geom_ncomp = 4;
  P.n = int32_t(bt->n);
  P.n_active = int32_t(bt->n);
  P.R = int32_t(bt->R);
  P.n_heavy = int32_t(bt->n_heavy);
  P.max_u = int32_t(bt->max_u);
  P.max_uy = 0;
  P.max_nf = int32_t(bt->max_nf);
  P.n_iso = int32_t(bt->n_iso);
  return P;
}

// The batch as the direct kernels see it: headers in item order and the
// padded foreign ids.
static DevPlan dev_batch_direct(const epk_batch *bt) {
  DevPlan P = dev_batch(bt);
  P.hdr = dptr<int32_t>(bt->d_image, bt->lay.hdr_items);
  P.pfid = dptr<int32_t>(bt->d_image, bt->lay.pfid);
  return P;
}

// Grid of a pipelined launch: per_cu workgroups on each of cus CUs, at most
// one per part, a multiple of 8 under the XCD-aware part lists.
static int64_t pipe_grid(int cus, int per_cu, int64_t k, bool swizzle) {
  int64_t g = std::max<int64_t>(1, std::min<int64_t>(int64_t(cus) * per_cu, k));
  if (swizzle) g = (g + 7) / 8 * 8;
  return g;
}

static int hip_status(hipError_t e, const char *what) {
  if (e == hipSuccess) return EPK_OK;
  return fail(EPK_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

extern "C" int epk_batch_set_launch(epk_batch *b, int32_t wg, int32_t direct);
static void size_batch_grids(epk_batch *b);

// ------------------------------------------------------------------ batch merge

template <typename T>
static const T *hptr(const epk_plan *p, size_t off) {
  return reinterpret_cast<const T *>(p->image.data() + off);
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static int batch_build(int32_t n_graphs, epk_plan *const *plans, epk_batch **out) {
  if (n_graphs < 1 || !plans) return fail(EPK_EINVAL, "need at least one plan");
  for (int32_t g = 0; g < n_graphs; ++g) {
    if (!plans[g]) return fail(EPK_EINVAL, "plan " + std::to_string(g) + " is NULL");
    if (plans[g]->kind != EPK_FLUX5 || plans[g]->geom_ncomp != 4)
      return fail(EPK_ESTATE, "batched plans must be FLUX5 with 4 geometry components");
  }
  epk_batch *B = new epk_batch();
  B->n_graphs = n_graphs;
  B->voff.assign(size_t(n_graphs) + 1, 0);
  std::vector<int32_t> hdr, fid, rvid, roff(1, 0), sidx, rslot, heavy, iso;
  std::vector<uint32_t> eloc;
  std::vector<float> geom;
  std::vector<uint16_t> inc, loff;
  int64_t eoff = 0, foff = 0, lofs_off = 0, rbase = 0, extra_pm = 0, extra_vm = 0;
  for (int32_t g = 0; g < n_graphs; ++g) {
    const epk_plan *p = plans[g];
    const ImageLayout &L = p->lay;
    const int64_t voff = B->voff[g];
    const int64_t C = int64_t(p->foreign_ids.size());
    const int64_t nloff = p->n_loff;
    const int32_t *h = hptr<int32_t>(p, L.hdr);
    for (int64_t q = 0; q < p->k; ++q) {
      const int32_t *hq = h + q * kHdrInts;
      hdr.push_back(int32_t(hq[0] + eoff));
      hdr.push_back(hq[1]);
      hdr.push_back(int32_t(hq[2] + voff));
      hdr.push_back(hq[3]);
      hdr.push_back(int32_t(hq[4] + foff));
      hdr.push_back(hq[5]);
      hdr.push_back(int32_t(hq[6] + lofs_off));
      hdr.push_back(hq[7]);
    }
    eloc.insert(eloc.end(), hptr<uint32_t>(p, L.eloc), hptr<uint32_t>(p, L.eloc) + p->me);
    geom.insert(geom.end(), hptr<float>(p, L.geom), hptr<float>(p, L.geom) + 3 * p->me);
    inc.insert(inc.end(), hptr<uint16_t>(p, L.inc), hptr<uint16_t>(p, L.inc) + 2 * p->me);
    loff.insert(loff.end(), hptr<uint16_t>(p, L.loff), hptr<uint16_t>(p, L.loff) + nloff);
    for (int64_t i = 0; i < C; ++i) fid.push_back(int32_t(hptr<int32_t>(p, L.fid)[i] + voff));
    for (int64_t i = 0; i < p->R; ++i) {
      rvid.push_back(int32_t(hptr<int32_t>(p, L.rvid)[i] + voff));
      roff.push_back(int32_t(hptr<int32_t>(p, L.roff)[i + 1] + foff));
    }
    for (int64_t i = 0; i < C; ++i) {
      sidx.push_back(int32_t(hptr<int32_t>(p, L.sidx)[i] + foff));
      rslot.push_back(int32_t(hptr<int32_t>(p, L.rslot)[i] + foff));
    }
    for (int64_t i = 0; i < p->n_heavy; ++i) heavy.push_back(int32_t(hptr<int32_t>(p, L.heavy)[i] + rbase));
    for (int64_t v = p->n_active_out; v < p->n_out; ++v) iso.push_back(int32_t(v + voff));
    B->voff[g + 1] = voff + p->n;
    B->max_u = std::max<int64_t>(B->max_u, p->max_u);
    B->max_nf = std::max<int64_t>(B->max_nf, p->max_nf);
    B->max_cap = std::max<int64_t>(B->max_cap, p->cap);
    // per launch pair: the slot indices (vertex-major) or the records and
    // long slot lists (part-major); added once the layout is known
    B->bytes_fwd += p->bytes_fwd_kernel + p->bytes_reduce;
    B->bytes_bwd += p->bytes_bwd_kernel + p->bytes_reduce;
    extra_pm += p->rec_delta;
    extra_vm += 4 * p->n_slots;
    eoff += p->me;
    B->m += p->m;
    foff += C;
    lofs_off += nloff;
    rbase += p->R;
    B->k += p->k;
  }
  B->me = eoff;
  B->n = B->voff[n_graphs];
  B->R = rbase;
  B->vmajor = int64_t(sidx.size()) > 4 * B->R;
  B->bytes_fwd += B->vmajor ? extra_vm : extra_pm;
  B->bytes_bwd += B->vmajor ? extra_vm : extra_pm;
  B->n_heavy = int64_t(heavy.size());
  B->n_iso = int64_t(iso.size());
  if (B->k >= (int64_t(1) << 31) || B->n >= (int64_t(1) << 31) || B->me >= (int64_t(1) << 31)) {
    delete B;
    return fail(EPK_ERANGE, "batch too large for 32-bit ids");
  }
  // The direct launch (one workgroup per item) finds item i's edge records at
  // i * cap and its foreign ids at i * max_nf before its header arrives, as
  // for a single plan: possible when every plan has the same capacity.
  B->direct_ok = true;
  for (int32_t g = 0; g < n_graphs; ++g)
    if (plans[g]->cap != plans[0]->cap || plans[g]->me != int64_t(plans[g]->k) * plans[g]->cap)
      B->direct_ok = false;
  std::vector<int32_t> hdr_items, pfid;
  if (B->direct_ok) {
    hdr_items = hdr;
    pfid.assign(size_t(B->k * std::max<int64_t>(B->max_nf, 1)), -1);
    int64_t item = 0;
    for (int32_t g = 0; g < n_graphs; ++g) {
      const epk_plan *p = plans[g];
      const int32_t *src = hptr<int32_t>(p, p->lay.pfid);
      for (int64_t q = 0; q < p->k; ++q, ++item)
        for (int64_t j = 0; j < p->max_nf; ++j) {
          const int32_t v = src[q * p->max_nf + j];
          pfid[size_t(item * B->max_nf + j)] = v < 0 ? -1 : int32_t(v + B->voff[g]);
        }
    }
  }
  // headers in processing order: largest parts first (ties: lower id first);
  // the pipelined kernel deals them round-robin over its workgroups
  {
    std::vector<int32_t> order(static_cast<size_t>(B->k));
    for (int64_t i = 0; i < B->k; ++i) order[i] = int32_t(i);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return hdr[size_t(a) * kHdrInts + 1] > hdr[size_t(b) * kHdrInts + 1];
    });
    std::vector<int32_t> sorted(hdr.size());
    for (int64_t i = 0; i < B->k; ++i)
      std::memcpy(&sorted[size_t(i) * kHdrInts], &hdr[size_t(order[i]) * kHdrInts], sizeof(int32_t) * kHdrInts);
    hdr.swap(sorted);
  }
  B->wg = std::min<int64_t>(256, std::max<int64_t>(64, ((B->max_cap + 63) / 64) * 64));
  B->lds_fwd = flux_pipe_lds(B->max_u, B->max_nf, B->max_cap, false, false, B->vmajor);
  B->lds_bwd = flux_pipe_lds(B->max_u, B->max_nf, B->max_cap, true, false, B->vmajor);
  B->lds_fwd_direct = flux_fwd_lds(B->max_u, B->max_nf, B->max_cap, B->vmajor);
  B->lds_bwd_direct = flux_bwd_lds(B->max_u, B->max_nf, B->max_cap, B->vmajor);
  if (B->lds_fwd_direct > kMaxLdsBytes || B->lds_bwd_direct > kMaxLdsBytes) B->direct_ok = false;
  B->direct = B->direct_ok;  // the faster kind on the meshes measured, where it can run
  if (B->lds_fwd > kMaxLdsBytes || B->lds_bwd > kMaxLdsBytes) {
    delete B;
    return fail(EPK_ERANGE, "batch needs more LDS than a workgroup may use");
  }
  ImageLayout &L = B->lay;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.hdr = take(hdr.size() * 4);
  L.eloc = take(eloc.size() * 4);
  L.geom = take(geom.size() * 4);
  L.inc = take(inc.size() * 2);
  L.loff = take(loff.size() * 2);
  L.fid = take(fid.size() * 4);
  L.rvid = take(rvid.size() * 4);
  L.roff = take(roff.size() * 4);
  L.sidx = take(sidx.size() * 4);
  L.rslot = take(rslot.size() * 4);
  const std::vector<int32_t> rrec = reduction_records(rvid, roff, rslot);
  L.rrec = take(rrec.size() * 4);
  L.heavy = take(heavy.size() * 4);
  L.iso = take(iso.size() * 4);
  L.hdr_items = take(hdr_items.size() * 4);
  L.pfid = take(pfid.size() * 4);
  L.total = off;
  B->image.assign(L.total, 0);
  auto put = [&](size_t o, const void *src, size_t bytes) {
    if (bytes) std::memcpy(B->image.data() + o, src, bytes);
  };
  put(L.hdr, hdr.data(), hdr.size() * 4);
  put(L.eloc, eloc.data(), eloc.size() * 4);
  put(L.geom, geom.data(), geom.size() * 4);
  put(L.inc, inc.data(), inc.size() * 2);
  put(L.loff, loff.data(), loff.size() * 2);
  put(L.fid, fid.data(), fid.size() * 4);
  put(L.rvid, rvid.data(), rvid.size() * 4);
  put(L.roff, roff.data(), roff.size() * 4);
  put(L.sidx, sidx.data(), sidx.size() * 4);
  put(L.rslot, rslot.data(), rslot.size() * 4);
  put(L.rrec, rrec.data(), rrec.size() * 4);
  put(L.heavy, heavy.data(), heavy.size() * 4);
  put(L.iso, iso.data(), iso.size() * 4);
  put(L.hdr_items, hdr_items.data(), hdr_items.size() * 4);
  put(L.pfid, pfid.data(), pfid.size() * 4);
  B->ws_bytes = align256(std::max<size_t>(size_t(foff) * 5 * 4, 4));
  *out = B;
  return EPK_OK;
}

// ------------------------------------------------------------------ autotune

__global__ void fill_kernel(float *p, int64_t n, float v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Key of a tuning problem: the graphs' sizes and the candidate capacities.
static std::string tune_key(const epk_graph *gs, int32_t n_graphs, const int32_t *caps, int32_t n_caps) {
  std::ostringstream os;
  int64_t n = 0, m = 0;
  for (int32_t g = 0; g < n_graphs; ++g) {
    n += gs[g].n_vertices;
    m += gs[g].n_edges;
  }
  os << "batch " << n_graphs << ' ' << n << ' ' << m;
  for (int32_t i = 0; i < n_caps; ++i) os << ' ' << caps[i];
  return os.str();
}

// Plans of all graphs at one capacity, built on up to 16 host threads.
static int build_plans(const epk_graph *gs, int32_t n_graphs, int32_t cap, std::vector<epk_plan *> &plans) {
  plans.assign(size_t(n_graphs), nullptr);
  const int nth = int(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  std::vector<int> status(static_cast<size_t>(nth), EPK_OK);
  std::vector<std::string> msg(static_cast<size_t>(nth));
  std::atomic<int32_t> next{0};
  auto work = [&](int w) {
    for (int32_t g; (g = next.fetch_add(1)) < n_graphs;) {
      const int st = epk_plan_create(&gs[g], cap, EPK_ORDER_EP, EPK_FLUX5, &plans[size_t(g)]);
      if (st && status[size_t(w)] == EPK_OK) {
        status[size_t(w)] = st;
        msg[size_t(w)] = epk_last_error();  // the error text is per thread
      }
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < nth; ++w) pool.emplace_back(work, w);
  work(0);
  for (auto &t : pool) t.join();
  for (int w = 0; w < nth; ++w)
    if (status[size_t(w)]) {
      for (epk_plan *p : plans) epk_plan_destroy(p);
      plans.clear();
      return fail(status[size_t(w)], msg[size_t(w)]);
    }
  return EPK_OK;
}

// Time (ms) of one batched forward + adjoint pass over all graphs at one
// capacity, run out of d_scratch: the median of 5 timings of 5 back-to-back
// passes.  EPK_ERANGE if the batch does not fit in the scratch memory or in
// LDS.  Also returns the batch's algorithmic bytes per pass.
// Workgroup sizes the autotuner tries at capacity cap, largest first (ties go
// to the larger): multiples of 64 up to the pipelined kernels' 256 lanes, with
// at most two edges per lane.
static std::vector<int32_t> tune_wgs(int32_t cap) {
  std::vector<int32_t> w;
  for (int32_t wg : {256, 128, 64})
    if (2 * wg >= cap) w.push_back(wg);
  if (w.empty()) w.push_back(256);
  return w;
}

// Times the batched forward + adjoint launch of all graphs at capacity cap,
// once per launch shape (workgroup size, one workgroup per item or
// pipelined) in shapes (median of 5 timings of 5 passes each): ms_out[i] for
// shapes[i], 1e30 where that shape cannot run.  The plans and the merged
// image are built once per capacity.
struct LaunchShape {
  int32_t wg, direct;
};

static int time_batch(const epk_graph *gs, int32_t n_graphs, int32_t cap, const std::vector<LaunchShape> &shapes,
                      void *d_scratch, size_t scratch_bytes, hipStream_t s, std::vector<float> &ms_out,
                      int64_t *bytes_out) {
  ms_out.assign(shapes.size(), 1e30f);
  std::vector<epk_plan *> plans;
  int st = build_plans(gs, n_graphs, cap, plans);
  if (st) return st;
  epk_batch *b = nullptr;
  st = epk_batch_create(n_graphs, plans.data(), &b);
  for (epk_plan *p : plans) epk_plan_destroy(p);
  if (st) return st;
  size_t img = 0, ws = 0;
  epk_batch_device_bytes(b, &img, &ws);
  const size_t state = align256(size_t(b->n) * 5 * 4);
  if (img + ws + 3 * state > scratch_bytes) {
    epk_batch_destroy(b);
    return fail(EPK_ERANGE, "autotune scratch too small");
  }
  uint8_t *base = static_cast<uint8_t *>(d_scratch);
  float *q = reinterpret_cast<float *>(base + img + ws);
  float *g = reinterpret_cast<float *>(base + img + ws + state);
  float *o = reinterpret_cast<float *>(base + img + ws + 2 * state);
  const int64_t nq = b->n * 5;
  if (nq) {
    hipLaunchKernelGGL(fill_kernel, dim3(unsigned((nq + 255) / 256)), dim3(256), 0, s, q, nq, 1.0f);
    hipLaunchKernelGGL(fill_kernel, dim3(unsigned((nq + 255) / 256)), dim3(256), 0, s, g, nq, 1.0f);
  }
  st = epk_batch_upload(b, base, s);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  constexpr int kPasses = 5;
  for (size_t w = 0; w < shapes.size() && !st; ++w) {
    // a shape this batch cannot run (capacity too large for the lanes, or
    // mixed capacities for one workgroup per item) is skipped
    if (epk_batch_set_launch(b, shapes[w].wg, shapes[w].direct) != EPK_OK) continue;
    std::vector<float> t;
    for (int it = 0; it < 6 && !st; ++it) {  // the first timing warms up
      (void)hipEventRecord(e0, s);
      for (int l = 0; l < kPasses && !st; ++l) {
        st = epk_batch_forward(b, q, o, base + img, s);
        if (!st) st = epk_batch_backward(b, q, g, o, base + img, s);
      }
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (it >= 1) t.push_back(ms / kPasses);
    }
    if (!st) {
      std::sort(t.begin(), t.end());
      ms_out[w] = t[t.size() / 2];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *bytes_out = b->bytes_fwd + b->bytes_bwd;
  epk_batch_destroy(b);
  return st;
}


// The batch's persistent grids: as many workgroups of b->wg lanes as fit on
// the device's CUs (LDS, waves), at most one per work item.
static void size_batch_grids(epk_batch *b) {
  b->grid_fwd = pipe_grid(b->cus, pipe_blocks_per_cu(int(b->wg), size_t(b->lds_fwd), false, 4, false, int(b->max_cap)),
                          b->k, false);
  b->grid_bwd = pipe_grid(b->cus, pipe_blocks_per_cu(int(b->wg), size_t(b->lds_bwd), true, 4, false, int(b->max_cap)),
                          b->k, false);
}

}  // namespace epk

using namespace epk;

extern "C" {

int epk_plan_upload(epk_plan *p, void *d_image, void *stream) {
  clear_error();
  if (!p || !d_image) return fail(EPK_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(d_image) % 256) return fail(EPK_EINVAL, "d_image must be 256-byte aligned");
  const hipError_t e = hipMemcpyAsync(d_image, p->image.data(), p->lay.total, hipMemcpyHostToDevice,
                                      static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_status(e, "image upload");
  p->d_image = d_image;
  return EPK_OK;
}

int epk_plan_set_pipeline(epk_plan *p, int32_t blocks_per_cu) {
  clear_error();
  if (!p) return fail(EPK_EINVAL, "plan is NULL");
  if (blocks_per_cu < -1) return fail(EPK_EINVAL, "blocks_per_cu must be -1, 0 or positive");
  if (blocks_per_cu == 0) {
    p->pipe = 0;
    return EPK_OK;
  }
  if (p->kind != EPK_FLUX5) return fail(EPK_EINVAL, "the pipelined launch is for FLUX5 plans");
  if (!p->staging) return fail(EPK_ESTATE, "the pipelined launch stages states: set staging first");
  if (p->wg > 256) return fail(EPK_EINVAL, "the pipelined launch needs a workgroup of at most 256");
  if (p->lds_pipe_fwd_qn > kMaxLdsBytes || p->lds_pipe_bwd > kMaxLdsBytes)
    return fail(EPK_ERANGE, "parts too large for the pipelined launch's LDS buffers");
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_status(e, "CU count");
  const int G = p->geom_ncomp;
  const int occ[3] = {pipe_blocks_per_cu(p->wg, size_t(p->lds_pipe_fwd), false, G, false, p->cap),
                      pipe_blocks_per_cu(p->wg, size_t(p->lds_pipe_fwd_qn), false, G, true, p->cap),
                      pipe_blocks_per_cu(p->wg, size_t(p->lds_pipe_bwd), true, G, false, p->cap)};
  auto per = [&](int o) { return blocks_per_cu < 0 ? o : std::min(o, int(blocks_per_cu)); };
  p->grid_pipe_fwd = pipe_grid(cus, per(occ[0]), p->k, p->swizzle);
  p->grid_pipe_fwd_qn = pipe_grid(cus, per(occ[1]), p->k, p->swizzle);
  p->grid_pipe_bwd = pipe_grid(cus, per(occ[2]), p->k, p->swizzle);
  p->pipe = blocks_per_cu;
  return EPK_OK;
}

static int run_stage(const epk_plan *p, int32_t op, int32_t stage, const float *in, const float *g_r, float *out,
                     float dt, float *q_new, void *d_ws, void *stream) {
  if (!p) return fail(EPK_EINVAL, "plan is NULL");
  if (op < EPK_OP_FORWARD || op > EPK_OP_SPMV) return fail(EPK_EINVAL, "unknown op");
  if (stage < -1 || stage > 1) return fail(EPK_EINVAL, "stage must be 0 or 1");
  if ((op == EPK_OP_SPMV) != (p->kind == EPK_SPMV)) return fail(EPK_ESTATE, "op does not match the plan's kind");
  if (!p->d_image) return fail(EPK_ESTATE, "plan not uploaded");
  if (op == EPK_OP_SPMV) {
    if ((p->n_x > 0 && !in) || (p->n_out > 0 && !out)) return fail(EPK_EINVAL, "x or y is NULL");
    if (p->R > 0 && !d_ws) return fail(EPK_EINVAL, "workspace is NULL");
  } else {
    if (p->n > 0 && (!in || !out)) return fail(EPK_EINVAL, "state or output is NULL");
    if (op == EPK_OP_BACKWARD && p->n > 0 && !g_r) return fail(EPK_EINVAL, "g_r is NULL");
    if (p->stats.cost > 0 && !d_ws) return fail(EPK_EINVAL, "workspace is NULL");
  }
  const DevPlan P = dev_plan(p);
  hipStream_t s = static_cast<hipStream_t>(stream);
  float *ws = static_cast<float *>(d_ws);
  if (op == EPK_OP_BACKWARD) q_new = nullptr;
  if (op != EPK_OP_SPMV && fused_in_use(p)) {
    // single launch: the part kernel also sums the replicated vertices (stage 1 has nothing left)
    if (stage == 1) return EPK_OK;
    const hipError_t e =
        op == EPK_OP_FORWARD
            ? launch_flux_fwd(P, p->wg, size_t(q_new ? p->lds_fwd_qn : p->lds_fwd), in, out, q_new, dt, ws, p->swizzle,
                              s, true)
            : launch_flux_bwd(P, p->wg, size_t(p->lds_bwd), in, g_r, out, ws, p->swizzle, s, true);
    return e == hipSuccess ? EPK_OK : hip_status(e, "part kernel launch");
  }
  if (stage != 1) {  // -1 runs both
    hipError_t e = hipSuccess;
    if (op != EPK_OP_SPMV && !p->staging) {
      if (op == EPK_OP_FORWARD)
        e = launch_flux_cached(P, p->wg, size_t(p->lds_cached_fwd), in, nullptr, out, q_new, dt, ws, false, p->swizzle,
                               s);
      else
        e = launch_flux_cached(P, p->wg, size_t(p->lds_cached_bwd), in, g_r, out, nullptr, 0.f, ws, true, p->swizzle,
                               s);
    } else if (op != EPK_OP_SPMV && p->pipe) {
      if (op == EPK_OP_FORWARD)
        e = launch_flux_pipe(P, p->wg, int(q_new ? p->grid_pipe_fwd_qn : p->grid_pipe_fwd),
                             size_t(q_new ? p->lds_pipe_fwd_qn : p->lds_pipe_fwd), in, nullptr, out, q_new, dt, ws,
                             false, p->swizzle, s);
      else
        e = launch_flux_pipe(P, p->wg, int(p->grid_pipe_bwd), size_t(p->lds_pipe_bwd), in, g_r, out, nullptr, 0.f, ws,
                             true, p->swizzle, s);
    } else if (op == EPK_OP_FORWARD)
      e = launch_flux_fwd(P, p->wg, size_t(q_new ? p->lds_fwd_qn : p->lds_fwd), in, out, q_new, dt, ws, p->swizzle, s);
    else if (op == EPK_OP_BACKWARD)
      e = launch_flux_bwd(P, p->wg, size_t(p->lds_bwd), in, g_r, out, ws, p->swizzle, s);
    else
      e = launch_spmv(P, p->wg, size_t(p->lds_fwd), in, out, ws, p->swizzle, s);
    if (e != hipSuccess) return hip_status(e, "part kernel launch");
  }
  if (stage != 0) {
    const int nc = op == EPK_OP_SPMV ? 1 : 5;
    const float *qin = op == EPK_OP_FORWARD ? in : nullptr;
    return hip_status(launch_reduce(P, nc, out, ws, qin, q_new, dt, s), "reduce launch");
  }
  return EPK_OK;
}

int epk_run_stage(const epk_plan *p, int32_t op, int32_t stage, const float *in, const float *g_r, float *out,
                  float dt, float *q_new, void *d_ws, void *stream) {
  clear_error();
  if (stage != 0 && stage != 1) return fail(EPK_EINVAL, "stage must be 0 or 1");
  return run_stage(p, op, stage, in, g_r, out, dt, q_new, d_ws, stream);
}

int epk_run_stage_timed(const epk_plan *p, int32_t op, int32_t stage, const float *in, const float *g_r, float *out,
                        float dt, float *q_new, void *d_ws, void *stream, float *ms) {
  clear_error();
  if (!ms) return fail(EPK_EINVAL, "ms is NULL");
  *ms = 0.f;
  if (stage != 0 && stage != 1) return fail(EPK_EINVAL, "stage must be 0 or 1");
  if (!p) return fail(EPK_EINVAL, "plan is NULL");
  if (!p->d_image) return fail(EPK_ESTATE, "plan not uploaded");
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e != hipSuccess) {
    if (a) hipEventDestroy(a);
    return hip_status(e, "event create");
  }
  g_timing = LaunchTiming{a, b, 0};
  int st = run_stage(p, op, stage, in, g_r, out, dt, q_new, d_ws, stream);
  const int launched = g_timing.launched;
  g_timing = LaunchTiming{};
  if (st == EPK_OK && launched > 0) {
    e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    if (e != hipSuccess) st = hip_status(e, "kernel timing");
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  return st;
}

int epk_forward(const epk_plan *p, const float *q, float *r, float dt, float *q_new, void *d_ws, void *stream) {
  clear_error();
  return run_stage(p, EPK_OP_FORWARD, -1, q, nullptr, r, dt, q_new, d_ws, stream);
}

// ---- forward for callers that cannot allocate
//
// The replicated-vertex partials of epk_forward_scratch live in this fixed
// array instead of a caller workspace.  Each device holds its own copy from
// module load until the process ends.  In host code `scratch` names a host
// stand-in, never the device memory: the kernels get the address that
// hipGetSymbolAddress returns with the device current (kept per device).
// Nothing in the array has to start at zero: the part kernel writes every
// partial before the reduction reads it.  Calls that overlap on one device
// share the array and race.
constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::atomic<void *> g_scratch_ptr[kScratchDevices];

static int scratch_of_current_device(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "current device");
  if (dev < 0 || dev >= kScratchDevices) return fail(EPK_ERANGE, "device index beyond the scratch table");
  void *ptr = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (!ptr) {  // first call on this device: its copy's address (the same on every later call)
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_status(e, "address of the scratch array");
    if (!ptr) return fail(EPK_EHIP, "address of the scratch array is NULL");
    g_scratch_ptr[dev].store(ptr, std::memory_order_release);
  }
  *out = ptr;
  return EPK_OK;
}

int epk_forward_scratch(const epk_plan *p, const float *q, float *r, float dt, float *q_new, void *stream) {
  clear_error();
  if (!p) return fail(EPK_EINVAL, "plan is NULL");
  if (p->kind != EPK_FLUX5) return fail(EPK_ESTATE, "op does not match the plan's kind");
  if (p->ws_bytes > kScratchBytes) return fail(EPK_ERANGE, "the plan's partials exceed the 16 MiB scratch array");
  if (!p->d_image) return fail(EPK_ESTATE, "plan not uploaded");
  void *ws = nullptr;
  const int st = scratch_of_current_device(&ws);
  if (st) return st;
  return run_stage(p, EPK_OP_FORWARD, -1, q, nullptr, r, dt, q_new, ws, stream);
}

int epk_backward(const epk_plan *p, const float *q, const float *g_r, float *g_q, void *d_ws, void *stream) {
  clear_error();
  return run_stage(p, EPK_OP_BACKWARD, -1, q, g_r, g_q, 0.f, nullptr, d_ws, stream);
}

int epk_spmv(const epk_plan *p, const float *x, float *y, void *d_ws, void *stream) {
  clear_error();
  return run_stage(p, EPK_OP_SPMV, -1, x, nullptr, y, 0.f, nullptr, d_ws, stream);
}

int epk_spmv_adjoint(const epk_plan *p, const float *x, const float *g_y, float *g_x, float *g_w, void *d_ws,
                     void *stream) {
  clear_error();
  if (!p) return fail(EPK_EINVAL, "plan is NULL");
  if (p->kind != EPK_SPMV) return fail(EPK_ESTATE, "not an SpMV plan");
  if (!p->d_image) return fail(EPK_ESTATE, "plan not uploaded");
  if ((p->n_x > 0 && !g_x) || (p->n_out > 0 && !g_y)) return fail(EPK_EINVAL, "g_x or g_y is NULL");
  if (g_w && !x && p->n_x > 0) return fail(EPK_EINVAL, "g_w needs x");
  if (p->xn_slots > 0 && !d_ws) return fail(EPK_EINVAL, "workspace is NULL");
  if (p->lds_bwd > kMaxLdsBytes) return fail(EPK_ERANGE, "parts too large for the adjoint's LDS");
  const DevPlan P = dev_plan(p);
  hipStream_t s = static_cast<hipStream_t>(stream);
  float *ws = static_cast<float *>(d_ws);
  const int wg_adj = std::max(64, ((p->cap + 63) / 64) * 64);  // one edge per lane
  hipError_t e = launch_spmv_adjoint(P, wg_adj, size_t(p->lds_bwd), x, g_y, g_x, g_w, ws, p->swizzle, s);
  if (e != hipSuccess) return hip_status(e, "adjoint kernel launch");
  return hip_status(launch_reduce(dev_plan_xreduce(p), 1, g_x, ws, nullptr, nullptr, 0.f, s), "reduce launch");
}

int epk_permute_rows(const float *src, float *dst, const int32_t *idx, int64_t n_rows, int32_t ncomp, int32_t inverse,
                     void *stream) {
  clear_error();
  if (n_rows < 0 || ncomp < 1) return fail(EPK_EINVAL, "bad sizes");
  if (n_rows > 0 && (!src || !dst || !idx)) return fail(EPK_EINVAL, "NULL argument");
  return hip_status(launch_permute(src, dst, idx, n_rows, ncomp, inverse, static_cast<hipStream_t>(stream)),
                    "permute launch");
}

int epk_batch_create(int32_t n_graphs, epk_plan *const *plans, epk_batch **out) {
  clear_error();
  if (!out) return fail(EPK_EINVAL, "out is NULL");
  *out = nullptr;
  try {
    return batch_build(n_graphs, plans, out);
  } catch (const std::bad_alloc &) {
    return fail(EPK_ENOMEM, "host allocation failed while merging the batch");
  }
}

int epk_batch_device_bytes(const epk_batch *b, size_t *image_bytes, size_t *workspace_bytes) {
  clear_error();
  if (!b) return fail(EPK_EINVAL, "batch is NULL");
  if (image_bytes) *image_bytes = b->lay.total;
  if (workspace_bytes) *workspace_bytes = b->ws_bytes;
  return EPK_OK;
}

int epk_batch_upload(epk_batch *b, void *d_image, void *stream) {
  clear_error();
  if (!b || !d_image) return fail(EPK_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(d_image) % 256) return fail(EPK_EINVAL, "d_image must be 256-byte aligned");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "hipGetDevice");
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_status(e, "CU count");
  b->cus = cus;
  size_batch_grids(b);
  e = hipMemcpyAsync(d_image, b->image.data(), b->lay.total, hipMemcpyHostToDevice, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_status(e, "batch upload");
  b->d_image = d_image;
  return EPK_OK;
}

int epk_batch_set_launch(epk_batch *b, int32_t wg, int32_t direct) {
  clear_error();
  if (!b) return fail(EPK_EINVAL, "batch is NULL");
  if (direct < -1 || direct > 1) return fail(EPK_EINVAL, "direct must be -1, 0 or 1");
  if (wg != 0) {
    if (wg < 64 || wg > 256 || wg % 64) return fail(EPK_EINVAL, "batch workgroup must be 64..256, multiple of 64");
    if (b->max_cap > 8 * int64_t(wg)) return fail(EPK_EINVAL, "batch capacity exceeds 8 edges per lane");
  }
  if (direct == 1 && !b->direct_ok)
    return fail(EPK_ESTATE, "one workgroup per item needs one capacity for all graphs (and LDS for the largest part)");
  if (wg != 0) b->wg = wg;
  if (direct >= 0) b->direct = direct == 1;
  if (b->cus) size_batch_grids(b);
  return EPK_OK;
}

int epk_batch_vertex_offsets(const epk_batch *b, int64_t *vertex_offset) {
  clear_error();
  if (!b || !vertex_offset) return fail(EPK_EINVAL, "NULL argument");
  std::memcpy(vertex_offset, b->voff.data(), sizeof(int64_t) * b->voff.size());
  return EPK_OK;
}

int epk_batch_info(const epk_batch *b, int64_t *info, int32_t n_info) {
  clear_error();
  if (!b || !info) return fail(EPK_EINVAL, "NULL argument");
  const int64_t v[10] = {b->k,  b->grid_fwd, b->lds_fwd,  b->bytes_fwd,  b->bytes_bwd,
                         b->wg, b->m,        b->grid_bwd, int64_t(b->direct), int64_t(b->direct_ok)};
  for (int32_t i = 0; i < n_info && i < 10; ++i) info[i] = v[i];
  return EPK_OK;
}

int epk_batch_forward(const epk_batch *b, const float *q, float *r, void *d_ws, void *stream) {
  clear_error();
  if (!b) return fail(EPK_EINVAL, "batch is NULL");
  if (!b->d_image) return fail(EPK_ESTATE, "batch not uploaded");
  if (b->n > 0 && (!q || !r || !d_ws)) return fail(EPK_EINVAL, "NULL argument");
  const DevPlan P = dev_batch(b);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = b->direct ? launch_flux_fwd(dev_batch_direct(b), int(b->wg), size_t(b->lds_fwd_direct), q, r,
                                             nullptr, 0.f, static_cast<float *>(d_ws), 1, s)
                           : launch_flux_pipe(P, int(b->wg), int(b->grid_fwd), size_t(b->lds_fwd), q, nullptr, r,
                                              nullptr, 0.f, static_cast<float *>(d_ws), false, 0, s);
  if (e != hipSuccess) return hip_status(e, "batch forward launch");
  return hip_status(launch_reduce(P, 5, r, static_cast<const float *>(d_ws), q, nullptr, 0.f, s), "reduce launch");
}

int epk_batch_backward(const epk_batch *b, const float *q, const float *g_r, float *g_q, void *d_ws, void *stream) {
  clear_error();
  if (!b) return fail(EPK_EINVAL, "batch is NULL");
  if (!b->d_image) return fail(EPK_ESTATE, "batch not uploaded");
  if (b->n > 0 && (!q || !g_r || !g_q || !d_ws)) return fail(EPK_EINVAL, "NULL argument");
  const DevPlan P = dev_batch(b);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = b->direct ? launch_flux_bwd(dev_batch_direct(b), int(b->wg), size_t(b->lds_bwd_direct), q, g_r, g_q,
                                             static_cast<float *>(d_ws), 1, s)
                           : launch_flux_pipe(P, int(b->wg), int(b->grid_bwd), size_t(b->lds_bwd), q, g_r, g_q,
                                              nullptr, 0.f, static_cast<float *>(d_ws), true, 0, s);
  if (e != hipSuccess) return hip_status(e, "batch adjoint launch");
  return hip_status(launch_reduce(P, 5, g_q, static_cast<const float *>(d_ws), nullptr, nullptr, 0.f, s),
                    "reduce launch");
}

void epk_batch_destroy(epk_batch *b) { delete b; }

int epk_autotune(const epk_graph *gs, int32_t n_graphs, const int32_t *caps, int32_t n_caps, const char *cache_path,
                 void *d_scratch, size_t scratch_bytes, void *stream, int32_t *chosen_cap, int32_t *chosen_wg,
                 int32_t *chosen_direct) {
  clear_error();
  if (!gs || n_graphs < 1 || !caps || n_caps < 1 || !chosen_cap) return fail(EPK_EINVAL, "bad arguments");
  if (!d_scratch) return fail(EPK_EINVAL, "d_scratch is NULL");
  for (int32_t i = 0; i < n_caps; ++i)
    if (caps[i] < 1) return fail(EPK_EINVAL, "capacities must be >= 1");
  for (int32_t g = 0; g < n_graphs; ++g) {
    const int v = validate_graph(&gs[g], EPK_FLUX5);
    if (v) return v;
    if (gs[g].geom_ncomp != 4) return fail(EPK_EINVAL, "batched graphs need 4 geometry components");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const std::string key = tune_key(gs, n_graphs, caps, n_caps);
  int32_t best_cap = 0, best_wg = 0, best_direct = 0;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const size_t bar = line.find('|');
      if (bar == std::string::npos || line.substr(0, bar) != key) continue;
      std::istringstream rest(line.substr(bar + 1));
      int32_t c = 0, w = 0, d = 0;
      if (rest >> c >> w) {
        if (!(rest >> d)) d = 0;  // lines written before the launch kind was tuned
        best_cap = c;
        best_wg = w;
        best_direct = d;
      }
    }
  }
  if (!best_cap) {
    // one capacity for the whole batch: its launch sizes every workgroup's
    // LDS for the largest parts, so mixing capacities only lowers occupancy.
    // Timings within kTie of the fastest count as equal; among those the
    // fewest algorithmic bytes win, so that timing noise does not decide.
    constexpr float kTie = 1.02f;
    struct Trial {
      int32_t cap;
      LaunchShape shape;
      float ms;
      int64_t bytes;
    };
    std::vector<Trial> trials;
    float best = 1e30f;
    for (int32_t i = 0; i < n_caps; ++i) {
      std::vector<LaunchShape> shapes;  // one workgroup per item first, then pipelined; larger workgroups first
      for (int32_t direct : {1, 0})
        for (int32_t wg : tune_wgs(caps[i])) shapes.push_back({wg, direct});
      std::vector<float> ms;
      int64_t bytes = 0;
      const int st = time_batch(gs, n_graphs, caps[i], shapes, d_scratch, scratch_bytes, s, ms, &bytes);
      if (st == EPK_ERANGE) continue;  // capacity not runnable here
      if (st) return st;
      for (size_t w = 0; w < shapes.size(); ++w) {
        trials.push_back({caps[i], shapes[w], ms[w], bytes});
        best = std::min(best, ms[w]);
      }
    }
    if (best >= 1e30f) return fail(EPK_ERANGE, "no capacity could be timed (scratch or LDS too small)");
    int64_t fewest = -1;
    for (const Trial &t : trials)  // in trial order: caps as listed, then the shapes' order
      if (t.ms <= best * kTie && (fewest < 0 || t.bytes < fewest)) {
        fewest = t.bytes;
        best_cap = t.cap;
        best_wg = t.shape.wg;
        best_direct = t.shape.direct;
      }
    if (cache_path) {
      std::ofstream outf(cache_path, std::ios::app);
      outf << key << '|' << best_cap << ' ' << best_wg << ' ' << best_direct << '\n';
    }
  }
  clear_error();
  for (int32_t g = 0; g < n_graphs; ++g) {
    chosen_cap[g] = best_cap;
    if (chosen_wg) chosen_wg[g] = best_wg;
    if (chosen_direct) chosen_direct[g] = best_direct;
  }
  return EPK_OK;
}

}  // extern "C"
