// Internal declarations shared by the host (C++) and device (HIP) parts of libepk.
#pragma once

#include <atomic>
#include <cstddef>
#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "epk.h"

namespace epk {

constexpr int kHdrInts = 8;          // int32 per part header
constexpr int kMaxLdsBytes = 65536;  // per-workgroup LDS the kernels may ask for
constexpr int kHeavySlots = 64;      // replicated vertices with more partials get a workgroup each
constexpr int kReduceBlock = 256;
constexpr int kHeavyBlock = 256;

int fail(int status, const std::string &msg);
void clear_error();

// Cooperative cancellation of a partition running on a background thread: the
// thread sets its flag with set_cancel_flag; the partitioner calls
// check_cancel at its level and pass boundaries, which throws Cancelled.
struct Cancelled {};
void set_cancel_flag(const std::atomic<bool> *flag);
void check_cancel();

// ------------------------------------------------------------ partitioner

struct Incidence {
  std::vector<int64_t> off;  // [n + 1]
  std::vector<int32_t> adj;  // [2m] edge ids, ascending within each vertex
};

int validate_graph(const epk_graph *g, int32_t kind_or_minus1);
void build_incidence(int32_t n, int64_t m, const int32_t *uv, Incidence &inc);
// nbr[4e .. 4e+3]: predecessor/successor of e in inc[u_e] and inc[v_e], -1 if absent.
// nbw (optional): the weight of each link slot, the class weight of the chain's vertex (x: id below
// n_x, y: the rest; class_weight NULL: 1)
void contracted_links(int64_t m, const int32_t *uv, const Incidence &inc, std::vector<int32_t> &nbr,
                      std::vector<int32_t> *nbw = nullptr, int32_t n_x = 0, const int32_t *class_weight = nullptr);
constexpr int32_t kMaxClassWeight = 64;
void greedy_growing(int64_t m, int32_t cap, const std::vector<int32_t> &nbr, std::vector<int32_t> &part,
                    std::vector<int32_t> &task);
void input_order(int64_t m, int32_t cap, std::vector<int32_t> &part, std::vector<int32_t> &task);
// baselines.cpp: PowerGraph's random and greedy vertex-cut placements
uint64_t splitmix64(uint64_t x);
void random_order(int64_t m, int32_t cap, std::vector<int32_t> &part, std::vector<int32_t> &task);
void greedy_vertex_cut(int32_t n, int64_t m, const int32_t *uv, int32_t cap, std::vector<int32_t> &part,
                       std::vector<int32_t> &task);
// Thrown when a partitioner cannot place a node without passing the capacity.
struct CapacityExceeded {};
int64_t multilevel_parts(int64_t m, int32_t cap);
int32_t multilevel_max_node_weight(int32_t cap);
void multilevel(int64_t m, int32_t cap, const std::vector<int32_t> &nbr, const std::vector<int32_t> *nbw,
                std::vector<int32_t> &part, std::vector<int32_t> &task);
void partition_stats(int32_t n, int64_t m, const int32_t *uv, int64_t k, const std::vector<int32_t> &part,
                     const std::vector<int32_t> &task, const Incidence &inc, epk_stats &st);
// hub_degree > 0 (EP order only): the hub split (epk_partition_hub) before the multilevel partition.
int run_partition(const epk_graph *g, int32_t cap, int32_t order, std::vector<int32_t> &part,
                  std::vector<int32_t> &task, epk_stats &st, Incidence *inc_out,
                  const int32_t *class_weight = nullptr, int32_t hub_degree = 0);
// A caller's partition: part_in[m] in [0, k); task_in[m] (may be NULL: parts
// ascending, edge id inside a part) a permutation listing parts in order.
// Capacity is not checked here (plan_build refuses parts above it).
int given_partition(const epk_graph *g, int64_t k, const int32_t *part_in, const int32_t *task_in,
                    std::vector<int32_t> &part, std::vector<int32_t> &task, epk_stats &st, Incidence *inc_out);

// ------------------------------------------------------------ device image

// Offsets (bytes) of the arrays inside a plan's device image.
struct ImageLayout {
  size_t hdr = 0, eloc = 0, geom = 0, inc = 0, loff = 0, fid = 0, pfid = 0;
  size_t hdr_items = 0;  // batch: headers in item order (the direct launch), next to the dealt order in hdr
  size_t rvid = 0, roff = 0, sidx = 0, rslot = 0, rrec = 0, heavy = 0, iso = 0, eoff = 0;
  // SpMV adjoint: x incidence per part, y foreign ids, x-class reduction tables
  size_t xinc = 0, xlo = 0, xlofs = 0, rfid = 0, eid = 0, xrvid = 0, xroff = 0, xsidx = 0, xrslot = 0, xheavy = 0;
  // single-launch reduction (FLUX5): per part, the parts it signals (records {part, target, first
  // replicated vertex, end} from nfy_off[p] to nfy_off[p + 1]), the first replicated owned vertex,
  // and one counter per part (zero in the uploaded image and between launches)
  size_t nfy_off = 0, nfy = 0, rsuf = 0, cnt = 0;
  size_t total = 0;
};

// What a kernel needs of a plan (or of a merged batch), as device pointers.
struct DevPlan {
  const int32_t *hdr;
  const uint32_t *eloc;
  const float *geom;
  const uint16_t *inc;
  const uint16_t *loff;
  const int32_t *fid;
  const int32_t *pfid;   // FLUX5 plan: foreign ids again, part p's at p * max_nf (else NULL)
  const int32_t *rvid;
  const int32_t *roff;
  const int32_t *sidx;   // vertex-major workspace: slot of each foreign entry (else NULL)
  const int32_t *rslot;  // part-major workspace: the slots of each replicated vertex (else NULL)
  const int32_t *rrec;   // part-major workspace: [R][4] {vertex, slot, slot, slot} per replicated vertex (else NULL)
  const int32_t *heavy;
  const int32_t *iso;    // batch: untouched vertices (NULL: the range [n_active, n))
  const uint16_t *xinc;  // SpMV adjoint: kernel-order edges of each local x, per part
  const uint16_t *xlo;   // SpMV adjoint: list offsets (part's block at xlofs[part])
  const int32_t *xlofs;
  const int32_t *rfid;   // SpMV adjoint: packed ids (y numbering) of each part's foreign y
  const int32_t *eid;    // SpMV adjoint: original edge id of each kernel-order edge
  const int32_t *xsidx;  // SpMV adjoint: x slot of each foreign x (vertex-major x workspace, else NULL)
  const int32_t *eoff;   // [k + 1] first task of every part
  const int32_t *nfy_off;  // single-launch reduction: [k + 1] first signal record of each part (else NULL)
  const int32_t *nfy;      // single-launch reduction: [signals][4] {part, target, first, end}
  const int32_t *rsuf;   // single-launch reduction: local index of each part's first replicated owned vertex
  int32_t *cnt;          // single-launch reduction: per-part signal counters (in the image)
  int64_t m;          // edge records in the image (FLUX5 plan: k * cap, part p's from p * cap)
  int32_t k;
  int32_t cap;
  int32_t geom_ncomp;
  int32_t n;          // vertices (FLUX5) / y vertices (SPMV)
  int32_t n_active;   // FLUX5: active vertices; SPMV: active y vertices
  int32_t R;          // replicated (reduced) vertices
  int32_t n_heavy;
  int32_t max_u;      // max vertices per part (FLUX5) / max x vertices per part (SPMV)
  int32_t max_uy;     // SPMV: max y vertices per part
  int32_t max_nf;     // max foreign vertices per part
  int32_t n_iso;      // batch: entries of iso
  int32_t max_nfy;    // single-launch reduction: most signal records of a part
  int32_t n_slots;    // workspace rows (replicated partials)
};

}  // namespace epk

struct epk_plan {
  int32_t n = 0, n_x = 0, kind = 0, order = 0, cap = 0, geom_ncomp = 0, ncls = 1, wg = 256, swizzle = 1;
  int64_t m = 0, k = 0;
  int64_t me = 0;  // edge records in the image: FLUX5 k * cap (part p's edges from p * cap), SpMV m
  std::vector<int32_t> part, task, perm;
  std::vector<int32_t> own_begin, own_count;  // [k * ncls]
  std::vector<int64_t> foreign_off;           // [k * ncls + 1]
  std::vector<int32_t> foreign_ids;           // [cost]
  epk_stats stats{};
  // device image, host copy
  std::vector<uint8_t> image;
  epk::ImageLayout lay;
  size_t ws_bytes = 0;
  int64_t R = 0, n_heavy = 0, n_active_out = 0, n_out = 0, max_u = 0, max_uy = 0;
  int64_t lds_fwd = 0, lds_fwd_qn = 0, lds_bwd = 0, n_loff = 0, max_nf = 0;
  // pipelined persistent launch (FLUX5): workgroups per CU asked for (0: one
  // workgroup per part), LDS bytes and grid sizes of the three kernels
  int32_t pipe = 0;
  int32_t staging = 1;  // FLUX5: 1 states staged in LDS, 0 read through the caches
  int64_t lds_cached_fwd = 0, lds_cached_bwd = 0;
  int64_t lds_pipe_fwd = 0, lds_pipe_fwd_qn = 0, lds_pipe_bwd = 0;
  int64_t grid_pipe_fwd = 0, grid_pipe_fwd_qn = 0, grid_pipe_bwd = 0;
  // bytes without the slot tables; see plan_bytes
  int64_t bytes_fwd_kernel = 0, bytes_bwd_kernel = 0, bytes_reduce = 0, bytes_reduce_qnew = 0;
  int64_t n_slots = 0;  // foreign entries of the reduced class = workspace rows
  int64_t rec_delta = 0;  // part-major reduction bytes with records, minus those without (see plan_bytes)
  bool vmajor = false;  // workspace layout: vertex-major (true) or part-major
  // SpMV adjoint's x-class reduction
  int64_t xR = 0, xn_heavy = 0, xn_active = 0, xn_slots = 0;
  bool xvmajor = false;
  // single-launch reduction (FLUX5): possible for this plan, switched on, signal records per part
  bool fused_ok = false, fused = false;
  int64_t max_nfy = 0, n_signals = 0;
  void *d_image = nullptr;
};

struct epk_batch {
  int32_t n_graphs = 0;
  std::vector<int64_t> voff;  // [n_graphs + 1]
  int64_t m = 0, k = 0, n = 0;
  int64_t me = 0;  // edge records in the merged image
  std::vector<uint8_t> image;
  epk::ImageLayout lay;
  size_t ws_bytes = 0;
  int64_t R = 0, n_heavy = 0, n_iso = 0, max_u = 0, max_nf = 0, max_cap = 0, wg = 256;
  bool vmajor = false;
  int64_t grid_fwd = 0, grid_bwd = 0;  // pipelined persistent grids
  int32_t cus = 0;                     // compute units of the device uploaded to
  // one workgroup per item (all plans share one capacity, so item i's edge
  // records start at i * cap and its padded foreign ids at i * max_nf)
  bool direct_ok = false, direct = false;
  int64_t lds_fwd_direct = 0, lds_bwd_direct = 0;
  int64_t lds_fwd = 0, lds_bwd = 0, bytes_fwd = 0, bytes_bwd = 0;
  void *d_image = nullptr;
};

namespace epk {
// LDS bytes of the FLUX5 kernels for a given part shape (must match the kernels' carve-up).
// sidx: the vertex-major workspace's slot indices take LDS too.
int64_t flux_fwd_lds(int64_t max_u, int64_t max_nf, int64_t cap, bool sidx);
int64_t flux_bwd_lds(int64_t max_u, int64_t max_nf, int64_t cap, bool sidx);
int64_t flux_pipe_lds(int64_t max_u, int64_t max_nf, int64_t cap, bool bwd, bool qnew, bool sidx);
int64_t flux_cached_lds(int64_t max_u, int64_t max_nf, int64_t cap, bool bwd, bool sidx);
void set_flux_lds(epk_plan *p);  // all of a FLUX5 plan's LDS sizes for its current layout
int64_t spmv_lds(int64_t max_ux, int64_t max_uy, int64_t wg, int64_t max_nf);
bool auto_vmajor(const epk_plan *p);
int64_t spmv_adj_lds(int64_t max_ux, int64_t max_uy, int64_t cap);
int64_t plan_bytes(const epk_plan *p, int which);
// The single-launch reduction applies to FLUX5 plans that allow it (part-major workspace, no vertex
// with more partials than one thread sums) when it is switched on and the direct staged kernels run.
// The completion list (two int32 per signal record of a part) reuses the kernels' LDS.
inline bool fused_in_use(const epk_plan *p) {
  return p->kind == EPK_FLUX5 && p->fused_ok && p->fused && p->staging && !p->pipe && !p->vmajor &&
         8 * p->max_nfy <= std::min(p->lds_fwd, p->lds_bwd);
}
// order < 0: the partition comes from the caller (given_k parts, given_part,
// given_task as for given_partition).
epk_plan *plan_build(const epk_graph *g, int32_t cap, int32_t order, int32_t kind, int *status,
                     int64_t given_k = 0, const int32_t *given_part = nullptr, const int32_t *given_task = nullptr,
                     const int32_t *class_weight = nullptr, int32_t hub_degree = 0);
// Reduction records, one per replicated vertex: its packed id and its (at
// most kRecSlots) slots, -1 past the last; a first slot of -1 sends the
// vertex to the slot lists (more slots than a record holds).
constexpr int kRecSlots = 3;
constexpr int kMaxSignals = 1024;  // single-launch reduction: parts one part may signal (one lane each)
#ifndef EPK_CNT_STRIDE
#define EPK_CNT_STRIDE 32
#endif
// single-launch reduction: int32 per part counter (32: one 128-byte line each, so that atomics on
// different parts' counters never share a line)
constexpr int kCntStride = EPK_CNT_STRIDE;
std::vector<int32_t> reduction_records(const std::vector<int32_t> &rvid, const std::vector<int32_t> &roff,
                                       const std::vector<int32_t> &rslot);
DevPlan dev_plan(const epk_plan *p);
DevPlan dev_plan_xreduce(const epk_plan *p);  // the SpMV adjoint's x-class reduction
DevPlan dev_batch(const epk_batch *b);
}  // namespace epk
