// Device kernels of libepk (gfx950).
//
// One workgroup runs one part of the edge partition, the paper's "one
// partition per thread block" (Section 4; Section 5.2 for SpMV):
//   1. stage the part's distinct vertices in LDS: the owned range as one
//      contiguous block, foreign vertices through their packed ids;
//   2. run the per-edge task out of LDS;
//   3. sum per-vertex partials in LDS in a fixed order (FLUX5: local
//      incidence lists; SpMV: segmented scan over edges sorted by local y);
//   4. owned vertices' sums go straight to the output, foreign (replicated)
//      ones to workspace slots: from registers in the one-part-per-workgroup
//      kernels, from LDS one iteration later in the pipelined ones.
// A reduction kernel then adds, for every replicated vertex, the slots to the
// owner's partial in ascending part order.  Nothing uses atomics on data, so
// every result is bitwise reproducible.  No MFMA: the work is gather/scatter.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "epk_internal.h"
#include "kernels.h"

namespace epk {

constexpr float kG1 = 0.4f;     // gamma - 1, gamma = 1.4
constexpr float kSigma = 1.0f;  // dissipation coefficient

// Workgroup -> part map.  Workgroups are dispatched round-robin over the 8
// XCDs; giving XCD x the consecutive parts [x*chunk, (x+1)*chunk) keeps
// neighbouring parts (which share vertices) on one L2.
__device__ __forceinline__ int part_of_block(int b, int k, int swizzle) {
  if (!swizzle) return b;
  const int chunk = (k + 7) >> 3;
  return (b & 7) * chunk + (b >> 3);
}

int grid_of_parts(int k, int swizzle) { return swizzle ? 8 * ((k + 7) / 8) : k; }

// ------------------------------------------------------------------ FLUX5

// 1 / x by the hardware reciprocal (within 1 ulp): one instruction where an
// IEEE division takes about ten, and the kernels are bound by instruction issue.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Edge flux a * F(q_u, q_v, n) of the cfd-style interaction, evaluated from
// the area vector A = a n: the Euler normal flux is linear in the normal, so
// a f(q, n) = f(q, A), and only the dissipation term needs a = |A| itself.
__device__ __forceinline__ void edge_flux(const float *qu, const float *qv, float n1, float n2, float n3, float a,
                                          float F[5]) {
  float fu[5], fv[5];
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const float *q = w ? qv : qu;
    float *f = w ? fv : fu;
    const float rho = q[0], m1 = q[1], m2 = q[2], m3 = q[3], E = q[4];
    const float ir = rcp(rho);
    const float mn = m1 * n1 + m2 * n2 + m3 * n3;
    const float mm = m1 * m1 + m2 * m2 + m3 * m3;
    const float s = mn * ir;
    const float p = kG1 * (E - 0.5f * mm * ir);
    f[0] = mn;  // rho * s
    f[1] = m1 * s + p * n1;
    f[2] = m2 * s + p * n2;
    f[3] = m3 * s + p * n3;
    f[4] = (E + p) * s;
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) F[c] = 0.5f * (fu[c] + fv[c]) - (0.5f * kSigma * a) * (qv[c] - qu[c]);
}

// Vector-Jacobian product of the Euler normal flux: out = J(q, n)^T d.
// With s = m.n/rho, p = (gamma-1)(E - |m|^2/(2 rho)), A = d_m.m + d4 (E + p),
// B = d_m.n + d4 s:  out_rho = -A s/rho + B (gamma-1)|m|^2/(2 rho^2),
// out_mi = d0 n_i + d_i s + A n_i/rho - B (gamma-1) m_i/rho, out_E = B (gamma-1) + d4 s.
__device__ __forceinline__ void euler_vjp(const float *q, float n1, float n2, float n3, const float d[5],
                                          float out[5]) {
  const float rho = q[0], m1 = q[1], m2 = q[2], m3 = q[3], E = q[4];
  const float ir = rcp(rho);
  const float mn = m1 * n1 + m2 * n2 + m3 * n3;
  const float mm = m1 * m1 + m2 * m2 + m3 * m3;
  const float s = mn * ir;
  const float p = kG1 * (E - 0.5f * mm * ir);
  const float A = d[1] * m1 + d[2] * m2 + d[3] * m3 + d[4] * (E + p);
  const float B = d[1] * n1 + d[2] * n2 + d[3] * n3 + d[4] * s;
  const float Bg = B * kG1 * ir;
  out[0] = -A * s * ir + Bg * 0.5f * mm * ir;
  out[1] = d[0] * n1 + d[1] * s + A * n1 * ir - Bg * m1;
  out[2] = d[0] * n2 + d[2] * s + A * n2 * ir - Bg * m2;
  out[3] = d[0] * n3 + d[3] * s + A * n3 * ir - Bg * m3;
  out[4] = B * kG1 + d[4] * s;
}

// 3D edges carry the area vector A = a n (3 floats); 2D edges the unit normal.
constexpr int geom_floats(int G) { return G == 4 ? 3 : 2; }

// Geometry of edge base + t, from the wave-uniform base pointer gb = geom +
// geom_floats(G) * base and a 32-bit lane offset t.  The address is then an
// SGPR base plus a 32-bit VGPR offset: with 64-bit lane arithmetic the
// compiler can read the destination register of a load still in flight as a
// don't-care half of the address, and must wait for that load first.
template <int G>
__device__ __forceinline__ float4 load_geom(const float *gb, uint32_t t) {
  if constexpr (G == 4) {
    const float *g = gb + 3u * t;
    return make_float4(g[0], g[1], g[2], 0.f);
  } else {
    const float2 g = reinterpret_cast<const float2 *>(gb)[t];
    return make_float4(g.x, g.y, 0.f, 0.f);
  }
}

// The face area: |A| in 3D (hardware square root, within 1 ulp), 1 in 2D.
// Evaluated once the loads have landed, so that no arithmetic sits between a
// load and the next one.
template <int G>
__device__ __forceinline__ float geom_area(const float4 &g) {
  if constexpr (G == 4)
    return __builtin_amdgcn_sqrtf(g.x * g.x + g.y * g.y + g.z * g.z);
  else
    return 1.0f;
}

// ------------------------------------------------------------------ staging

#define EPK_LDS(p) ((__attribute__((address_space(3))) void *)(p))

// First element of this wave's share in a lane-strided loop (wave-uniform).
__device__ __forceinline__ int wave_first(int tid) { return __builtin_amdgcn_readfirstlane(tid & ~63); }

// Copy src[0, n) to LDS dst[0, n) with direct-to-LDS loads: in each step a
// wave copies 64 consecutive dwords, lane l's to (wave base + 4 l).  The loop
// bound and both bases are wave-uniform, so only the lane predicate is vector
// work.
__device__ __forceinline__ void dma_block(float *dst, const float *src, int n, int tid, int nt) {
  const int lane = tid & 63;
  for (int b = wave_first(tid); b < n; b += nt)
    if (b + lane < n) __builtin_amdgcn_global_load_lds(src + b + lane, EPK_LDS(dst + b), 4, 0, 0);
}

// Stage NC * nf dwords of the rows src[ids[i]] (ids already in LDS) into
// dst[i][NC].  A lane's dword d = tid + j nt sits in row d / NC, column
// d % NC; both advance by fixed steps from one iteration to the next, so no
// division runs inside the loop.
template <int NC>
__device__ __forceinline__ void dma_rows(float *dst, const float *__restrict__ src, const int32_t *ids, int nf, int tid,
                                         int nt) {
  const int lane = tid & 63;
  const int nd = nf * NC;
  const int sv = nt / NC, sc = nt - NC * (nt / NC);
  int v = tid / NC, c = tid - NC * (tid / NC);
  for (int b = wave_first(tid); b < nd; b += nt) {
    if (b + lane < nd)
      __builtin_amdgcn_global_load_lds(src + (int64_t(ids[v]) * NC + c), EPK_LDS(dst + b), 4, 0, 0);
    v += sv;
    c += sc;
    if (c >= NC) {
      c -= NC;
      ++v;
    }
  }
}

// Two blocks of different lengths in one loop: fewer loop steps than two
// loops, and both blocks' loads are issued side by side.
__device__ __forceinline__ void dma_pair(float *dst0, const float *src0, int n0, float *dst1, const float *src1, int n1,
                                         int tid, int nt) {
  const int lane = tid & 63;
  const int n = max(n0, n1);
  for (int b = wave_first(tid); b < n; b += nt) {
    if (b + lane < n0) __builtin_amdgcn_global_load_lds(src0 + b + lane, EPK_LDS(dst0 + b), 4, 0, 0);
    if (b + lane < n1) __builtin_amdgcn_global_load_lds(src1 + b + lane, EPK_LDS(dst1 + b), 4, 0, 0);
  }
}

// Two arrays staged with the same indices (the adjoint's states and upstream
// gradients): one loop, so the ids and addresses are computed once for both.
__device__ __forceinline__ void dma_block2(float *dst0, const float *src0, float *dst1, const float *src1, int n,
                                           int tid, int nt) {
  const int lane = tid & 63;
  for (int b = wave_first(tid); b < n; b += nt)
    if (b + lane < n) {
      __builtin_amdgcn_global_load_lds(src0 + b + lane, EPK_LDS(dst0 + b), 4, 0, 0);
      __builtin_amdgcn_global_load_lds(src1 + b + lane, EPK_LDS(dst1 + b), 4, 0, 0);
    }
}

template <int NC>
__device__ __forceinline__ void dma_rows2(float *dst0, const float *__restrict__ src0, float *dst1,
                                          const float *__restrict__ src1, const int32_t *ids, int nf, int tid, int nt) {
  const int lane = tid & 63;
  const int nd = nf * NC;
  const int sv = nt / NC, sc = nt - NC * (nt / NC);
  int v = tid / NC, c = tid - NC * (tid / NC);
  for (int b = wave_first(tid); b < nd; b += nt) {
    if (b + lane < nd) {
      const int64_t e = int64_t(ids[v]) * NC + c;
      __builtin_amdgcn_global_load_lds(src0 + e, EPK_LDS(dst0 + b), 4, 0, 0);
      __builtin_amdgcn_global_load_lds(src1 + e, EPK_LDS(dst1 + b), 4, 0, 0);
    }
    v += sv;
    c += sc;
    if (c >= NC) {
      c -= NC;
      ++v;
    }
  }
}

// dma_block with 16-byte direct-to-LDS loads (gfx950): in each step a wave
// copies 64 chunks of four dwords, lane l's chunk to (wave base + 16 l bytes);
// the last n mod 4 dwords go as single dwords.  Sources and destinations need
// only 4-byte alignment.  A quarter of the load instructions, which matters
// where the address units bound a kernel (SpMV).
__device__ __forceinline__ void dma_block16(float *dst, const float *src, int n, int tid, int nt) {
  const int lane = tid & 63;
  const int n4 = n & ~3;
  for (int b = 4 * wave_first(tid); b < n4; b += 4 * nt)
    if (b + 4 * lane < n4) __builtin_amdgcn_global_load_lds(src + b + 4 * lane, EPK_LDS(dst + b), 16, 0, 0);
  for (int b = n4 + wave_first(tid); b < n; b += nt)
    if (b + lane < n) __builtin_amdgcn_global_load_lds(src + b + lane, EPK_LDS(dst + b), 4, 0, 0);
}

__device__ __forceinline__ void wait_staged() {
  __builtin_amdgcn_s_waitcnt(0);  // all direct-to-LDS loads of this wave have landed
  __syncthreads();
}

// Workgroup barrier for LDS traffic: waits for this wave's LDS accesses only.
// A __syncthreads() would also wait for every direct-to-LDS load still in
// flight, which the pipelined kernels issue for the next part on purpose.
// The memory clobber keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

constexpr int kIncBatch = 4;  // incidence entries per vertex read as one batch (mesh degrees are <= 4)

// The first kIncBatch incidence entries of the list [t0, t1) and a mask per
// entry (all ones inside the list, zero past its end), read as one batch
// whatever the list length.  The empty asm hides the masks from the compiler,
// which would otherwise turn each masked use into a branch.
__device__ __forceinline__ void inc_batch(const uint16_t *inc, int t0, int t1, int y[kIncBatch],
                                          int in[kIncBatch]) {
  static_assert(kIncBatch == 4, "one asm operand per entry");
#pragma unroll
  for (int k = 0; k < kIncBatch; ++k) {
    y[k] = inc[t0 + k];
    in[k] = -int(t0 + k < t1);
  }
  asm volatile("" : "+v"(in[0]), "+v"(in[1]), "+v"(in[2]), "+v"(in[3]));
}

struct PartHdr {
  int e0, ne, own0, nown, f0, nf, lofs, U;
};

__device__ __forceinline__ PartHdr load_hdr(const DevPlan &P, int part) {
  const int4 *h = reinterpret_cast<const int4 *>(P.hdr + int64_t(part) * kHdrInts);
  const int4 a = h[0], b = h[1];
  return {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
}

// Header of a part as one dword per lane (lane l holds field l mod 8); zero
// for a part past the end.  Read into scalars (hdr_unpack) only after the
// wait for the load, so that the load itself never waits.
__device__ __forceinline__ int hdr_lanes(const DevPlan &P, int part) {
  if (part < 0) return 0;
  return P.hdr[int64_t(part) * kHdrInts + (threadIdx.x & 7)];
}

__device__ __forceinline__ PartHdr hdr_unpack(int v) {
  return {__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 1), __builtin_amdgcn_readlane(v, 2),
          __builtin_amdgcn_readlane(v, 3), __builtin_amdgcn_readlane(v, 4), __builtin_amdgcn_readlane(v, 5),
          __builtin_amdgcn_readlane(v, 6), __builtin_amdgcn_readlane(v, 7)};
}

// Incidence entries (2 u16 per edge, one dword) and offsets (U + 1 u16 from an
// even index, read as whole dwords) into LDS.
__device__ __forceinline__ void dma_incidence(uint16_t *inc, uint16_t *lo, const DevPlan &P, const PartHdr &h, int tid,
                                              int nt) {
  dma_block(reinterpret_cast<float *>(inc), reinterpret_cast<const float *>(P.inc) + h.e0, h.ne, tid, nt);
  dma_block(reinterpret_cast<float *>(lo), reinterpret_cast<const float *>(P.loff) + (h.lofs >> 1), (h.U + 2) >> 1,
            tid, nt);
}

// Edge index of lane j of a part, clamped into [e0, e0 + ne) and, for an
// empty part, into the edge array: lanes past the last edge re-read an edge
// they never use, so every lane issues the same loads and no branch (and no
// wait for the header) separates them.
__device__ __forceinline__ int64_t clamp_edge(const DevPlan &P, int e0, int ne, int j) {
  return min(int64_t(e0) + max(min(j, ne - 1), 0), P.m - 1);
}

// Edge endpoints and geometry into registers, for the edges clamp_edge
// gives: eb = min(e0, m - 1) is wave-uniform, and the lane's offset from it
// min(max(min(j, ne - 1), 0), m - 1 - eb) is 32-bit.
template <int G, int EPT>
__device__ __forceinline__ void load_edges(const DevPlan &P, const PartHdr &h, int tid, int nt, uint32_t ew[EPT],
                                           float4 eg[EPT]) {
  const int64_t eb = min(int64_t(h.e0), P.m - 1);
  const int lim = int(min(int64_t(h.ne - 1), P.m - 1 - eb));
  const uint32_t *el = P.eloc + eb;
  const float *gb = P.geom + geom_floats(G) * eb;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const uint32_t t = uint32_t(min(max(min(tid + k * nt, h.ne - 1), 0), max(lim, 0)));
    ew[k] = el[t];
    eg[k] = load_geom<G>(gb, t);
  }
}

// Edge records of a single plan's part from its fixed block [e0, e0 + cap):
// every lane reads a record (past ne, zero padding it never uses), so the
// loads need no header.
template <int G, int EPT>
__device__ __forceinline__ void load_edge_block(const DevPlan &P, int64_t e0, int tid, int nt, uint32_t ew[EPT],
                                                float4 eg[EPT]) {
  const uint32_t *el = P.eloc + e0;
  const float *gb = P.geom + geom_floats(G) * e0;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const uint32_t t = uint32_t(min(tid + k * nt, P.cap - 1));
    ew[k] = el[t];
    eg[k] = load_geom<G>(gb, t);
  }
}

// ------------------------------------------------------------------ FLUX5 parts
//
// A part goes through three dependent loads and a compute stage:
//   H  its header (8 dwords);
//   A  its foreign ids into an LDS id buffer (addresses from H);
//   B  owned rows and foreign rows (by id) into an LDS state buffer, the local
//      incidence lists and offsets into LDS, edge data into registers;
//   C  flux from LDS, per-vertex sums in a fixed order, the writes.
// The direct kernels run one part per workgroup.  A single plan keeps a
// part's edge records at p cap and its foreign ids at p max_nf, so H, A and
// the edge data are issued together; B's rows follow after one wait.  The
// pipelined kernels run a fixed grid that overlaps the stages of
// consecutive parts of one workgroup (see flux_*_pipe).

__device__ __forceinline__ void stage_ids(const DevPlan &P, const PartHdr &h, int32_t *ids, int tid, int nt) {
  dma_block(reinterpret_cast<float *>(ids), reinterpret_cast<const float *>(P.fid + h.f0), h.nf, tid, nt);
}

// Rows of one [n][5] state array for a part: owned block, then foreign rows.
__device__ __forceinline__ void stage_state(const PartHdr &h, const float *__restrict__ src, float *dst,
                                            const int32_t *ids, int tid, int nt) {
  dma_block(dst, src + int64_t(h.own0) * 5, h.nown * 5, tid, nt);
  dma_rows<5>(dst + h.nown * 5, src, ids, h.nf, tid, nt);
}

// The same rows of two state arrays (states and upstream gradients) in one pass.
__device__ __forceinline__ void stage_state2(const PartHdr &h, const float *__restrict__ src0, float *dst0,
                                             const float *__restrict__ src1, float *dst1, const int32_t *ids, int tid,
                                             int nt) {
  dma_block2(dst0, src0 + int64_t(h.own0) * 5, dst1, src1 + int64_t(h.own0) * 5, h.nown * 5, tid, nt);
  dma_rows2<5>(dst0 + h.nown * 5, src0, dst1 + h.nown * 5, src1, ids, h.nf, tid, nt);
}

// Sum of the signed per-edge fluxes at local vertex i, over its incidence
// list in ascending (edge, side) order: the first kIncBatch entries, then
// their rows, each as one batch of LDS reads.
__device__ __forceinline__ void vertex_sum_fwd(const float *flx, const uint16_t *inc, const uint16_t *lo, int i,
                                               float s[5]) {
  const int t0 = lo[i], t1 = lo[i + 1];
  // the first kIncBatch entries, then their rows, each as one batch of LDS
  // reads and with no branch.  An entry past the list (the next vertex's, or
  // padding) gets weight 0 and reads row 0 (a finite flux); the sum still runs
  // in list order.
  int y[kIncBatch], in[kIncBatch], x[kIncBatch];
  float w[kIncBatch];
  inc_batch(inc, t0, t1, y, in);
#pragma unroll
  for (int k = 0; k < kIncBatch; ++k) {
    x[k] = ((y[k] >> 1) * 5) & in[k];
    // +1 or -1 by the side bit (the sign bit of the float), 0 past the list
    w[k] = __int_as_float((0x3f800000 | ((y[k] & 1) << 31)) & in[k]);
  }
  float v[kIncBatch][5];
#pragma unroll
  for (int k = 0; k < kIncBatch; ++k) {
#pragma unroll
    for (int c = 0; c < 5; ++c) v[k][c] = flx[x[k] + c];
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) s[c] = w[0] * v[0][c];
#pragma unroll
  for (int k = 1; k < kIncBatch; ++k) {
#pragma unroll
    for (int c = 0; c < 5; ++c) s[c] += w[k] * v[k][c];
  }
  for (int t = t0 + kIncBatch; t < t1; ++t) {
    const int e = inc[t];
    const float *f = flx + (e >> 1) * 5;
    const float sg = (e & 1) ? -1.f : 1.f;
#pragma unroll
    for (int c = 0; c < 5; ++c) s[c] += sg * f[c];
  }
}

// Adjoint: sum of the u-side (vu) or v-side (vv) per-edge values at local
// vertex i, in the same order.
__device__ __forceinline__ void vertex_sum_bwd(const float *vu, const float *vv, const uint16_t *inc,
                                               const uint16_t *lo, int i, float s[5]) {
  const int t0 = lo[i], t1 = lo[i + 1];
  const int dv = int(vv - vu);  // the v-side rows, as an offset from vu
  int y[kIncBatch], in[kIncBatch], x[kIncBatch];
  float w[kIncBatch];
  inc_batch(inc, t0, t1, y, in);
#pragma unroll
  for (int k = 0; k < kIncBatch; ++k) {  // as in vertex_sum_fwd: past the list, weight 0 on row 0
    x[k] = ((y[k] >> 1) * 5 + (y[k] & 1) * dv) & in[k];
    w[k] = __int_as_float(0x3f800000 & in[k]);
  }
  float v[kIncBatch][5];
#pragma unroll
  for (int k = 0; k < kIncBatch; ++k) {
#pragma unroll
    for (int c = 0; c < 5; ++c) v[k][c] = vu[x[k] + c];
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) s[c] = w[0] * v[0][c];
#pragma unroll
  for (int k = 1; k < kIncBatch; ++k) {
#pragma unroll
    for (int c = 0; c < 5; ++c) s[c] += w[k] * v[k][c];
  }
  for (int t = t0 + kIncBatch; t < t1; ++t) {
    const int e = inc[t];
    const float *g = vu + (e >> 1) * 5 + (e & 1) * dv;
#pragma unroll
    for (int c = 0; c < 5; ++c) s[c] += g[c];
  }
}

// A part's foreign partials (nf rows of 5) to their workspace slots.
// Part-major workspace (sidx NULL): one contiguous block at the part's slot
// offset.  Vertex-major: sidx (in LDS) gives each foreign entry's slot, so
// that the reduction reads each vertex's slots as one contiguous run.
__device__ __forceinline__ void write_slots(const PartHdr &h, const float *src, const int32_t *sidx,
                                            float *__restrict__ ws, int tid, int nt) {
  if (!sidx) {
    float *wo = ws + int64_t(h.f0) * 5;
    for (int d = tid; d < h.nf * 5; d += nt) wo[d] = src[d];
    return;
  }
  for (int d = tid; d < h.nf * 5; d += nt) {
    const int i = d / 5;
    ws[int64_t(sidx[i]) * 5 + (d - 5 * i)] = src[d];
  }
}

// The slot indices of a part's foreign entries (vertex-major workspace only).
__device__ __forceinline__ void stage_sidx(const DevPlan &P, const PartHdr &h, int32_t *sidx, int tid, int nt) {
  if (P.sidx)
    dma_block(reinterpret_cast<float *>(sidx), reinterpret_cast<const float *>(P.sidx + h.f0), h.nf, tid, nt);
}

// Per-edge fluxes of a part from the staged states st into flx (cap rows of
// 5), then a barrier.
template <int G, int EPT>
__device__ __forceinline__ void edge_stage_fwd(const PartHdr &h, const float *st, float *flx, const uint32_t ew[EPT],
                                               const float4 eg[EPT], int tid, int nt) {
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int j = tid + k * nt;
    if (j < h.ne) {
      float F[5];
      edge_flux(st + (ew[k] & 0xffffu) * 5, st + (ew[k] >> 16) * 5, eg[k].x, eg[k].y, eg[k].z, geom_area<G>(eg[k]),
                F);
#pragma unroll
      for (int c = 0; c < 5; ++c) flx[j * 5 + c] = F[c];
    }
  }
  lds_sync();
}

// The pipelined kernels' compute stage: the sums go to acc in LDS (acc may be
// st when q_new is not written) and leave with write_fwd one iteration later.
// On gfx950 a wait for loads also waits for stores, so stores issued at the
// end of an iteration would stall the next iteration's wait.
template <int G, int EPT>
__device__ __forceinline__ void compute_fwd(const PartHdr &h, const float *st, float *acc, float *flx,
                                            const uint16_t *inc, const uint16_t *lo, const uint32_t ew[EPT],
                                            const float4 eg[EPT], int tid, int nt) {
  edge_stage_fwd<G, EPT>(h, st, flx, ew, eg, tid, nt);
  for (int i = tid; i < h.U; i += nt) {
    float s[5];
    vertex_sum_fwd(flx, inc, lo, i, s);
#pragma unroll
    for (int c = 0; c < 5; ++c) acc[i * 5 + c] = s[c];
  }
  lds_sync();
}

// Forward writes of a computed part: owned sums (and q_new) to the output,
// foreign sums to the part's workspace slots.
template <bool QNEW>
__device__ __forceinline__ void write_fwd(const PartHdr &h, const float *st, const float *acc, const int32_t *sidx,
                                          float *__restrict__ r, float *__restrict__ qn, float dt,
                                          float *__restrict__ ws, int tid, int nt) {
  float *ro = r + int64_t(h.own0) * 5;
  for (int d = tid; d < h.nown * 5; d += nt) {
    ro[d] = acc[d];
    if constexpr (QNEW) qn[int64_t(h.own0) * 5 + d] = st[d] + dt * acc[d];
  }
  write_slots(h, acc + h.nown * 5, sidx, ws, tid, nt);
}

// Adjoint compute stage.  st: states, gs: upstream gradients (overwritten by
// the per-vertex sums); vu, vv: cap * 5 floats each.
// Per-edge adjoint values of a part into vu, vv (then a barrier).
template <int G, int EPT>
__device__ __forceinline__ void edge_stage_bwd(const PartHdr &h, const float *st, const float *gs, float *vu,
                                               float *vv, const uint32_t ew[EPT], const float4 eg[EPT], int tid,
                                               int nt) {
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int j = tid + k * nt;
    if (j < h.ne) {
      const int lu = ew[k] & 0xffffu, lv = ew[k] >> 16;
      // d(a F)/dq = a J(q, n) / 2 +- a sigma I / 2 = J(q, A) / 2 +- a sigma I / 2 (J linear in n)
      const float hs = 0.5f * kSigma * geom_area<G>(eg[k]);
      float d[5], ju[5], jv[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) d[c] = gs[lu * 5 + c] - gs[lv * 5 + c];
      euler_vjp(st + lu * 5, eg[k].x, eg[k].y, eg[k].z, d, ju);
      euler_vjp(st + lv * 5, eg[k].x, eg[k].y, eg[k].z, d, jv);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        vu[j * 5 + c] = 0.5f * ju[c] + hs * d[c];
        vv[j * 5 + c] = 0.5f * jv[c] - hs * d[c];
      }
    }
  }
  lds_sync();
}

template <int G, int EPT>
__device__ __forceinline__ void compute_bwd(const PartHdr &h, const float *st, float *gs, float *vu, float *vv,
                                            const uint16_t *inc, const uint16_t *lo, const uint32_t ew[EPT],
                                            const float4 eg[EPT], int tid, int nt) {
  edge_stage_bwd<G, EPT>(h, st, gs, vu, vv, ew, eg, tid, nt);
  for (int i = tid; i < h.U; i += nt) {
    float s[5];
    vertex_sum_bwd(vu, vv, inc, lo, i, s);
#pragma unroll
    for (int c = 0; c < 5; ++c) gs[i * 5 + c] = s[c];
  }
  lds_sync();
}

__device__ __forceinline__ void write_bwd(const PartHdr &h, const float *gs, const int32_t *sidx,
                                          float *__restrict__ gq, float *__restrict__ ws, int tid, int nt) {
  float *go = gq + int64_t(h.own0) * 5;
  for (int d = tid; d < h.nown * 5; d += nt) go[d] = gs[d];
  write_slots(h, gs + h.nown * 5, sidx, ws, tid, nt);
}

// A row of NC floats of one lane, 4-byte aligned: for NC = 5 one 16-byte and
// one 4-byte access instead of five 4-byte ones (a wave's rows are scattered,
// so every access instruction costs the cache lines it touches).
struct __attribute__((aligned(4))) Float4u {
  float x, y, z, w;
};
template <int NC = 5>
__device__ __forceinline__ void store_row(float *dst, const float *v) {
  if constexpr (NC == 5) {
    *reinterpret_cast<Float4u *>(dst) = {v[0], v[1], v[2], v[3]};
    dst[4] = v[4];
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) dst[c] = v[c];
  }
}
template <int NC = 5>
__device__ __forceinline__ void load_row(const float *src, float *v) {
  if constexpr (NC == 5) {
    const Float4u a = *reinterpret_cast<const Float4u *>(src);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
    v[4] = src[4];
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = src[c];
  }
}

// ---- device-scope rows (single-launch reduction)
//
// A replicated vertex's partials come from several workgroups, possibly on
// different XCDs, whose L2s are not coherent with one another.  An
// agent-scope release (an L2 write-back) at the end of every part made the
// part kernels about 12x slower on tet55, so the partials that another
// workgroup sums within the same launch move through device-scope accesses
// instead: buffer stores with the device-scope cache policy (sc1) write
// through the XCD's L2 to the device's coherence point, and device-scope
// loads read from it.  Rows are addressed by 32-bit byte offsets inside a
// buffer resource covering the array.
constexpr int kDeviceScope = 16;  // cache-policy operand of a buffer access: sc1, device scope
typedef float f32x4 __attribute__((ext_vector_type(4)));

// An array of rows for device-scope access (NULL base: not used).
struct DevRows {
  const float *base;
  int64_t rows;
};
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(DevRows a) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(a.base), 0, int(a.rows * 20), 0x00020000);
}
__device__ __forceinline__ void store_row_dev(DevRows a, int64_t row, const float *v) {
  const __amdgpu_buffer_rsrc_t rs = rsrc_of(a);
  const int o = int(row * 20);
  const f32x4 x = {v[0], v[1], v[2], v[3]};
  __builtin_amdgcn_raw_buffer_store_b128(x, rs, o, 0, kDeviceScope);
  // the 32-bit buffer builtins move an integer: pass the float's bits, not its value
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[4]), rs, o + 16, 0, kDeviceScope);
}
__device__ __forceinline__ void load_row_dev(DevRows a, int64_t row, float *v) {
  const __amdgpu_buffer_rsrc_t rs = rsrc_of(a);
  const int o = int(row * 20);
  const f32x4 x = __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, kDeviceScope);
  v[4] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, o + 16, 0, kDeviceScope));
  v[0] = x.x;
  v[1] = x.y;
  v[2] = x.z;
  v[3] = x.w;
}

// The destination row of local vertex i's sum: owned vertices go to out (row
// own0 + i), foreign ones to their workspace slot.
__device__ __forceinline__ float *sum_row(const PartHdr &h, const int32_t *sidx, float *out, float *ws, int i) {
  if (i < h.nown) return out + (int64_t(h.own0) + i) * 5;
  const int f = i - h.nown;
  return ws + (sidx ? int64_t(sidx[f]) : int64_t(h.f0) + f) * 5;
}

// Per-vertex forward sums, each lane storing its vertex's row from registers
// (owned: r and q_new; foreign: the slot), so no LDS round trip or barrier
// follows the sums.
// FUSED (single-launch reduction, part-major workspace): local vertices from
// rsuf on are replicated (the owned ones, then the foreign ones); their rows
// are stored at device scope for the workgroup that will sum them, and the
// q_new of replicated owned vertices is left to that workgroup.
template <bool QNEW, bool FUSED = false>
__device__ __forceinline__ void sum_store_fwd(const PartHdr &h, const float *st, const float *flx, const uint16_t *inc,
                                              const uint16_t *lo, const int32_t *sidx, float *__restrict__ r,
                                              float *__restrict__ qn, float dt, float *__restrict__ ws, int tid,
                                              int nt, int rsuf = 0, DevRows rr = {nullptr, 0},
                                              DevRows rw = {nullptr, 0}) {
  for (int i = tid; i < h.U; i += nt) {
    float s[5];
    vertex_sum_fwd(flx, inc, lo, i, s);
    if constexpr (FUSED) {
      if (i >= rsuf) {
        if (i < h.nown)
          store_row_dev(rr, int64_t(h.own0) + i, s);
        else
          store_row_dev(rw, int64_t(h.f0) + (i - h.nown), s);
        continue;
      }
    }
    store_row(sum_row(h, sidx, r, ws, i), s);
    if constexpr (QNEW) {
      if (i < h.nown) {
        float t[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) t[c] = st[i * 5 + c] + dt * s[c];
        store_row(qn + (int64_t(h.own0) + i) * 5, t);
      }
    }
  }
}

// Adjoint counterpart: owned sums to gq, foreign ones to their slots.
template <bool FUSED = false>
__device__ __forceinline__ void sum_store_bwd(const PartHdr &h, const float *vu, const float *vv, const uint16_t *inc,
                                              const uint16_t *lo, const int32_t *sidx, float *__restrict__ gq,
                                              float *__restrict__ ws, int tid, int nt, int rsuf = 0,
                                              DevRows rr = {nullptr, 0}, DevRows rw = {nullptr, 0}) {
  for (int i = tid; i < h.U; i += nt) {
    float s[5];
    vertex_sum_bwd(vu, vv, inc, lo, i, s);
    if constexpr (FUSED) {
      if (i >= rsuf) {
        if (i < h.nown)
          store_row_dev(rr, int64_t(h.own0) + i, s);
        else
          store_row_dev(rw, int64_t(h.f0) + (i - h.nown), s);
        continue;
      }
    }
    store_row(sum_row(h, sidx, gq, ws, i), s);
  }
}

// ---- reduction of one light replicated vertex
//
// r_v = (((own + s_1) + s_2) + ...) over at most kHeavySlots (64) partials in
// ascending part order, then q_new.  A part-major workspace lists a vertex's
// slots in its record (up to kRecSlots) or through rslot; a vertex-major one
// keeps them as one run.  DEV: the owner partial and the slots are read at
// device scope (the single-launch reduction sums partials that other
// workgroups stored in the same launch).  The reduction kernel and the
// single-launch reduction share this function, so their sums agree bit for bit.
template <int NC, bool QNEW, bool DEV>
__device__ __forceinline__ void reduce_light(const DevPlan &P, int64_t rho, float *__restrict__ r,
                                             const float *__restrict__ ws, const float *__restrict__ q,
                                             float *__restrict__ qn, float dt, DevRows rr, DevRows rw) {
  auto ld_r = [&](int64_t row, float *v) {
    if constexpr (DEV)
      load_row_dev(rr, row, v);
    else
      load_row<NC>(r + row * NC, v);
  };
  auto ld_w = [&](int64_t row, float *v) {
    if constexpr (DEV)
      load_row_dev(rw, row, v);
    else
      load_row<NC>(ws + row * NC, v);
  };
  // The whole record is read before the branch on it, so that the rows are
  // the second and last dependent load of the record path.
  int4 rec = make_int4(-1, -1, -1, -1);
  if (P.rrec) rec = reinterpret_cast<const int4 *>(P.rrec)[rho];
  int64_t o;
  float s[NC];
  if (rec.y >= 0) {
    // up to kRecSlots slots, all in the vertex's record: one dependent load
    // fewer than the slot lists; absent slots re-read the first with
    // weight 0 (the sum's bits are those of the list path)
    o = int64_t(rec.x);
    const int sl[3] = {rec.y, rec.z, rec.w};
    float v[3][NC];
    ld_r(o, s);
#pragma unroll
    for (int u = 0; u < 3; ++u) ld_w(int64_t(sl[u] < 0 ? rec.y : sl[u]), v[u]);
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const float w = sl[u] < 0 ? 0.f : 1.f;
#pragma unroll
      for (int c = 0; c < NC; ++c) s[c] += w * v[u][c];
    }
  } else {
    const int s0 = P.roff[rho], s1 = P.roff[rho + 1];
    if (s1 - s0 > kHeavySlots) return;
    o = int64_t(P.rvid[rho]);
    ld_r(o, s);
    if (P.rslot) {
      for (int t = s0; t < s1; t += 4) {
        // four slots per batch of loads, with no branch: past the vertex's
        // last slot, its first slot is read again with weight 0 (adding
        // zero leaves the sum's bits unchanged)
        int in[4], sl[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) in[u] = -int(t + u < s1);
        asm volatile("" : "+v"(in[0]), "+v"(in[1]), "+v"(in[2]), "+v"(in[3]));
#pragma unroll
        for (int u = 0; u < 4; ++u) sl[u] = P.rslot[s0 + ((t + u - s0) & in[u])];
        float v[4][NC];
#pragma unroll
        for (int u = 0; u < 4; ++u) ld_w(int64_t(sl[u]), v[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float w = __int_as_float(0x3f800000 & in[u]);
#pragma unroll
          for (int c = 0; c < NC; ++c) s[c] += w * v[u][c];
        }
      }
    } else {
      for (int t = s0; t < s1; ++t) {
        float v[NC];
        ld_w(int64_t(t), v);
#pragma unroll
        for (int c = 0; c < NC; ++c) s[c] += v[c];
      }
    }
  }
  store_row<NC>(r + o * NC, s);
  if constexpr (QNEW) {
    float qv[NC], t[NC];
    load_row<NC>(q + o * NC, qv);
#pragma unroll
    for (int c = 0; c < NC; ++c) t[c] = qv[c] + dt * s[c];
    store_row<NC>(qn + o * NC, t);
  }
}

// ---- single-launch reduction, at the end of a direct part kernel
//
// Part p signals itself (if it owns replicated vertices) and the owner of
// each of its foreign vertices: one relaxed device-scope atomic add on that
// part's counter, by lane t for p's t-th signal record {part q, target, q's
// first replicated vertex, end}.  Before it, every wave has waited for its
// own stores, which the device-scope ones complete at the device's coherence
// point.  A part's target counts the parts that signal it, so the workgroup
// that brings q's counter to its target comes after every partial of q's
// replicated vertices: it sums them (reduce_light, with device-scope loads)
// and sets the counter back to zero for the next launch.  Untouched vertices
// (past n_active) are zeroed part by part, a slice each.  n_done: an LDS
// counter set to zero before the kernel's first barrier.
__device__ __forceinline__ void signal_one(const DevPlan &P, int4 sig, int32_t *lds, int32_t *n_done) {
  if (sig.x < 0) return;
  int32_t *c = P.cnt + int64_t(sig.x) * kCntStride;
  const int old = __hip_atomic_fetch_add(c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (old == sig.y - 1) {
    __hip_atomic_store(c, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int at = atomicAdd(n_done, 1);
    lds[2 * at] = sig.z;
    lds[2 * at + 1] = sig.w;
  }
}

// sig: lane tid's record (loaded with the rows); records past the first nt
// (parts signalling more parts than the workgroup has lanes) are read here.
template <bool QNEW>
__device__ __forceinline__ void fused_reduce(const DevPlan &P, int part, int4 sig, int s0, int s1,
                                             float *__restrict__ r, float *__restrict__ qn,
                                             const float *__restrict__ q, float dt, const float *__restrict__ ws,
                                             int32_t *lds, int32_t *n_done, DevRows rr, DevRows rw, int tid, int nt) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores are complete
  __syncthreads();                                   // ... and every other wave's; LDS is free again
  signal_one(P, sig, lds, n_done);
  for (int t = tid + nt; t < s1 - s0; t += nt) signal_one(P, reinterpret_cast<const int4 *>(P.nfy)[s0 + t], lds, n_done);
  __syncthreads();
  const int nd = *n_done;
  for (int d = 0; d < nd; ++d) {
    const int b = lds[2 * d], e = lds[2 * d + 1];
    for (int j = b + tid; j < e; j += nt) reduce_light<5, QNEW, true>(P, j, r, ws, q, qn, dt, rr, rw);
  }
  const int n_iso = P.n - P.n_active;
  if (n_iso > 0) {
    const int per = (n_iso + P.k - 1) / P.k;
    const int v0 = P.n_active + part * per, v1 = min(P.n, v0 + per);
    for (int v = v0 + tid; v < v1; v += nt) {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        r[int64_t(v) * 5 + c] = 0.0f;
        if constexpr (QNEW) qn[int64_t(v) * 5 + c] = q[int64_t(v) * 5 + c];
      }
    }
  }
}

// Signal records of a part for the single-launch reduction: lane t holds the
// t-th (part -1 past the last).  Issued after the header wait, next to the
// row gathers, so that it lands with them.
__device__ __forceinline__ int4 load_signal(const DevPlan &P, int s0, int s1, int tid) {
  int4 sig = make_int4(-1, 0, 0, 0);
  if (tid < s1 - s0) sig = reinterpret_cast<const int4 *>(P.nfy)[s0 + tid];
  return sig;
}

// ---- direct kernels: one part per workgroup

// LDS: st[max_u][5] | flx[cap][5] (the ids until the flux stage) |
// inc[2 cap] u16 | lo[nlo] u16 | (vertex-major workspace: sidx[max_nf]),
// nlo = max_u + 2 rounded up to even.  The sums leave from registers.
template <int G, bool QNEW, int EPT, bool FUSED = false>
__global__ void __launch_bounds__(1024) flux_fwd_kernel(DevPlan P, const float *__restrict__ q, float *__restrict__ r,
                                                        float *__restrict__ qn, float dt, float *__restrict__ ws,
                                                        int swizzle) {
  extern __shared__ float smem[];
  const int part = part_of_block(blockIdx.x, P.k, swizzle);
  if (part >= P.k) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ int32_t n_done;
  int s0 = 0, s1 = 0, rsuf = 0;
  if constexpr (FUSED) {
    s0 = P.nfy_off[part];
    s1 = P.nfy_off[part + 1];
    rsuf = P.rsuf[part];
    if (tid == 0) n_done = 0;
  }
  float *st = smem;
  float *flx = st + P.max_u * 5;
  uint16_t *inc = reinterpret_cast<uint16_t *>(flx + P.cap * 5);
  uint16_t *lo = inc + 2 * P.cap;
  int32_t *sidx = reinterpret_cast<int32_t *>(lo + ((P.max_u + 3) & ~1));
  int32_t *ids = reinterpret_cast<int32_t *>(flx);
  // foreign ids, edge records and header: none waits for another
  dma_block(reinterpret_cast<float *>(ids), reinterpret_cast<const float *>(P.pfid) + int64_t(part) * P.max_nf,
            P.max_nf, tid, nt);
  uint32_t ew[EPT];
  float4 eg[EPT];
  load_edge_block<G, EPT>(P, int64_t(part) * P.cap, tid, nt, ew, eg);
  const int hv = hdr_lanes(P, part);
  wait_staged();
  const PartHdr h = hdr_unpack(hv);
  // owned and foreign rows, incidence lists and offsets, slot indices
  dma_pair(st, q + int64_t(h.own0) * 5, h.nown * 5, reinterpret_cast<float *>(inc),
           reinterpret_cast<const float *>(P.inc) + h.e0, h.ne, tid, nt);
  dma_pair(reinterpret_cast<float *>(lo), reinterpret_cast<const float *>(P.loff) + (h.lofs >> 1), (h.U + 2) >> 1,
           reinterpret_cast<float *>(sidx), P.sidx ? reinterpret_cast<const float *>(P.sidx + h.f0) : nullptr,
           P.sidx ? h.nf : 0, tid, nt);
  dma_rows<5>(st + h.nown * 5, q, ids, h.nf, tid, nt);
  int4 sig = make_int4(-1, 0, 0, 0);
  if constexpr (FUSED) sig = load_signal(P, s0, s1, tid);
  wait_staged();
  edge_stage_fwd<G, EPT>(h, st, flx, ew, eg, tid, nt);
  if constexpr (FUSED) {
    const DevRows rr = {r, P.n}, rw = {ws, P.n_slots};
    sum_store_fwd<QNEW, true>(h, st, flx, inc, lo, nullptr, r, qn, dt, ws, tid, nt, rsuf, rr, rw);
    fused_reduce<QNEW>(P, part, sig, s0, s1, r, qn, q, dt, ws, reinterpret_cast<int32_t *>(smem), &n_done, rr, rw, tid,
                       nt);
  } else {
    sum_store_fwd<QNEW>(h, st, flx, inc, lo, P.sidx ? sidx : nullptr, r, qn, dt, ws, tid, nt);
  }
}

// LDS: st[max_u][5] | gs[max_u][5] | vu[cap][5] (the ids until the flux
// stage) | vv[cap][5] | inc | lo | sidx.
template <int G, int EPT, bool FUSED = false>
__global__ void __launch_bounds__(1024) flux_bwd_kernel(DevPlan P, const float *__restrict__ q,
                                                        const float *__restrict__ gr, float *__restrict__ gq,
                                                        float *__restrict__ ws, int swizzle) {
  extern __shared__ float smem[];
  const int part = part_of_block(blockIdx.x, P.k, swizzle);
  if (part >= P.k) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ int32_t n_done;
  int s0 = 0, s1 = 0, rsuf = 0;
  if constexpr (FUSED) {
    s0 = P.nfy_off[part];
    s1 = P.nfy_off[part + 1];
    rsuf = P.rsuf[part];
    if (tid == 0) n_done = 0;
  }
  float *st = smem;
  float *gs = st + P.max_u * 5;
  float *vu = gs + P.max_u * 5;
  float *vv = vu + P.cap * 5;
  uint16_t *inc = reinterpret_cast<uint16_t *>(vv + P.cap * 5);
  uint16_t *lo = inc + 2 * P.cap;
  int32_t *sidx = reinterpret_cast<int32_t *>(lo + ((P.max_u + 3) & ~1));
  int32_t *ids = reinterpret_cast<int32_t *>(vu);
  dma_block(reinterpret_cast<float *>(ids), reinterpret_cast<const float *>(P.pfid) + int64_t(part) * P.max_nf,
            P.max_nf, tid, nt);
  uint32_t ew[EPT];
  float4 eg[EPT];
  load_edge_block<G, EPT>(P, int64_t(part) * P.cap, tid, nt, ew, eg);
  const int hv = hdr_lanes(P, part);
  wait_staged();
  const PartHdr h = hdr_unpack(hv);
  stage_sidx(P, h, sidx, tid, nt);
  dma_pair(reinterpret_cast<float *>(inc), reinterpret_cast<const float *>(P.inc) + h.e0, h.ne,
           reinterpret_cast<float *>(lo), reinterpret_cast<const float *>(P.loff) + (h.lofs >> 1), (h.U + 2) >> 1, tid,
           nt);
  dma_block2(st, q + int64_t(h.own0) * 5, gs, gr + int64_t(h.own0) * 5, h.nown * 5, tid, nt);
  dma_rows2<5>(st + h.nown * 5, q, gs + h.nown * 5, gr, ids, h.nf, tid, nt);
  int4 sig = make_int4(-1, 0, 0, 0);
  if constexpr (FUSED) sig = load_signal(P, s0, s1, tid);
  wait_staged();
  edge_stage_bwd<G, EPT>(h, st, gs, vu, vv, ew, eg, tid, nt);
  if constexpr (FUSED) {
    const DevRows rr = {gq, P.n}, rw = {ws, P.n_slots};
    sum_store_bwd<true>(h, vu, vv, inc, lo, nullptr, gq, ws, tid, nt, rsuf, rr, rw);
    fused_reduce<false>(P, part, sig, s0, s1, gq, nullptr, nullptr, 0.f, ws, reinterpret_cast<int32_t *>(smem),
                        &n_done, rr, rw, tid, nt);
  } else {
    sum_store_bwd(h, vu, vv, inc, lo, P.sidx ? sidx : nullptr, gq, ws, tid, nt);
  }
}

// ---- cache-only kernels: no LDS staging of states
//
// The paper's alternative to shared-memory staging relies on the hardware
// caches alone (its texture-cache variant, Section 5.2): the same parts, task
// order and packed layout, but each edge reads the states of its endpoints
// straight from global memory, so repeated vertices of a part hit L1/L2
// instead of an LDS copy.  Only the foreign ids (to map local to packed
// vertex ids), the incidence lists and the per-edge values live in LDS; the
// per-vertex sums, writes and reduction are the staged kernels' own, so the
// results agree up to rounding (the edge arithmetic is compiled separately and
// may fuse multiplies and adds differently).

__device__ __forceinline__ int64_t packed_of(const PartHdr &h, const int32_t *ids, int l) {
  return l < h.nown ? int64_t(h.own0) + l : int64_t(ids[l - h.nown]);
}

__device__ __forceinline__ void load_row(const float *__restrict__ src, int64_t v, float out[5]) {
#pragma unroll
  for (int c = 0; c < 5; ++c) out[c] = src[v * 5 + c];
}

// LDS: flx[cap][5] | ids[max_nf] | inc[2 cap] u16 | lo[nlo] u16 | sidx[max_nf].
template <int G, bool QNEW, int EPT>
__global__ void __launch_bounds__(1024) flux_fwd_cached(DevPlan P, const float *__restrict__ q, float *__restrict__ r,
                                                        float *__restrict__ qn, float dt, float *__restrict__ ws,
                                                        int swizzle) {
  extern __shared__ float smem[];
  const int part = part_of_block(blockIdx.x, P.k, swizzle);
  if (part >= P.k) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  float *flx = smem;
  int32_t *ids = reinterpret_cast<int32_t *>(flx + P.cap * 5);
  uint16_t *inc = reinterpret_cast<uint16_t *>(ids + P.max_nf);
  uint16_t *lo = inc + 2 * P.cap;
  int32_t *sidx = reinterpret_cast<int32_t *>(lo + ((P.max_u + 3) & ~1));
  const PartHdr h = load_hdr(P, part);
  stage_ids(P, h, ids, tid, nt);
  stage_sidx(P, h, sidx, tid, nt);
  uint32_t ew[EPT];
  float4 eg[EPT];
  load_edges<G, EPT>(P, h, tid, nt, ew, eg);
  dma_incidence(inc, lo, P, h, tid, nt);
  wait_staged();
  float qu[EPT][5], qv[EPT][5];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {  // every row load of the part in one batch; idle lanes read row 0
    const bool ok = tid + k * nt < h.ne;
    load_row(q, ok ? packed_of(h, ids, ew[k] & 0xffffu) : 0, qu[k]);
    load_row(q, ok ? packed_of(h, ids, ew[k] >> 16) : 0, qv[k]);
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int j = tid + k * nt;
    if (j < h.ne) {
      float F[5];
      edge_flux(qu[k], qv[k], eg[k].x, eg[k].y, eg[k].z, geom_area<G>(eg[k]), F);
#pragma unroll
      for (int c = 0; c < 5; ++c) flx[j * 5 + c] = F[c];
    }
  }
  __syncthreads();
  // per-vertex sums in registers, in the staged kernels' order, then written out
  float *ro = r + int64_t(h.own0) * 5;
  for (int i = tid; i < h.U; i += nt) {
    float s[5];
    vertex_sum_fwd(flx, inc, lo, i, s);
    if (i < h.nown) {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        ro[i * 5 + c] = s[c];
        if constexpr (QNEW) qn[(int64_t(h.own0) + i) * 5 + c] = q[(int64_t(h.own0) + i) * 5 + c] + dt * s[c];
      }
    } else {
      const int f = i - h.nown;
      const int64_t slot = P.sidx ? int64_t(sidx[f]) : int64_t(h.f0) + f;
#pragma unroll
      for (int c = 0; c < 5; ++c) ws[slot * 5 + c] = s[c];
    }
  }
}

// LDS: vu[cap][5] | vv[cap][5] | ids | inc | lo | sidx.
template <int G, int EPT>
__global__ void __launch_bounds__(1024) flux_bwd_cached(DevPlan P, const float *__restrict__ q,
                                                        const float *__restrict__ gr, float *__restrict__ gq,
                                                        float *__restrict__ ws, int swizzle) {
  extern __shared__ float smem[];
  const int part = part_of_block(blockIdx.x, P.k, swizzle);
  if (part >= P.k) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  float *vu = smem;
  float *vv = vu + P.cap * 5;
  int32_t *ids = reinterpret_cast<int32_t *>(vv + P.cap * 5);
  uint16_t *inc = reinterpret_cast<uint16_t *>(ids + P.max_nf);
  uint16_t *lo = inc + 2 * P.cap;
  int32_t *sidx = reinterpret_cast<int32_t *>(lo + ((P.max_u + 3) & ~1));
  const PartHdr h = load_hdr(P, part);
  stage_ids(P, h, ids, tid, nt);
  stage_sidx(P, h, sidx, tid, nt);
  uint32_t ew[EPT];
  float4 eg[EPT];
  load_edges<G, EPT>(P, h, tid, nt, ew, eg);
  dma_incidence(inc, lo, P, h, tid, nt);
  wait_staged();
  float qu[EPT][5], qv[EPT][5], gu[EPT][5], gv[EPT][5];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {  // idle lanes read row 0
    const bool ok = tid + k * nt < h.ne;
    const int64_t pu = ok ? packed_of(h, ids, ew[k] & 0xffffu) : 0, pv = ok ? packed_of(h, ids, ew[k] >> 16) : 0;
    load_row(q, pu, qu[k]);
    load_row(q, pv, qv[k]);
    load_row(gr, pu, gu[k]);
    load_row(gr, pv, gv[k]);
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int j = tid + k * nt;
    if (j < h.ne) {
      const float hs = 0.5f * kSigma * geom_area<G>(eg[k]);
      float d[5], ju[5], jv[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) d[c] = gu[k][c] - gv[k][c];
      euler_vjp(qu[k], eg[k].x, eg[k].y, eg[k].z, d, ju);
      euler_vjp(qv[k], eg[k].x, eg[k].y, eg[k].z, d, jv);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        vu[j * 5 + c] = 0.5f * ju[c] + hs * d[c];
        vv[j * 5 + c] = 0.5f * jv[c] - hs * d[c];
      }
    }
  }
  __syncthreads();
  float *go = gq + int64_t(h.own0) * 5;
  for (int i = tid; i < h.U; i += nt) {
    float s[5];
    vertex_sum_bwd(vu, vv, inc, lo, i, s);
    if (i < h.nown) {
#pragma unroll
      for (int c = 0; c < 5; ++c) go[i * 5 + c] = s[c];
    } else {
      const int f = i - h.nown;
      const int64_t slot = P.sidx ? int64_t(sidx[f]) : int64_t(h.f0) + f;
#pragma unroll
      for (int c = 0; c < 5; ++c) ws[slot * 5 + c] = s[c];
    }
  }
}

// ---- pipelined persistent kernels
//
// Workgroup b walks its own list of parts, t = 0, 1, ...  Iteration t waits
// once for every load issued before it, then issues B(t+1), A(t+2) and H(t+3)
// and computes C(t), so the loads of three parts overlap the compute of a
// fourth.  LDS holds two id buffers, two state buffers and two incidence
// buffers; a buffer is reloaded only after the barrier that follows its last
// reader.  A header of a part past the end of the list is all zero, which
// makes its stages empty (edge loads read edge 0 and are never used).
//
// Part lists.  swizzle = 1: workgroup b runs on XCD b mod 8 and takes the
// parts x*chunk + b/8 + t*(grid/8) of that XCD's range (grid a multiple of 8),
// so the workgroups of one XCD work on neighbouring parts at the same time.
// swizzle = 0: part b + t*grid (a batch image stores its headers in
// processing order, largest parts first).

__device__ __forceinline__ int pipe_part(int k, int t, int swizzle) {
  const int b = blockIdx.x, G = gridDim.x;
  if (swizzle) {
    const int chunk = (k + 7) >> 3;
    const int i = (b >> 3) + t * (G >> 3);
    const int part = (b & 7) * chunk + i;
    return (i < chunk && part < k) ? part : -1;
  }
  const int part = b + t * G;
  return part < k ? part : -1;
}

// LDS carve-up of the pipelined kernels (host mirror: flux_pipe_lds):
// st[2][max_u][5] | (adjoint: gs[2][max_u][5]) | (q_new: acc[max_u][5]) |
// f0[cap][5] | (adjoint: f1[cap][5]) | ids[2][max_nf] | inc[2][2 cap] u16 |
// lo[2][nlo] u16 | (vertex-major workspace only: sidx[2][max_nf]).  Buffers are addressed by arithmetic on the one LDS base,
// so every pointer stays an LDS pointer (no indexed pointer arrays).
struct PipeLds {
  float *base;
  int su, sf, nf, cap, nlo, o_gs, o_acc, o_f0, o_f1, o_ids, o_sx;
  __device__ float *st(int b) const { return base + b * su; }
  __device__ float *gs(int b) const { return base + o_gs + b * su; }
  __device__ float *acc() const { return base + o_acc; }
  __device__ float *f0() const { return base + o_f0; }
  __device__ float *f1() const { return base + o_f1; }
  __device__ int32_t *ids(int b) const { return reinterpret_cast<int32_t *>(base + o_ids) + b * nf; }
  __device__ uint16_t *inc(int b) const {
    return reinterpret_cast<uint16_t *>(base + o_ids + 2 * nf) + b * (2 * cap);
  }
  __device__ uint16_t *lo(int b) const {
    return reinterpret_cast<uint16_t *>(base + o_ids + 2 * nf) + 4 * cap + b * nlo;
  }
  __device__ int32_t *sidx(int b) const { return reinterpret_cast<int32_t *>(base + o_sx) + b * nf; }
};

__device__ __forceinline__ PipeLds pipe_lds(const DevPlan &P, float *smem, bool bwd, bool qnew) {
  PipeLds L;
  L.base = smem;
  L.su = P.max_u * 5;
  L.sf = P.cap * 5;
  L.nf = P.max_nf;
  L.cap = P.cap;
  L.nlo = (P.max_u + 3) & ~1;  // U + 1 offsets, read as whole dwords
  int o = 2 * L.su;
  L.o_gs = o;
  o += bwd ? 2 * L.su : 0;
  L.o_acc = o;
  o += qnew ? L.su : 0;
  L.o_f0 = o;
  o += L.sf;
  L.o_f1 = o;
  o += bwd ? L.sf : 0;
  L.o_ids = o;
  L.o_sx = o + 2 * L.nf + 2 * L.cap + L.nlo;  // after ids, inc and lo (nlo is even)
  return L;
}

template <int G, bool QNEW, int EPT>
__global__ void __launch_bounds__(256) flux_fwd_pipe(DevPlan P, const float *__restrict__ q, float *__restrict__ r,
                                                     float *__restrict__ qn, float dt, float *__restrict__ ws,
                                                     int swizzle) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const PipeLds L = pipe_lds(P, smem, false, QNEW);
  uint32_t ew[EPT], ewn[EPT];
  float4 eg[EPT], egn[EPT];

  // prologue: H(0); A(0), H(1); B(0), A(1), H(2)
  int hv = hdr_lanes(P, pipe_part(P.k, 0, swizzle));
  wait_staged();
  PartHdr h0 = hdr_unpack(hv);
  hv = hdr_lanes(P, pipe_part(P.k, 1, swizzle));
  stage_ids(P, h0, L.ids(0), tid, nt);
  wait_staged();
  PartHdr h1 = hdr_unpack(hv);
  hv = hdr_lanes(P, pipe_part(P.k, 2, swizzle));
  stage_ids(P, h1, L.ids(1), tid, nt);
  stage_state(h0, q, L.st(0), L.ids(0), tid, nt);
  stage_sidx(P, h0, L.sidx(0), tid, nt);
  dma_incidence(L.inc(0), L.lo(0), P, h0, tid, nt);
  load_edges<G, EPT>(P, h0, tid, nt, ew, eg);

  // The writes of part t-1 open iteration t: issued right after the wait,
  // they complete while part t is computed instead of delaying the next wait.
  PartHdr hp = {0, 0, 0, 0, 0, 0, 0, 0};  // part t-1 (none yet: writes nothing)
  int t = 0;
  for (; pipe_part(P.k, t, swizzle) >= 0; ++t) {
    const int b = t & 1, nb = b ^ 1;
    wait_staged();
    const PartHdr h2 = hdr_unpack(hv);
    write_fwd<QNEW>(hp, L.st(nb), QNEW ? L.acc() : L.st(nb), P.sidx ? L.sidx(nb) : nullptr, r, qn, dt, ws, tid,
                    nt);  // W(t-1)
    lds_sync();                                           // buffers nb and acc are free again
    hv = hdr_lanes(P, pipe_part(P.k, t + 3, swizzle));   // H(t+3)
    stage_state(h1, q, L.st(nb), L.ids(nb), tid, nt);     // B(t+1)
    stage_sidx(P, h1, L.sidx(nb), tid, nt);
    dma_incidence(L.inc(nb), L.lo(nb), P, h1, tid, nt);
    load_edges<G, EPT>(P, h1, tid, nt, ewn, egn);
    stage_ids(P, h2, L.ids(b), tid, nt);                  // A(t+2)
    compute_fwd<G, EPT>(h0, L.st(b), QNEW ? L.acc() : L.st(b), L.f0(), L.inc(b), L.lo(b), ew, eg, tid, nt);  // C(t)
    hp = h0;
    h0 = h1;
    h1 = h2;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      ew[k] = ewn[k];
      eg[k] = egn[k];
    }
  }
  const int pb = (t + 1) & 1;  // buffer of part t-1
  write_fwd<QNEW>(hp, L.st(pb), QNEW ? L.acc() : L.st(pb), P.sidx ? L.sidx(pb) : nullptr, r, qn, dt, ws, tid, nt);
  __builtin_amdgcn_s_waitcnt(0);  // no load into LDS outlives the workgroup
}

template <int G, int EPT>
__global__ void __launch_bounds__(256) flux_bwd_pipe(DevPlan P, const float *__restrict__ q,
                                                     const float *__restrict__ gr, float *__restrict__ gq,
                                                     float *__restrict__ ws, int swizzle) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const PipeLds L = pipe_lds(P, smem, true, false);
  uint32_t ew[EPT], ewn[EPT];
  float4 eg[EPT], egn[EPT];

  int hv = hdr_lanes(P, pipe_part(P.k, 0, swizzle));
  wait_staged();
  PartHdr h0 = hdr_unpack(hv);
  hv = hdr_lanes(P, pipe_part(P.k, 1, swizzle));
  stage_ids(P, h0, L.ids(0), tid, nt);
  wait_staged();
  PartHdr h1 = hdr_unpack(hv);
  hv = hdr_lanes(P, pipe_part(P.k, 2, swizzle));
  stage_ids(P, h1, L.ids(1), tid, nt);
  stage_state2(h0, q, L.st(0), gr, L.gs(0), L.ids(0), tid, nt);
  stage_sidx(P, h0, L.sidx(0), tid, nt);
  dma_incidence(L.inc(0), L.lo(0), P, h0, tid, nt);
  load_edges<G, EPT>(P, h0, tid, nt, ew, eg);

  PartHdr hp = {0, 0, 0, 0, 0, 0, 0, 0};
  int t = 0;
  for (; pipe_part(P.k, t, swizzle) >= 0; ++t) {
    const int b = t & 1, nb = b ^ 1;
    wait_staged();
    const PartHdr h2 = hdr_unpack(hv);
    write_bwd(hp, L.gs(nb), P.sidx ? L.sidx(nb) : nullptr, gq, ws, tid, nt);
    lds_sync();
    hv = hdr_lanes(P, pipe_part(P.k, t + 3, swizzle));
    stage_state2(h1, q, L.st(nb), gr, L.gs(nb), L.ids(nb), tid, nt);
    stage_sidx(P, h1, L.sidx(nb), tid, nt);
    dma_incidence(L.inc(nb), L.lo(nb), P, h1, tid, nt);
    load_edges<G, EPT>(P, h1, tid, nt, ewn, egn);
    stage_ids(P, h2, L.ids(b), tid, nt);
    compute_bwd<G, EPT>(h0, L.st(b), L.gs(b), L.f0(), L.f1(), L.inc(b), L.lo(b), ew, eg, tid, nt);
    hp = h0;
    h0 = h1;
    h1 = h2;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      ew[k] = ewn[k];
      eg[k] = egn[k];
    }
  }
  write_bwd(hp, L.gs((t + 1) & 1), P.sidx ? L.sidx((t + 1) & 1) : nullptr, gq, ws, tid, nt);
  __builtin_amdgcn_s_waitcnt(0);
}

// ------------------------------------------------------------------ SpMV

// LDS: xs[max_ux] | ys[max_uy] | ysl[max_uy] (slots of the foreign y) |
// xid[max_nf] (foreign x ids) | per-wave carry keys and values.
// EPT consecutive edges per lane (EPT * blockDim.x >= cap).
template <int EPT>
__global__ void __launch_bounds__(1024) spmv_kernel(DevPlan P, const float *__restrict__ x, float *__restrict__ y,
                                                    float *__restrict__ ws, int swizzle) {
  extern __shared__ float smem[];
  const int part = part_of_block(blockIdx.x, P.k, swizzle);
  if (part >= P.k) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  float *xs = smem;
  float *ys = xs + P.max_u;
  int32_t *ysl = reinterpret_cast<int32_t *>(ys + P.max_uy);
  int32_t *xid = ysl + P.max_uy;
  int *tkey = xid + P.max_nf;
  float *tval = reinterpret_cast<float *>(tkey + (nt >> 6));
  const int lane = tid & 63, wave = tid >> 6;

  // batch 1, all addressed from the part index: header, edge count, foreign x
  // ids (fixed-stride copy) and edge records (part p's at p cap, zero past its
  // count; positions past the capacity re-read the last record).  The kernel
  // is bound by its address units (one cache line per x gather), so the other
  // loads take as few instructions as they can: the ids in 16-byte chunks, a
  // lane's EPT records and weights as one vector load each, and the record
  // after a wave's last only in its last lane, the one lane that uses it.
  const int4 *h4 = reinterpret_cast<const int4 *>(P.hdr + int64_t(part) * kHdrInts);
  const int4 ha = h4[0], hb = h4[1];
  const int ne = int(P.eoff[part + 1] - P.eoff[part]);
  dma_block16(reinterpret_cast<float *>(xid), reinterpret_cast<const float *>(P.pfid) + int64_t(part) * P.max_nf,
              P.max_nf, tid, nt);
  const uint32_t *el = P.eloc + int64_t(part) * P.cap;
  const float *eg = P.geom + int64_t(part) * P.cap;
  const int j0 = tid * EPT;
  uint32_t w[EPT];
  float wt[EPT];
  if (EPT > 1 && P.cap % EPT == 0 && j0 + EPT <= P.cap) {  // aligned, inside the block
    typedef uint32_t vu __attribute__((ext_vector_type(EPT)));
    typedef float vf __attribute__((ext_vector_type(EPT)));
    const vu a = *reinterpret_cast<const vu *>(el + j0);
    const vf b = *reinterpret_cast<const vf *>(eg + j0);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      w[i] = a[i];
      wt[i] = b[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int j = min(j0 + i, P.cap - 1);
      w[i] = el[j];
      wt[i] = eg[j];
    }
  }
  uint32_t w_next = 0;
  if (lane == 63) w_next = el[min(j0 + EPT, P.cap - 1)];
  wait_staged();
  const int xo = ha.x, xn = ha.y, xnf = ha.w, yo = hb.x, yn = hb.y, yf0 = hb.z, ynf = hb.w;
  // batch 2: owned x block, foreign x values by id, slot indices of the foreign y
  dma_block(xs, x + xo, xn, tid, nt);
  if (P.sidx) dma_block(reinterpret_cast<float *>(ysl), reinterpret_cast<const float *>(P.sidx + yf0), ynf, tid, nt);
  for (int d = tid; d < xnf; d += nt) __builtin_amdgcn_global_load_lds(x + xid[d], EPK_LDS(xs + xn + (d - lane)), 4, 0, 0);
  wait_staged();

  // edges sorted by local y: the lane's EPT edges summed run by run, then an
  // inclusive segmented scan of the lanes' last runs per wavefront
  int k[EPT];
  float sv[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const bool ok = j0 + i < ne;
    k[i] = ok ? int(w[i] >> 16) : 0x7fffffff;
    const float v = ok ? wt[i] * xs[w[i] & 0xffffu] : 0.0f;
    sv[i] = (i > 0 && k[i] == k[i - 1]) ? sv[i - 1] + v : v;
  }
  const int key = k[EPT - 1];
  float v = sv[EPT - 1];
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const float vu = __shfl_up(v, d, 64);
    const int ku = __shfl_up(key, d, 64);
    if (lane >= d && ku == key) v = vu + v;
  }
  // the earlier lanes' sum of this lane's first key (runs that start at its first edge)
  const float vp = __shfl_up(v, 1, 64);
  const int kp = __shfl_up(key, 1, 64);
  const bool carry_in = lane > 0 && kp == k[0];
  int key_next = __shfl_down(k[0], 1, 64);
  if (lane == 63) key_next = (j0 + EPT < ne) ? int(w_next >> 16) : 0x7ffffffe;
  const bool last_ok = j0 + EPT - 1 < ne;
  if (lane == 63) {
    tkey[wave] = (last_ok && key_next == key) ? key : -1;
    tval[wave] = v;
  }
  __syncthreads();
  // ends of segments: add the carries of earlier wavefronts
  auto finish = [&](int kk, float t) {
    float carry = 0.0f;
    bool has = false;
    for (int wp = wave - 1; wp >= 0 && tkey[wp] == kk; --wp) {
      carry = has ? carry + tval[wp] : tval[wp];
      has = true;
    }
    ys[kk] = has ? carry + t : t;
  };
#pragma unroll
  for (int i = 0; i < EPT - 1; ++i) {
    if (j0 + i < ne && k[i + 1] != k[i]) finish(k[i], (carry_in && k[i] == k[0]) ? vp + sv[i] : sv[i]);
  }
  if (last_ok && key_next != key) finish(key, v);
  __syncthreads();
  for (int d = tid; d < yn; d += nt) y[yo + d] = ys[d];
  if (P.sidx) {
    for (int d = tid; d < ynf; d += nt) ws[ysl[d]] = ys[yn + d];
  } else {
    for (int d = tid; d < ynf; d += nt) ws[yf0 + d] = ys[yn + d];
  }
}

// SpMV adjoint over the same parts (Section 5.2's graph, gradients flowing
// back): g_x = A^T g_y, i.e. g_x[j] = sum over the edges (j, i) of w g_y[i],
// and, if g_w is not NULL, the weight gradient g_w[e] = g_y[i] x[j] in
// original edge order.  The part's y gradients (owned block, then foreign y by
// id) and, for g_w, its x values are staged in LDS like the forward's x; each
// local x sums its edges' values over a per-part incidence list in ascending
// kernel order; owned x are written directly, foreign x partials go to the
// workspace and an x-class reduction adds them in ascending part order.
// LDS: gys[max_uy] | xs[max_ux] | val[cap] | xinc[cap, even] u16 | xlo[nlo] u16 | xsl[max_ux].
__global__ void __launch_bounds__(1024) spmv_adj_kernel(DevPlan P, const float *__restrict__ x,
                                                        const float *__restrict__ gy, float *__restrict__ gx,
                                                        float *__restrict__ gw, float *__restrict__ ws, int swizzle) {
  extern __shared__ float smem[];
  const int part = part_of_block(blockIdx.x, P.k, swizzle);
  if (part >= P.k) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int4 *h4 = reinterpret_cast<const int4 *>(P.hdr + int64_t(part) * kHdrInts);
  const int4 ha = h4[0], hb = h4[1];
  const int xo = ha.x, xn = ha.y, xf0 = ha.z, xnf = ha.w, yo = hb.x, yn = hb.y, yf0 = hb.z, ynf = hb.w;
  const int64_t e0 = int64_t(part) * P.cap;  // the part's record block
  const int ne = int(P.eoff[part + 1] - P.eoff[part]);
  const int ux = xn + xnf;
  float *gys = smem;
  float *xs = gys + P.max_uy;
  float *val = xs + P.max_u;
  uint16_t *xinc = reinterpret_cast<uint16_t *>(val + P.cap);
  uint16_t *xlo = xinc + ((P.cap + 1) & ~1);
  int32_t *xsl = reinterpret_cast<int32_t *>(xlo + ((P.max_u + 3) & ~1));
  const int lane = tid & 63;

  // batch 1: owned blocks, foreign ids (into the slots their values take), edges, x incidence
  int32_t *yid = reinterpret_cast<int32_t *>(gys + yn);
  dma_block(gys, gy + yo, yn, tid, nt);
  dma_block(reinterpret_cast<float *>(yid), reinterpret_cast<const float *>(P.rfid + yf0), ynf, tid, nt);
  int32_t *xid = reinterpret_cast<int32_t *>(xs + xn);
  if (gw) {
    dma_block(xs, x + xo, xn, tid, nt);
    dma_block(reinterpret_cast<float *>(xid), reinterpret_cast<const float *>(P.fid + xf0), xnf, tid, nt);
  }
  if (P.xsidx) dma_block(reinterpret_cast<float *>(xsl), reinterpret_cast<const float *>(P.xsidx + xf0), xnf, tid, nt);
  dma_block(reinterpret_cast<float *>(xinc), reinterpret_cast<const float *>(P.xinc) + e0, (ne + 1) >> 1, tid, nt);
  dma_block(reinterpret_cast<float *>(xlo), reinterpret_cast<const float *>(P.xlo + P.xlofs[part]), (ux + 2) >> 1, tid,
            nt);
  const bool valid = tid < ne;
  const int64_t ec = clamp_edge(P, int(e0), ne, tid);
  const uint32_t w = P.eloc[ec];
  const float wt = P.geom[ec];
  const int32_t oe = gw ? P.eid[ec] : 0;
  wait_staged();
  // batch 2: foreign values, each lane overwriting the id it read
  for (int d = tid; d < ynf; d += nt) __builtin_amdgcn_global_load_lds(gy + yid[d], EPK_LDS(gys + yn + (d - lane)), 4, 0, 0);
  if (gw)
    for (int d = tid; d < xnf; d += nt) __builtin_amdgcn_global_load_lds(x + xid[d], EPK_LDS(xs + xn + (d - lane)), 4, 0, 0);
  wait_staged();

  if (valid) {
    const float g = gys[w >> 16];
    val[tid] = wt * g;
    if (gw) gw[oe] = g * xs[w & 0xffffu];
  }
  __syncthreads();
  for (int i = tid; i < ux; i += nt) {
    float s = 0.0f;
    const int t1 = xlo[i + 1];
    for (int t = xlo[i]; t < t1; ++t) s += val[xinc[t]];
    if (i < xn)
      gx[xo + i] = s;
    else
      ws[P.xsidx ? int64_t(xsl[i - xn]) : int64_t(xf0) + (i - xn)] = s;
  }
}

// ------------------------------------------------------------------ reduction

// Light vertices (<= kHeavySlots partials): one thread per vertex
// (reduce_light).  Heavy vertices: one workgroup each, strided partial sums
// then a fixed tree.  Untouched vertices are zeroed here as well.
template <int NC, bool QNEW>
__global__ void __launch_bounds__(256) reduce_kernel(DevPlan P, float *__restrict__ r, const float *__restrict__ ws,
                                                     const float *__restrict__ q, float *__restrict__ qn, float dt,
                                                     int nb_light) {
  __shared__ float red[kHeavyBlock];
  if (int(blockIdx.x) < nb_light) {
    const int64_t rho = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (rho < P.R) {
      reduce_light<NC, QNEW, false>(P, rho, r, ws, q, qn, dt, {nullptr, 0}, {nullptr, 0});
    } else if (rho < int64_t(P.R) + (P.iso ? P.n_iso : P.n - P.n_active)) {
      const int64_t v = P.iso ? int64_t(P.iso[rho - P.R]) : int64_t(P.n_active) + (rho - P.R);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        r[v * NC + c] = 0.0f;
        if constexpr (QNEW) qn[v * NC + c] = q[v * NC + c];
      }
    }
    return;
  }
  const int rho = P.heavy[blockIdx.x - nb_light];
  const int s0 = P.roff[rho], s1 = P.roff[rho + 1];
  const int64_t base = int64_t(P.rvid[rho]) * NC;
  for (int c = 0; c < NC; ++c) {
    float s = 0.0f;
    for (int t = s0 + threadIdx.x; t < s1; t += kHeavyBlock) s += ws[int64_t(P.rslot ? P.rslot[t] : t) * NC + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kHeavyBlock / 2; w > 0; w >>= 1) {
      if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const float tot = r[base + c] + red[0];
      r[base + c] = tot;
      if constexpr (QNEW) qn[base + c] = q[base + c] + dt * tot;
    }
    __syncthreads();
  }
}

__global__ void permute_rows_kernel(const float *__restrict__ src, float *__restrict__ dst,
                                    const int32_t *__restrict__ idx, int64_t n_rows, int ncomp, int inverse) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_rows * ncomp) return;
  const int64_t i = t / ncomp;
  const int c = int(t - i * ncomp);
  const int64_t j = idx[i];
  if (inverse)
    dst[j * ncomp + c] = src[i * ncomp + c];
  else
    dst[i * ncomp + c] = src[j * ncomp + c];
}

// ------------------------------------------------------------------ launchers

int edges_per_thread(int cap, int wg) {
  const int e = (cap + wg - 1) / wg;
  return e <= 1 ? 1 : e <= 2 ? 2 : e <= 4 ? 4 : e <= 8 ? 8 : -1;
}

thread_local LaunchTiming g_timing;

// A kernel launch; with g_timing set, through hipExtLaunchKernelGGL so that the events take the
// dispatch's own timestamps.
#define EPK_LAUNCH(K, grid, block, lds, s, ...)                                                  \
  do {                                                                                           \
    if (g_timing.start) {                                                                        \
      hipExtLaunchKernelGGL(K, grid, block, uint32_t(lds), s, g_timing.start, g_timing.stop, 0u, \
                            __VA_ARGS__);                                                        \
      ++g_timing.launched;                                                                       \
    } else {                                                                                     \
      hipLaunchKernelGGL(K, grid, block, lds, s, __VA_ARGS__);                                   \
    }                                                                                            \
  } while (0)

#define EPK_EPT_SWITCH(ept, CALL) \
  switch (ept) {                  \
    case 1: {                     \
      constexpr int E = 1;        \
      CALL;                       \
    } break;                      \
    case 2: {                     \
      constexpr int E = 2;        \
      CALL;                       \
    } break;                      \
    case 4: {                     \
      constexpr int E = 4;        \
      CALL;                       \
    } break;                      \
    case 8: {                     \
      constexpr int E = 8;        \
      CALL;                       \
    } break;                      \
    default:                      \
      return hipErrorInvalidValue; \
  }

// fused: the single-launch reduction (P.nfy_off, P.nfy, P.rsuf and P.cnt set).
hipError_t launch_flux_fwd(const DevPlan &P, int wg, size_t lds, const float *q, float *r, float *qn, float dt,
                           float *ws, int swizzle, hipStream_t s, bool fused) {
  if (P.k == 0) return hipSuccess;
  const dim3 grid(grid_of_parts(P.k, swizzle)), block(wg);
  const int ept = edges_per_thread(P.cap, wg);
#define EPK_FWD(G, QN, F) \
  EPK_EPT_SWITCH(ept, EPK_LAUNCH((flux_fwd_kernel<G, QN, E, F>), grid, block, lds, s, P, q, r, qn, dt, ws, swizzle))
  if (P.geom_ncomp == 4) {
    if (qn) {
      if (fused) { EPK_FWD(4, true, true) } else { EPK_FWD(4, true, false) }
    } else {
      if (fused) { EPK_FWD(4, false, true) } else { EPK_FWD(4, false, false) }
    }
  } else {
    if (qn) {
      if (fused) { EPK_FWD(2, true, true) } else { EPK_FWD(2, true, false) }
    } else {
      if (fused) { EPK_FWD(2, false, true) } else { EPK_FWD(2, false, false) }
    }
  }
#undef EPK_FWD
  return hipGetLastError();
}

hipError_t launch_flux_bwd(const DevPlan &P, int wg, size_t lds, const float *q, const float *gr, float *gq, float *ws,
                           int swizzle, hipStream_t s, bool fused) {
  if (P.k == 0) return hipSuccess;
  const dim3 grid(grid_of_parts(P.k, swizzle)), block(wg);
  const int ept = edges_per_thread(P.cap, wg);
#define EPK_BWD(G, F) \
  EPK_EPT_SWITCH(ept, EPK_LAUNCH((flux_bwd_kernel<G, E, F>), grid, block, lds, s, P, q, gr, gq, ws, swizzle))
  if (P.geom_ncomp == 4) {
    if (fused) { EPK_BWD(4, true) } else { EPK_BWD(4, false) }
  } else {
    if (fused) { EPK_BWD(2, true) } else { EPK_BWD(2, false) }
  }
#undef EPK_BWD
  return hipGetLastError();
}

hipError_t launch_flux_cached(const DevPlan &P, int wg, size_t lds, const float *q, const float *gr, float *out,
                              float *qn, float dt, float *ws, bool backward, int swizzle, hipStream_t s) {
  if (P.k == 0) return hipSuccess;
  const dim3 grid(grid_of_parts(P.k, swizzle)), block(wg);
  const int ept = edges_per_thread(P.cap, wg);
  if (backward) {
    if (P.geom_ncomp == 4) {
      EPK_EPT_SWITCH(ept, EPK_LAUNCH((flux_bwd_cached<4, E>), grid, block, lds, s, P, q, gr, out, ws, swizzle))
    } else {
      EPK_EPT_SWITCH(ept, EPK_LAUNCH((flux_bwd_cached<2, E>), grid, block, lds, s, P, q, gr, out, ws, swizzle))
    }
  } else if (P.geom_ncomp == 4) {
    if (qn) {
      EPK_EPT_SWITCH(ept, EPK_LAUNCH((flux_fwd_cached<4, true, E>), grid, block, lds, s, P, q, out, qn, dt, ws,
                                             swizzle))
    } else {
      EPK_EPT_SWITCH(ept, EPK_LAUNCH((flux_fwd_cached<4, false, E>), grid, block, lds, s, P, q, out, qn, dt, ws,
                                             swizzle))
    }
  } else {
    if (qn) {
      EPK_EPT_SWITCH(ept, EPK_LAUNCH((flux_fwd_cached<2, true, E>), grid, block, lds, s, P, q, out, qn, dt, ws,
                                             swizzle))
    } else {
      EPK_EPT_SWITCH(ept, EPK_LAUNCH((flux_fwd_cached<2, false, E>), grid, block, lds, s, P, q, out, qn, dt, ws,
                                             swizzle))
    }
  }
  return hipGetLastError();
}

// The pipelined kernel instance for (adjoint?, geometry width, q_new?, edges per thread).
static const void *pipe_fn(bool bwd, int G, bool qnew, int ept) {
#define EPK_PIPE_FN(E)                                                                                        \
  if (ept == E) {                                                                                              \
    if (bwd) return G == 4 ? reinterpret_cast<const void *>(&flux_bwd_pipe<4, E>)                             \
                           : reinterpret_cast<const void *>(&flux_bwd_pipe<2, E>);                            \
    if (G == 4) return qnew ? reinterpret_cast<const void *>(&flux_fwd_pipe<4, true, E>)                       \
                            : reinterpret_cast<const void *>(&flux_fwd_pipe<4, false, E>);                     \
    return qnew ? reinterpret_cast<const void *>(&flux_fwd_pipe<2, true, E>)                                   \
                : reinterpret_cast<const void *>(&flux_fwd_pipe<2, false, E>);                                 \
  }
  EPK_PIPE_FN(1)
  EPK_PIPE_FN(2)
  EPK_PIPE_FN(4)
  EPK_PIPE_FN(8)
#undef EPK_PIPE_FN
  return nullptr;
}

hipError_t launch_flux_pipe(const DevPlan &P, int wg, int grid, size_t lds, const float *q, const float *gr,
                            float *out, float *qn, float dt, float *ws, bool backward, int swizzle, hipStream_t s) {
  if (P.k == 0) return hipSuccess;
  const void *fn = pipe_fn(backward, P.geom_ncomp, qn != nullptr, edges_per_thread(P.cap, wg));
  if (!fn || grid < 1 || (swizzle && grid % 8)) return hipErrorInvalidValue;
  DevPlan Pa = P;
  void *args_bwd[] = {&Pa, &q, &gr, &out, &ws, &swizzle};
  void *args_fwd[] = {&Pa, &q, &out, &qn, &dt, &ws, &swizzle};
  void **args = backward ? args_bwd : args_fwd;
  if (g_timing.start) {
    ++g_timing.launched;
    return hipExtLaunchKernel(fn, dim3(grid), dim3(wg), args, lds, s, g_timing.start, g_timing.stop, 0);
  }
  return hipLaunchKernel(fn, dim3(grid), dim3(wg), args, lds, s);
}

hipError_t launch_spmv(const DevPlan &P, int wg, size_t lds, const float *x, float *y, float *ws, int swizzle,
                       hipStream_t s) {
  if (P.k == 0) return hipSuccess;
  const dim3 grid(grid_of_parts(P.k, swizzle)), block(wg);
  const int ept = (P.cap + wg - 1) / wg;
  if (ept <= 1)
    EPK_LAUNCH((spmv_kernel<1>), grid, block, lds, s, P, x, y, ws, swizzle);
  else if (ept == 2)
    EPK_LAUNCH((spmv_kernel<2>), grid, block, lds, s, P, x, y, ws, swizzle);
  else if (ept <= 4)
    EPK_LAUNCH((spmv_kernel<4>), grid, block, lds, s, P, x, y, ws, swizzle);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_spmv_adjoint(const DevPlan &P, int wg, size_t lds, const float *x, const float *gy, float *gx,
                               float *gw, float *ws, int swizzle, hipStream_t s) {
  if (P.k == 0) return hipSuccess;
  EPK_LAUNCH(spmv_adj_kernel, dim3(grid_of_parts(P.k, swizzle)), dim3(wg), lds, s, P, x, gy, gx, gw, ws,
                     swizzle);
  return hipGetLastError();
}

hipError_t launch_reduce(const DevPlan &P, int nc, float *r, const float *ws, const float *q, float *qn, float dt,
                         hipStream_t s) {
  const int64_t light = int64_t(P.R) + (P.iso ? P.n_iso : P.n - P.n_active);
  const int nb_light = int((light + kReduceBlock - 1) / kReduceBlock);
  const int grid = nb_light + P.n_heavy;
  if (grid == 0) return hipSuccess;
  if (nc == 5) {
    if (qn)
      EPK_LAUNCH((reduce_kernel<5, true>), dim3(grid), dim3(kReduceBlock), 0, s, P, r, ws, q, qn, dt, nb_light);
    else
      EPK_LAUNCH((reduce_kernel<5, false>), dim3(grid), dim3(kReduceBlock), 0, s, P, r, ws, q, qn, dt,
                         nb_light);
  } else {
    EPK_LAUNCH((reduce_kernel<1, false>), dim3(grid), dim3(kReduceBlock), 0, s, P, r, ws, q, qn, dt, nb_light);
  }
  return hipGetLastError();
}

hipError_t launch_permute(const float *src, float *dst, const int32_t *idx, int64_t n_rows, int ncomp, int inverse,
                          hipStream_t s) {
  const int64_t tot = n_rows * ncomp;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(permute_rows_kernel, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s, src, dst, idx, n_rows,
                     ncomp, inverse);
  return hipGetLastError();
}

int pipe_blocks_per_cu(int wg, size_t lds, bool backward, int G, bool qnew, int cap) {
  const void *fn = pipe_fn(backward, G, qnew, edges_per_thread(cap, wg));
  int nb = 0;
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, wg, lds) != hipSuccess || nb < 1) return 1;
  return nb;
}

}  // namespace epk
