// Device kernels of libepk (gfx950).
//
// One workgroup runs one part of the edge partition, the paper's "one
// partition per thread block" (Section 4; Section 5.2 for SpMV):
//   1. stage the part's distinct vertices in LDS: the owned range as one
//      contiguous block, foreign vertices through their packed ids;
//   2. run the per-edge task out of LDS;
//   3. sum per-vertex partials in LDS in a fixed order (FLUX5: local
//      incidence lists; SpMV: segmented scan over edges sorted by local y);
//   4. write owned vertices straight to the output and the partials of
//      foreign (replicated) vertices to workspace slots, both as contiguous
//      blocks.
// A reduction kernel then adds, for every replicated vertex, the slots to the
// owner's partial in ascending part order.  Nothing uses atomics on data, so
// every result is bitwise reproducible.  No MFMA: the work is gather/scatter.
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
    const float mn = m1 * n1 + m2 * n2 + m3 * n3;
    const float mm = m1 * m1 + m2 * m2 + m3 * m3;
    const float s = mn / rho;
    const float p = kG1 * (E - 0.5f * mm / rho);
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
  const float ir = 1.0f / rho;
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

// 3D edges carry the area vector A = a n (3 floats); 2D edges the unit normal (a = 1).
template <int G>
__device__ __forceinline__ void load_geom(const float *geom, int64_t e, float &n1, float &n2, float &n3, float &a) {
  if constexpr (G == 4) {
    const float *g = geom + 3 * e;
    n1 = g[0];
    n2 = g[1];
    n3 = g[2];
    a = sqrtf(n1 * n1 + n2 * n2 + n3 * n3);
  } else {
    const float2 g = reinterpret_cast<const float2 *>(geom)[e];
    n1 = g.x;
    n2 = g.y;
    n3 = 0.0f;
    a = 1.0f;
  }
}

// ------------------------------------------------------------------ staging

#define EPK_LDS(p) ((__attribute__((address_space(3))) void *)(p))

constexpr int kMaxFI = 16;  // foreign-state dwords prefetched per thread (covers 16 * wg / 5 vertices)

// Copy src[0, n) to LDS dst[0, n) with direct-to-LDS loads: lane l of a wave
// writes its dword at (wave base + 4 l); the base d - lane is wave-uniform
// because the block size is a multiple of 64.
__device__ __forceinline__ void dma_block(float *dst, const float *src, int n, int tid, int nt) {
  const int lane = tid & 63;
  for (int d = tid; d < n; d += nt) __builtin_amdgcn_global_load_lds(src + d, EPK_LDS(dst + (d - lane)), 4, 0, 0);
}

// Stage 5 * nf foreign state dwords: every foreign id is read first (one batch
// of independent loads), then the states are fetched straight into LDS.
__device__ __forceinline__ void dma_foreign(float *dst, const float *__restrict__ src, const int32_t *__restrict__ fids,
                                            int nf, int tid, int nt) {
  const int lane = tid & 63;
  const int nfd = nf * 5;
  int fr[kMaxFI];
#pragma unroll
  for (int k = 0; k < kMaxFI; ++k) {
    const int d = tid + k * nt;
    fr[k] = d < nfd ? fids[d / 5] : 0;
  }
#pragma unroll
  for (int k = 0; k < kMaxFI; ++k) {
    const int d = tid + k * nt;
    if (d < nfd)
      __builtin_amdgcn_global_load_lds(src + int64_t(fr[k]) * 5 + (d - 5 * (d / 5)), EPK_LDS(dst + (d - lane)), 4, 0, 0);
  }
  for (int d = tid + kMaxFI * nt; d < nfd; d += nt)  // parts wider than the prefetch window
    __builtin_amdgcn_global_load_lds(src + int64_t(fids[d / 5]) * 5 + (d - 5 * (d / 5)), EPK_LDS(dst + (d - lane)), 4,
                                     0, 0);
}

__device__ __forceinline__ void wait_staged() {
  __builtin_amdgcn_s_waitcnt(0);  // all direct-to-LDS loads of this wave have landed
  __syncthreads();
}

struct PartHdr {
  int e0, ne, own0, nown, f0, nf, lofs, U;
};

__device__ __forceinline__ PartHdr load_hdr(const DevPlan &P, int part) {
  const int4 *h = reinterpret_cast<const int4 *>(P.hdr + int64_t(part) * kHdrInts);
  const int4 a = h[0], b = h[1];
  return {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
}

// Incidence entries (2 u16 per edge, one dword) and offsets (U + 1 u16 from an
// even index, read as whole dwords) into LDS.
__device__ __forceinline__ void dma_incidence(uint16_t *inc, uint16_t *lo, const DevPlan &P, const PartHdr &h, int tid,
                                              int nt) {
  dma_block(reinterpret_cast<float *>(inc), reinterpret_cast<const float *>(P.inc) + h.e0, h.ne, tid, nt);
  dma_block(reinterpret_cast<float *>(lo), reinterpret_cast<const float *>(P.loff) + (h.lofs >> 1), (h.U + 2) >> 1,
            tid, nt);
}

template <int G, int EPT>
__device__ __forceinline__ void load_edges(const DevPlan &P, const PartHdr &h, int tid, int nt, uint32_t ew[EPT],
                                           float4 eg[EPT]) {
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int j = tid + k * nt;
    ew[k] = 0u;
    eg[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (j < h.ne) {
      ew[k] = P.eloc[h.e0 + j];
      load_geom<G>(P.geom, int64_t(h.e0) + j, eg[k].x, eg[k].y, eg[k].z, eg[k].w);
    }
  }
}

// ------------------------------------------------------------------ FLUX5 parts

// LDS: st[max_u][5] | (QNEW: acc[max_u][5]) | flx[cap][5] | inc[2 cap] u16 | lo[max_u + 2] u16.
// Without q_new the per-vertex sums overwrite st (no thread reads st then).
template <int G, bool QNEW, int EPT>
__device__ __forceinline__ void flux_fwd_part(const DevPlan &P, int part, const float *__restrict__ q,
                                              float *__restrict__ r, float *__restrict__ qn, float dt,
                                              float *__restrict__ ws, float *smem) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const PartHdr h = load_hdr(P, part);
  float *st = smem;
  float *acc = QNEW ? st + P.max_u * 5 : st;
  float *flx = (QNEW ? acc : st) + P.max_u * 5;
  uint16_t *inc = reinterpret_cast<uint16_t *>(flx + P.cap * 5);
  uint16_t *lo = inc + 2 * P.cap;

  dma_block(st, q + int64_t(h.own0) * 5, h.nown * 5, tid, nt);
  dma_incidence(inc, lo, P, h, tid, nt);
  uint32_t ew[EPT];
  float4 eg[EPT];
  load_edges<G, EPT>(P, h, tid, nt, ew, eg);
  dma_foreign(st + h.nown * 5, q, P.fid + h.f0, h.nf, tid, nt);
  wait_staged();

#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int j = tid + k * nt;
    if (j < h.ne) {
      float F[5];
      edge_flux(st + (ew[k] & 0xffffu) * 5, st + (ew[k] >> 16) * 5, eg[k].x, eg[k].y, eg[k].z, eg[k].w, F);
#pragma unroll
      for (int c = 0; c < 5; ++c) flx[j * 5 + c] = F[c];
    }
  }
  __syncthreads();

  for (int i = tid; i < h.U; i += nt) {
    float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    const int t1 = lo[i + 1];
    for (int t = lo[i]; t < t1; ++t) {
      const int x = inc[t];
      const float *f = flx + (x >> 1) * 5;
      if (x & 1) {
#pragma unroll
        for (int c = 0; c < 5; ++c) s[c] -= f[c];
      } else {
#pragma unroll
        for (int c = 0; c < 5; ++c) s[c] += f[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) acc[i * 5 + c] = s[c];
  }
  __syncthreads();

  float *ro = r + int64_t(h.own0) * 5;
  for (int d = tid; d < h.nown * 5; d += nt) {
    ro[d] = acc[d];
    if constexpr (QNEW) qn[int64_t(h.own0) * 5 + d] = st[d] + dt * acc[d];
  }
  float *wo = ws + int64_t(h.f0) * 5;
  for (int d = tid; d < h.nf * 5; d += nt) wo[d] = acc[h.nown * 5 + d];
}

// LDS: st[max_u][5] | gs[max_u][5] (then the per-vertex sums) | vu[cap][5] | vv[cap][5] | inc | lo.
template <int G, int EPT>
__device__ __forceinline__ void flux_bwd_part(const DevPlan &P, int part, const float *__restrict__ q,
                                              const float *__restrict__ gr, float *__restrict__ gq,
                                              float *__restrict__ ws, float *smem) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const PartHdr h = load_hdr(P, part);
  float *st = smem;
  float *gs = st + P.max_u * 5;
  float *vu = gs + P.max_u * 5;
  float *vv = vu + P.cap * 5;
  uint16_t *inc = reinterpret_cast<uint16_t *>(vv + P.cap * 5);
  uint16_t *lo = inc + 2 * P.cap;

  dma_block(st, q + int64_t(h.own0) * 5, h.nown * 5, tid, nt);
  dma_block(gs, gr + int64_t(h.own0) * 5, h.nown * 5, tid, nt);
  dma_incidence(inc, lo, P, h, tid, nt);
  uint32_t ew[EPT];
  float4 eg[EPT];
  load_edges<G, EPT>(P, h, tid, nt, ew, eg);
  dma_foreign(st + h.nown * 5, q, P.fid + h.f0, h.nf, tid, nt);
  dma_foreign(gs + h.nown * 5, gr, P.fid + h.f0, h.nf, tid, nt);
  wait_staged();

#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int j = tid + k * nt;
    if (j < h.ne) {
      const int lu = ew[k] & 0xffffu, lv = ew[k] >> 16;
      // d(a F)/dq = a J(q, n) / 2 +- a sigma I / 2 = J(q, A) / 2 +- a sigma I / 2 (J linear in n)
      const float hs = 0.5f * kSigma * eg[k].w;
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
  __syncthreads();

  for (int i = tid; i < h.U; i += nt) {
    float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    const int t1 = lo[i + 1];
    for (int t = lo[i]; t < t1; ++t) {
      const int x = inc[t];
      const float *f = ((x & 1) ? vv : vu) + (x >> 1) * 5;
#pragma unroll
      for (int c = 0; c < 5; ++c) s[c] += f[c];
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) gs[i * 5 + c] = s[c];
  }
  __syncthreads();

  float *go = gq + int64_t(h.own0) * 5;
  for (int d = tid; d < h.nown * 5; d += nt) go[d] = gs[d];
  float *wo = ws + int64_t(h.f0) * 5;
  for (int d = tid; d < h.nf * 5; d += nt) wo[d] = gs[h.nown * 5 + d];
}

template <int G, bool QNEW, int EPT>
__global__ void __launch_bounds__(1024) flux_fwd_kernel(DevPlan P, const float *__restrict__ q, float *__restrict__ r,
                                                        float *__restrict__ qn, float dt, float *__restrict__ ws,
                                                        int swizzle) {
  extern __shared__ float smem[];
  const int part = part_of_block(blockIdx.x, P.k, swizzle);
  if (part >= P.k) return;
  flux_fwd_part<G, QNEW, EPT>(P, part, q, r, qn, dt, ws, smem);
}

template <int G, int EPT>
__global__ void __launch_bounds__(1024) flux_bwd_kernel(DevPlan P, const float *__restrict__ q,
                                                        const float *__restrict__ gr, float *__restrict__ gq,
                                                        float *__restrict__ ws, int swizzle) {
  extern __shared__ float smem[];
  const int part = part_of_block(blockIdx.x, P.k, swizzle);
  if (part >= P.k) return;
  flux_bwd_part<G, EPT>(P, part, q, gr, gq, ws, smem);
}

// Persistent variant: a fixed grid takes parts from a queue (largest first).
// Every workgroup stops after drawing one ticket past the last item; the
// workgroup that stops last resets both counters, so the next launch (and
// every replay of a captured graph) starts from zero.
__device__ __forceinline__ int next_item(const DevPlan &P, int *s_item) {
  if (threadIdx.x == 0) {
    const uint32_t t = atomicAdd(&P.queue[0], 1u);
    int item = -1;
    if (t < uint32_t(P.k)) {
      item = P.items[t];
    } else {
      const uint32_t done = atomicAdd(&P.queue[1], 1u);
      if (done == uint32_t(P.grid) - 1u) {
        atomicExch(&P.queue[0], 0u);
        atomicExch(&P.queue[1], 0u);
      }
    }
    *s_item = item;
  }
  __syncthreads();
  const int item = *s_item;
  __syncthreads();
  return item;
}

template <int EPT>
__global__ void __launch_bounds__(256) flux_fwd_persistent(DevPlan P, const float *__restrict__ q,
                                                            float *__restrict__ r, float *__restrict__ ws) {
  extern __shared__ float smem[];
  __shared__ int s_item;
  for (;;) {
    const int part = next_item(P, &s_item);
    if (part < 0) break;
    flux_fwd_part<4, false, EPT>(P, part, q, r, nullptr, 0.f, ws, smem);
    __syncthreads();
  }
}

template <int EPT>
__global__ void __launch_bounds__(256) flux_bwd_persistent(DevPlan P, const float *__restrict__ q,
                                                            const float *__restrict__ gr, float *__restrict__ gq,
                                                            float *__restrict__ ws) {
  extern __shared__ float smem[];
  __shared__ int s_item;
  for (;;) {
    const int part = next_item(P, &s_item);
    if (part < 0) break;
    flux_bwd_part<4, EPT>(P, part, q, gr, gq, ws, smem);
    __syncthreads();
  }
}

// ------------------------------------------------------------------ SpMV

// LDS: xs[max_ux] | ys[max_uy] | per-wave carry keys and values.
__global__ void __launch_bounds__(1024) spmv_kernel(DevPlan P, const float *__restrict__ x, float *__restrict__ y,
                                                    float *__restrict__ ws, int swizzle) {
  extern __shared__ float smem[];
  const int part = part_of_block(blockIdx.x, P.k, swizzle);
  if (part >= P.k) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int4 *h4 = reinterpret_cast<const int4 *>(P.hdr + int64_t(part) * kHdrInts);
  const int4 ha = h4[0], hb = h4[1];
  const int xo = ha.x, xn = ha.y, xf0 = ha.z, xnf = ha.w, yo = hb.x, yn = hb.y, yf0 = hb.z, ynf = hb.w;
  const int64_t e0 = P.eoff[part];
  const int ne = int(P.eoff[part + 1] - e0);
  float *xs = smem;
  float *ys = xs + P.max_u;
  int *tkey = reinterpret_cast<int *>(ys + P.max_uy);
  float *tval = reinterpret_cast<float *>(tkey + (nt >> 6));
  const int lane = tid & 63, wave = tid >> 6;

  // owned x block straight to LDS; edge data and foreign x ids in one batch of loads
  dma_block(xs, x + xo, xn, tid, nt);
  const bool valid = tid < ne;
  const uint32_t w = valid ? P.eloc[e0 + tid] : 0u;
  const float wt = valid ? P.geom[e0 + tid] : 0.0f;
  const uint32_t w_next = (lane == 63 && tid + 1 < ne) ? P.eloc[e0 + tid + 1] : 0u;
  const int32_t *fids = P.fid + xf0;
  int fr[kMaxFI];
#pragma unroll
  for (int k = 0; k < kMaxFI; ++k) {
    const int d = tid + k * nt;
    fr[k] = d < xnf ? fids[d] : 0;
  }
#pragma unroll
  for (int k = 0; k < kMaxFI; ++k) {
    const int d = tid + k * nt;
    if (d < xnf) __builtin_amdgcn_global_load_lds(x + fr[k], EPK_LDS(xs + xn + (d - lane)), 4, 0, 0);
  }
  for (int d = tid + kMaxFI * nt; d < xnf; d += nt)
    __builtin_amdgcn_global_load_lds(x + fids[d], EPK_LDS(xs + xn + (d - lane)), 4, 0, 0);
  wait_staged();

  // one edge per thread, edges sorted by local y: inclusive segmented scan per wavefront
  const int key = valid ? int(w >> 16) : 0x7fffffff;
  float v = valid ? wt * xs[w & 0xffffu] : 0.0f;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const float vu = __shfl_up(v, d, 64);
    const int ku = __shfl_up(key, d, 64);
    if (lane >= d && ku == key) v = vu + v;
  }
  int key_next = __shfl_down(key, 1, 64);
  if (lane == 63) key_next = (tid + 1 < ne) ? int(w_next >> 16) : 0x7ffffffe;
  if (lane == 63) {
    tkey[wave] = (valid && key_next == key) ? key : -1;
    tval[wave] = v;
  }
  __syncthreads();
  if (valid && key_next != key) {  // end of a segment: add the carries of earlier wavefronts
    float carry = 0.0f;
    bool has = false;
    for (int wp = wave - 1; wp >= 0 && tkey[wp] == key; --wp) {
      carry = has ? carry + tval[wp] : tval[wp];
      has = true;
    }
    ys[key] = has ? carry + v : v;
  }
  __syncthreads();
  for (int d = tid; d < yn; d += nt) y[yo + d] = ys[d];
  float *wo = ws + yf0;
  for (int d = tid; d < ynf; d += nt) wo[d] = ys[yn + d];
}

// ------------------------------------------------------------------ reduction

// Light vertices (<= kHeavySlots partials): one thread per vertex,
// r_v = (((own + s_1) + s_2) + ...) in ascending part order.  Heavy vertices:
// one workgroup each, strided partial sums then a fixed tree.  Untouched
// vertices are zeroed here as well.
template <int NC, bool QNEW>
__global__ void __launch_bounds__(256) reduce_kernel(DevPlan P, float *__restrict__ r, const float *__restrict__ ws,
                                                     const float *__restrict__ q, float *__restrict__ qn, float dt,
                                                     int nb_light) {
  __shared__ float red[kHeavyBlock];
  if (int(blockIdx.x) < nb_light) {
    const int64_t rho = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (rho < P.R) {
      const int s0 = P.roff[rho], s1 = P.roff[rho + 1];
      if (s1 - s0 > kHeavySlots) return;
      const int64_t o = int64_t(P.rvid[rho]) * NC;
      float s[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) s[c] = r[o + c];
      for (int t = s0; t < s1; t += 4) {  // four slot ids per batch of loads
        int sl[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) sl[u] = t + u < s1 ? P.rslot[t + u] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (sl[u] >= 0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) s[c] += ws[int64_t(sl[u]) * NC + c];
          }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        r[o + c] = s[c];
        if constexpr (QNEW) qn[o + c] = q[o + c] + dt * s[c];
      }
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
    for (int t = s0 + threadIdx.x; t < s1; t += kHeavyBlock) s += ws[int64_t(P.rslot[t]) * NC + c];
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

hipError_t launch_flux_fwd(const DevPlan &P, int wg, size_t lds, const float *q, float *r, float *qn, float dt,
                           float *ws, int swizzle, hipStream_t s) {
  if (P.k == 0) return hipSuccess;
  const dim3 grid(grid_of_parts(P.k, swizzle)), block(wg);
  const int ept = edges_per_thread(P.cap, wg);
  if (P.geom_ncomp == 4) {
    if (qn) {
      EPK_EPT_SWITCH(ept, hipLaunchKernelGGL((flux_fwd_kernel<4, true, E>), grid, block, lds, s, P, q, r, qn, dt, ws,
                                             swizzle))
    } else {
      EPK_EPT_SWITCH(ept, hipLaunchKernelGGL((flux_fwd_kernel<4, false, E>), grid, block, lds, s, P, q, r, qn, dt, ws,
                                             swizzle))
    }
  } else {
    if (qn) {
      EPK_EPT_SWITCH(ept, hipLaunchKernelGGL((flux_fwd_kernel<2, true, E>), grid, block, lds, s, P, q, r, qn, dt, ws,
                                             swizzle))
    } else {
      EPK_EPT_SWITCH(ept, hipLaunchKernelGGL((flux_fwd_kernel<2, false, E>), grid, block, lds, s, P, q, r, qn, dt, ws,
                                             swizzle))
    }
  }
  return hipGetLastError();
}

hipError_t launch_flux_bwd(const DevPlan &P, int wg, size_t lds, const float *q, const float *gr, float *gq, float *ws,
                           int swizzle, hipStream_t s) {
  if (P.k == 0) return hipSuccess;
  const dim3 grid(grid_of_parts(P.k, swizzle)), block(wg);
  const int ept = edges_per_thread(P.cap, wg);
  if (P.geom_ncomp == 4) {
    EPK_EPT_SWITCH(ept, hipLaunchKernelGGL((flux_bwd_kernel<4, E>), grid, block, lds, s, P, q, gr, gq, ws, swizzle))
  } else {
    EPK_EPT_SWITCH(ept, hipLaunchKernelGGL((flux_bwd_kernel<2, E>), grid, block, lds, s, P, q, gr, gq, ws, swizzle))
  }
  return hipGetLastError();
}

hipError_t launch_flux_persistent(const DevPlan &P, int wg, size_t lds, const float *q, const float *gr, float *out,
                                  float *ws, bool backward, hipStream_t s) {
  if (P.k == 0) return hipSuccess;
  const dim3 grid(P.grid), block(wg);
  const int ept = edges_per_thread(P.cap, wg);
  if (backward) {
    EPK_EPT_SWITCH(ept, hipLaunchKernelGGL((flux_bwd_persistent<E>), grid, block, lds, s, P, q, gr, out, ws))
  } else {
    EPK_EPT_SWITCH(ept, hipLaunchKernelGGL((flux_fwd_persistent<E>), grid, block, lds, s, P, q, out, ws))
  }
  return hipGetLastError();
}

hipError_t launch_spmv(const DevPlan &P, int wg, size_t lds, const float *x, float *y, float *ws, int swizzle,
                       hipStream_t s) {
  if (P.k == 0) return hipSuccess;
  hipLaunchKernelGGL(spmv_kernel, dim3(grid_of_parts(P.k, swizzle)), dim3(wg), lds, s, P, x, y, ws, swizzle);
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
      hipLaunchKernelGGL((reduce_kernel<5, true>), dim3(grid), dim3(kReduceBlock), 0, s, P, r, ws, q, qn, dt, nb_light);
    else
      hipLaunchKernelGGL((reduce_kernel<5, false>), dim3(grid), dim3(kReduceBlock), 0, s, P, r, ws, q, qn, dt,
                         nb_light);
  } else {
    hipLaunchKernelGGL((reduce_kernel<1, false>), dim3(grid), dim3(kReduceBlock), 0, s, P, r, ws, q, qn, dt, nb_light);
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

int persistent_blocks_per_cu(int wg, size_t lds, bool backward, int cap) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  const int ept = edges_per_thread(cap, wg);
  const void *fn = nullptr;
  if (backward)
    fn = ept == 1 ? reinterpret_cast<const void *>(&flux_bwd_persistent<1>)
       : ept == 2 ? reinterpret_cast<const void *>(&flux_bwd_persistent<2>)
       : ept == 4 ? reinterpret_cast<const void *>(&flux_bwd_persistent<4>)
                  : reinterpret_cast<const void *>(&flux_bwd_persistent<8>);
  else
    fn = ept == 1 ? reinterpret_cast<const void *>(&flux_fwd_persistent<1>)
       : ept == 2 ? reinterpret_cast<const void *>(&flux_fwd_persistent<2>)
       : ept == 4 ? reinterpret_cast<const void *>(&flux_fwd_persistent<4>)
                  : reinterpret_cast<const void *>(&flux_fwd_persistent<8>);
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, wg, lds);
  if (e != hipSuccess || nb < 1) return 1;
  return nb;
}

}  // namespace epk
