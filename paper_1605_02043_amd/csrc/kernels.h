// Launchers of the device kernels (kernels.hip); used by the device API (api.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "epk_internal.h"

namespace epk {

// Dispatch timestamps for benchmarking: while `start` is set, the launchers on this thread pass
// start/stop to hipExtLaunchKernel, which records the kernel's own start and end times into them;
// `launched` counts those launches.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
  int launched = 0;
};
extern thread_local LaunchTiming g_timing;

int grid_of_parts(int k, int swizzle);
// fused: the single-launch reduction (the plan's signal records and counters are set in P)
hipError_t launch_flux_fwd(const DevPlan &P, int wg, size_t lds, const float *q, float *r, float *qn, float dt,
                           float *ws, int swizzle, hipStream_t s, bool fused = false);
hipError_t launch_flux_bwd(const DevPlan &P, int wg, size_t lds, const float *q, const float *gr, float *gq, float *ws,
                           int swizzle, hipStream_t s, bool fused = false);
hipError_t launch_flux_cached(const DevPlan &P, int wg, size_t lds, const float *q, const float *gr, float *out,
                              float *qn, float dt, float *ws, bool backward, int swizzle, hipStream_t s);
hipError_t launch_flux_pipe(const DevPlan &P, int wg, int grid, size_t lds, const float *q, const float *gr,
                            float *out, float *qn, float dt, float *ws, bool backward, int swizzle, hipStream_t s);
hipError_t launch_spmv(const DevPlan &P, int wg, size_t lds, const float *x, float *y, float *ws, int swizzle,
                       hipStream_t s);
hipError_t launch_spmv_adjoint(const DevPlan &P, int wg, size_t lds, const float *x, const float *gy, float *gx,
                               float *gw, float *ws, int swizzle, hipStream_t s);
hipError_t launch_reduce(const DevPlan &P, int nc, float *r, const float *ws, const float *q, float *qn, float dt,
                         hipStream_t s);
hipError_t launch_permute(const float *src, float *dst, const int32_t *idx, int64_t n_rows, int ncomp, int inverse,
                          hipStream_t s);
int pipe_blocks_per_cu(int wg, size_t lds, bool backward, int G, bool qnew, int cap);
int edges_per_thread(int cap, int wg);

}  // namespace epk
