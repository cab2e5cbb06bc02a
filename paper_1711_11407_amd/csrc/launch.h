// Launchers of the gfx950 kernels, called by the host plan.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "types.h"

namespace fpssft {

// Device tables every kernel reads.
struct LaunchCtx {
  const CubeDesc* descs;
  const int32_t* sched;
  const float2* tw;
};

hipError_t launch_lines_single(const LaunchCtx& ctx, int cube, const float2* x, int t0, int count,
                               int G, float2* out, size_t lds, int threads, hipStream_t st);
hipError_t launch_lines_items(const LaunchCtx& ctx, const LineItem* items, int nitems,
                              const float2* const* xs, float2* out, size_t lds, int threads,
                              hipStream_t st);
hipError_t launch_solve_plain(const LaunchCtx& ctx, int cube, const float2* x, const OutPtrs& out,
                              const float2* pre, int pre_count, size_t lds, int threads, hipStream_t st);
hipError_t launch_solve_batched(const LaunchCtx& ctx, const float2* const* xs, const OutPtrs* outs,
                                const int32_t* order, int ncubes, int* queue, int grid, size_t lds,
                                int threads, hipStream_t st);
hipError_t launch_zero_single(float2* p, int64_t n, hipStream_t st);
hipError_t launch_zero_multi(float2* const* bufs, const int64_t* lens, int nbufs, int64_t maxlen,
                             hipStream_t st);
hipError_t launch_backward_single(const LaunchCtx& ctx, int cube, const OutPtrs& fwd, const float2* ga,
                                  float2* gx, size_t lds, int threads, hipStream_t st);
hipError_t launch_backward_batched(const LaunchCtx& ctx, int ncubes, const OutPtrs* fwds,
                                   const float2* const* gas, float2* const* gxs, size_t lds, int threads,
                                   hipStream_t st);

const void* kernel_solve_batched();
const void* kernel_solve_plain();
const void* kernel_lines();
const void* kernel_backward();

}  // namespace fpssft
