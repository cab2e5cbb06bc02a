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
  char* rec_ws;  // record stores of the cubes whose records exceed LDS, and
                 // line workspaces of the cubes whose lines do
};

// Which kernel instantiation serves a cube: dimension count, power-of-two
// line length (all N_k are then powers of two), records kept in LDS.
struct KernelKey {
  int D;
  bool pow2;
  bool rec_lds;
  bool wave;  // solve kernels: one wave per line (64 <= L <= 512, >= D+1 waves)
  bool lines_ws;  // solve kernels: lines in a device workspace (too long for LDS)
  bool operator==(const KernelKey& o) const {
    return D == o.D && pow2 == o.pow2 && rec_lds == o.rec_lds && wave == o.wave && lines_ws == o.lines_ws;
  }
};

enum class KernelKind { kLines, kSolvePlain, kSolveBatched, kBackward };

// The allocation-free plain entry point takes its scratch (the pre-chunk
// spectra and a record store in device memory) from one static device
// array per GPU of this many bytes.
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;

// Address of that array on `device`, which must be the current device;
// looked up once per device (hipGetSymbolAddress) and cached.
hipError_t noalloc_scratch(int device, void** out);

const void* kernel_ptr(KernelKind kind, const KernelKey& key);

hipError_t launch_lines_single(const LaunchCtx& ctx, const KernelKey& key, int cube, const float2* x, int t0,
                               int count, float2* out, int maxL, size_t lds, int threads, hipStream_t st);
hipError_t launch_lines_items(const LaunchCtx& ctx, const KernelKey& key, const LineItem* items,
                              const int32_t* ranges, int* queues, int grid, const float2* const* xs, float2* out,
                              int maxL, size_t lds, int threads, hipStream_t st);
hipError_t launch_solve_plain(const LaunchCtx& ctx, const KernelKey& key, int cube, const float2* x,
                              const OutPtrs& out, const float2* pre, int pre_count, char* rec_store, char* lines_ws,
                              size_t lds, int threads, hipStream_t st);
hipError_t launch_reset(int* p, int n, hipStream_t st);
hipError_t launch_solve_batched(const LaunchCtx& ctx, const KernelKey& key, const float2* const* xs,
                                const OutPtrs* outs, const int32_t* order, int ncubes, int* queue, int grid,
                                size_t lds, int threads, hipStream_t st);
hipError_t launch_zero_single(float2* p, int64_t n, hipStream_t st);
hipError_t launch_zero_multi(float2* const* bufs, const int64_t* lens, int nbufs, int64_t maxlen, hipStream_t st);
hipError_t launch_backward_single(const LaunchCtx& ctx, const KernelKey& key, int cube, const OutPtrs& fwd,
                                  const float2* ga, float2* gx, size_t lds, int threads, hipStream_t st);
hipError_t launch_backward_batched(const LaunchCtx& ctx, const KernelKey& key, const int32_t* order, int ncubes,
                                   const OutPtrs* fwds, const float2* const* gas, float2* const* gxs, size_t lds,
                                   int threads, hipStream_t st);

}  // namespace fpssft
