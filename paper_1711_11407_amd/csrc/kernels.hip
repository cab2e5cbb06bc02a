// gfx950 kernels of the FPS-SFT hot path.
//
//  k_lines          line gather + L-point FFT of whole iterations (D+1 lines
//                   each) into a spectra buffer (Eq. sample_slice, Eq. hs);
//                   many work-groups, HBM-bound.
//  k_solve_plain    one cube in one work-group: for every iteration, the
//                   spectra (precomputed by k_lines for the first chunk,
//                   gathered and transformed in LDS after it), the peel of
//                   the recovered list (construction-subtraction, Sec. 2.2,
//                   done on the spectra), the 1-sparsity test, the phase
//                   decode and the amplitude (Eq. decoding), the ordered
//                   append, and the stopping rule.
//  k_solve_batched  the same per cube, persistent: work-groups take cube
//                   indices from a device queue until it is empty.
//  k_backward       adjoint of the amplitudes with the decisions fixed.
//  k_reset, k_zero  counter reset and zero fill (kernels, so that they can
//                   sit inside a captured graph).
#include <hip/hip_runtime.h>

#include "device.h"
#include "launch.h"

namespace fpssft {

static constexpr float kInv2Pi = (float)(1.0 / (2.0 * 3.14159265358979323846));

// ---------------------------------------------------------------------------
// Line gather + FFT
// ---------------------------------------------------------------------------
__global__ void k_lines(const CubeDesc* __restrict__ descs, const LineItem* __restrict__ items,
                        int nitems, int per_xcd, int single_cube, int t0, int count, int G,
                        const float2* __restrict__ x_single, const float2* const* __restrict__ xs,
                        const int32_t* __restrict__ sched, const float2* __restrict__ tw,
                        float2* __restrict__ out) {
  extern __shared__ float2 lds_lines[];
  int cube, tb, tc;
  int64_t ooff;
  const float2* x;
  if (items) {
    // XCD-aware order: work-groups are dispatched round-robin over the 8
    // XCDs, so consecutive items (the same cube) go to one XCD and share its
    // L2.
    const int b = blockIdx.x;
    const int it = (b & 7) * per_xcd + (b >> 3);
    if (it >= nitems) return;
    const LineItem li = items[it];
    cube = li.cube;
    tb = li.t0;
    tc = li.count;
    ooff = li.out_off;
    x = xs[cube];
  } else {
    cube = single_cube;
    tb = t0 + blockIdx.x * G;
    tc = min(G, t0 + count - tb);
    if (tc <= 0) return;
    x = x_single;
    ooff = (int64_t)(tb - t0) * (descs[cube].D + 1) * descs[cube].L;
  }
  const CubeDesc& cd = descs[cube];
  const int nl = tc * (cd.D + 1);
  float2* a = lds_lines;
  float2* b2 = a + nl * cd.L;
  gather_lines(a, x, cd, sched + cd.sched_off + tb * 2 * cd.D, tc, cd.inv_L);
  __syncthreads();
  float2* S = block_fft(a, b2, nl, cd, tw + cd.tw_off);
  float2* o = out + ooff;
  const int n = nl * cd.L;
  for (int e = threadIdx.x; e < n; e += blockDim.x) o[e] = S[e];
}

// ---------------------------------------------------------------------------
// One cube, one work-group.
// ---------------------------------------------------------------------------
struct SolveLds {
  float2* bufA;
  float2* bufB;
  int32_t* rec_f;  // [rec_lds][D] frequency indices
  float2* rec_a;   // [rec_lds] amplitudes
  int* wsum;       // [16]
};

__device__ __forceinline__ SolveLds carve_solve_lds(char* smem, const CubeDesc& cd) {
  SolveLds s;
  const int nl = cd.D + 1;
  s.bufA = (float2*)smem;
  s.bufB = s.bufA + nl * cd.L;
  char* p = (char*)(s.bufB + nl * cd.L);
  s.rec_a = (float2*)p;
  p += (size_t)cd.rec_lds * sizeof(float2);
  s.rec_f = (int32_t*)p;
  p += (size_t)cd.rec_lds * cd.D * sizeof(int32_t);
  s.wsum = (int*)p;
  return s;
}

// Samples (or precomputed spectra) of one iteration held in registers: the
// D+1 values at l = tid + u * blockDim.x, u < kPfU. Loaded one iteration
// ahead so that their latency overlaps the current iteration's work.
constexpr int kPfU = 4;

struct Prefetch {
  float2 v[kPfU][5];
};

__device__ __forceinline__ void prefetch_issue(Prefetch& pf, const CubeDesc& cd, const float2* __restrict__ x,
                                               const int32_t* __restrict__ sched,
                                               const float2* __restrict__ pre, int pre_count, int t) {
  const int D = cd.D;
  const int L = cd.L;
  if (t < pre_count) {
    const float2* src = pre + (int64_t)t * (D + 1) * L;
#pragma unroll
    for (int u = 0; u < kPfU; ++u) {
      const int l = threadIdx.x + u * blockDim.x;
      if (l < L) {
#pragma unroll
        for (int i = 0; i < 5; ++i)
          if (i <= D) pf.v[u][i] = src[i * L + l];
      }
    }
    return;
  }
  const int32_t* row = sched + cd.sched_off + t * 2 * D;
#pragma unroll
  for (int u = 0; u < kPfU; ++u) {
    const int l = threadIdx.x + u * blockDim.x;
    if (l < L) {
      uint32_t n[4];
      int64_t flat = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k < D) {
          const uint32_t v = (uint32_t)row[k] * (uint32_t)l + (uint32_t)row[D + k];
          n[k] = umod(v, (uint32_t)cd.dims[k], cd.dmask[k]);
          flat += (int64_t)n[k] * cd.stride[k];
        }
      }
      pf.v[u][0] = x[flat];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k < D) {
          const int64_t step = (n[k] + 1 == (uint32_t)cd.dims[k]) ? -(int64_t)(cd.dims[k] - 1) * cd.stride[k]
                                                                     : cd.stride[k];
          pf.v[u][k + 1] = x[flat + step];
        }
      }
    }
  }
}

__device__ __forceinline__ void prefetch_store(const Prefetch& pf, const CubeDesc& cd, float2* __restrict__ dst,
                                               float scale) {
  const int D = cd.D;
  const int L = cd.L;
#pragma unroll
  for (int u = 0; u < kPfU; ++u) {
    const int l = threadIdx.x + u * blockDim.x;
    if (l < L) {
#pragma unroll
      for (int i = 0; i < 5; ++i)
        if (i <= D) dst[i * L + l] = c_scale(pf.v[u][i], scale);
    }
  }
}

__device__ __forceinline__ void solve_cube(const CubeDesc& cd, const float2* __restrict__ x, const OutPtrs out,
                                           const int32_t* __restrict__ sched, const float2* __restrict__ twall,
                                           const float2* __restrict__ pre, int pre_count, char* smem) {
  const int D = cd.D;
  const int L = cd.L;
  const int T = cd.T;
  const int nl = D + 1;
  const int tid = threadIdx.x;
  const int B = blockDim.x;
  const float2* __restrict__ tw = twall + cd.tw_off;
  SolveLds s = carve_solve_lds(smem, cd);
  // Records: LDS copies when they fit, else the output arrays themselves.
  int32_t* rf = cd.rec_lds ? s.rec_f : out.freqs;
  float2* ra = cd.rec_lds ? s.rec_a : (float2*)out.amps;
  float2* oamps = (float2*)out.amps;

  const float th0 = cd.zero_thresh;
  const float rho = cd.mag_rel_tol;
  const float gtol = cd.grid_tol;
  const bool use_pf = L <= kPfU * B;

  Prefetch pf;
  if (use_pf && T > 0) prefetch_issue(pf, cd, x, sched, pre, pre_count, 0);

  int kc = 0;
  int status = kStatusIncomplete;
  int iters = T;
  for (int t = 0; t < T; ++t) {
    const int32_t* at = sched + cd.sched_off + t * 2 * D;
    const bool precomputed = t < pre_count;
    if (use_pf) {
      prefetch_store(pf, cd, s.bufA, precomputed ? 1.0f : cd.inv_L);
      if (t + 1 < T) prefetch_issue(pf, cd, x, sched, pre, pre_count, t + 1);
    } else if (precomputed) {
      const float2* src = pre + (int64_t)t * nl * L;
      for (int e = tid; e < nl * L; e += B) s.bufA[e] = src[e];
    } else {
      gather_lines(s.bufA, x, cd, at, 1, cd.inv_L);
    }
    lds_barrier();
    float2* S = precomputed ? s.bufA : block_fft(s.bufA, s.bufB, nl, cd, tw);
    uint32_t al[4], ta[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      al[k] = k < D ? (uint32_t)at[k] : 0u;
      ta[k] = k < D ? (uint32_t)at[D + k] : 0u;
    }

    // Peel: subtract every earlier record's projection a e^{+j 2 pi p / L}
    // from bin b of each line, b = [sum_k alpha_k c_k m_k]_L and
    // p = [sum_k tau_k^{(i)} c_k m_k]_L (Eq. freqSum, Eq. orthogonality).
    for (int j = tid; j < kc; j += B) {
      uint32_t g[4];
      uint32_t b = 0, p0 = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k < D) {
          g[k] = (uint32_t)cd.c[k] * (uint32_t)rf[j * D + k];
          b = umod(b + al[k] * g[k], L, cd.Lmask);
          p0 = umod(p0 + ta[k] * g[k], L, cd.Lmask);
        }
      }
      const float2 a = ra[j];
      float2 c = c_mulc(a, tw[p0]);
      atomicAdd(&S[b].x, -c.x);
      atomicAdd(&S[b].y, -c.y);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k < D) {
          uint32_t p = p0 + g[k];
          if (p >= (uint32_t)L) p -= L;
          c = c_mulc(a, tw[p]);
          atomicAdd(&S[(k + 1) * L + b].x, -c.x);
          atomicAdd(&S[(k + 1) * L + b].y, -c.y);
        }
      }
    }
    lds_barrier();

    // Test, decode and append, bins in ascending order.
    bool nonzero = false;
    bool full = false;
    for (int m0 = 0; m0 < L; m0 += B) {
      const int m = m0 + tid;
      bool cand = false;
      int f[4] = {0, 0, 0, 0};
      float2 amp = make_float2(0.f, 0.f);
      if (m < L) {
        const float2 r0 = S[m];
        const float mag0 = sqrtf(r0.x * r0.x + r0.y * r0.y);
        nonzero |= mag0 > th0;
        cand = mag0 > th0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (k < D) {
            const float2 ri = S[(k + 1) * L + m];
            const float mi = sqrtf(ri.x * ri.x + ri.y * ri.y);
            nonzero |= mi > th0;
            cand = cand && (fabsf(mi - mag0) <= rho * mag0);
            const float2 z = c_mulc(ri, r0);
            const float phi = atan2f(z.y, z.x);
            const float u = ((float)cd.dims[k] * phi) * kInv2Pi;
            const float v = rintf(u);
            if (gtol >= 0.f) cand = cand && (fabsf(u - v) <= gtol);
            int fi = (int)v % cd.dims[k];
            if (fi < 0) fi += cd.dims[k];
            f[k] = fi;
          }
        }
        if (cand) {
          uint32_t b = 0, q = 0;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            if (k < D) {
              const uint32_t g = (uint32_t)cd.c[k] * (uint32_t)f[k];
              b = umod(b + al[k] * g, L, cd.Lmask);
              q = umod(q + ta[k] * g, L, cd.Lmask);
            }
          }
          cand = (b == (uint32_t)m);
          amp = c_mul(r0, tw[q]);  // r0 exp(-j 2 pi q / L)
        }
      }
      int tot;
      const int pos = block_prefix(cand, s.wsum, &tot);
      if (cand) {
        const int idx = kc + pos;
        if (idx < cd.max_k) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            if (k < D) {
              rf[idx * D + k] = f[k];
              if (cd.rec_lds) out.freqs[idx * D + k] = f[k];
            }
          }
          ra[idx] = amp;
          if (cd.rec_lds) oamps[idx] = amp;
          out.rec_iter[idx] = t;
          out.rec_bin[idx] = m;
        }
      }
      if (kc + tot > cd.max_k) {
        full = true;
        kc = cd.max_k;
        break;
      }
      kc += tot;
    }
    const bool nz = block_any(nonzero, s.wsum);
    // Records kept in global memory are read by other threads next
    // iteration: make the stores visible across the work-group.
    if (!cd.rec_lds) __syncthreads();
    if (full) {
      status = kStatusCapacity;
      iters = t + 1;
      break;
    }
    if (!nz) {
      status = kStatusOk;
      iters = t + 1;
      break;
    }
  }
  if (tid == 0) {
    out.info[0] = kc;
    out.info[1] = iters;
    out.info[2] = status;
    out.info[3] = 0;
  }
  __syncthreads();
}

__global__ void k_solve_plain(const CubeDesc* __restrict__ descs, int cube, const float2* __restrict__ x,
                              OutPtrs out, const int32_t* __restrict__ sched,
                              const float2* __restrict__ tw, const float2* __restrict__ pre,
                              int pre_count) {
  extern __shared__ char lds_solve[];
  solve_cube(descs[cube], x, out, sched, tw, pre, pre_count, lds_solve);
}

// Persistent: every work-group loops taking the next cube of `order` from
// the queue counter; it leaves when the counter passes the cube count, so
// every wave reaches the exit.
__global__ void k_solve_batched(const CubeDesc* __restrict__ descs, const float2* const* __restrict__ xs,
                                const OutPtrs* __restrict__ outs, const int32_t* __restrict__ sched,
                                const float2* __restrict__ tw, const int32_t* __restrict__ order,
                                int ncubes, int* __restrict__ queue) {
  extern __shared__ char lds_solve[];
  __shared__ int s_idx;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(queue, 1);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= ncubes) break;
    const int c = order[idx];
    solve_cube(descs[c], xs[c], outs[c], sched, tw, nullptr, 0, lds_solve);
  }
}

__global__ void k_reset(int* __restrict__ p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Zero fill of one buffer per blockIdx.y (float2 elements).
__global__ void k_zero(float2* const* __restrict__ bufs, const int64_t* __restrict__ lens,
                       float2* single, int64_t single_len) {
  float2* p = single ? single : bufs[blockIdx.y];
  const int64_t n = single ? single_len : lens[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    p[i] = make_float2(0.f, 0.f);
}

// ---------------------------------------------------------------------------
// Adjoint of the amplitudes (decisions fixed). Forward, per record i found
// at iteration t in bin m:  a_i = W^{p_i} (s_hat^{(t,0)}(m) - sum_j a_j
// W^{-p_j^{(t)}}) over records j of earlier iterations in bin m, with
// W = exp(-j 2 pi / L), p = [sum_k tau_k^{(t)} c_k m_k]_L. Reverse order:
// r_bar = W^{-p_i} a_bar_i flows to bin m of line 0 of iteration t and,
// negated and rotated by W^{p_j^{(t)}}, to the earlier records j in that bin.
// The line cotangent goes back through the 1/L DFT (an inverse DFT with 1/L)
// and is added at the line-0 sample positions.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void backward_cube(const CubeDesc& cd, const OutPtrs fwd, const float2* __restrict__ ga,
                              float2* __restrict__ gx, const int32_t* __restrict__ sched,
                              const float2* __restrict__ twall, char* smem) {
  const int D = cd.D;
  const int L = cd.L;
  const int tid = threadIdx.x;
  const int B = blockDim.x;
  const float2* __restrict__ tw = twall + cd.tw_off;
  float2* rbar = (float2*)smem;     // [L] line-0 spectrum cotangent
  float2* scratch = rbar + L;       // [L] FFT ping-pong
  float2* abar = scratch + L;       // [max_k]
  __shared__ int sh_s, sh_t;

  const int k = min(fwd.info[0], cd.max_k);
  for (int i = tid; i < k; i += B) abar[i] = ga[i];
  __syncthreads();
  int e = k;
  while (e > 0) {
    if (tid == 0) {
      const int tt = fwd.rec_iter[e - 1];
      int s0 = e - 1;
      while (s0 > 0 && fwd.rec_iter[s0 - 1] == tt) --s0;
      sh_s = s0;
      sh_t = tt;
    }
    for (int m = tid; m < L; m += B) rbar[m] = make_float2(0.f, 0.f);
    __syncthreads();
    const int s0 = sh_s;
    const int t = sh_t;
    const int32_t* at = sched + cd.sched_off + ((t >= 0 && t < cd.T) ? t : 0) * 2 * D;
    uint32_t al[4], ta[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      al[q] = q < D ? (uint32_t)at[q] : 0u;
      ta[q] = q < D ? (uint32_t)at[D + q] : 0u;
    }
    // Records of iteration t: distinct bins, so plain stores. Entries that
    // no forward run can have written (bin or iteration out of range) are
    // skipped rather than trusted as LDS or schedule indices.
    const bool t_ok = t >= 0 && t < cd.T;
    for (int i = s0 + tid; i < e; i += B) {
      const int m = fwd.rec_bin[i];
      if (!t_ok || m < 0 || m >= L) continue;
      uint32_t p = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < D) p = umod(p + ta[q] * ((uint32_t)cd.c[q] * (uint32_t)fwd.freqs[i * D + q]), L, cd.Lmask);
      rbar[m] = c_mulc(abar[i], tw[p]);
    }
    __syncthreads();
    // Earlier records that iteration t's peel subtracted.
    for (int j = tid; j < s0; j += B) {
      uint32_t b = 0, p = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < D) {
          const uint32_t g = (uint32_t)cd.c[q] * (uint32_t)fwd.freqs[j * D + q];
          b = umod(b + al[q] * g, L, cd.Lmask);
          p = umod(p + ta[q] * g, L, cd.Lmask);
        }
      }
      const float2 v = rbar[b];
      abar[j] = c_sub(abar[j], c_mul(tw[p], v));
    }
    __syncthreads();
    // s_bar(l) = (1/L) sum_m r_bar(m) e^{+j 2 pi l m / L}
    //          = (1/L) conj(FFT(conj(r_bar)))(l).
    for (int m = tid; m < L; m += B) rbar[m] = c_scale(c_conj(rbar[m]), cd.inv_L);
    __syncthreads();
    const float2* S = block_fft(rbar, scratch, 1, cd, tw);
    for (int l = tid; l < L; l += B) {
      int64_t flat = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < D) {
          const uint32_t v = al[q] * (uint32_t)l + ta[q];
          flat += (int64_t)umod(v, (uint32_t)cd.dims[q], cd.dmask[q]) * cd.stride[q];
        }
      }
      const float2 g = c_conj(S[l]);
      unsafeAtomicAdd(&gx[flat].x, g.x);
      unsafeAtomicAdd(&gx[flat].y, g.y);
    }
    __syncthreads();
    e = s0;
  }
}

__global__ void k_backward(const CubeDesc* __restrict__ descs, int cube, OutPtrs fwd_single,
                           const float2* __restrict__ ga_single, float2* __restrict__ gx_single,
                           const OutPtrs* __restrict__ fwds, const float2* const* __restrict__ gas,
                           float2* const* __restrict__ gxs, const int32_t* __restrict__ sched,
                           const float2* __restrict__ tw) {
  extern __shared__ char lds_bwd[];
  if (cube >= 0) {
    backward_cube(descs[cube], fwd_single, ga_single, gx_single, sched, tw, lds_bwd);
  } else {
    const int c = blockIdx.x;
    backward_cube(descs[c], fwds[c], gas[c], gxs[c], sched, tw, lds_bwd);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
hipError_t launch_lines_single(const LaunchCtx& ctx, int cube, const float2* x, int t0, int count,
                               int G, float2* out, size_t lds, int threads, hipStream_t st) {
  const int grid = (count + G - 1) / G;
  hipLaunchKernelGGL(k_lines, dim3(grid), dim3(threads), lds, st, ctx.descs, (const LineItem*)nullptr, 0,
                     0, cube, t0, count, G, x, (const float2* const*)nullptr, ctx.sched, ctx.tw, out);
  return hipGetLastError();
}

hipError_t launch_lines_items(const LaunchCtx& ctx, const LineItem* items, int nitems,
                              const float2* const* xs, float2* out, size_t lds, int threads,
                              hipStream_t st) {
  const int per_xcd = (nitems + 7) / 8;
  hipLaunchKernelGGL(k_lines, dim3(per_xcd * 8), dim3(threads), lds, st, ctx.descs, items, nitems,
                     per_xcd, 0, 0, 0, 0, (const float2*)nullptr, xs, ctx.sched, ctx.tw, out);
  return hipGetLastError();
}

hipError_t launch_solve_plain(const LaunchCtx& ctx, int cube, const float2* x, const OutPtrs& out,
                              const float2* pre, int pre_count, size_t lds, int threads, hipStream_t st) {
  hipLaunchKernelGGL(k_solve_plain, dim3(1), dim3(threads), lds, st, ctx.descs, cube, x, out, ctx.sched,
                     ctx.tw, pre, pre_count);
  return hipGetLastError();
}

hipError_t launch_solve_batched(const LaunchCtx& ctx, const float2* const* xs, const OutPtrs* outs,
                                const int32_t* order, int ncubes, int* queue, int grid, size_t lds,
                                int threads, hipStream_t st) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, queue, 1);
  hipLaunchKernelGGL(k_solve_batched, dim3(grid), dim3(threads), lds, st, ctx.descs, xs, outs, ctx.sched,
                     ctx.tw, order, ncubes, queue);
  return hipGetLastError();
}

hipError_t launch_zero_single(float2* p, int64_t n, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, (float2* const*)nullptr,
                     (const int64_t*)nullptr, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_multi(float2* const* bufs, const int64_t* lens, int nbufs, int64_t maxlen,
                             hipStream_t st) {
  int64_t blocks = (maxlen + 255) / 256;
  if (blocks > 512) blocks = 512;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks, nbufs), dim3(256), 0, st, bufs, lens,
                     (float2*)nullptr, (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_backward_single(const LaunchCtx& ctx, int cube, const OutPtrs& fwd, const float2* ga,
                                  float2* gx, size_t lds, int threads, hipStream_t st) {
  hipLaunchKernelGGL(k_backward, dim3(1), dim3(threads), lds, st, ctx.descs, cube, fwd, ga, gx,
                     (const OutPtrs*)nullptr, (const float2* const*)nullptr, (float2* const*)nullptr,
                     ctx.sched, ctx.tw);
  return hipGetLastError();
}

hipError_t launch_backward_batched(const LaunchCtx& ctx, int ncubes, const OutPtrs* fwds,
                                   const float2* const* gas, float2* const* gxs, size_t lds, int threads,
                                   hipStream_t st) {
  OutPtrs none{};
  hipLaunchKernelGGL(k_backward, dim3(ncubes), dim3(threads), lds, st, ctx.descs, -1, none,
                     (const float2*)nullptr, (float2*)nullptr, fwds, gas, gxs, ctx.sched, ctx.tw);
  return hipGetLastError();
}

const void* kernel_solve_batched() { return (const void*)k_solve_batched; }
const void* kernel_solve_plain() { return (const void*)k_solve_plain; }
const void* kernel_lines() { return (const void*)k_lines; }
const void* kernel_backward() { return (const void*)k_backward; }

}  // namespace fpssft
