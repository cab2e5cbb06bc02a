// gfx950 kernels of the FPS-SFT hot path.
//
//  k_lines          line gather + L-point FFT of whole iterations (D+1 lines
//                   each) into a spectra buffer (Eq. sample_slice, Eq. hs);
//                   many work-groups, HBM-bound.
//  k_solve_plain    one cube in one work-group: for every iteration, the
//                   spectra (precomputed by k_lines for the first chunk,
//                   gathered and transformed after it: one wave per line in
//                   registers, a block FFT in LDS, or line by line for long
//                   lines, in LDS or in a device workspace), the subtraction
//                   of the recovered set (construction-subtraction, Sec. 2.2:
//                   on the spectra as exact per-bin sums, or in time on
//                   request), the 1-sparsity test, the phase decode and the
//                   amplitude (Eq. decoding), the merge of a frequency
//                   detected again (found through a hash of the set's
//                   frequencies), the ordered record, and the stopping rule.
//  k_solve_batched  the same per cube, persistent: each work-group solves
//                   the cube of its index, then takes cube indices from a
//                   device queue until it is empty.
//  k_backward       adjoint of the set amplitudes with the decisions fixed.
//  k_reset, k_zero  counter reset and zero fill (kernels, so that they can
//                   sit inside a captured graph).
//
// Kernels are instantiated per (D, power-of-two L, records in LDS, path:
// block FFT, wave per line, or lines in a device workspace); the host groups
// cubes by instantiation.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device.h"
#include "launch.h"

namespace fpssft {

static constexpr float kInv2Pi = (float)(1.0 / (2.0 * 3.14159265358979323846));

// Samples (or precomputed spectra) of one iteration held in registers: the
// D+1 values at l = tid + u * blockDim.x, u < kPfU. Loaded one iteration
// ahead so that their latency overlaps the current iteration's work.
constexpr int kPfU = 4;

template <int D>
struct Prefetch {
  float2 v[kPfU][D + 1];
};

template <int D, bool kPow2>
__device__ __forceinline__ void prefetch_issue(Prefetch<D>& pf, const Geo<D>& g, const float2* __restrict__ x,
                                               const int32_t* __restrict__ row, const float2* __restrict__ pre,
                                               bool precomputed) {
  const uint32_t L = g.L;
#pragma unroll
  for (int u = 0; u < kPfU; ++u) {
    const uint32_t l = threadIdx.x + u * blockDim.x;
    if (l < L) {
      if (precomputed) {
#pragma unroll
        for (int i = 0; i <= D; ++i) pf.v[u][i] = ld_g(pre, i * L + l);
      } else {
        int64_t step[D];
        const int64_t flat = line_sample<D, kPow2>(g, row, l, step);
        load_line_samples<D>(x, flat, step, pf.v[u]);
      }
    }
  }
}

template <int D>
__device__ __forceinline__ void prefetch_store(const Prefetch<D>& pf, uint32_t L, float2* __restrict__ dst,
                                               float scale) {
#pragma unroll
  for (int u = 0; u < kPfU; ++u) {
    const uint32_t l = threadIdx.x + u * blockDim.x;
    if (l < L) {
#pragma unroll
      for (int i = 0; i <= D; ++i) dst[i * L + l] = c_scale(pf.v[u][i], scale);
    }
  }
}

// ---------------------------------------------------------------------------
// Line gather + FFT. Work items are runs of consecutive iterations of one
// cube. Work-groups are persistent: each takes items from the queue of its
// XCD (work-groups are dispatched round-robin over the 8 XCDs, and each XCD
// owns a contiguous, cube-ordered slice of the items, so a cube's lines are
// gathered through one L2). Within an item the next iteration's samples are
// loaded into registers while the current one is transformed and written.
// Single-cube calls (`items` == null) run one iteration per work-group.
// ---------------------------------------------------------------------------
template <int D, bool kPow2>
__device__ __forceinline__ void lines_item(const CubeDesc& cd, const float2* __restrict__ x,
                                           const int32_t* __restrict__ sched, const float2* __restrict__ twall,
                                           int tb, int tc, float2* __restrict__ out, float2* bufA, float2* bufB,
                                           float2* tw, int* tw_cached) {
  const Geo<D> g = load_geo<D>(cd);
  const uint32_t L = g.L;
  const int B = blockDim.x;
  if (cd.serial) {
    // Long lines: one line at a time through two line buffers at the start
    // of LDS (which may cover the cached twiddles: the cache is dropped),
    // twiddles from global memory.
    float2* X = bufA;
    float2* Y = X + L;
    const float2* twg = twall + cd.tw_off;
    const int32_t* sch = sched + cd.sched_off + tb * 2 * D;
    for (int i = 0; i < tc; ++i) {
      for (int line = 0; line <= D; ++line) {
        gather_one_line<D, kPow2>(X, x, g, sch + i * 2 * D, line, cd.inv_L);
        lds_barrier();
        const float2* S = block_fft<kPow2>(X, Y, 1, (int)L, cd.nstages, cd.radix, twg);
        float2* o = out + ((int64_t)i * (D + 1) + line) * L;
        for (uint32_t e = threadIdx.x; e < L; e += B) st_g(o, e, S[e]);
        lds_barrier();
      }
    }
    *tw_cached = -1;
    return;
  }
  if (*tw_cached != cd.tw_off) {  // uniform
    lds_barrier();
    for (uint32_t e = threadIdx.x; e < L; e += B) tw[e] = ld_g(twall, cd.tw_off + e);
    *tw_cached = cd.tw_off;
  }
  const int32_t* sch = sched + cd.sched_off + tb * 2 * D;
  const bool use_pf = L <= (uint32_t)(kPfU * B);
  Prefetch<D> pf;
  if (use_pf) prefetch_issue<D, kPow2>(pf, g, x, sch, nullptr, false);
  for (int i = 0; i < tc; ++i) {
    if (use_pf) {
      prefetch_store<D>(pf, L, bufA, cd.inv_L);
    } else {
      gather_lines<D, kPow2>(bufA, x, g, sch + i * 2 * D, 1, cd.inv_L);
    }
    lds_barrier();
    const float2* S = block_fft<kPow2>(bufA, bufB, D + 1, (int)L, cd.nstages, cd.radix, tw);
    // Next iteration's gathers go out after the transform (scattered loads in
    // flight slow the LDS traffic of the butterflies).
    if (use_pf && i + 1 < tc) prefetch_issue<D, kPow2>(pf, g, x, sch + (i + 1) * 2 * D, nullptr, false);
    // Two elements per lane and store: half the store instructions.
    float2* o = out + (int64_t)i * (D + 1) * L;
    const uint32_t n = (D + 1) * L;
    for (uint32_t e = 2 * threadIdx.x; e + 1 < n; e += 2 * B) st_g_pair(o, e, S[e], S[e + 1]);
    if ((n & 1u) && threadIdx.x == 0) st_g(o, n - 1, S[n - 1]);
    lds_barrier();
  }
}

template <int D, bool kPow2>
__global__ void k_lines(const CubeDesc* __restrict__ descs, const LineItem* __restrict__ items,
                        const int32_t* __restrict__ ranges, int* __restrict__ queues, int single_cube, int t0,
                        int count, const float2* __restrict__ x_single, const float2* const* __restrict__ xs,
                        const int32_t* __restrict__ sched, const float2* __restrict__ tw,
                        float2* __restrict__ out, int maxL) {
  extern __shared__ float2 lds_lines[];
  __shared__ int s_item;
  __shared__ int s_tw;
  float2* bufA = lds_lines;
  float2* bufB = bufA + (D + 1) * maxL;
  float2* twl = bufB + (D + 1) * maxL;
  if (threadIdx.x == 0) s_tw = -1;
  __syncthreads();
  if (!items) {
    const int t = t0 + blockIdx.x;
    if (t >= t0 + count) return;
    const CubeDesc& cd = descs[single_cube];
    lines_item<D, kPow2>(cd, x_single, sched, tw, t, 1, out + (int64_t)(t - t0) * (D + 1) * cd.L, bufA, bufB, twl,
                         &s_tw);
    return;
  }
  const int xcd = blockIdx.x & 7;
  const int lo = ranges[2 * xcd];
  const int hi = ranges[2 * xcd + 1];
  for (;;) {
    if (threadIdx.x == 0) s_item = lo + atomicAdd(&queues[xcd], 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= hi) break;
    const LineItem li = items[it];
    const int c = __builtin_amdgcn_readfirstlane(li.cube);
    lines_item<D, kPow2>(descs[c], xs[c], sched, tw, li.t0, li.count, out + li.out_off, bufA, bufB, twl, &s_tw);
  }
}

// ---------------------------------------------------------------------------
// One cube, one work-group.
// ---------------------------------------------------------------------------

// Record store of one cube: the recovered set, one slot per distinct
// frequency, in the order the work-group's waves appended them. It lives in
// LDS (kRecLds) or in the plan's device workspace, `cap` entries per array.
// The detection trace goes to the outputs as it is found.
struct RecStore {
  float2* sa;   // [cap] amplitude of a set entry: the sum of its detections
  int32_t* sf;  // [cap][D] its frequency indices
  int32_t* sp;  // [cap] its canonical set index; the sign bit marks a
                // frequency detected more than once
  int32_t* nx;  // [cap] long lines: next entry projecting onto the same
                // bin in this iteration (-1 ends a list); at the end of the
                // cube, the slot, then the output position, of each
                // canonical index
  int32_t* ht;  // [hash slots] slot of each set frequency, -1: empty
  uint32_t hmask;  // hash slots - 1
  int hshift;      // 32 - log2(hash slots)
};

template <int D>
__device__ __forceinline__ RecStore carve_records(char* base, int cap) {
  RecStore r;
  r.sa = (float2*)base;
  r.sf = (int32_t*)(r.sa + cap);
  r.sp = r.sf + cap * D;
  r.nx = r.sp + cap;
  r.ht = r.nx + cap;
  const int hs = fps_rec_hash_slots(cap);
  r.hmask = (uint32_t)hs - 1u;
  r.hshift = __clz(hs) + 1;
  return r;
}

// Record-store accessors: LDS, or device memory through address-space-1
// instructions.
template <bool kLds>
__device__ __forceinline__ int32_t rs_ld(const int32_t* p, int i) {
  if constexpr (kLds) return p[i];
  else return ld_gi(p, i);
}
template <bool kLds>
__device__ __forceinline__ void rs_st(int32_t* p, int i, int32_t v) {
  if constexpr (kLds) p[i] = v;
  else st_gi(p, i, v);
}
template <bool kLds>
__device__ __forceinline__ float2 rs_ld(const float2* p, int i) {
  if constexpr (kLds) return p[i];
  else return ld_g(p, i);
}
template <bool kLds>
__device__ __forceinline__ void rs_st(float2* p, int i, float2 v) {
  if constexpr (kLds) p[i] = v;
  else st_g(p, i, v);
}

// Barrier after record-store writes that other threads read next: LDS only,
// or every memory access when the store is in device memory.
template <bool kLds>
__device__ __forceinline__ void rec_barrier() {
  if constexpr (kLds) lds_barrier();
  else __syncthreads();
}

// Solve-kernel paths: the block FFT in LDS, one wave per line (registers),
// and long lines whose spectra and scratch line are in a device workspace.
constexpr int kPathBlock = 0;
constexpr int kPathWave = 1;
constexpr int kPathLinesWs = 2;

struct SolveLds {
  float2* bufA;  // [(D+1) L] the line spectra, row i = line i
  float2* bufB;  // block path: the FFT's second buffer [(D+1) L]; long
                 // lines: one line of scratch [L]
  float2* P;     // [(D+1) L] constructed spectra (time-domain
                 // construction-subtraction only)
  float2* tw;    // [L] twiddles W_L^k (long lines: none, read from memory)
  int* head;     // long lines: [L] first set entry of each bin's list, in
                 // the scratch line once the transforms are done
  uint32_t* bmax;  // [L] largest amplitude component of the set entries
                   // projecting onto each bin (float bits)
  int* bcnt;     // [L] number of those entries (not with long lines)
  int2* Q;       // [(D+1) L] each bin's projection sums per line, fixed point
                 // (not with long lines)
  RecStore rec;  // the record store when it is in LDS
  int* wsum;     // [2][16] per-wave exchange words (two per wave),
                 // double-buffered
  int* cnt;      // [4]: slots appended; unused; set size after a pass that
                 // filled the store
};

// Layout (the host's solve_lds_bytes mirrors it): the wave path keeps the
// D+1 spectra (each wave's transform writes its row), the block path two
// line buffers; then the twiddles, the constructed spectra of the
// time-domain construction-subtraction, the per-bin words (largest
// amplitudes, entry counts) and fixed-point projection sums, the records
// with their frequency hash and the exchange words.
template <int D, int kPath>
__device__ __forceinline__ SolveLds carve_solve_lds(char* smem, int L, int rec_cap, bool serial, bool literal,
                                                    char* lines_ws) {
  constexpr bool kWave = kPath == kPathWave;
  SolveLds s;
  s.bufA = (float2*)smem;
  s.P = nullptr;
  float2* end;
  if constexpr (kPath == kPathLinesWs) {
    // lines longer still: the same buffers in device memory, LDS keeps the
    // records only
    s.bufA = (float2*)lines_ws;
    s.bufB = s.bufA + (D + 1) * L;
    s.tw = nullptr;
    s.head = (int*)s.bufB;
    s.bmax = (uint32_t*)(s.head + L);
    s.bcnt = nullptr;
    s.Q = nullptr;
    end = (float2*)smem;
  } else if (!kWave && serial) {
    s.bufB = s.bufA + (D + 1) * L;
    s.tw = nullptr;
    s.head = (int*)s.bufB;
    s.bmax = (uint32_t*)(s.head + L);
    s.bcnt = nullptr;
    s.Q = nullptr;
    end = s.bufB + L;
  } else {
    if constexpr (kWave) {
      s.bufB = nullptr;
      s.tw = s.bufA + (D + 1) * L;
    } else {
      s.bufB = s.bufA + (D + 1) * L;
      s.tw = s.bufB + (D + 1) * L;
    }
    end = s.tw + L;
    if (!kWave && literal) {
      s.P = end;
      end += (D + 1) * L;
    }
    const int Lr = (L + 1) & ~1;
    s.head = nullptr;
    s.bmax = (uint32_t*)end;
    s.bcnt = (int*)(s.bmax + Lr);
    // the time-domain construction-subtraction converts the sums into its
    // constructed spectra in place
    s.Q = s.P ? (int2*)s.P : (int2*)(s.bcnt + Lr);
    end = s.P ? (float2*)(s.bcnt + Lr) : (float2*)(s.Q + (D + 1) * L);
  }
  s.rec = carve_records<D>((char*)end, rec_cap);
  s.wsum = (int*)((char*)end + fps_rec_bytes(D, rec_cap));
  s.cnt = s.wsum + 32;
  return s;
}

// Exact, order-independent sums of the records' projections on one bin
// (long lines, where a bin's owner sums its list): each term is truncated to
// an integer multiple of 2^-e in 32 bits, the integers are added in 64 bits,
// and the sum is converted back once, so the result does not depend on the
// order of the list. The scale comes from the largest amplitude component
// in the bin's list (amax < 2^ea): a term is
// below sqrt(2) amax < 2^(ea + 1), so e = 29 - ea keeps it below 2^30, and
// the truncation error of a term is below 2^(ea - 29), about 4e-9 of amax.
__device__ __forceinline__ int bin_exponent(uint32_t amax_bits) {
  return 29 - ((int)((amax_bits >> 23) & 0xffu) - 126);
}
__device__ __forceinline__ long long fixed_term(float v, int e) { return (long long)(int)__builtin_ldexpf(v, e); }
__device__ __forceinline__ float fixed_value(long long v, int e) { return (float)__builtin_ldexp((double)v, -e); }

// The same with 32-bit sums, when the bin's entry count n is known: e =
// 29 - ea - en with n < 2^en keeps every term below 2^(30 - en) and the sum
// below 2^30. Integer addition is exact and commutative, so the sums can be
// accumulated with LDS atomics in any order (wrapping partial sums included).
__device__ __forceinline__ int bin_exponent32(uint32_t amax_bits, int n) {
  return bin_exponent(amax_bits) - (32 - __clz(n > 1 ? n : 1));
}
__device__ __forceinline__ int fixed_term32(float v, int e) { return (int)__builtin_ldexpf(v, e); }
__device__ __forceinline__ float fixed_value32(int v, int e) { return __builtin_ldexpf((float)v, -e); }

// Wave path of the solve loop (L = 64 E, 64 <= L <= 512, one wave per
// line): wave w holds line w's values at l = lane + 64 e in registers.
constexpr int kEMax = 8;
// Bins per thread in one decode pass (one exchange barrier per pass).
constexpr int kDecodeBins = 2;

template <int D, bool kPow2>
__device__ __forceinline__ void wave_prefetch(float2 (&pf)[kEMax], int E, const Geo<D>& g,
                                              const float2* __restrict__ x, const int32_t* __restrict__ row,
                                              const float2* __restrict__ pre, bool precomputed, int w) {
  const int lane = threadIdx.x & 63;
  const uint32_t L = g.L;
  if (precomputed) {
#pragma unroll
    for (int e = 0; e < kEMax; ++e)
      if (e < E) pf[e] = ld_g(pre, w * L + lane + 64 * e);
    return;
  }
  // Line w has offsets tau + e_{w-1} (line 0: tau); slope and offsets are
  // read once, uniform across the wave. alpha_k l + tau_k + 1 < N_k L + N_k
  // stays below 2^32 (the plan checks N_k L < 2^31).
  const int ws = __builtin_amdgcn_readfirstlane(w);
  uint32_t al[D], ta[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    al[k] = (uint32_t)__builtin_amdgcn_readfirstlane(row[k]);
    ta[k] = (uint32_t)__builtin_amdgcn_readfirstlane(row[D + k]) + (k + 1 == ws ? 1u : 0u);
  }
#pragma unroll
  for (int e = 0; e < kEMax; ++e) {
    if (e < E) {
      // the wave transform takes sample e + E q in register e of lane q
      const uint32_t l = (uint32_t)E * lane + e;
      int64_t flat = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) flat += (int64_t)umod<kPow2>(al[k] * l + ta[k], g.dims[k]) * g.stride[k];
      pf[e] = ld_g(x, flat);
    }
  }
}

template <int E>
__device__ __forceinline__ void wave_fft_to_lds(const float2 (&in)[kEMax], const float2* tw, float2* dst) {
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = in[e];
  wave_fft_lanes<E>(v, tw, [&](int k, float2 val) { dst[k] = val; });
}

// The set's frequency hash: key = the frequency's flat index, slot = its
// record slot. The entries an iteration opens enter it while the next
// iteration links the set, before the barrier that precedes that
// iteration's lookups; an iteration never looks up a frequency it opened
// itself (a frequency projects onto one bin, the one that found it). Slots
// are never emptied during a cube, so a lookup that meets an empty slot has
// seen every entry of its probe sequence.
template <int D>
__device__ __forceinline__ uint32_t freq_key(const Geo<D>& g, const int (&f)[D]) {
  uint32_t key = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) key += (uint32_t)f[k] * (uint32_t)g.stride[k];
  return key;
}
__device__ __forceinline__ uint32_t hash_home(const RecStore& rs, uint32_t key) {
  return (key * 0x9E3779B1u) >> rs.hshift;
}
template <int D, bool kRecLds>
__device__ __forceinline__ int hash_find(const RecStore& rs, uint32_t key, const int (&f)[D]) {
  uint32_t h = hash_home(rs, key);
  for (uint32_t steps = 0; steps <= rs.hmask; ++steps) {
    const int j = rs_ld<kRecLds>(rs.ht, (int)h);
    if (j < 0) return -1;
    bool eq = true;
#pragma unroll
    for (int k = 0; k < D; ++k) eq = eq && rs_ld<kRecLds>(rs.sf, j * D + k) == f[k];
    if (eq) return j;
    h = (h + 1u) & rs.hmask;
  }
  return -1;
}
// Entries j = j0, j0 + js, ... of [from, n) enter the hash.
template <int D, bool kRecLds>
__device__ __forceinline__ void hash_insert(const Geo<D>& g, const RecStore& rs, int from, int j0, int js, int n) {
  for (int j = from + j0; j < n; j += js) {
    int f[D];
#pragma unroll
    for (int k = 0; k < D; ++k) f[k] = rs_ld<kRecLds>(rs.sf, j * D + k);
    uint32_t h = hash_home(rs, freq_key<D>(g, f));
    for (uint32_t steps = 0; steps <= rs.hmask; ++steps) {
      if (atomicCAS(&rs.ht[h], -1, j) == -1) break;
      h = (h + 1u) & rs.hmask;
    }
  }
}

// Construction-subtraction (Sec. 2.2): the recovered sinusoid (m_j, a_j)
// contributes a_j e^{+j 2 pi p_j^{(i)} / L} to bin b_j = [sum_k alpha_k c_k
// m_jk]_L of line i, p_j^{(i)} = [sum_k tau_k^{(i)} c_k m_jk]_L (Eq.
// freqSum, Eq. orthogonality). First, for each set entry j = j0, j0 + js,
// ... < n, its bin's largest amplitude component is raised to the entry's
// and the bin's entry count incremented; with long lines (no counts) the
// entry is linked into its bin's list instead. The same threads enter the
// entries of slots hfrom .. n-1 into the frequency hash.
template <int D, bool kPow2, bool kRecLds>
__device__ __forceinline__ uint32_t entry_bin(const Geo<D>& g, const uint32_t (&al)[D], const RecStore& rs, int j) {
  uint32_t b = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) b = umod<kPow2>(b + al[k] * (g.c[k] * (uint32_t)rs_ld<kRecLds>(rs.sf, j * D + k)), g.L);
  return b;
}
__device__ __forceinline__ uint32_t amp_bits(float2 a) { return __float_as_uint(fmaxf(fabsf(a.x), fabsf(a.y))); }

template <int D, bool kPow2, bool kRecLds>
__device__ __forceinline__ void link_bins(const Geo<D>& g, const uint32_t (&al)[D], const RecStore& rs, int* head,
                                          uint32_t* bmax, int* bcnt, int j0, int js, int n, int hfrom) {
  // the entries the last iteration opened (slots hfrom .. n-1)
  hash_insert<D, kRecLds>(g, rs, hfrom, j0, js, n);
  if (bcnt) {
    // two entries per step, so that their loads overlap
    int j = j0;
    for (; j + js < n; j += 2 * js) {
      const uint32_t b0 = entry_bin<D, kPow2, kRecLds>(g, al, rs, j);
      const uint32_t b1 = entry_bin<D, kPow2, kRecLds>(g, al, rs, j + js);
      const float2 a0 = rs_ld<kRecLds>(rs.sa, j);
      const float2 a1 = rs_ld<kRecLds>(rs.sa, j + js);
      atomicMax(&bmax[b0], amp_bits(a0));
      atomicAdd(&bcnt[b0], 1);
      atomicMax(&bmax[b1], amp_bits(a1));
      atomicAdd(&bcnt[b1], 1);
    }
    if (j < n) {
      const uint32_t b = entry_bin<D, kPow2, kRecLds>(g, al, rs, j);
      atomicMax(&bmax[b], amp_bits(rs_ld<kRecLds>(rs.sa, j)));
      atomicAdd(&bcnt[b], 1);
    }
    return;
  }
  for (int j = j0; j < n; j += js) {
    const uint32_t b = entry_bin<D, kPow2, kRecLds>(g, al, rs, j);
    rs_st<kRecLds>(rs.nx, j, atomicExch(&head[b], j));
    atomicMax(&bmax[b], amp_bits(rs_ld<kRecLds>(rs.sa, j)));
  }
}

// One entry's contribution: the bin, the fixed-point scale and the terms on
// the D+1 lines. Every read comes before the first atomic (the compiler does
// not move reads across them), so that they go out in one round.
template <int D, bool kPow2, bool kRecLds>
__device__ __forceinline__ uint32_t entry_reads(const Geo<D>& g, const uint32_t (&al)[D], const uint32_t (&ta)[D],
                                                const RecStore& rs, const float2* tw, const uint32_t* bmax,
                                                const int* bcnt, int j, float2& a, uint32_t& bm, int& bc,
                                                float2 (&w)[D + 1]) {
  const uint32_t L = g.L;
  uint32_t gk[D];
  uint32_t b = 0, p0 = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    gk[k] = g.c[k] * (uint32_t)rs_ld<kRecLds>(rs.sf, j * D + k);
    b = umod<kPow2>(b + al[k] * gk[k], L);
    p0 = umod<kPow2>(p0 + ta[k] * gk[k], L);
  }
  a = rs_ld<kRecLds>(rs.sa, j);
  bm = bmax[b];
  bc = bcnt[b];
  w[0] = tw[p0];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    uint32_t p = p0 + gk[k];
    if (p >= L) p -= L;
    w[k + 1] = tw[p];
  }
  return b;
}
template <int D>
__device__ __forceinline__ void entry_add(int2* Q, uint32_t L, uint32_t b, float2 a, uint32_t bm, int bc,
                                          const float2 (&w)[D + 1]) {
  const int e = bin_exponent32(bm, bc);
#pragma unroll
  for (int i = 0; i <= D; ++i) {
    const float2 c = c_mulc(a, w[i]);
    atomicAdd(&Q[i * L + b].x, fixed_term32(c.x, e));
    atomicAdd(&Q[i * L + b].y, fixed_term32(c.y, e));
  }
}

// Then every thread takes set entries j = j0, j0 + js, ... < n and adds
// their projections on the D+1 lines to their bin's fixed-point sums in Q
// (scale from the bin's largest amplitude and entry count; LDS integer
// atomics, exact in any order).
template <int D, bool kPow2, bool kRecLds>
__device__ __forceinline__ void accumulate_bins(const Geo<D>& g, const uint32_t (&al)[D], const uint32_t (&ta)[D],
                                                const RecStore& rs, const float2* tw, const uint32_t* bmax,
                                                const int* bcnt, int2* Q, int j0, int js, int n) {
  const uint32_t L = g.L;
  for (int j = j0; j < n; j += js) {
    float2 a, w[D + 1];
    uint32_t bm;
    int bc;
    const uint32_t b = entry_reads<D, kPow2, kRecLds>(g, al, ta, rs, tw, bmax, bcnt, j, a, bm, bc, w);
    entry_add<D>(Q, L, b, a, bm, bc, w);
  }
}

// Long lines, where LDS has no room for the per-bin sums: the thread that
// owns a bin sums its list's contributions on the D+1 lines (fixed point at
// scale 2^e from the bin's largest amplitude, so the sum is the same for any
// list order) into sum[i]. A list holds at most the n set entries, all with
// slots below n; the walk stops there whatever the links say.
template <int D, bool kPow2, bool kRecLds>
__device__ __forceinline__ void list_sum(const Geo<D>& g, const uint32_t (&ta)[D], const RecStore& rs,
                                         const float2* tw, int h, int n, int e, float2 (&sum)[D + 1]) {
  const uint32_t L = g.L;
  long long sr[D + 1], si[D + 1];
#pragma unroll
  for (int i = 0; i <= D; ++i) sr[i] = si[i] = 0;
  for (int j = h, steps = 0; (unsigned)j < (unsigned)n && steps < n; ++steps) {
    const int nxt = rs_ld<kRecLds>(rs.nx, j);
    uint32_t gk[D];
    uint32_t p0 = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      gk[k] = g.c[k] * (uint32_t)rs_ld<kRecLds>(rs.sf, j * D + k);
      p0 = umod<kPow2>(p0 + ta[k] * gk[k], L);
    }
    const float2 a = rs_ld<kRecLds>(rs.sa, j);
    float2 c = c_mulc(a, tw[p0]);
    sr[0] += fixed_term(c.x, e);
    si[0] += fixed_term(c.y, e);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      uint32_t p = p0 + gk[k];
      if (p >= L) p -= L;
      c = c_mulc(a, tw[p]);
      sr[k + 1] += fixed_term(c.x, e);
      si[k + 1] += fixed_term(c.y, e);
    }
    j = nxt;
  }
#pragma unroll
  for (int i = 0; i <= D; ++i) sum[i] = make_float2(fixed_value(sr[i], e), fixed_value(si[i], e));
}

// Bin m of one iteration (r: its value on lines 0..D after the peel): the
// nonzero and magnitude-equality tests (Sec. 2.1), the phase decode of the
// frequency (Eq. decoding) with the on-grid check, the projection-consistency
// check, and the amplitude r_0 exp(-j 2 pi q / L) (with `avg`, the mean over
// the D+1 lines of r_i exp(-j 2 pi q_i / L)). All decisions in float32; the
// magnitudes take the hardware square root (within 1 ulp), without the
// correctly rounded expansion.
template <int D, bool kPow2>
__device__ __forceinline__ bool decode_bin(const Geo<D>& g, const uint32_t (&al)[D], const uint32_t (&ta)[D],
                                           const float2 (&r)[D + 1], uint32_t m, float th0, float rho, float gtol,
                                           const float2* tw, bool avg, bool& nonzero, int (&f)[D],
                                           float2& amp) {
  const uint32_t L = g.L;
  const float2 r0 = r[0];
  const float mag0 = __builtin_amdgcn_sqrtf(r0.x * r0.x + r0.y * r0.y);
  nonzero |= mag0 > th0;
  bool cand = mag0 > th0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float2 ri = r[k + 1];
    const float mi = __builtin_amdgcn_sqrtf(ri.x * ri.x + ri.y * ri.y);
    nonzero |= mi > th0;
    cand = cand && (fabsf(mi - mag0) <= rho * mag0);
  }
  // The phase decode only for bins that pass the magnitude tests (the same
  // decisions: every test must hold); waves without such a bin skip it.
  // With D >= 3 every bin takes it, branch-free, which lets the D phase
  // decodes of a bin overlap (a 128^3 cube 2.5% faster; 2-D cubes are
  // faster skipping it).
  if (D >= 3 || cand) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const float2 z = c_mulc(r[k + 1], r0);
      const float phi = atan2f(z.y, z.x);
      const float u = ((float)g.dims[k] * phi) * kInv2Pi;
      const float v = rintf(u);
      if (gtol >= 0.f) cand = cand && (fabsf(u - v) <= gtol);
      // [v]_{N_k}: a mask for power-of-two sides (two's complement)
      int fi;
      if constexpr (kPow2) {
        fi = (int)v & ((int)g.dims[k] - 1);
      } else {
        fi = (int)v % (int)g.dims[k];
        if (fi < 0) fi += (int)g.dims[k];
      }
      f[k] = fi;
    }
  }
  if (cand) {
    uint32_t b = 0, q = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const uint32_t gk = g.c[k] * (uint32_t)f[k];
      b = umod<kPow2>(b + al[k] * gk, L);
      q = umod<kPow2>(q + ta[k] * gk, L);
    }
    cand = (b == m);
    amp = c_mul(r0, tw[q]);  // r0 exp(-j 2 pi q / L)
    if (avg) {
      // line i's offset adds c_{i-1} m_{i-1} to the phase index
#pragma unroll
      for (int k = 0; k < D; ++k) {
        uint32_t qk = q + g.c[k] * (uint32_t)f[k];
        if (qk >= L) qk -= L;
        amp = c_add(amp, c_mul(r[k + 1], tw[qk]));
      }
      amp = c_scale(amp, 1.0f / (float)(D + 1));
    }
  }
  return cand;
}

// One cube in one work-group, iteration by iteration (Sec. 2.2).
//
// One iteration (wave path, more waves than lines): waves 0..D transform
// their line into bufA while the remaining waves count the set entries per
// bin (largest amplitude component and number, which fix the bin's
// fixed-point scale); one barrier; every thread adds entries' projections
// to their bins' sums; one barrier; the owner of each bin subtracts the
// sums from the spectra (construction-subtraction) and tests and decodes
// the bin (Eq. decoding); one barrier per pass of bins exchanges the
// per-wave counts of detections and new frequencies and the nonzero flags.
// Other configurations count the entries after the transform, with a
// barrier on each side; long lines link them into per-bin lists that the
// bin's owner sums.
//
// A detection whose frequency is already in the set (found through the
// set's frequency hash) adds its amplitude to that entry; otherwise it
// opens a new entry. Every entry contributes to the one bin it projects
// onto, so the subtraction is the same as summing every detection (the set
// amplitudes are sums of detections).
template <int D, bool kPow2, bool kRecLds, int kPath>
__device__ __forceinline__ void solve_cube(const CubeDesc& cd, const float2* __restrict__ x, const OutPtrs out,
                                           const int32_t* __restrict__ sched, const float2* __restrict__ twall,
                                           const float2* __restrict__ pre, int pre_count, char* smem,
                                           char* rec_store, char* lines_ws) {
  const Geo<D> g = load_geo<D>(cd);
  const uint32_t L = g.L;
  const int T = cd.T;
  const int max_k = cd.max_k;
  const int tid = threadIdx.x;
  const int B = blockDim.x;
  const float th0 = cd.zero_thresh;
  const float rho = cd.mag_rel_tol;
  const float gtol = cd.grid_tol;
  const float inv_L = cd.inv_L;
  const int32_t* sch = sched + cd.sched_off;
  // Long lines (block path only): lines transformed one at a time, twiddles
  // read from global memory (the host sends no precomputed spectra).
  constexpr bool kWave = kPath == kPathWave;
  constexpr bool gmem = kPath == kPathLinesWs;  // the host sends only such cubes here
  const bool serial = gmem || (!(kWave && kPow2) && cd.serial != 0);
  // Time-domain construction-subtraction (block path; the host sends such
  // cubes nowhere else) and line-averaged amplitudes.
  const bool literal = !(kWave && kPow2) && !serial && (cd.flags & FPS_LITERAL_PEEL) != 0;
  const bool avg = (cd.flags & FPS_AMP_AVERAGE) != 0;
  // Longer lines still: the spectra and the scratch line in device memory
  // (barriers that order the line buffers then order every memory access).
  SolveLds s = carve_solve_lds<D, kPath>(smem, (int)L, kRecLds ? cd.rec_lds : 0, serial, literal, lines_ws);
  const RecStore rs = kRecLds ? s.rec : carve_records<D>(rec_store, max_k);
  for (uint32_t e = tid; e <= rs.hmask; e += B) rs_st<kRecLds>(rs.ht, (int)e, -1);
  if (!serial) {
    for (uint32_t e = tid; e < L; e += B) {
      s.tw[e] = ld_g(twall, cd.tw_off + e);
      s.bmax[e] = 0u;
      s.bcnt[e] = 0;
    }
    for (uint32_t e = tid; e < (D + 1) * L; e += B) s.Q[e] = make_int2(0, 0);
  }
  const float2* tw = serial ? twall + cd.tw_off : s.tw;
  float2* oamps = (float2*)out.amps;
  const bool use_pf = !serial && L <= (uint32_t)(kPfU * B);
  const int wv = tid >> 6;
  const int lane = tid & 63;
  const int nw = (B + 63) >> 6;
  const int E = (int)(L >> 6);
  // The host sends a cube here only if 64 <= L <= 512 and blockDim has at
  // least D+1 waves.
  constexpr bool wave_path = kWave && kPow2;
  // Link the entries concurrently with the transforms when some waves have
  // no line.
  const bool conc = wave_path && nw > D + 1;
  if (tid < 4) s.cnt[tid] = 0;

  Prefetch<D> pf;
  float2 pfw[kEMax];
  if constexpr (wave_path) {
    if (wv <= D) wave_prefetch<D, kPow2>(pfw, E, g, x, sch, pre, 0 < pre_count, wv);
    // The wave transforms read twiddles that other threads staged above.
    lds_barrier();
  } else if (use_pf) {
    prefetch_issue<D, kPow2>(pf, g, x, sch, pre, 0 < pre_count);
  }

  int kc_det = 0;   // detections recorded (the capacity counts these)
  int kc_set = 0;   // distinct frequencies recorded
  int kc_hash = 0;  // of which in the frequency hash (or entering it)
  bool any_merge = false;
  int xpar = 0;
  int status = kStatusIncomplete;
  int iters = T;
  bool full = false;
  for (int t = 0; t < T; ++t) {
    const int32_t* at = sch + t * 2 * D;
    // the entries of slots hfrom .. kc_set-1 enter the hash while linking
    const int hfrom = kc_hash;
    kc_hash = kc_set;
    const bool precomputed = t < pre_count;
    uint32_t al[D], ta[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      al[k] = (uint32_t)at[k];
      ta[k] = (uint32_t)at[D + k];
    }
    const float2* S;
    if constexpr (wave_path) {
      if (wv <= D) {
        // Consume the prefetched samples first, so that the registers they
        // occupy are free when the next iteration's loads are issued into
        // them; otherwise the compiler carries the new loads through a
        // register copy that waits for them right after the transform.
        const float sc = precomputed ? 1.0f : inv_L;
        float2 cur[kEMax];
#pragma unroll
        for (int e = 0; e < kEMax; ++e) {
          cur[e] = c_scale(pfw[e], sc);
          __asm__ volatile("" : "+v"(cur[e].x), "+v"(cur[e].y));
        }
        float2* dst = s.bufA + wv * L;
        if (precomputed) {
#pragma unroll
          for (int e = 0; e < kEMax; ++e)
            if (e < E) dst[lane + 64 * e] = cur[e];
        } else {
          switch (E) {
            case 1: wave_fft_to_lds<1>(cur, tw, dst); break;
            case 2: wave_fft_to_lds<2>(cur, tw, dst); break;
            case 4: wave_fft_to_lds<4>(cur, tw, dst); break;
            default: wave_fft_to_lds<8>(cur, tw, dst); break;
          }
        }
        // The next iteration's gathers are issued after the transform: in
        // flight, scattered loads slow this wave's LDS traffic several-fold;
        // they overlap the entry counts, the sums and the decode instead.
        if (t + 1 < T)
          wave_prefetch<D, kPow2>(pfw, E, g, x, at + 2 * D, pre + (int64_t)(t + 1) * (D + 1) * L, t + 1 < pre_count,
                                  wv);
      } else if (conc) {
        link_bins<D, kPow2, kRecLds>(g, al, rs, s.head, s.bmax, s.bcnt, tid - (D + 1) * 64, B - (D + 1) * 64,
                                     kc_set, hfrom);
      }
      rec_barrier<kRecLds>();
      S = s.bufA;
    } else if (serial) {
      // the last iteration's reads of the line buffers come first
      if (gmem) __syncthreads();
      for (int line = 0; line <= D; ++line) {
        gather_one_line<D, kPow2>(s.bufB, x, g, at, line, inv_L);
        if (gmem)
          __syncthreads();
        else
          lds_barrier();
        float2* dst = s.bufA + line * L;
        const float2* R = block_fft<kPow2>(s.bufB, dst, 1, (int)L, cd.nstages, cd.radix, tw, gmem);
        if (R != dst) {
          for (uint32_t e = tid; e < L; e += B) dst[e] = R[e];
          if (gmem)
            __syncthreads();
          else
            lds_barrier();
        }
      }
      S = s.bufA;
    } else {
      if (use_pf) {
        prefetch_store<D>(pf, L, s.bufA, precomputed ? 1.0f : inv_L);
      } else if (precomputed) {
        const float2* src = pre + (int64_t)t * (D + 1) * L;
        for (uint32_t e = tid; e < (D + 1) * L; e += B) s.bufA[e] = ld_g(src, e);
      } else {
        gather_lines<D, kPow2>(s.bufA, x, g, at, 1, inv_L);
      }
      lds_barrier();
      if (literal) {
        // Construction-subtraction as stated in Sec. 2.2: the records' line
        // spectra (Eq. freqSum) go through an unnormalised inverse DFT, read
        // as the forward DFT at index (L - l) mod L, and are subtracted from
        // the samples (held divided by L, hence the constructed ones too).
        link_bins<D, kPow2, kRecLds>(g, al, rs, s.head, s.bmax, s.bcnt, tid, B, kc_set, hfrom);
        rec_barrier<kRecLds>();
        accumulate_bins<D, kPow2, kRecLds>(g, al, ta, rs, tw, s.bmax, s.bcnt, s.Q, tid, B, kc_set);
        lds_barrier();
        for (uint32_t m = tid; m < L; m += B) {
          const int n = s.bcnt[m];
          const int e = n > 0 ? bin_exponent32(s.bmax[m], n) : 0;
#pragma unroll
          for (int i = 0; i <= D; ++i) {
            const int2 q = s.Q[i * L + m];
            s.P[i * L + m] = n > 0 ? make_float2(fixed_value32(q.x, e), fixed_value32(q.y, e)) : make_float2(0.f, 0.f);
          }
        }
        lds_barrier();
        const float2* R = block_fft<kPow2>(s.P, s.bufB, D + 1, (int)L, cd.nstages, cd.radix, tw);
        for (int i = 0; i <= D; ++i)
          for (uint32_t l = tid; l < L; l += B) {
            const uint32_t lr = l ? L - l : 0u;
            s.bufA[i * L + l] = c_sub(s.bufA[i * L + l], c_scale(R[i * L + lr], inv_L));
          }
        lds_barrier();
        // the sums (in the same buffer) start at zero next iteration
        for (uint32_t e = tid; e < (D + 1) * L; e += B) s.Q[e] = make_int2(0, 0);
      }
      S = precomputed ? s.bufA : block_fft<kPow2>(s.bufA, s.bufB, D + 1, (int)L, cd.nstages, cd.radix, tw);
      if (use_pf && t + 1 < T)
        prefetch_issue<D, kPow2>(pf, g, x, at + 2 * D, pre + (int64_t)(t + 1) * (D + 1) * L, t + 1 < pre_count);
    }
    if (!conc && !literal) {
      if (serial) {
        // the heads live in the scratch line, free once the lines are done
        for (uint32_t e = tid; e < L; e += B) {
          s.head[e] = -1;
          s.bmax[e] = 0u;
        }
        if (gmem)
          __syncthreads();
        else
          lds_barrier();
      }
      link_bins<D, kPow2, kRecLds>(g, al, rs, s.head, s.bmax, serial ? nullptr : s.bcnt, tid, B, kc_set, hfrom);
      if (gmem)
        __syncthreads();
      else
        rec_barrier<kRecLds>();
    }
    if (!serial && !literal && kc_set > 0) {
      // all threads add the entries' projections to their bins' sums
      accumulate_bins<D, kPow2, kRecLds>(g, al, ta, rs, tw, s.bmax, s.bcnt, s.Q, tid, B, kc_set);
      lds_barrier();
    }

    // Test, decode and record, bins in ascending order: a pass covers up to
    // kDecodeBins bins per thread (bin m0 + j B + tid for the j-th), with one
    // exchange barrier for all of them.
    bool nonzero = false;
    bool any = false;
    constexpr int kNB = D >= 4 ? 1 : kDecodeBins;  // 4-D: register budget
    const int nbp = min(kNB, (int)((L + (uint32_t)B - 1) / (uint32_t)B));
    for (uint32_t m0 = 0; m0 < L; m0 += (uint32_t)(B * nbp)) {
      bool cand[kNB], isnew[kNB];
      int f[kNB][D];
      float2 amp[kNB];
      int mslot[kNB], slot[kNB], bdet[kNB], bnew[kNB], wdet[kNB], wnew[kNB];
      int wall = 0;
      const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        const uint32_t m = m0 + (uint32_t)(j * B) + tid;
        cand[j] = false;
        isnew[j] = false;
        amp[j] = make_float2(0.f, 0.f);
        mslot[j] = -1;
        slot[j] = -1;
        if (j < nbp && m < L) {
          float2 r[D + 1];
#pragma unroll
          for (int i = 0; i <= D; ++i) r[i] = S[i * L + m];
          // entries of the set project onto this bin
          const int h = serial ? s.head[m] : -1;
          // The bin's count, scale word and sums are read together (only the
          // count decides whether they are used), except where the block
          // path's registers are short (D >= 3).
          constexpr bool kEarly = (kWave && kPow2) || D <= 2;
          int nb = 0;
          uint32_t bm = 0u;
          int2 q[D + 1];
          if (!serial) {
            nb = s.bcnt[m];
            if constexpr (kEarly) {
              bm = s.bmax[m];
#pragma unroll
              for (int i = 0; i <= D; ++i) q[i] = s.Q[i * L + m];
            }
          }
          const bool hs = serial ? h >= 0 : nb > 0;
          if (hs && !literal) {
            float2 sum[D + 1];
            if (serial) {
              list_sum<D, kPow2, kRecLds>(g, ta, rs, tw, h, kc_set, bin_exponent(s.bmax[m]), sum);
            } else {
              if constexpr (!kEarly) {
                bm = s.bmax[m];
#pragma unroll
                for (int i = 0; i <= D; ++i) q[i] = s.Q[i * L + m];
              }
              const int e = bin_exponent32(bm, nb);
#pragma unroll
              for (int i = 0; i <= D; ++i) sum[i] = make_float2(fixed_value32(q[i].x, e), fixed_value32(q[i].y, e));
            }
#pragma unroll
            for (int i = 0; i <= D; ++i) r[i] = c_sub(r[i], sum[i]);
          }
          cand[j] = decode_bin<D, kPow2>(g, al, ta, r, m, th0, rho, gtol, tw, avg, nonzero, f[j], amp[j]);
          if (hs) {
            // a frequency already in the set projects onto this bin
            if (cand[j]) mslot[j] = hash_find<D, kRecLds>(rs, freq_key<D>(g, f[j]), f[j]);
            if (serial) s.head[m] = -1;  // the list is rebuilt next iteration
            s.bmax[m] = 0u;
            if (!serial) {
              s.bcnt[m] = 0;
#pragma unroll
              for (int i = 0; i <= D; ++i) s.Q[i * L + m] = make_int2(0, 0);
            }
          }
          isnew[j] = cand[j] && mslot[j] < 0;
        }
        const unsigned long long bd = __ballot(cand[j] ? 1 : 0);
        const unsigned long long bn = __ballot(isnew[j] ? 1 : 0);
        wdet[j] = __popcll(bd);
        bdet[j] = __popcll(bd & lt);
        wnew[j] = __popcll(bn);
        bnew[j] = __popcll(bn & lt);
        wall += wnew[j];
      }
      // New frequencies go to the store and detected ones join their entry
      // now (one slot atomic per wave), so that the next iteration can link
      // and sum them with no barrier after the exchange below. A merge that
      // turns out not to fit the capacity is undone after the exchange.
      float2 mold[kNB];
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        mold[j] = make_float2(0.f, 0.f);
        if (mslot[j] >= 0) {
          mold[j] = rs_ld<kRecLds>(rs.sa, mslot[j]);
          const float2 av = c_add(mold[j], amp[j]);
          rs_st<kRecLds>(rs.sa, mslot[j], av);
        }
      }
      if (wall > 0) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&s.cnt[0], wall);
        base = __builtin_amdgcn_readlane(base, 0);
#pragma unroll
        for (int j = 0; j < kNB; ++j) {
          slot[j] = base + bnew[j];
          base += wnew[j];
          if (isnew[j] && slot[j] < max_k) {
#pragma unroll
            for (int k = 0; k < D; ++k) rs_st<kRecLds>(rs.sf, slot[j] * D + k, f[j][k]);
            rs_st<kRecLds>(rs.sa, slot[j], amp[j]);
          }
        }
      }
      // exchange words of a wave: its detection counts per bin set in 16-bit
      // fields (at most 64 each, at most 512 summed over 8 waves) with the
      // nonzero flag in bit 31, and its new-frequency counts the same way
      static_assert(kNB <= 2, "two 16-bit count fields per exchange word");
      const bool wnz = __ballot(nonzero ? 1 : 0) != 0ull;
      uint32_t wa = wnz ? 0x80000000u : 0u, wb = 0u;
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        wa |= (uint32_t)wdet[j] << (16 * j);
        wb |= (uint32_t)wnew[j] << (16 * j);
      }
      if (lane == 0) {
        s.wsum[xpar * 16 + 2 * wv] = (int)wa;
        s.wsum[xpar * 16 + 2 * wv + 1] = (int)wb;
      }
      lds_barrier();
      // one LDS read per lane (zero past the last wave), then the words are
      // taken from fixed lanes and summed as packed fields
      const int word = lane < 2 * nw ? s.wsum[xpar * 16 + lane] : 0;
      uint32_t sa = 0u, sb = 0u, pa = 0u, pb = 0u, fl = 0u;
      const int wvu = __builtin_amdgcn_readfirstlane(wv);
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        const uint32_t va = (uint32_t)__builtin_amdgcn_readlane(word, 2 * w);
        const uint32_t vb = (uint32_t)__builtin_amdgcn_readlane(word, 2 * w + 1);
        fl |= va;
        sa += va & 0x7fffffffu;
        sb += vb;
        pa += w < wvu ? (va & 0x7fffffffu) : 0u;
        pb += w < wvu ? vb : 0u;
      }
      any = (fl >> 31) != 0u;
      int pdet[kNB], tdet[kNB], pnew[kNB], tnew[kNB];
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        pdet[j] = (int)((pa >> (16 * j)) & 0xffffu);
        tdet[j] = (int)((sa >> (16 * j)) & 0xffffu);
        pnew[j] = (int)((pb >> (16 * j)) & 0xffffu);
        tnew[j] = (int)((sb >> (16 * j)) & 0xffffu);
      }
      xpar ^= 1;
      int sum_det = 0, sum_new = 0;
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        sum_det += tdet[j];
        sum_new += tnew[j];
      }
      // The store is full: the detections up to capacity are kept, in
      // canonical order, and the run stops.
      const bool fullp = kc_det + sum_det > max_k;
      any_merge |= sum_det != sum_new;
      int done_det = 0, done_new = 0;  // counts of the earlier bin sets
      // (device-memory store: the wave-order writes of a full pass must land
      // before the canonical ones below)
      if constexpr (!kRecLds) {
        if (fullp) __syncthreads();
      }
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        if (cand[j]) {
          const int di = kc_det + done_det + pdet[j] + bdet[j];
          if (di < max_k) {
            int si;
            if (isnew[j]) {
              si = kc_set + done_new + pnew[j] + bnew[j];
              int sl = slot[j];
              if (fullp) {
                // Slots went to this pass's new frequencies in wave order;
                // the ones kept move to their canonical slots (all of them
                // hold their values in registers).
                sl = si;
#pragma unroll
                for (int k = 0; k < D; ++k) rs_st<kRecLds>(rs.sf, sl * D + k, f[j][k]);
                rs_st<kRecLds>(rs.sa, sl, amp[j]);
                atomicMax(&s.cnt[2], si + 1);
              }
              if (sl < max_k) rs_st<kRecLds>(rs.sp, sl, si);
            } else {
              // detected again: the amplitude joined the first record
              si = rs_ld<kRecLds>(rs.sp, mslot[j]) & 0x7fffffff;
              rs_st<kRecLds>(rs.sp, mslot[j], (int32_t)((uint32_t)si | 0x80000000u));
            }
            st_gi(out.rec_iter, di, t);
            st_gi(out.rec_bin, di, (int32_t)(m0 + (uint32_t)(j * B) + tid));
            st_gi(out.rec_sin, di, si);
          } else if (!isnew[j]) {
            rs_st<kRecLds>(rs.sa, mslot[j], mold[j]);
          }
        }
        done_det += tdet[j];
        done_new += tnew[j];
      }
      if (fullp) {
        full = true;
        break;
      }
      kc_det += done_det;
      kc_set += done_new;
    }
    // Records kept in device memory are read by other threads next
    // iteration: make the stores visible across the work-group.
    if (!kRecLds) __syncthreads();
    if (full) {
      status = kStatusCapacity;
      iters = t + 1;
      break;
    }
    if (!any) {
      status = kStatusOk;
      iters = t + 1;
      break;
    }
  }

  // End of the cube: the set and the detections go to the outputs. Without
  // a re-detection the set is in first-detection order at the canonical
  // indices; otherwise a merged frequency whose amplitude sum has |a| <=
  // theta0 is not part of the set (Eq. sigModel2: a != 0) and moves behind
  // the kept ones, both groups in first-detection order.
  // (a full barrier: the detection trace in the outputs is read below)
  __syncthreads();
  if (full) {
    kc_det = max_k;
    kc_set = max(kc_set, s.cnt[2]);
  }
  const int nset = kc_set;
  int kept = nset;
  if (!any_merge) {
    for (int j = tid; j < nset; j += B) {
      const int pos = rs_ld<kRecLds>(rs.sp, j);
#pragma unroll
      for (int k = 0; k < D; ++k) st_gi(out.freqs, pos * D + k, rs_ld<kRecLds>(rs.sf, j * D + k));
      st_g(oamps, pos, rs_ld<kRecLds>(rs.sa, j));
    }
  } else {
    for (int j = tid; j < nset; j += B) rs_st<kRecLds>(rs.nx, rs_ld<kRecLds>(rs.sp, j) & 0x7fffffff, j);
    rec_barrier<kRecLds>();
    const unsigned long long lt = (1ull << lane) - 1ull;
    int ck = 0, cdrop = 0;
    for (int base = 0; base < nset; base += B) {
      const int pos = base + tid;
      int j = -1;
      bool drop = false, keep = false;
      if (pos < nset) {
        j = rs_ld<kRecLds>(rs.nx, pos);
        const float2 a = rs_ld<kRecLds>(rs.sa, j);
        drop = rs_ld<kRecLds>(rs.sp, j) < 0 && sqrtf(a.x * a.x + a.y * a.y) <= th0;
        keep = !drop;
      }
      const unsigned long long bd = __ballot(drop ? 1 : 0);
      const unsigned long long bk = __ballot(keep ? 1 : 0);
      if (lane == 0) s.wsum[xpar * 16 + wv] = __popcll(bd) | (__popcll(bk) << 8);
      lds_barrier();
      const int word = lane < nw ? s.wsum[xpar * 16 + lane] : 0;
      int pd = 0, pk = 0, td = 0, tk = 0;
      for (int w = 0; w < nw; ++w) {
        const int v = __builtin_amdgcn_readlane(word, w);
        pd += (w < wv) ? (v & 0xff) : 0;
        pk += (w < wv) ? ((v >> 8) & 0xff) : 0;
        td += v & 0xff;
        tk += (v >> 8) & 0xff;
      }
      xpar ^= 1;
      // rank among the kept (>= 0) or among the dropped (~rank < 0)
      if (pos < nset)
        rs_st<kRecLds>(rs.sp, j, drop ? ~(cdrop + pd + __popcll(bd & lt)) : ck + pk + __popcll(bk & lt));
      cdrop += td;
      ck += tk;
    }
    rec_barrier<kRecLds>();
    kept = ck;
    for (int pos = tid; pos < nset; pos += B) {
      const int j = rs_ld<kRecLds>(rs.nx, pos);
      const int enc = rs_ld<kRecLds>(rs.sp, j);
      const int fin = enc >= 0 ? enc : kept + ~enc;
#pragma unroll
      for (int k = 0; k < D; ++k) st_gi(out.freqs, fin * D + k, rs_ld<kRecLds>(rs.sf, j * D + k));
      st_g(oamps, fin, rs_ld<kRecLds>(rs.sa, j));
      rs_st<kRecLds>(rs.nx, pos, fin);
    }
    rec_barrier<kRecLds>();
  }
  if (any_merge) {
    // detections point at canonical set indices: map them to output positions
    for (int i = tid; i < kc_det; i += B) st_gi(out.rec_sin, i, rs_ld<kRecLds>(rs.nx, ld_gi(out.rec_sin, i)));
  }
  if (tid == 0) {
    st_gi(out.info, 0, kept);
    st_gi(out.info, 1, iters);
    st_gi(out.info, 2, status);
    st_gi(out.info, 3, kc_det);
    st_gi(out.info, 4, nset - kept);
    for (int q = 5; q < FPS_INFO_LEN; ++q) st_gi(out.info, q, 0);
  }
  __syncthreads();
}

// Solve kernels run 64..512 threads per work-group; the register budget is
// set for three waves per SIMD.
#define FPS_SOLVE_ATTRS __attribute__((amdgpu_flat_work_group_size(64, 512), amdgpu_waves_per_eu(3, 3)))

template <int D, bool kPow2, bool kRecLds, int kPath>
__global__ FPS_SOLVE_ATTRS void k_solve_plain(const CubeDesc* __restrict__ descs, int cube, const float2* __restrict__ x,
                                              OutPtrs out, const int32_t* __restrict__ sched,
                                              const float2* __restrict__ tw, const float2* __restrict__ pre,
                                              int pre_count, char* rec_store, char* lines_ws) {
  extern __shared__ __attribute__((aligned(16))) char lds_solve[];
  solve_cube<D, kPow2, kRecLds, kPath>(descs[cube], x, out, sched, tw, pre, pre_count, lds_solve, rec_store,
                                       lines_ws);
}

// Persistent: work-group b first solves cube order[b] (the grid is at most
// the cube count), so the launch's first takes wait on no atomic at one
// address; then it loops taking order[gridDim.x + queue[0]++] and leaves
// when that index passes the cube count, so every wave reaches the exit.
// Leaving, it counts itself in queue[1]; the last work-group out (every
// other one has made its final take) sets both counters back to zero for
// the next launch, so no reset kernel precedes the launch.
template <int D, bool kPow2, bool kRecLds, int kPath>
__global__ FPS_SOLVE_ATTRS void k_solve_batched(const CubeDesc* __restrict__ descs, const float2* const* __restrict__ xs,
                                                const OutPtrs* __restrict__ outs, const int32_t* __restrict__ sched,
                                                const float2* __restrict__ tw, const int32_t* __restrict__ order,
                                                int ncubes, int* __restrict__ queue, char* recws) {
  extern __shared__ __attribute__((aligned(16))) char lds_solve[];
  __shared__ int s_idx;
  int idx = (int)blockIdx.x;
  for (;; idx = -1) {
    if (idx < 0) {
      if (threadIdx.x == 0) s_idx = (int)gridDim.x + atomicAdd(queue, 1);
      __syncthreads();
      // uniform across the work-group: keep it in a scalar register
      idx = __builtin_amdgcn_readfirstlane(s_idx);
      __syncthreads();
    }
    if (idx >= ncubes) {
      if (threadIdx.x == 0 && atomicAdd(queue + 1, 1) == (int)gridDim.x - 1) {
        atomicExch(queue, 0);
        atomicExch(queue + 1, 0);
      }
      break;
    }
    const int c = __builtin_amdgcn_readfirstlane(order[idx]);
    const CubeDesc& cd = descs[c];
    solve_cube<D, kPow2, kRecLds, kPath>(cd, xs[c], outs[c], sched, tw, nullptr, 0, lds_solve,
                                         kRecLds ? nullptr : recws + cd.rec_off,
                                         kPath == kPathLinesWs ? recws + cd.lws_off : nullptr);
  }
}

__global__ void k_reset(int* __restrict__ p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Zero fill of one buffer per blockIdx.y (float2 elements): 16-byte stores
// of two elements, after one leading element when the buffer is only 8-byte
// aligned, and a trailing one when the rest is odd.
__global__ void k_zero(float2* const* __restrict__ bufs, const int64_t* __restrict__ lens, float2* single,
                       int64_t single_len) {
  float2* p = single ? single : bufs[blockIdx.y];
  const int64_t n = single ? single_len : lens[blockIdx.y];
  if (n <= 0) return;
  const int64_t head = ((uintptr_t)p & 15u) ? 1 : 0;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (head && gid == 0) st_g(p, 0, make_float2(0.f, 0.f));
  float2* q = p + head;
  const int64_t m = n - head;
  const int64_t pairs = m >> 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = gid; i < pairs; i += stride) st_g_pair(q, 2 * i, make_float2(0.f, 0.f), make_float2(0.f, 0.f));
  if ((m & 1) && gid == 0) st_g(q, m - 1, make_float2(0.f, 0.f));
}

// ---------------------------------------------------------------------------
// Adjoint of the set amplitudes (decisions fixed). Forward, per detection i
// found at iteration t in bin m:  a_i = W^{p_i} (s_hat^{(t,0)}(m) - sum_j
// a_j W^{-p_j^{(t)}}) over detections j of earlier iterations in bin m, with
// W = exp(-j 2 pi / L), p = [sum_k tau_k^{(t)} c_k m_k]_L; a set amplitude is
// the sum of its detections, so a detection's cotangent starts as its
// entry's. Reverse order: r_bar =
// W^{-p_i} a_bar_i flows to bin m of line 0 of iteration t and, negated and
// rotated by W^{p_j^{(t)}}, to the earlier detections j in that bin. The
// line cotangent goes back through the 1/L DFT (an inverse DFT with 1/L) and
// is added at the line-0 sample positions.
//
// The line cotangent and the FFT's second buffer are in LDS, with the
// twiddles beside them, or for long lines read from device memory; with
// kLinesWs (lines too long for LDS) the two line buffers are in the cube's
// device workspace.
// ---------------------------------------------------------------------------
// First index of the run of equal iterations that ends at e - 1 (the
// detection trace is in iteration order), found by one wave: each round
// probes 64 evenly spaced indices of the remaining range at once. The
// result is below e whatever the trace holds.
__device__ __forceinline__ int run_first(const int* riter, int e) {
  const int lane = threadIdx.x & 63;
  const int tt = riter[e - 1];
  int lo = 0, hi = e - 1;  // indices below lo hold earlier iterations
  while (hi > lo) {
    const int step = (hi - lo + 63) >> 6;
    const int idx = lo + lane * step;
    const bool below = idx <= hi && riter[idx] < tt;
    const int cnt = __popcll(__ballot(below ? 1 : 0));
    if (cnt == 0) break;
    const int nlo = lo + (cnt - 1) * step + 1;
    hi = min(lo + cnt * step, hi);
    lo = nlo;
  }
  return min(lo, e - 1);
}

// The deferred iterations of the adjoint (64 <= L <= 512, a power of two):
// up to two waves each take an iteration, spread its detections' values
// over the line in their own LDS buffer, transform it in registers and add
// the conjugate at the line-0 sample positions. A wave reads back only
// what it wrote itself, in program order (no block barrier).
template <int D, bool kPow2>
__device__ __forceinline__ void backward_deferred(const CubeDesc& cd, const Geo<D>& g, const float2* abar,
                                                  const int* riter, const int* rbin, const int* rstart, int nr,
                                                  int n, const int32_t* __restrict__ sched, const float2* tw,
                                                  float2* buf0, float2* buf1, float2* __restrict__ gx) {
  const uint32_t L = g.L;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int npw = min((int)(blockDim.x >> 6), 2);
  if (wv >= npw) return;
  const int E = (int)(L >> 6);
  float2* buf = wv ? buf1 : buf0;
  for (int r = wv; r < nr; r += npw) {
    const int s0 = rstart[r];
    const int e = r ? rstart[r - 1] : n;
    const int t = riter[s0];
    if (t < 0 || t >= cd.T) continue;
    for (uint32_t m = lane; m < L; m += 64) buf[m] = make_float2(0.f, 0.f);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the detections' bins are distinct within an iteration
    for (int i = s0 + lane; i < e; i += 64) {
      const int m = rbin[i];
      if (m >= 0 && m < (int)L) buf[m] = c_scale(c_conj(abar[i]), cd.inv_L);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the wave transform takes line element E q + e in register e of lane q
    float2 v[kEMax];
#pragma unroll
    for (int q = 0; q < kEMax; ++q) v[q] = q < E ? buf[E * lane + q] : make_float2(0.f, 0.f);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int32_t row[2 * D];
#pragma unroll
    for (int q = 0; q < 2 * D; ++q) row[q] = sched[cd.sched_off + t * 2 * D + q];
    // s_bar(l) = conj(FFT(conj(r_bar) / L))(l), added at sample l of line 0
    auto add = [&](int l, float2 val) {
      int64_t step[D];
      const int64_t flat = line_sample<D, kPow2>(g, row, (uint32_t)l, step);
      unsafeAtomicAdd(&gx[flat].x, val.x);
      unsafeAtomicAdd(&gx[flat].y, -val.y);
    };
    switch (E) {
      case 1: {
        float2 w[1] = {v[0]};
        wave_fft_lanes<1>(w, tw, add);
        break;
      }
      case 2: {
        float2 w[2] = {v[0], v[1]};
        wave_fft_lanes<2>(w, tw, add);
        break;
      }
      case 4: {
        float2 w[4] = {v[0], v[1], v[2], v[3]};
        wave_fft_lanes<4>(w, tw, add);
        break;
      }
      default: {
        float2 w[8] = {v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
        wave_fft_lanes<8>(w, tw, add);
        break;
      }
    }
  }
}

template <int D, bool kPow2, bool kLinesWs>
__device__ __forceinline__ void backward_cube(const CubeDesc& cd, const OutPtrs fwd, const float2* __restrict__ ga,
                                              float2* __restrict__ gx, const int32_t* __restrict__ sched,
                                              const float2* __restrict__ twall, char* smem, char* lines_ws) {
  const Geo<D> g = load_geo<D>(cd);
  const uint32_t L = g.L;
  const int tid = threadIdx.x;
  const int B = blockDim.x;
  const bool twg = kLinesWs || cd.serial != 0;   // twiddles from device memory
  float2* rbar;     // [L] line-0 spectrum cotangent
  float2* scratch;  // [L] FFT ping-pong
  float2* abar;     // [max_k] detection cotangents (LDS)
  int* riter;       // [max_k] detection iterations (LDS, after abar)
  uint32_t* dgk;    // [max_k][D] c_k m_k of each detection's frequency
                    // (LDS); ~0 first: no valid set index
  int* rbin;        // [max_k] detection bins (LDS)
  int* rstart;      // [min(T, max_k)] first detection of each iteration
                    // whose line transform is deferred, last iteration
                    // first (LDS)
  const float2* tw;
  if constexpr (kLinesWs) {
    rbar = (float2*)lines_ws;
    scratch = rbar + L;
    abar = (float2*)smem;
    tw = twall + cd.tw_off;
  } else {
    rbar = (float2*)smem;
    scratch = rbar + L;
    float2* twl = scratch + L;
    abar = twg ? twl : twl + L;
    if (twg) {
      tw = twall + cd.tw_off;
    } else {
      for (uint32_t e = tid; e < L; e += B) twl[e] = ld_g(twall, cd.tw_off + e);
      tw = twl;
    }
  }
  riter = (int*)(abar + cd.max_k);
  dgk = (uint32_t*)(riter + cd.max_k);
  rbin = (int*)(dgk + cd.max_k * D);
  rstart = rbin + cd.max_k;
  const int rcap = min(cd.T, cd.max_k);
  __shared__ int sh_s, sh_t, sh_nr, sh_def;
  __shared__ int32_t sh_row[2 * D];
  // Lines a wave can transform in registers (twiddles in LDS): the reverse
  // recursion runs first, storing each detection's line-spectrum cotangent
  // in its slot, and the iterations' inverse transforms and gradient adds
  // follow, one iteration per wave, in parallel.
  const bool par = kPow2 && !twg && L >= 64 && L <= 512 && B >= 64;

  // the set and the merged frequencies left out of it: every entry the
  // forward wrote is a sum of detections
  const int nent = min(max(ld_gi(fwd.info, 0), 0) + max(ld_gi(fwd.info, 4), 0), cd.max_k);
  const int n = min(max(ld_gi(fwd.info, 3), 0), cd.max_k);
  // Entries that no forward run can have written (set index, bin or
  // iteration out of range) are skipped rather than trusted as indices.
  for (int i = tid; i < n; i += B) {
    const int si = ld_gi(fwd.rec_sin, i);
    abar[i] = (si >= 0 && si < nent) ? ld_g(ga, si) : make_float2(0.f, 0.f);
    riter[i] = ld_gi(fwd.rec_iter, i);
    rbin[i] = ld_gi(fwd.rec_bin, i);
    const bool fok = si >= 0 && si < cd.max_k;
#pragma unroll
    for (int q = 0; q < D; ++q)
      dgk[i * D + q] = fok ? g.c[q] * (uint32_t)ld_gi(fwd.freqs, si * D + q) : (q == 0 ? ~0u : 0u);
  }
  // The last wave finds each iteration's run and reads its schedule row
  // while the others work on the iteration before; its lane 0 publishes
  // them at the barrier that ends that iteration.
  const int wl = (B >> 6) - 1;
  const bool finder = (tid >> 6) == wl;
  const bool pub = tid == (wl << 6);
  int nx_s = 0, nx_t = 0;
  int32_t nx_row[2 * D];
  auto find_next = [&](int end) {
    nx_s = run_first(riter, end);
    nx_t = riter[nx_s];
    const bool ok = nx_t >= 0 && nx_t < cd.T;
#pragma unroll
    for (int q = 0; q < 2 * D; ++q) nx_row[q] = ok ? sched[cd.sched_off + nx_t * 2 * D + q] : 0;
  };
  auto publish = [&]() {
    sh_s = nx_s;
    sh_t = nx_t;
#pragma unroll
    for (int q = 0; q < 2 * D; ++q) sh_row[q] = nx_row[q];
    int d = 0;
    if (par && sh_nr < rcap) {
      rstart[sh_nr] = nx_s;
      sh_nr = sh_nr + 1;
      d = 1;
    }
    sh_def = d;
  };
  if (tid == 0) sh_nr = 0;
  __syncthreads();
  if (finder && n > 0) find_next(n);
  if (pub && n > 0) publish();
  for (uint32_t m = tid; m < L; m += B) rbar[m] = make_float2(0.f, 0.f);
  __syncthreads();
  int e = n;
  while (e > 0) {
    const int s0 = sh_s;
    const int t = sh_t;
    const bool deferred = sh_def != 0;
    const bool t_ok = t >= 0 && t < cd.T;
    uint32_t al[D], ta[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
      al[q] = (uint32_t)sh_row[q];
      ta[q] = (uint32_t)sh_row[D + q];
    }
    const int32_t* at = sched + cd.sched_off + (t_ok ? t : 0) * 2 * D;
    // Detections of iteration t: distinct bins, so plain stores.
    // A deferred iteration keeps each detection's value in its own slot
    // (zero for a skipped one), which nothing reads again in this loop.
    for (int i = s0 + tid; i < e; i += B) {
      const int m = rbin[i];
      if (!t_ok || m < 0 || m >= (int)L || dgk[i * D] == ~0u) {
        if (deferred) abar[i] = make_float2(0.f, 0.f);
        continue;
      }
      uint32_t p = 0;
#pragma unroll
      for (int q = 0; q < D; ++q) p = umod<kPow2>(p + ta[q] * dgk[i * D + q], L);
      const float2 r = c_mulc(abar[i], tw[p]);
      rbar[m] = r;
      if (deferred) abar[i] = r;
    }
    if (finder && s0 > 0) find_next(s0);
    __syncthreads();
    // Earlier detections that iteration t's construction-subtraction removed.
    for (int j = tid; j < s0; j += B) {
      if (dgk[j * D] == ~0u) continue;
      uint32_t b = 0, p = 0;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const uint32_t gq = dgk[j * D + q];
        b = umod<kPow2>(b + al[q] * gq, L);
        p = umod<kPow2>(p + ta[q] * gq, L);
      }
      const float2 v = rbar[b];
      abar[j] = c_sub(abar[j], c_mul(tw[p], v));
    }
    __syncthreads();
    if (!deferred) {
      // s_bar(l) = (1/L) sum_m r_bar(m) e^{+j 2 pi l m / L}
      //          = (1/L) conj(FFT(conj(r_bar)))(l).
      for (uint32_t m = tid; m < L; m += B) rbar[m] = c_scale(c_conj(rbar[m]), cd.inv_L);
      __syncthreads();
      const float2* S = block_fft<kPow2>(rbar, scratch, 1, (int)L, cd.nstages, cd.radix, tw, kLinesWs);
      if (t_ok) {
        for (uint32_t l = tid; l < L; l += B) {
          int64_t step[D];
          const int64_t flat = line_sample<D, kPow2>(g, at, l, step);
          const float2 v = c_conj(S[l]);
          unsafeAtomicAdd(&gx[flat].x, v.x);
          unsafeAtomicAdd(&gx[flat].y, v.y);
        }
      }
      __syncthreads();
    }
    // the next iteration
    for (uint32_t m = tid; m < L; m += B) rbar[m] = make_float2(0.f, 0.f);
    if (pub && s0 > 0) publish();
    __syncthreads();
    e = s0;
  }
  if (par) backward_deferred<D, kPow2>(cd, g, abar, riter, rbin, rstart, sh_nr, n, sched, tw, rbar, scratch, gx);
}

template <int D, bool kPow2, bool kLinesWs>
__global__ void k_backward(const CubeDesc* __restrict__ descs, int cube, OutPtrs fwd_single,
                           const float2* __restrict__ ga_single, float2* __restrict__ gx_single,
                           const int32_t* __restrict__ order, const OutPtrs* __restrict__ fwds,
                           const float2* const* __restrict__ gas, float2* const* __restrict__ gxs,
                           const int32_t* __restrict__ sched, const float2* __restrict__ tw, char* ws) {
  extern __shared__ __attribute__((aligned(16))) char lds_bwd[];
  const int c = cube >= 0 ? cube : order[blockIdx.x];
  const CubeDesc& cd = descs[c];
  char* lws = kLinesWs ? ws + cd.lws_off : nullptr;
  if (cube >= 0)
    backward_cube<D, kPow2, kLinesWs>(cd, fwd_single, ga_single, gx_single, sched, tw, lds_bwd, lws);
  else
    backward_cube<D, kPow2, kLinesWs>(cd, fwds[c], gas[c], gxs[c], sched, tw, lds_bwd, lws);
}

// ---------------------------------------------------------------------------
// Instantiation tables and host-side launchers.
// ---------------------------------------------------------------------------
#define FPS_DISPATCH_D(D_, ...)                 \
  switch (D_) {                                 \
    case 1: {                                   \
      constexpr int kD = 1;                     \
      __VA_ARGS__;                              \
      break;                                    \
    }                                           \
    case 2: {                                   \
      constexpr int kD = 2;                     \
      __VA_ARGS__;                              \
      break;                                    \
    }                                           \
    case 3: {                                   \
      constexpr int kD = 3;                     \
      __VA_ARGS__;                              \
      break;                                    \
    }                                           \
    default: {                                  \
      constexpr int kD = 4;                     \
      __VA_ARGS__;                              \
      break;                                    \
    }                                           \
  }

#define FPS_DISPATCH_B(flag, name, ...) \
  if (flag) {                           \
    constexpr bool name = true;         \
    __VA_ARGS__;                        \
  } else {                              \
    constexpr bool name = false;        \
    __VA_ARGS__;                        \
  }

// Solve kernels: the wave path exists only for power-of-two lines.
#define FPS_DISPATCH_SOLVE(key, ...)                                                          \
  FPS_DISPATCH_D(key.D, FPS_DISPATCH_B(key.rec_lds, kR, {                                     \
    if (key.pow2 && key.wave) {                                                               \
      constexpr bool kP = true;                                                               \
      constexpr int kW = kPathWave;                                                           \
      __VA_ARGS__;                                                                            \
    } else if (key.pow2 && key.lines_ws) {                                                    \
      constexpr bool kP = true;                                                               \
      constexpr int kW = kPathLinesWs;                                                        \
      __VA_ARGS__;                                                                            \
    } else if (key.pow2) {                                                                    \
      constexpr bool kP = true;                                                               \
      constexpr int kW = kPathBlock;                                                          \
      __VA_ARGS__;                                                                            \
    } else if (key.lines_ws) {                                                                \
      constexpr bool kP = false;                                                              \
      constexpr int kW = kPathLinesWs;                                                        \
      __VA_ARGS__;                                                                            \
    } else {                                                                                  \
      constexpr bool kP = false;                                                              \
      constexpr int kW = kPathBlock;                                                          \
      __VA_ARGS__;                                                                            \
    }                                                                                         \
  }))

const void* kernel_ptr(KernelKind kind, const KernelKey& key) {
  const void* fn = nullptr;
  if (kind == KernelKind::kSolvePlain || kind == KernelKind::kSolveBatched) {
    FPS_DISPATCH_SOLVE(key, {
      fn = kind == KernelKind::kSolvePlain ? (const void*)k_solve_plain<kD, kP, kR, kW>
                                           : (const void*)k_solve_batched<kD, kP, kR, kW>;
    })
    return fn;
  }
  if (kind == KernelKind::kBackward) {
    FPS_DISPATCH_D(key.D, FPS_DISPATCH_B(key.pow2, kP, FPS_DISPATCH_B(key.lines_ws, kL, {
      fn = (const void*)k_backward<kD, kP, kL>;
    })))
    return fn;
  }
  FPS_DISPATCH_D(key.D, FPS_DISPATCH_B(key.pow2, kP, { fn = (const void*)k_lines<kD, kP>; }))
  return fn;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free plain entry point: one static array, of
// which every GPU the library runs on holds its own copy until the process
// ends. Host code uses the address hipGetSymbolAddress returns for the
// current device, never the array's name.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(int device, void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    addr[device] = ptr;
  }
  *out = addr[device];
  return hipSuccess;
}

hipError_t launch_lines_single(const LaunchCtx& ctx, const KernelKey& key, int cube, const float2* x, int t0,
                               int count, float2* out, int maxL, size_t lds, int threads, hipStream_t st) {
  FPS_DISPATCH_D(key.D, FPS_DISPATCH_B(key.pow2, kP, {
    hipLaunchKernelGGL((k_lines<kD, kP>), dim3(count), dim3(threads), lds, st, ctx.descs,
                       (const LineItem*)nullptr, (const int32_t*)nullptr, (int*)nullptr, cube, t0, count, x,
                       (const float2* const*)nullptr, ctx.sched, ctx.tw, out, maxL);
  }))
  return hipGetLastError();
}

hipError_t launch_lines_items(const LaunchCtx& ctx, const KernelKey& key, const LineItem* items,
                              const int32_t* ranges, int* queues, int grid, const float2* const* xs, float2* out,
                              int maxL, size_t lds, int threads, hipStream_t st) {
  FPS_DISPATCH_D(key.D, FPS_DISPATCH_B(key.pow2, kP, {
    hipLaunchKernelGGL((k_lines<kD, kP>), dim3(grid), dim3(threads), lds, st, ctx.descs, items, ranges, queues, 0,
                       0, 0, (const float2*)nullptr, xs, ctx.sched, ctx.tw, out, maxL);
  }))
  return hipGetLastError();
}

hipError_t launch_solve_plain(const LaunchCtx& ctx, const KernelKey& key, int cube, const float2* x,
                              const OutPtrs& out, const float2* pre, int pre_count, char* rec_store, char* lines_ws,
                              size_t lds, int threads, hipStream_t st) {
  FPS_DISPATCH_SOLVE(key, {
    hipLaunchKernelGGL((k_solve_plain<kD, kP, kR, kW>), dim3(1), dim3(threads), lds, st, ctx.descs, cube, x, out,
                       ctx.sched, ctx.tw, pre, pre_count, rec_store, lines_ws);
  })
  return hipGetLastError();
}

hipError_t launch_reset(int* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_solve_batched(const LaunchCtx& ctx, const KernelKey& key, const float2* const* xs,
                                const OutPtrs* outs, const int32_t* order, int ncubes, int* queue, int grid,
                                size_t lds, int threads, hipStream_t st) {
  FPS_DISPATCH_SOLVE(key, {
    hipLaunchKernelGGL((k_solve_batched<kD, kP, kR, kW>), dim3(grid), dim3(threads), lds, st, ctx.descs, xs, outs,
                       ctx.sched, ctx.tw, order, ncubes, queue, ctx.rec_ws);
  })
  return hipGetLastError();
}

hipError_t launch_zero_single(float2* p, int64_t n, hipStream_t st) {
  // about four 16-byte stores per thread
  int64_t blocks = (n + 2047) / 2048;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, (float2* const*)nullptr,
                     (const int64_t*)nullptr, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_multi(float2* const* bufs, const int64_t* lens, int nbufs, int64_t maxlen, hipStream_t st) {
  // about four 16-byte stores per thread
  int64_t blocks = (maxlen + 2047) / 2048;
  if (blocks > 512) blocks = 512;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks, nbufs), dim3(256), 0, st, bufs, lens, (float2*)nullptr,
                     (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_backward_single(const LaunchCtx& ctx, const KernelKey& key, int cube, const OutPtrs& fwd,
                                  const float2* ga, float2* gx, size_t lds, int threads, hipStream_t st) {
  FPS_DISPATCH_D(key.D, FPS_DISPATCH_B(key.pow2, kP, FPS_DISPATCH_B(key.lines_ws, kL, {
    hipLaunchKernelGGL((k_backward<kD, kP, kL>), dim3(1), dim3(threads), lds, st, ctx.descs, cube, fwd, ga, gx,
                       (const int32_t*)nullptr, (const OutPtrs*)nullptr, (const float2* const*)nullptr,
                       (float2* const*)nullptr, ctx.sched, ctx.tw, ctx.rec_ws);
  })))
  return hipGetLastError();
}

hipError_t launch_backward_batched(const LaunchCtx& ctx, const KernelKey& key, const int32_t* order, int ncubes,
                                   const OutPtrs* fwds, const float2* const* gas, float2* const* gxs, size_t lds,
                                   int threads, hipStream_t st) {
  OutPtrs none{};
  FPS_DISPATCH_D(key.D, FPS_DISPATCH_B(key.pow2, kP, FPS_DISPATCH_B(key.lines_ws, kL, {
    hipLaunchKernelGGL((k_backward<kD, kP, kL>), dim3(ncubes), dim3(threads), lds, st, ctx.descs, -1, none,
                       (const float2*)nullptr, (float2*)nullptr, order, fwds, gas, gxs, ctx.sched, ctx.tw,
                       ctx.rec_ws);
  })))
  return hipGetLastError();
}

}  // namespace fpssft
