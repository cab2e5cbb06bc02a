// Device building blocks of the FPS-SFT kernels (gfx950, wave64).
//
//  * exact-integer line indexing (Eq. sample_slice): n_k(l) = [alpha_k l +
//    tau_k]_{N_k}, computed in 32-bit unsigned arithmetic (the plan checks
//    N_k * L < 2^31) and a 64-bit flat offset;
//  * a block-wide Stockham FFT over several lines held in LDS, radix 2/4/8
//    butterflies in registers and a generic radix for other prime factors,
//    twiddles read from one table W_L^k = exp(-j 2 pi k / L) with exact
//    integer exponents (Eq. hs);
//  * a block prefix count built from wave64 ballots.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "types.h"

namespace fpssft {

constexpr int kStatusOk = 0;
constexpr int kStatusIncomplete = 1;
constexpr int kStatusCapacity = 2;

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 c_mulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }

// x mod n for x < 2^32; `mask` is n - 1 for a power-of-two n, else -1.
__device__ __forceinline__ uint32_t umod(uint32_t x, uint32_t n, int32_t mask) {
  return mask >= 0 ? (x & (uint32_t)mask) : (x % n);
}

// ---------------------------------------------------------------------------
// Small DFTs (forward, exp(-j ...)) in registers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = c_add(t, b);
  b = c_sub(t, b);
}

__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
  float2 s02 = c_add(v0, v2), d02 = c_sub(v0, v2);
  float2 s13 = c_add(v1, v3), d13 = c_sub(v1, v3);
  float2 md = make_float2(d13.y, -d13.x);  // -j * d13
  v0 = c_add(s02, s13);
  v2 = c_sub(s02, s13);
  v1 = c_add(d02, md);
  v3 = c_sub(d02, md);
}

__device__ __forceinline__ void dft8(float2* v) {
  const float h = 0.70710678118654752440f;
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  // twiddles W8^1 = h(1 - j), W8^2 = -j, W8^3 = -h(1 + j)
  float2 t1 = make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x));
  float2 t2 = make_float2(o2.y, -o2.x);
  float2 t3 = make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y));
  v[0] = c_add(e0, o0);
  v[4] = c_sub(e0, o0);
  v[1] = c_add(e1, t1);
  v[5] = c_sub(e1, t1);
  v[2] = c_add(e2, t2);
  v[6] = c_sub(e2, t2);
  v[3] = c_add(e3, t3);
  v[7] = c_sub(e3, t3);
}

// ---------------------------------------------------------------------------
// One Stockham stage over `nl` lines: in -> out, radix r, Ns = product of
// the radices of earlier stages. Butterfly j of a line reads in[j + q L/r]
// (q < r), rotates input q by W_{Ns r}^{q (j mod Ns)}, takes an r-point DFT
// and writes output p to out[(j - j mod Ns) r + j mod Ns + p Ns].
// ---------------------------------------------------------------------------
template <int R>
__device__ __forceinline__ void stage_fixed(const float2* __restrict__ in, float2* __restrict__ out,
                                            int nl, int L, int Ns, int lg_nb, int lg_ns, bool pow2,
                                            const float2* __restrict__ tw) {
  const int nb = L / R;
  const int total = nl * nb;
  const int ts = L / (Ns * R);
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    int line, j, k;
    if (pow2) {
      line = w >> lg_nb;
      j = w & (nb - 1);
      k = j & (Ns - 1);
    } else {
      line = w / nb;
      j = w - line * nb;
      k = j % Ns;
    }
    const float2* src = in + line * L;
    float2* dst = out + line * L;
    float2 v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = src[j + q * nb];
    if (k != 0) {
#pragma unroll
      for (int q = 1; q < R; ++q) v[q] = c_mul(v[q], tw[q * k * ts]);
    }
    if (R == 2) {
      dft2(v[0], v[1]);
    } else if (R == 4) {
      dft4(v[0], v[1], v[2], v[3]);
    } else if (R == 8) {
      dft8(v);
    }
    const int ob = (j - k) * R + k;
#pragma unroll
    for (int p = 0; p < R; ++p) dst[ob + p * Ns] = v[p];
  }
}

// Any radix r (used for odd prime factors): each butterfly output is an
// r-term sum read straight from LDS.
__device__ __forceinline__ void stage_generic(const float2* __restrict__ in, float2* __restrict__ out,
                                              int nl, int L, int Ns, int r,
                                              const float2* __restrict__ tw) {
  const int nb = L / r;
  const int total = nl * nb * r;
  const int ts = L / (Ns * r);
  const int tr = L / r;  // W_r^1 = W_L^{L/r}
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    const int p = w % r;
    const int bw = w / r;
    const int line = bw / nb;
    const int j = bw - line * nb;
    const int k = j % Ns;
    const float2* src = in + line * L;
    float2 acc = make_float2(0.f, 0.f);
    for (int q = 0; q < r; ++q) {
      float2 v = src[j + q * nb];
      v = c_mul(v, tw[q * k * ts]);
      v = c_mul(v, tw[((p * q) % r) * tr]);
      acc = c_add(acc, v);
    }
    out[line * L + (j - k) * r + k + p * Ns] = acc;
  }
}

__device__ __forceinline__ int ilog2_pow2(int v) { return 31 - __clz(v); }

// Work-group barrier that orders LDS only. Global loads issued before it stay
// in flight (HIP's __syncthreads also waits for every outstanding global
// access, which would serialise the register prefetch of the next
// iteration's samples behind each barrier).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Forward, unnormalised FFT of `nl` contiguous lines of length cd.L held in
// LDS buffer a (b is scratch of the same size). Returns the buffer that holds
// the result. Must be called by the whole block; ends with a barrier.
__device__ __forceinline__ float2* block_fft(float2* a, float2* b, int nl, const CubeDesc& cd,
                             const float2* __restrict__ tw) {
  const int L = cd.L;
  const bool pow2 = cd.Lmask >= 0;
  float2* in = a;
  float2* out = b;
  int Ns = 1;
  for (int s = 0; s < cd.nstages; ++s) {
    const int r = cd.radix[s];
    const int lg_nb = pow2 ? ilog2_pow2(L / r) : 0;
    const int lg_ns = pow2 ? ilog2_pow2(Ns) : 0;
    if (r == 8)
      stage_fixed<8>(in, out, nl, L, Ns, lg_nb, lg_ns, pow2, tw);
    else if (r == 4)
      stage_fixed<4>(in, out, nl, L, Ns, lg_nb, lg_ns, pow2, tw);
    else if (r == 2)
      stage_fixed<2>(in, out, nl, L, Ns, lg_nb, lg_ns, pow2, tw);
    else
      stage_generic(in, out, nl, L, Ns, r, tw);
    lds_barrier();
    float2* t = in;
    in = out;
    out = t;
    Ns *= r;
  }
  return in;
}

// ---------------------------------------------------------------------------
// Exclusive prefix count of `flag` over the block in thread order (wave64
// ballots, per-wave counts in LDS `wsum`). Two barriers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int block_prefix(bool flag, int* wsum, int* total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  const unsigned long long bal = __ballot(flag ? 1 : 0);
  const int before = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) wsum[wave] = __popcll(bal);
  lds_barrier();
  int base = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    const int c = wsum[w];
    base += (w < wave) ? c : 0;
    tot += c;
  }
  lds_barrier();
  *total = tot;
  return base + before;
}

// True on every thread iff `flag` is true on some thread. Two barriers.
__device__ __forceinline__ bool block_any(bool flag, int* wsum) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  const unsigned long long bal = __ballot(flag ? 1 : 0);
  if (lane == 0) wsum[wave] = bal != 0ull;
  lds_barrier();
  int any = 0;
  for (int w = 0; w < nw; ++w) any |= wsum[w];
  lds_barrier();
  return any != 0;
}

// ---------------------------------------------------------------------------
// Line gather (Eq. sample_slice): the D+1 lines of `nt` consecutive
// iterations, sample l of line i of iteration tt written (times `scale`) to
// dst[(tt (D+1) + i) L + l]. Line 0 starts at tau, line i >= 1 at tau with
// coordinate i-1 advanced by one (mod N_{i-1}). at: the schedule rows
// [nt][2][D] (slope then offset per iteration).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gather_lines(float2* __restrict__ dst, const float2* __restrict__ x,
                                             const CubeDesc& cd, const int32_t* __restrict__ at,
                                             int nt, float scale) {
  const int D = cd.D;
  const int L = cd.L;
  const int total = nt * L;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int tt, l;
    if (cd.Lmask >= 0) {
      tt = e >> ilog2_pow2(L);
      l = e & cd.Lmask;
    } else {
      tt = e / L;
      l = e - tt * L;
    }
    const int32_t* row = at + tt * 2 * D;
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
    float2 s[5];
    s[0] = x[flat];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k < D) {
        const int64_t step = (n[k] + 1 == (uint32_t)cd.dims[k])
                                 ? -(int64_t)(cd.dims[k] - 1) * cd.stride[k]
                                 : cd.stride[k];
        s[k + 1] = x[flat + step];
      }
    }
    float2* base = dst + (int64_t)tt * (D + 1) * L + l;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      if (i <= D) base[i * L] = c_scale(s[i], scale);
    }
  }
}

}  // namespace fpssft
