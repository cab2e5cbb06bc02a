// Device building blocks of the FPS-SFT kernels (gfx950, wave64).
//
//  * exact-integer line indexing (Eq. sample_slice): n_k(l) = [alpha_k l +
//    tau_k]_{N_k}, computed in 32-bit unsigned arithmetic (the plan checks
//    N_k * L < 2^31) and a 64-bit flat offset;
//  * a block-wide Stockham FFT over several lines held in LDS, radix 2/4/8
//    butterflies in registers and a generic radix for other prime factors,
//    twiddles read from one table W_L^k = exp(-j 2 pi k / L) with exact
//    integer exponents (Eq. hs);
//  * a register-only wave FFT for power-of-two lines of 64..512 points, its
//    cross-lane butterflies on DPP row rotations, quad permutations and the
//    gfx950 permlane swaps;
//  * a work-group barrier that orders LDS only.
//
// Everything is templated on the dimension count D and on whether the line
// length (hence every N_k, which divides it) is a power of two, so that each
// kernel instantiation holds only the code it runs: the solve loop is walked
// once per iteration and must stay small for the instruction cache.
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

// Global-memory accessors. Pointers read from tables (per-cube inputs and
// outputs) are generic to the compiler, which then emits flat instructions;
// those count against the LDS counter too, so every LDS barrier would wait
// for in-flight global loads. Address-space-1 accesses keep them apart.
#define FPS_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ float2 ld_g(const float2* p, int64_t i) {
  return __builtin_bit_cast(float2, ((const FPS_GLOBAL unsigned long long*)p)[i]);
}
__device__ __forceinline__ void st_g(float2* p, int64_t i, float2 v) {
  ((FPS_GLOBAL unsigned long long*)p)[i] = __builtin_bit_cast(unsigned long long, v);
}
__device__ __forceinline__ int32_t ld_gi(const int32_t* p, int64_t i) { return ((const FPS_GLOBAL int32_t*)p)[i]; }
// Elements i and i+1 in one 16-byte load (8-byte aligned).
typedef float fps_f4a8 __attribute__((ext_vector_type(4), aligned(8)));
__device__ __forceinline__ void ld_g_pair(const float2* p, int64_t i, float2& u, float2& v) {
  const fps_f4a8 q = *(const FPS_GLOBAL fps_f4a8*)((const FPS_GLOBAL char*)p + i * 8);
  u = make_float2(q.x, q.y);
  v = make_float2(q.z, q.w);
}
// Elements i and i+1 in one 16-byte store (8-byte aligned).
__device__ __forceinline__ void st_g_pair(float2* p, int64_t i, float2 u, float2 v) {
  *(FPS_GLOBAL fps_f4a8*)((FPS_GLOBAL char*)p + i * 8) = fps_f4a8{u.x, u.y, v.x, v.y};
}
__device__ __forceinline__ void st_gi(int32_t* p, int64_t i, int32_t v) { ((FPS_GLOBAL int32_t*)p)[i] = v; }

// x mod n for x < 2^32 (n a power of two when kPow2).
template <bool kPow2>
__device__ __forceinline__ uint32_t umod(uint32_t x, uint32_t n) {
  return kPow2 ? (x & (n - 1u)) : (x % n);
}

__device__ __forceinline__ int ilog2_pow2(uint32_t v) { return 31 - __clz(v); }

// Per-cube geometry, uniform across the work-group (scalar registers).
template <int D>
struct Geo {
  uint32_t L;
  uint32_t dims[D];
  uint32_t c[D];  // L / N_k
  int64_t stride[D];
};

template <int D>
__device__ __forceinline__ Geo<D> load_geo(const CubeDesc& cd) {
  Geo<D> g;
  g.L = (uint32_t)cd.L;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    g.dims[k] = (uint32_t)cd.dims[k];
    g.c[k] = (uint32_t)cd.c[k];
    g.stride[k] = cd.stride[k];
  }
  return g;
}

// Flat offset of sample l of the line with slope/offset `row` ([2][D]) and
// the offset steps to the same sample on the shifted lines i = 1..D (the
// coordinate i-1 advanced by one, wrapping at N_{i-1}).
template <int D, bool kPow2>
__device__ __forceinline__ int64_t line_sample(const Geo<D>& g, const int32_t* row, uint32_t l,
                                               int64_t* step) {
  int64_t flat = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const uint32_t n = umod<kPow2>((uint32_t)row[k] * l + (uint32_t)row[D + k], g.dims[k]);
    flat += (int64_t)n * g.stride[k];
    step[k] = (n + 1u == g.dims[k]) ? -(int64_t)(g.dims[k] - 1u) * g.stride[k] : g.stride[k];
  }
  return flat;
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

// 16-point DFT as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.
__device__ __forceinline__ void dft16(float2* v) {
  const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f, h = 0.70710678118654752440f;
  float2 T[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    float2 a0 = v[n2], a1 = v[4 + n2], a2 = v[8 + n2], a3 = v[12 + n2];
    dft4(a0, a1, a2, a3);
    T[n2 * 4 + 0] = a0;
    T[n2 * 4 + 1] = a1;
    T[n2 * 4 + 2] = a2;
    T[n2 * 4 + 3] = a3;
  }
  // W16^m for m = n2 k1: 1, 2, 3, 2, 4, 6, 3, 6, 9
  T[1 * 4 + 1] = c_mul(T[1 * 4 + 1], make_float2(c1, -s1));
  T[1 * 4 + 2] = c_mul(T[1 * 4 + 2], make_float2(h, -h));
  T[1 * 4 + 3] = c_mul(T[1 * 4 + 3], make_float2(s1, -c1));
  T[2 * 4 + 1] = c_mul(T[2 * 4 + 1], make_float2(h, -h));
  T[2 * 4 + 2] = make_float2(T[2 * 4 + 2].y, -T[2 * 4 + 2].x);
  T[2 * 4 + 3] = c_mul(T[2 * 4 + 3], make_float2(-h, -h));
  T[3 * 4 + 1] = c_mul(T[3 * 4 + 1], make_float2(s1, -c1));
  T[3 * 4 + 2] = c_mul(T[3 * 4 + 2], make_float2(-h, -h));
  T[3 * 4 + 3] = c_mul(T[3 * 4 + 3], make_float2(-c1, s1));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 b0 = T[k1], b1 = T[4 + k1], b2 = T[8 + k1], b3 = T[12 + k1];
    dft4(b0, b1, b2, b3);
    v[k1] = b0;
    v[k1 + 4] = b1;
    v[k1 + 8] = b2;
    v[k1 + 12] = b3;
  }
}

template <int E>
__device__ __forceinline__ void dft_small(float2* v) {
  if constexpr (E == 2) dft2(v[0], v[1]);
  if constexpr (E == 4) dft4(v[0], v[1], v[2], v[3]);
  if constexpr (E == 8) dft8(v);
  if constexpr (E == 16) dft16(v);
}

// ---------------------------------------------------------------------------
// Register-only wave FFT: one wave transforms one line of L = 64 E points
// (E = 1, 2, 4, 8), forward and unnormalised, without LDS scratch. On entry
// lane q holds v[e] = x[e + E q]. Cooley-Tukey with n = e + E q and
// k = k2 + 64 k1:
//   1. for each e, the 64-point DFT over the lanes q, radix 2 with
//      decimation in frequency: six butterfly stages exchange values between
//      lanes q and q ^ h (h = 32, 16: permlane swaps; h = 8, 4, 2, 1: DPP
//      row rotations and quad permutations), leaving bin k2 = bitrev6(q) in
//      lane q;
//   2. twiddles W_L^{e k2};
//   3. the E-point DFT over e in registers gives X[k2 + 64 k1] in v[k1].
// store(k, X[k]) receives the result; each store instruction of the wave
// covers 64 consecutive bins in bit-reversed lane order. tw: W_L^k, k < L
// (W_64^j = W_L^{E j}).
// ---------------------------------------------------------------------------

// Values of lanes q and q ^ H (H = 32, 16) as (lower, upper) of the pair.
template <int H>
__device__ __forceinline__ void lane_pair_swap(float v, float& lo, float& hi) {
  const unsigned u = __float_as_uint(v);
  if constexpr (H == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    lo = __uint_as_float(r[0]);
    hi = __uint_as_float(r[1]);
  } else {
    static_assert(H == 16, "permlane swaps cover lane distances 32 and 16");
    const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    lo = __uint_as_float(r[0]);
    hi = __uint_as_float(r[1]);
  }
}

// Value of lane q ^ H for H = 8, 4, 2, 1 (within a row of 16 lanes).
template <int H>
__device__ __forceinline__ float lane_partner_dpp(float v, int lane) {
  const int u = __float_as_int(v);
  int p;
  if constexpr (H == 8) {
    p = __builtin_amdgcn_update_dpp(0, u, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (H == 4) {
    const int up = __builtin_amdgcn_update_dpp(0, u, 0x12C, 0xF, 0xF, false);  // row_ror:12: lane + 4
    const int dn = __builtin_amdgcn_update_dpp(0, u, 0x124, 0xF, 0xF, false);  // row_ror:4: lane - 4
    p = (lane & 4) ? dn : up;
  } else if constexpr (H == 2) {
    p = __builtin_amdgcn_update_dpp(0, u, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
  } else {
    static_assert(H == 1, "DPP partners cover lane distances 8, 4, 2, 1");
    p = __builtin_amdgcn_update_dpp(0, u, 0xB1, 0xF, 0xF, false);  // quad_perm 1,0,3,2
  }
  return __int_as_float(p);
}

// One decimation-in-frequency stage over lane bit H: the lower lane of a
// pair keeps lo + hi, the upper lane (lo - hi) W_{2H}^{q mod H}; w is that
// twiddle in upper lanes and 1 in lower ones, sgn -1 in upper lanes.
template <int H>
__device__ __forceinline__ float2 lane_butterfly(float2 v, float sgn, float2 w, int lane) {
  float2 t;
  if constexpr (H >= 16) {
    float lx, hx, ly, hy;
    lane_pair_swap<H>(v.x, lx, hx);
    lane_pair_swap<H>(v.y, ly, hy);
    t = make_float2(fmaf(sgn, hx, lx), fmaf(sgn, hy, ly));
  } else {
    // partner p: lower lane p + v = lo + hi, upper lane p - v = lo - hi
    const float2 p = make_float2(lane_partner_dpp<H>(v.x, lane), lane_partner_dpp<H>(v.y, lane));
    t = make_float2(fmaf(sgn, v.x, p.x), fmaf(sgn, v.y, p.y));
  }
  if constexpr (H > 1) t = c_mul(t, w);
  return t;
}

template <int E, class Store>
__device__ __forceinline__ void wave_fft_lanes(float2 (&v)[E], const float2* __restrict__ tw, Store&& store) {
  const int lane = threadIdx.x & 63;
  const int k2 = (int)(__builtin_bitreverse32((unsigned)lane) >> 26);
  // Stage twiddles W_64^{(q mod h) 32/h} (upper lanes; W^0 = 1 below) and
  // the W_L^{e k2} of step 2, read together ahead of the arithmetic.
  float2 ws[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const int h = 32 >> s;
    ws[s] = tw[(lane & h) ? E * (lane & (h - 1)) * (32 / h) : 0];
  }
  float2 w2[E];
#pragma unroll
  for (int e = 1; e < E; ++e) w2[e] = tw[e * k2];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    float2 a = v[e];
    a = lane_butterfly<32>(a, (lane & 32) ? -1.f : 1.f, ws[0], lane);
    a = lane_butterfly<16>(a, (lane & 16) ? -1.f : 1.f, ws[1], lane);
    a = lane_butterfly<8>(a, (lane & 8) ? -1.f : 1.f, ws[2], lane);
    a = lane_butterfly<4>(a, (lane & 4) ? -1.f : 1.f, ws[3], lane);
    a = lane_butterfly<2>(a, (lane & 2) ? -1.f : 1.f, ws[4], lane);
    a = lane_butterfly<1>(a, (lane & 1) ? -1.f : 1.f, make_float2(1.f, 0.f), lane);
    v[e] = e ? c_mul(a, w2[e]) : a;
  }
  dft_small<E>(v);
#pragma unroll
  for (int k1 = 0; k1 < E; ++k1) store(k2 + 64 * k1, v[k1]);
}

// ---------------------------------------------------------------------------
// One Stockham stage over `nl` lines: in -> out, radix R, Ns = product of
// the radices of earlier stages. Butterfly j of a line reads in[j + q L/R]
// (q < R), rotates input q by W_{Ns R}^{q (j mod Ns)}, takes an R-point DFT
// and writes output p to out[(j - j mod Ns) R + j mod Ns + p Ns].
// ---------------------------------------------------------------------------
template <int R, bool kPow2>
__device__ __forceinline__ void stage_fixed(const float2* __restrict__ in, float2* __restrict__ out, int nl,
                                            int L, int Ns, const float2* __restrict__ tw) {
  const int nb = L / R;
  const int total = nl * nb;
  const int ts = L / (Ns * R);
  const int lg_nb = kPow2 ? ilog2_pow2(nb) : 0;
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    int line, j, k;
    if (kPow2) {
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
    } else {
      dft8(v);
    }
    const int ob = (j - k) * R + k;
#pragma unroll
    for (int p = 0; p < R; ++p) dst[ob + p * Ns] = v[p];
  }
}

// Any radix r (odd prime factors): each butterfly output is an r-term sum
// read straight from LDS.
__device__ __forceinline__ void stage_generic(const float2* __restrict__ in, float2* __restrict__ out, int nl,
                                              int L, int Ns, int r, const float2* __restrict__ tw) {
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

// Work-group barrier that orders LDS only. Global loads issued before it stay
// in flight (HIP's __syncthreads also waits for every outstanding global
// access, which would serialise the register prefetch of the next
// iteration's samples behind each barrier).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Forward, unnormalised FFT of `nl` contiguous lines of length L held in
// buffer a (b is scratch of the same size); radix[] lists the stages (powers
// of two only when kPow2). Returns the buffer holding the result. Whole
// work-group; ends with a barrier. The buffers are in LDS, or with `gmem`
// in device memory, where each stage's barrier orders every memory access.
template <bool kPow2>
__device__ __forceinline__ float2* block_fft(float2* a, float2* b, int nl, int L, int nstages,
                                             const int32_t* radix, const float2* __restrict__ tw,
                                             bool gmem = false) {
  float2* in = a;
  float2* out = b;
  int Ns = 1;
  for (int s = 0; s < nstages; ++s) {
    const int r = radix[s];
    if (r == 8)
      stage_fixed<8, kPow2>(in, out, nl, L, Ns, tw);
    else if (r == 4)
      stage_fixed<4, kPow2>(in, out, nl, L, Ns, tw);
    else if (kPow2 || r == 2)
      stage_fixed<2, kPow2>(in, out, nl, L, Ns, tw);
    else
      stage_generic(in, out, nl, L, Ns, r, tw);
    if (gmem)
      __syncthreads();
    else
      lds_barrier();
    float2* t = in;
    in = out;
    out = t;
    Ns *= r;
  }
  return in;
}

// ---------------------------------------------------------------------------
// The D+1 samples of line position l (Eq. sample_slice): line 0 at `flat`,
// line i at flat + step[i-1]. Line D is the shift along the contiguous last
// dimension, so unless that coordinate wraps its sample is the next element:
// both come from one 16-byte load.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void load_line_samples(const float2* __restrict__ x, int64_t flat,
                                                  const int64_t* step, float2* s) {
  if (step[D - 1] == 1) {
    ld_g_pair(x, flat, s[0], s[D]);
  } else {
    s[0] = ld_g(x, flat);
    s[D] = ld_g(x, flat + step[D - 1]);
  }
#pragma unroll
  for (int k = 0; k < D - 1; ++k) s[k + 1] = ld_g(x, flat + step[k]);
}

// ---------------------------------------------------------------------------
// Line i (0..D) of one iteration alone: dst[l] = scale * sample l (Eq.
// sample_slice), row: the iteration's slope and offsets [2][D]. Whole
// work-group.
// ---------------------------------------------------------------------------
template <int D, bool kPow2>
__device__ __forceinline__ void gather_one_line(float2* __restrict__ dst, const float2* __restrict__ x,
                                                const Geo<D>& g, const int32_t* __restrict__ row, int i,
                                                float scale) {
  for (uint32_t l = threadIdx.x; l < g.L; l += blockDim.x) {
    int64_t step[D];
    int64_t flat = line_sample<D, kPow2>(g, row, l, step);
#pragma unroll
    for (int k = 0; k < D; ++k)
      if (i == k + 1) flat += step[k];
    dst[l] = c_scale(ld_g(x, flat), scale);
  }
}

// ---------------------------------------------------------------------------
// Line gather: the D+1 lines of `nt` consecutive iterations, sample l of
// line i of iteration tt written (times `scale`) to dst[(tt (D+1) + i) L + l].
// at: the schedule rows [nt][2][D]. Each thread issues the loads of kU
// positions before storing any, to keep more gathers in flight.
// ---------------------------------------------------------------------------
template <int D, bool kPow2>
__device__ __forceinline__ void gather_lines(float2* __restrict__ dst, const float2* __restrict__ x,
                                             const Geo<D>& g, const int32_t* __restrict__ at, int nt,
                                             float scale) {
  constexpr int kU = 4;
  const uint32_t L = g.L;
  const int total = nt * (int)L;
  const int B = blockDim.x;
  for (int e0 = threadIdx.x; e0 < total; e0 += kU * B) {
    float2 s[kU][D + 1];
    uint32_t tt[kU], l[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + u * B;
      tt[u] = kPow2 ? ((uint32_t)e >> ilog2_pow2(L)) : (uint32_t)e / L;
      l[u] = (uint32_t)e - tt[u] * L;
      if (e < total) {
        int64_t step[D];
        const int64_t flat = line_sample<D, kPow2>(g, at + tt[u] * 2 * D, l[u], step);
        load_line_samples<D>(x, flat, step, s[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (e0 + u * B < total) {
        float2* base = dst + (int64_t)tt[u] * (D + 1) * L + l[u];
#pragma unroll
        for (int i = 0; i <= D; ++i) base[i * L] = c_scale(s[u][i], scale);
      }
    }
  }
}

}  // namespace fpssft
