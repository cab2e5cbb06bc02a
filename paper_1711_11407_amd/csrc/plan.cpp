// Host side of the FPS-SFT C ABI: validation, line schedules, FFT
// factorisations, twiddle tables, plans (device tables + workspace), the
// launch sequences of the plain, batched, line-FFT and adjoint entry points,
// and the HIP graph of the batched path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/fpssft.h"
#include "launch.h"
#include "types.h"

using fpssft::LaunchCtx;

namespace {

// ---------------------------------------------------------------------------
// Exact integer helpers.
// ---------------------------------------------------------------------------
int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a < 0 ? -a : a;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// L = LCM(N_k) (Lemma 1); returns -1 if it exceeds `cap`.
int64_t lcm_dims(const int32_t* dims, int D, int64_t cap) {
  int64_t L = 1;
  for (int k = 0; k < D; ++k) {
    L = L / gcd64(L, dims[k]) * dims[k];
    if (L > cap) return -1;
  }
  return L;
}

constexpr int64_t kMaxL = 65536;

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood 2014): output i of the stream started at
// `seed` is the published mix of seed + (i+1) * golden gamma.
// ---------------------------------------------------------------------------
uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// floor(z * n / 2^64)
uint32_t draw_below(uint64_t z, uint32_t n) {
  return (uint32_t)(((unsigned __int128)z * n) >> 64);
}

fpssft_status validate(const fpssft_desc* d, int32_t* L_out, int32_t* T_out) {
  if (!d) return FPSSFT_ERR_INVALID_ARG;
  if (d->ndim < 1 || d->ndim > FPSSFT_MAX_D) return FPSSFT_ERR_INVALID_ARG;
  int64_t N = 1;
  for (int k = 0; k < d->ndim; ++k) {
    if (d->dims[k] < 1) return FPSSFT_ERR_INVALID_ARG;
    N *= d->dims[k];
    if (N >= (int64_t(1) << 40)) return FPSSFT_ERR_UNSUPPORTED;
  }
  if (d->max_k < 1 || d->max_k > FPS_MAX_K || d->max_iters < 0) return FPSSFT_ERR_INVALID_ARG;
  if (!std::isfinite(d->zero_thresh) || d->zero_thresh < 0.f) return FPSSFT_ERR_INVALID_ARG;
  if (!std::isfinite(d->mag_rel_tol) || d->mag_rel_tol < 0.f) return FPSSFT_ERR_INVALID_ARG;
  if (!std::isfinite(d->grid_tol)) return FPSSFT_ERR_INVALID_ARG;
  if (d->schedule && d->max_iters == 0) return FPSSFT_ERR_INVALID_ARG;
  if (d->flags & ~(FPSSFT_FLAG_AXIS_SCHEDULE | FPSSFT_FLAG_AMP_AVERAGE | FPSSFT_FLAG_LITERAL_PEEL |
                   FPSSFT_FLAG_DETERMINISTIC))
    return FPSSFT_ERR_INVALID_ARG;
  const int64_t L = lcm_dims(d->dims, d->ndim, kMaxL);
  if (L < 0) return FPSSFT_ERR_UNSUPPORTED;
  for (int k = 0; k < d->ndim; ++k)
    if ((int64_t)d->dims[k] * L >= (int64_t(1) << 31)) return FPSSFT_ERR_UNSUPPORTED;
  int64_t T = d->max_iters;
  if (T == 0) T = std::max<int64_t>(1, N / ((int64_t)(d->ndim + 1) * L));
  if (T > (int64_t(1) << 24)) return FPSSFT_ERR_UNSUPPORTED;
  if (d->schedule) {
    for (int64_t t = 0; t < T; ++t)
      for (int s = 0; s < 2; ++s)
        for (int k = 0; k < d->ndim; ++k) {
          const int32_t v = d->schedule[(t * 2 + s) * d->ndim + k];
          if (v < 0 || v >= d->dims[k]) return FPSSFT_ERR_INVALID_ARG;
        }
  }
  if (L_out) *L_out = (int32_t)L;
  if (T_out) *T_out = (int32_t)T;
  return FPSSFT_OK;
}

void generate_schedule(const fpssft_desc* d, int32_t L, int32_t T, int32_t* at) {
  const int D = d->ndim;
  const bool axis = (d->flags & FPSSFT_FLAG_AXIS_SCHEDULE) != 0;
  uint64_t ctr = 0;
  for (int32_t t = 0; t < T; ++t) {
    int32_t* row = at + (int64_t)t * 2 * D;
    if (axis) {
      // alpha = e_{t mod D} (reduced mod N_k for a side of 1)
      for (int k = 0; k < D; ++k) row[k] = (k == t % D ? 1 : 0) % d->dims[k];
    } else {
      for (;;) {
        int64_t g = 0;
        for (int k = 0; k < D; ++k) {
          row[k] = (int32_t)draw_below(splitmix64(d->seed, ctr++), (uint32_t)d->dims[k]);
          g = gcd64(g, (int64_t)(L / d->dims[k]) * row[k]);
        }
        if (g == 1) break;
      }
    }
    for (int k = 0; k < D; ++k)
      row[D + k] = (int32_t)draw_below(splitmix64(d->seed, ctr++), (uint32_t)d->dims[k]);
  }
}

// Stockham stage radices for length L: powers of two in chunks of at most
// `max_radix`, then odd primes ascending.
bool factor_fft(int32_t L, int max_radix, int32_t* radix, int32_t* nstages) {
  int n = L, s = 0;
  int lg = 0;
  while ((n & 1) == 0) {
    n >>= 1;
    ++lg;
  }
  const int lgr = max_radix >= 8 ? 3 : (max_radix >= 4 ? 2 : 1);
  while (lg > 0) {
    const int take = std::min(lg, lgr);
    if (s >= FPSSFT_MAX_STAGES) return false;
    radix[s++] = 1 << take;
    lg -= take;
  }
  for (int p = 3; n > 1; p += 2) {
    while (n % p == 0) {
      if (s >= FPSSFT_MAX_STAGES) return false;
      radix[s++] = p;
      n /= p;
    }
    if ((int64_t)p * p > n && n > 1) {
      if (s >= FPSSFT_MAX_STAGES) return false;
      radix[s++] = n;
      n = 1;
    }
  }
  *nstages = s;
  return true;
}

struct StagedTable {
  // A device table whose contents follow host arrays of pointers. The
  // pinned staging copy is reused only after the previous upload from it
  // has executed.
  void* dev = nullptr;
  void* pinned = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool valid = false;
  std::vector<char> last;

  hipError_t init(size_t nbytes) {
    bytes = nbytes;
    hipError_t e = hipMalloc(&dev, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) return e;
    e = hipHostMalloc(&pinned, std::max<size_t>(bytes, 16), hipHostMallocDefault);
    if (e != hipSuccess) return e;
    return hipEventCreateWithFlags(&done, hipEventDisableTiming);
  }
  // Upload `src` if it differs from the last upload. Stream-ordered.
  hipError_t update(const void* src, hipStream_t st) {
    if (valid && last.size() == bytes && std::memcmp(last.data(), src, bytes) == 0) return hipSuccess;
    hipError_t e = hipEventSynchronize(done);
    if (e != hipSuccess) return e;
    std::memcpy(pinned, src, bytes);
    e = hipMemcpyAsync(dev, pinned, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    e = hipEventRecord(done, st);
    if (e != hipSuccess) return e;
    last.assign((const char*)src, (const char*)src + bytes);
    valid = true;
    return hipSuccess;
  }
  void release() {
    if (done) hipEventSynchronize(done), hipEventDestroy(done);
    if (dev) hipFree(dev);
    if (pinned) hipHostFree(pinned);
    dev = pinned = nullptr;
    done = nullptr;
  }
};

fpssft_status hip_status(hipError_t e) {
  if (e == hipSuccess) return FPSSFT_OK;
  if (e == hipErrorOutOfMemory) return FPSSFT_ERR_NOMEM;
  if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return FPSSFT_ERR_NO_DEVICE;
  if (std::getenv("FPSSFT_LOG")) std::fprintf(stderr, "fpssft: HIP error %s\n", hipGetErrorString(e));
  return FPSSFT_ERR_HIP;
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return hip_status(_e);        \
  } while (0)

}  // namespace

// Cubes served by one kernel instantiation: a contiguous slice of the
// order array (shortest lines first, then smallest cubes) and of the
// line-FFT item list.
struct Group {
  fpssft::KernelKey key;
  int32_t L = 0;        // line length of its cubes (one-length groups), else 0
  int lines_threads = 0;  // line gather + FFT work-group size
  int first = 0;        // into order[]
  int count = 0;
  int item_first = 0;   // into items[]
  int item_count = 0;
  int grid = 0;         // persistent solve grid
  int threads = 0;      // solve work-group size
  size_t lds_solve = 0;
  size_t lds_bwd = 0;
  size_t lds_lines = 0;
  int lines_grid = 0;   // persistent line-FFT grid (multiple of 8)
  int32_t maxL = 1;         // longest line of the group's regular cubes
  int32_t maxL_serial = 0;  // longest line of its long-line cubes
  int64_t max_N = 0;
};

struct fpssft_plan_st {
  int device = 0;
  int B = 0;
  int ncu = 0;
  size_t lds_max = 0;
  fpssft_tuning tune{};
  std::vector<CubeDesc> descs;
  std::vector<int32_t> sched;
  std::vector<float2> tw;
  std::vector<int> group_of;   // per cube
  std::vector<int> cthreads;   // per cube: solve work-group size
  std::vector<int> clthreads;  // per cube: line-kernel work-group size
  std::vector<int> clsamples;  // per cube: line-kernel item size (samples)
  std::vector<Group> groups;
  // concurrent group launches: side streams joined back to the caller's
  static constexpr int kSide = 3;
  hipStream_t side[kSide] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kSide] = {};
  int64_t spec_elems = 0;
  LaunchCtx ctx{};
  CubeDesc* d_descs = nullptr;
  int32_t* d_sched = nullptr;
  float2* d_tw = nullptr;
  // plain path
  float2* d_pre = nullptr;
  // record stores of the cubes whose records do not fit in LDS
  char* d_recws = nullptr;
  // the static scratch array of the allocation-free entry point on this
  // plan's device
  void* noalloc_scratch = nullptr;
  bool lines_too_long = false;  // some cube's lines exceed the line kernel's LDS
  // batched path
  int32_t* d_order = nullptr;
  int* d_queue = nullptr;
  StagedTable xs_tab, outs_tab, ga_tab, gx_tab, len_tab;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;
  // line-FFT over the whole budget
  std::vector<LineItem> items;
  LineItem* d_items = nullptr;
  std::vector<int32_t> ranges;  // per group: 8 x [lo, hi) item ranges, one per XCD
  int32_t* d_ranges = nullptr;
  int* d_lqueue = nullptr;      // per group: 8 queue counters
  int64_t max_N = 0;
};

namespace {

// Cubes the one-wave-per-line path can take (power-of-two 64 <= L <= 512).
// The time-domain construction-subtraction runs on the block path only.
bool wave_eligible(const CubeDesc& c) {
  return c.Lmask >= 0 && c.L >= 64 && c.L <= 512 && !(c.flags & FPS_LITERAL_PEEL);
}

// Threads per work-group of the solve kernels for D dimensions: the tuned
// count, and for D >= 3 at least D+3 waves, so that two waves link records
// while the D+1 line waves transform (3-D: 117 against 126 us on a 128^3
// cube).
int solve_threads(int tuned, int D) {
  return D >= 3 ? std::max(tuned, std::min(512, 64 * (D + 3))) : tuned;
}

// The one-wave-per-line solve path: an eligible line and at least D+1 waves
// in a work-group of `threads`.
bool uses_wave_path(int threads, const CubeDesc& c) {
  return wave_eligible(c) && threads / 64 >= c.D + 1;
}

size_t solve_lds_bytes(const CubeDesc& c, int rec_cap, bool wave) {
  // The layout of carve_solve_lds: the D+1 spectra, and on the block path a
  // second buffer (the FFT's) or, with long lines, one line of scratch that
  // also holds the bin-list words; the twiddles; the constructed spectra of
  // the time-domain construction-subtraction; the bins' largest amplitudes
  // and entry counts (2 x L ints, each rounded to 8 bytes) and the
  // fixed-point projection sums ((D+1) L int pairs, in the constructed
  // spectra's buffer when there is one); the record store (per slot the set
  // entry, then the frequency hash); the exchange words and counters.
  const size_t lines = (size_t)(c.D + 1) * c.L;
  size_t b;
  if (c.serial == 2) {
    b = 0;  // spectra and scratch line in the device workspace
  } else if (c.serial) {
    b = (lines + c.L) * sizeof(float2);
  } else {
    b = (lines + (wave ? 0 : lines) + c.L + ((!wave && (c.flags & FPS_LITERAL_PEEL)) ? lines : 0)) * sizeof(float2);
    b += 2 * (size_t)((c.L + 1) & ~1) * sizeof(int);
    // the sums share the constructed spectra's buffer when there is one
    if (wave || !(c.flags & FPS_LITERAL_PEEL)) b += lines * 2 * sizeof(int);
  }
  b += (size_t)fps_rec_bytes(c.D, rec_cap);
  b += 64 * sizeof(int);
  return b;
}

// Device workspace of a cube whose lines do not fit in LDS: its D+1 spectra
// and one line of scratch, rounded to 256 bytes.
size_t lines_ws_bytes(const CubeDesc& c) {
  return ((size_t)(c.D + 2) * c.L * sizeof(float2) + 255) / 256 * 256;
}

// LDS of the adjoint: the line cotangent and the FFT's second buffer (in the
// line workspace when the lines are too long for LDS), the twiddles (read
// from device memory for long lines), per detection its cotangent, its
// iteration, c_k m_k of its frequency and its bin, and per iteration (at
// most max_k of them) the first detection of its run.
size_t bwd_lds_bytes(const CubeDesc& c) {
  const size_t lines = c.serial == 2 ? 0 : (c.serial ? 2 : 3) * (size_t)c.L * sizeof(float2);
  return lines + (size_t)c.max_k * (sizeof(float2) + (2 + (size_t)c.D) * sizeof(int)) +
         (size_t)std::min(c.T, c.max_k) * sizeof(int) + 64;
}

// Line-FFT work-group LDS: two line buffers and the twiddle table.
size_t lines_lds_bytes(int D, int L) { return (2 * (size_t)(D + 1) + 1) * L * sizeof(float2); }

size_t lines_single_lds_bytes(const CubeDesc& c) {
  return c.serial ? 2 * (size_t)c.L * sizeof(float2) : lines_lds_bytes(c.D, c.L);
}

fpssft::KernelKey key_of(const fpssft_plan_t p, int c) {
  const CubeDesc& cd = p->descs[c];
  const bool pow2 = cd.Lmask >= 0;
  return fpssft::KernelKey{cd.D, pow2, cd.rec_lds > 0, uses_wave_path(p->cthreads[c], cd), cd.serial == 2};
}

void destroy_plan(fpssft_plan_t p) {
  if (!p) return;
  int prev = -1;
  const bool restore = hipGetDevice(&prev) == hipSuccess && prev != p->device;
  hipSetDevice(p->device);
  hipDeviceSynchronize();
  if (p->gexec) hipGraphExecDestroy(p->gexec);
  if (p->graph) hipGraphDestroy(p->graph);
  if (p->cap_stream) hipStreamDestroy(p->cap_stream);
  for (int i = 0; i < fpssft_plan_st::kSide; ++i) {
    if (p->side[i]) hipStreamDestroy(p->side[i]);
    if (p->ev_join[i]) hipEventDestroy(p->ev_join[i]);
  }
  if (p->ev_fork) hipEventDestroy(p->ev_fork);
  p->xs_tab.release();
  p->outs_tab.release();
  p->ga_tab.release();
  p->gx_tab.release();
  p->len_tab.release();
  hipFree(p->d_descs);
  hipFree(p->d_sched);
  hipFree(p->d_tw);
  hipFree(p->d_pre);
  hipFree(p->d_recws);
  hipFree(p->d_order);
  hipFree(p->d_queue);
  hipFree(p->d_items);
  hipFree(p->d_ranges);
  hipFree(p->d_lqueue);
  delete p;
  if (restore) hipSetDevice(prev);
}

// The hot-path calls enqueue on the current device: it must be the plan's,
// or its device pointers would be used on another GPU.
bool on_plan_device(const fpssft_plan_t p) {
  int d = -1;
  return hipGetDevice(&d) == hipSuccess && d == p->device;
}

fpssft_status build_plan(const fpssft_desc* descs, int32_t batch, const fpssft_tuning* tuning,
                         fpssft_plan_t p) {
  HIP_TRY(hipGetDevice(&p->device));
  // set-up of the allocation-free entry point's scratch on this device
  HIP_TRY(fpssft::noalloc_scratch(p->device, &p->noalloc_scratch));
  int v = 0;
  HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, p->device));
  p->ncu = v;
  HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device));
  // Dynamic LDS budget; 1 KiB stays for the kernels' static __shared__ data.
  if (v <= 2048) return FPSSFT_ERR_UNSUPPORTED;
  p->lds_max = (size_t)v - 1024;
  p->B = batch;
  fpssft_tuning tn{256, 8, 8, 4, 256, 0, 3072, 0, 0, nullptr};
  std::vector<fpssft_shape_tuning> shapes;
  if (tuning) {
    if (tuning->block_threads) tn.block_threads = tuning->block_threads;
    if (tuning->max_radix) tn.max_radix = tuning->max_radix;
    if (tuning->chunk_iters >= 0) tn.chunk_iters = tuning->chunk_iters;
    if (tuning->lines_wg) tn.lines_wg = tuning->lines_wg;
    if (tuning->lines_threads) tn.lines_threads = tuning->lines_threads;
    tn.direct_launch = tuning->direct_launch != 0;
    if (tuning->lines_samples) tn.lines_samples = tuning->lines_samples;
    tn.group_by_length = tuning->group_by_length != 0;
    if (tuning->nshapes < 0 || (tuning->nshapes > 0 && !tuning->shapes)) return FPSSFT_ERR_INVALID_ARG;
    for (int i = 0; i < tuning->nshapes; ++i) {
      const fpssft_shape_tuning& sh = tuning->shapes[i];
      if (sh.ndim < 1 || sh.ndim > FPSSFT_MAX_D || sh.line_length < 1) return FPSSFT_ERR_INVALID_ARG;
      if (sh.block_threads && (sh.block_threads < 64 || sh.block_threads > 512 || sh.block_threads % 64))
        return FPSSFT_ERR_INVALID_ARG;
      if (sh.lines_samples < 0) return FPSSFT_ERR_INVALID_ARG;
      shapes.push_back(sh);
    }
  }
  tn.nshapes = 0;
  tn.shapes = nullptr;
  if (tn.block_threads < 64 || tn.block_threads > 512 || tn.block_threads % 64) return FPSSFT_ERR_INVALID_ARG;
  if (tn.lines_threads < 64 || tn.lines_threads > 1024 || tn.lines_threads % 64) return FPSSFT_ERR_INVALID_ARG;
  if (tn.max_radix != 2 && tn.max_radix != 4 && tn.max_radix != 8) return FPSSFT_ERR_INVALID_ARG;
  if (tn.lines_wg < 1) return FPSSFT_ERR_INVALID_ARG;
  p->tune = tn;

  std::map<int32_t, int32_t> tw_off;
  p->descs.resize(batch);
  p->cthreads.assign(batch, 0);
  p->clthreads.assign(batch, 0);
  p->clsamples.assign(batch, 0);
  int64_t max_pre = 0;
  int64_t rec_ws_bytes = 0;
  for (int32_t c = 0; c < batch; ++c) {
    const fpssft_desc& d = descs[c];
    int32_t L, T;
    fpssft_status st = validate(&d, &L, &T);
    if (st != FPSSFT_OK) return st;
    CubeDesc cd{};
    cd.D = d.ndim;
    cd.L = L;
    cd.T = T;
    cd.max_k = d.max_k;
    int64_t stride = 1;
    for (int k = d.ndim - 1; k >= 0; --k) {
      cd.stride[k] = stride;
      stride *= d.dims[k];
    }
    cd.N = stride;
    for (int k = 0; k < 4; ++k) {
      cd.dims[k] = k < d.ndim ? d.dims[k] : 1;
      cd.c[k] = k < d.ndim ? L / d.dims[k] : 1;
      cd.dmask[k] = (k < d.ndim && is_pow2(d.dims[k])) ? d.dims[k] - 1 : -1;
      if (k >= d.ndim) cd.stride[k] = 0;
    }
    cd.Lmask = is_pow2(L) ? L - 1 : -1;
    // launch shapes: the (D, L) class's tuned values over the plan-wide ones
    int bt = tn.block_threads, ls = tn.lines_samples;
    for (const fpssft_shape_tuning& sh : shapes) {
      if (sh.ndim != d.ndim || sh.line_length != L) continue;
      if (sh.block_threads) bt = sh.block_threads;
      if (sh.lines_samples) ls = sh.lines_samples;
    }
    p->cthreads[c] = solve_threads(bt, d.ndim);
    p->clthreads[c] = tn.lines_threads;
    p->clsamples[c] = ls;
    if (!factor_fft(L, tn.max_radix, cd.radix, &cd.nstages)) return FPSSFT_ERR_UNSUPPORTED;
    cd.inv_L = (float)(1.0 / (double)L);
    cd.zero_thresh = d.zero_thresh;
    cd.mag_rel_tol = d.mag_rel_tol;
    cd.grid_tol = d.grid_tol;
    cd.flags = d.flags;
    cd.sched_off = (int32_t)p->sched.size();
    if ((int64_t)p->sched.size() + (int64_t)T * 2 * d.ndim >= (int64_t(1) << 31)) return FPSSFT_ERR_UNSUPPORTED;
    p->sched.resize(p->sched.size() + (size_t)T * 2 * d.ndim);
    if (d.schedule)
      std::memcpy(p->sched.data() + cd.sched_off, d.schedule, sizeof(int32_t) * T * 2 * d.ndim);
    else
      generate_schedule(&d, L, T, p->sched.data() + cd.sched_off);
    auto it = tw_off.find(L);
    if (it == tw_off.end()) {
      const int32_t off = (int32_t)p->tw.size();
      for (int32_t k = 0; k < L; ++k) {
        const double ang = -2.0 * M_PI * (double)k / (double)L;
        p->tw.push_back(make_float2((float)std::cos(ang), (float)std::sin(ang)));
      }
      it = tw_off.emplace(L, off).first;
    }
    cd.tw_off = it->second;
    cd.spec_off = p->spec_elems;
    p->spec_elems += (int64_t)T * (d.ndim + 1) * L;
    // Lines too long for the D+1 spectra plus a second buffer and the
    // twiddles in LDS are transformed one at a time (no precomputed chunk).
    cd.serial = 0;
    cd.rec_off = -1;
    cd.lws_off = -1;
    if (!wave_eligible(cd) && solve_lds_bytes(cd, 0, false) > p->lds_max) cd.serial = 1;
    // longer still: the spectra and the scratch line in device memory
    if (cd.serial && solve_lds_bytes(cd, 0, false) > p->lds_max) {
      cd.serial = 2;
      cd.lws_off = rec_ws_bytes;
      rec_ws_bytes += (int64_t)lines_ws_bytes(cd);
    }
    if (cd.serial && (cd.flags & FPS_LITERAL_PEEL)) return FPSSFT_ERR_UNSUPPORTED;
    // the time-domain construction-subtraction needs the samples themselves
    const int32_t pre_T = (cd.serial || (cd.flags & FPS_LITERAL_PEEL)) ? 0 : std::min(T, tn.chunk_iters);
    max_pre = std::max<int64_t>(max_pre, (int64_t)pre_T * (d.ndim + 1) * L);
    p->max_N = std::max(p->max_N, cd.N);
    const bool wave = uses_wave_path(p->cthreads[c], cd);
    if (solve_lds_bytes(cd, 0, wave) > p->lds_max || (cd.serial != 2 && lines_single_lds_bytes(cd) > p->lds_max))
      return FPSSFT_ERR_UNSUPPORTED;
    // The record store stays in LDS when the cube's spectra and records fit;
    // otherwise it is a region of the plan's device workspace.
    if (solve_lds_bytes(cd, cd.max_k, wave) <= p->lds_max) {
      cd.rec_lds = cd.max_k;
    } else {
      cd.rec_lds = 0;
      cd.rec_off = rec_ws_bytes;
      rec_ws_bytes += (fps_rec_bytes(cd.D, cd.max_k) + 255) / 256 * 256;
    }
    p->descs[c] = cd;
  }

  // Group cubes by kernel instantiation; within a group, shortest lines
  // first, ties by index: short lines hold more sinusoids per bin, and their
  // long runs of cheap iterations set the makespan when started late.
  p->group_of.assign(batch, -1);
  for (int32_t c = 0; c < batch; ++c) {
    const fpssft::KernelKey k = key_of(p, c);
    const int32_t gl = tn.group_by_length ? p->descs[c].L : 0;
    int gi = -1;
    for (size_t i = 0; i < p->groups.size(); ++i) {
      const Group& g = p->groups[i];
      if (g.key == k && g.L == gl && g.threads == p->cthreads[c] && g.lines_threads == p->clthreads[c]) gi = (int)i;
    }
    if (gi < 0) {
      Group g;
      g.key = k;
      g.L = gl;
      g.threads = p->cthreads[c];
      g.lines_threads = p->clthreads[c];
      p->groups.push_back(g);
      gi = (int)p->groups.size() - 1;
    }
    p->group_of[c] = gi;
  }
  std::vector<int32_t> order(batch);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    if (p->group_of[a] != p->group_of[b]) return p->group_of[a] < p->group_of[b];
    const int64_t ca = (int64_t)(p->descs[a].D + 1) * p->descs[a].L;
    const int64_t cb = (int64_t)(p->descs[b].D + 1) * p->descs[b].L;
    if (ca != cb) return ca < cb;
    // for one line length, fewer samples means fewer distinct lines through
    // the cube, so collisions recur and the chain of iterations runs longer
    return p->descs[a].N < p->descs[b].N;
  });
  for (size_t gi = 0; gi < p->groups.size(); ++gi) {
    Group& g = p->groups[gi];
    g.first = -1;
    for (int i = 0; i < batch; ++i) {
      if (p->group_of[order[i]] != (int)gi) continue;
      if (g.first < 0) g.first = i;
      ++g.count;
      const CubeDesc& cd = p->descs[order[i]];
      g.lds_solve = std::max(g.lds_solve, solve_lds_bytes(cd, cd.rec_lds, g.key.wave));
      g.lds_bwd = std::max(g.lds_bwd, bwd_lds_bytes(cd));
      g.max_N = std::max(g.max_N, cd.N);
    }
    // Line-FFT items of this group, cube by cube in order: runs of at most
    // lines_wg consecutive iterations.
    g.item_first = (int)p->items.size();
    for (int i = g.first; i < g.first + g.count; ++i) {
      const int32_t c = order[i];
      const CubeDesc& cd = p->descs[c];
      // the line kernel keeps two lines in LDS: longer ones get no items
      if (lines_single_lds_bytes(cd) > p->lds_max) {
        p->lines_too_long = true;
        continue;
      }
      if (cd.serial)
        g.maxL_serial = std::max(g.maxL_serial, cd.L);
      else
        g.maxL = std::max(g.maxL, cd.L);
      // iterations per item: about lines_samples samples, else lines_wg
      const int32_t ls = p->clsamples[c];
      const int32_t wg = ls > 0 ? std::max<int32_t>(1, ls / ((cd.D + 1) * cd.L)) : tn.lines_wg;
      for (int32_t t = 0; t < cd.T; t += wg) {
        LineItem li{};
        li.cube = c;
        li.t0 = t;
        li.count = std::min(wg, cd.T - t);
        li.out_off = cd.spec_off + (int64_t)t * (cd.D + 1) * cd.L;
        p->items.push_back(li);
      }
    }
    g.item_count = (int)p->items.size() - g.item_first;
    g.lds_lines = std::max(lines_lds_bytes(g.key.D, g.maxL), 2 * (size_t)g.maxL_serial * sizeof(float2));
    if (g.lds_lines > p->lds_max) return FPSSFT_ERR_UNSUPPORTED;
    // Eight contiguous item ranges of about equal work ((D+1) L per iteration).
    {
      int64_t total = 0;
      for (int i = 0; i < g.item_count; ++i) {
        const LineItem& li = p->items[g.item_first + i];
        total += (int64_t)li.count * (p->descs[li.cube].D + 1) * p->descs[li.cube].L;
      }
      int64_t acc = 0;
      int x = 0;
      int lo = 0;
      for (int i = 0; i < g.item_count && x < 7; ++i) {
        const LineItem& li = p->items[g.item_first + i];
        acc += (int64_t)li.count * (p->descs[li.cube].D + 1) * p->descs[li.cube].L;
        if (acc * 8 >= total * (x + 1)) {
          p->ranges.push_back(lo);
          p->ranges.push_back(i + 1);
          lo = i + 1;
          ++x;
        }
      }
      for (; x < 8; ++x) {
        p->ranges.push_back(lo);
        p->ranges.push_back(x == 7 ? g.item_count : lo);
        lo = x == 7 ? g.item_count : lo;
      }
    }
    for (fpssft::KernelKind kind : {fpssft::KernelKind::kLines, fpssft::KernelKind::kSolvePlain,
                                    fpssft::KernelKind::kSolveBatched, fpssft::KernelKind::kBackward}) {
      HIP_TRY(hipFuncSetAttribute(fpssft::kernel_ptr(kind, g.key), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)p->lds_max));
    }
    int occ = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &occ, fpssft::kernel_ptr(fpssft::KernelKind::kSolveBatched, g.key), g.threads, g.lds_solve));
    if (occ < 1) return FPSSFT_ERR_UNSUPPORTED;
    g.grid = (int)std::max<int64_t>(1, std::min<int64_t>(g.count, (int64_t)occ * p->ncu));
    int locc = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &locc, fpssft::kernel_ptr(fpssft::KernelKind::kLines, g.key), g.lines_threads, g.lds_lines));
    if (locc < 1) return FPSSFT_ERR_UNSUPPORTED;
    const int64_t lg = std::min<int64_t>((int64_t)locc * p->ncu, ((int64_t)g.item_count + 7) / 8 * 8);
    g.lines_grid = (int)std::max<int64_t>(8, lg / 8 * 8);
  }

  HIP_TRY(hipMalloc(&p->d_descs, sizeof(CubeDesc) * batch));
  HIP_TRY(hipMemcpy(p->d_descs, p->descs.data(), sizeof(CubeDesc) * batch, hipMemcpyHostToDevice));
  HIP_TRY(hipMalloc(&p->d_sched, sizeof(int32_t) * std::max<size_t>(p->sched.size(), 1)));
  HIP_TRY(hipMemcpy(p->d_sched, p->sched.data(), sizeof(int32_t) * p->sched.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMalloc(&p->d_tw, sizeof(float2) * p->tw.size()));
  HIP_TRY(hipMemcpy(p->d_tw, p->tw.data(), sizeof(float2) * p->tw.size(), hipMemcpyHostToDevice));
  if (max_pre > 0) HIP_TRY(hipMalloc(&p->d_pre, sizeof(float2) * max_pre));
  if (rec_ws_bytes > 0) HIP_TRY(hipMalloc(&p->d_recws, (size_t)rec_ws_bytes));
  HIP_TRY(hipMalloc(&p->d_order, sizeof(int32_t) * batch));
  HIP_TRY(hipMemcpy(p->d_order, order.data(), sizeof(int32_t) * batch, hipMemcpyHostToDevice));
  // per group: the persistent solve's queue counter and exit counter (the
  // kernel leaves both at zero)
  HIP_TRY(hipMalloc(&p->d_queue, 2 * sizeof(int) * std::max<size_t>(p->groups.size(), 1)));
  HIP_TRY(hipMemset(p->d_queue, 0, 2 * sizeof(int) * std::max<size_t>(p->groups.size(), 1)));
  HIP_TRY(hipMalloc(&p->d_items, sizeof(LineItem) * std::max<size_t>(p->items.size(), 1)));
  HIP_TRY(hipMemcpy(p->d_items, p->items.data(), sizeof(LineItem) * p->items.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMalloc(&p->d_ranges, sizeof(int32_t) * p->ranges.size()));
  HIP_TRY(hipMemcpy(p->d_ranges, p->ranges.data(), sizeof(int32_t) * p->ranges.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMalloc(&p->d_lqueue, sizeof(int) * 8 * p->groups.size()));
  HIP_TRY(hipMemset(p->d_lqueue, 0, sizeof(int) * 8 * p->groups.size()));
  HIP_TRY(p->xs_tab.init(sizeof(void*) * batch));
  HIP_TRY(p->outs_tab.init(sizeof(OutPtrs) * batch));
  HIP_TRY(p->ga_tab.init(sizeof(void*) * batch));
  HIP_TRY(p->gx_tab.init(sizeof(void*) * batch));
  HIP_TRY(p->len_tab.init(sizeof(int64_t) * batch));
  p->ctx.descs = p->d_descs;
  p->ctx.sched = p->d_sched;
  p->ctx.tw = p->d_tw;
  p->ctx.rec_ws = p->d_recws;
  HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  if (p->groups.size() > 1) {
    // default-priority side streams for the concurrent group launches
    for (int i = 0; i < fpssft_plan_st::kSide; ++i) {
      HIP_TRY(hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&p->ev_join[i], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
  }
  return FPSSFT_OK;
}

bool check_out(const fpssft_out* o) {
  return o && o->freqs && o->amps && o->rec_iter && o->rec_bin && o->rec_sin && o->info;
}

OutPtrs to_ptrs(const fpssft_out& o) {
  OutPtrs p;
  p.freqs = o.freqs;
  p.amps = o.amps;
  p.rec_iter = o.rec_iter;
  p.rec_bin = o.rec_bin;
  p.rec_sin = o.rec_sin;
  p.info = o.info;
  return p;
}

// Runs launch(group index, stream) for every group: on `st` when there is
// one, else concurrently, the first on `st` and the others on the side
// streams, forked from `st` by an event and joined back into it (inside a
// stream capture, the side streams become parallel branches of the graph).
template <class Launch>
fpssft_status launch_groups(fpssft_plan_t p, hipStream_t st, Launch&& launch) {
  const int ng = (int)p->groups.size();
  if (ng <= 1 || !p->ev_fork) {
    for (int gi = 0; gi < ng; ++gi) HIP_TRY(launch(gi, st));
    return FPSSFT_OK;
  }
  const int nside = std::min(fpssft_plan_st::kSide, ng - 1);
  HIP_TRY(hipEventRecord(p->ev_fork, st));
  for (int i = 0; i < nside; ++i) HIP_TRY(hipStreamWaitEvent(p->side[i], p->ev_fork, 0));
  for (int gi = 0; gi < ng; ++gi) HIP_TRY(launch(gi, gi == 0 ? st : p->side[(gi - 1) % fpssft_plan_st::kSide]));
  for (int i = 0; i < nside; ++i) {
    HIP_TRY(hipEventRecord(p->ev_join[i], p->side[i]));
    HIP_TRY(hipStreamWaitEvent(st, p->ev_join[i], 0));
  }
  return FPSSFT_OK;
}

}  // namespace

extern "C" {

const char* fpssft_strerror(int32_t s) {
  switch (s) {
    case FPSSFT_OK: return "ok";
    case FPSSFT_INCOMPLETE: return "incomplete: iteration budget reached with a nonzero residual";
    case FPSSFT_CAPACITY: return "capacity: the record list is full";
    case FPSSFT_ERR_INVALID_ARG: return "invalid argument";
    case FPSSFT_ERR_UNSUPPORTED: return "valid but unsupported by the library (LDS or index range)";
    case FPSSFT_ERR_HIP: return "HIP runtime error";
    case FPSSFT_ERR_NOMEM: return "out of device memory";
    case FPSSFT_ERR_NO_DEVICE: return "no HIP device";
    default: return "unknown status";
  }
}

int32_t fpssft_abi_version(void) { return FPSSFT_ABI_VERSION; }

fpssft_status fpssft_validate(const fpssft_desc* desc, int32_t* line_length, int32_t* max_iters) {
  return validate(desc, line_length, max_iters);
}

fpssft_status fpssft_schedule_generate(const fpssft_desc* desc, int32_t T, int32_t* alpha_tau) {
  if (!desc) return FPSSFT_ERR_INVALID_ARG;
  int32_t L, Tm;
  fpssft_desc d = *desc;
  d.schedule = nullptr;
  fpssft_status st = validate(&d, &L, &Tm);
  if (st != FPSSFT_OK) return st;
  if (T < 0 || (T > 0 && !alpha_tau)) return FPSSFT_ERR_INVALID_ARG;
  generate_schedule(&d, L, T, alpha_tau);
  return FPSSFT_OK;
}

fpssft_status fpssft_plan_create(const fpssft_desc* descs, int32_t batch, const fpssft_tuning* tuning,
                                 fpssft_plan_t* plan) {
  if (!descs || batch < 1 || !plan) return FPSSFT_ERR_INVALID_ARG;
  *plan = nullptr;
  for (int32_t c = 0; c < batch; ++c) {
    fpssft_status st = validate(&descs[c], nullptr, nullptr);
    if (st != FPSSFT_OK) return st;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return FPSSFT_ERR_NO_DEVICE;
  fpssft_plan_t p = new (std::nothrow) fpssft_plan_st();
  if (!p) return FPSSFT_ERR_NOMEM;
  fpssft_status st = build_plan(descs, batch, tuning, p);
  if (st != FPSSFT_OK) {
    destroy_plan(p);
    return st;
  }
  *plan = p;
  return FPSSFT_OK;
}

fpssft_status fpssft_plan(const fpssft_desc* descs, int32_t batch, fpssft_plan_t* plan) {
  return fpssft_plan_create(descs, batch, nullptr, plan);
}

fpssft_status fpssft_plan_destroy(fpssft_plan_t plan) {
  if (!plan) return FPSSFT_ERR_INVALID_ARG;
  destroy_plan(plan);
  return FPSSFT_OK;
}

fpssft_status fpssft_plan_get_schedule(fpssft_plan_t p, int32_t cube, int32_t* alpha_tau) {
  if (!p || cube < 0 || cube >= p->B || !alpha_tau) return FPSSFT_ERR_INVALID_ARG;
  const CubeDesc& cd = p->descs[cube];
  std::memcpy(alpha_tau, p->sched.data() + cd.sched_off, sizeof(int32_t) * cd.T * 2 * cd.D);
  return FPSSFT_OK;
}

fpssft_status fpssft_plan_cube_info(fpssft_plan_t p, int32_t cube, int32_t* line_length, int32_t* max_iters,
                                    int64_t* spectra_offset) {
  if (!p || cube < 0 || cube >= p->B) return FPSSFT_ERR_INVALID_ARG;
  const CubeDesc& cd = p->descs[cube];
  if (line_length) *line_length = cd.L;
  if (max_iters) *max_iters = cd.T;
  if (spectra_offset) *spectra_offset = cd.spec_off;
  return FPSSFT_OK;
}

int64_t fpssft_plan_spectra_elems(fpssft_plan_t p) { return p ? p->spec_elems : -1; }

fpssft_status fpssft_execute(fpssft_plan_t p, int32_t cube, const void* x, const fpssft_out* out,
                             void* stream) {
  if (!p || cube < 0 || cube >= p->B || !x || !check_out(out)) return FPSSFT_ERR_INVALID_ARG;
  if (!on_plan_device(p)) return FPSSFT_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const CubeDesc& cd = p->descs[cube];
  const fpssft::KernelKey key = key_of(p, cube);
  const Group& g = p->groups[p->group_of[cube]];
  const int pre = (cd.serial || (cd.flags & FPS_LITERAL_PEEL)) ? 0 : std::min(cd.T, p->tune.chunk_iters);
  if (pre > 0) {
    HIP_TRY(fpssft::launch_lines_single(p->ctx, key, cube, (const float2*)x, 0, pre, p->d_pre, cd.L,
                                        lines_single_lds_bytes(cd), p->clthreads[cube], st));
  }
  char* rec = cd.rec_lds ? nullptr : p->d_recws + cd.rec_off;
  char* lws = cd.lws_off >= 0 ? p->d_recws + cd.lws_off : nullptr;
  HIP_TRY(fpssft::launch_solve_plain(p->ctx, key, cube, (const float2*)x, to_ptrs(*out), p->d_pre, pre, rec, lws,
                                     g.lds_solve, g.threads, st));
  return FPSSFT_OK;
}

fpssft_status fpssft_execute_noalloc(fpssft_plan_t p, int32_t cube, const void* x, const fpssft_out* out,
                                     void* stream) {
  if (!p || cube < 0 || cube >= p->B || !x || !check_out(out)) return FPSSFT_ERR_INVALID_ARG;
  if (!on_plan_device(p)) return FPSSFT_ERR_INVALID_ARG;
  const CubeDesc& cd = p->descs[cube];
  const int pre = (cd.serial || (cd.flags & FPS_LITERAL_PEEL)) ? 0 : std::min(cd.T, p->tune.chunk_iters);
  // the pre-chunk spectra, the record store when it is not in LDS, then the
  // line workspace when the lines are not
  const size_t pre_span = ((size_t)pre * (cd.D + 1) * cd.L * sizeof(float2) + 255) / 256 * 256;
  const size_t rec_bytes = cd.rec_lds ? 0 : ((size_t)fps_rec_bytes(cd.D, cd.max_k) + 255) / 256 * 256;
  const size_t lws_bytes = cd.lws_off >= 0 ? lines_ws_bytes(cd) : 0;
  if (pre_span + rec_bytes + lws_bytes > fpssft::kNoAllocScratchBytes) return FPSSFT_ERR_UNSUPPORTED;
  char* base = (char*)p->noalloc_scratch;
  float2* pre_buf = (float2*)base;
  char* rec = cd.rec_lds ? nullptr : base + pre_span;
  char* lws = cd.lws_off >= 0 ? base + pre_span + rec_bytes : nullptr;
  hipStream_t st = (hipStream_t)stream;
  const fpssft::KernelKey key = key_of(p, cube);
  const Group& g = p->groups[p->group_of[cube]];
  if (pre > 0) {
    HIP_TRY(fpssft::launch_lines_single(p->ctx, key, cube, (const float2*)x, 0, pre, pre_buf, cd.L,
                                        lines_single_lds_bytes(cd), p->clthreads[cube], st));
  }
  HIP_TRY(fpssft::launch_solve_plain(p->ctx, key, cube, (const float2*)x, to_ptrs(*out), pre_buf, pre, rec, lws,
                                     g.lds_solve, g.threads, st));
  return FPSSFT_OK;
}

fpssft_status fpssft_execute_batched(fpssft_plan_t p, const void* const* xs, const fpssft_out* outs,
                                     void* stream) {
  if (!p || !xs || !outs) return FPSSFT_ERR_INVALID_ARG;
  if (!on_plan_device(p)) return FPSSFT_ERR_INVALID_ARG;
  std::vector<OutPtrs> op(p->B);
  for (int c = 0; c < p->B; ++c) {
    if (!xs[c] || !check_out(&outs[c])) return FPSSFT_ERR_INVALID_ARG;
    op[c] = to_ptrs(outs[c]);
  }
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(p->xs_tab.update(xs, st));
  HIP_TRY(p->outs_tab.update(op.data(), st));
  auto solve = [&](int gi, hipStream_t s) {
    const Group& g = p->groups[gi];
    return fpssft::launch_solve_batched(p->ctx, g.key, (const float2* const*)p->xs_tab.dev,
                                        (const OutPtrs*)p->outs_tab.dev, p->d_order + g.first, g.count,
                                        p->d_queue + 2 * gi, g.grid, g.lds_solve, g.threads, s);
  };
  if (p->tune.direct_launch) {
    // The persistent launches straight on the stream (concurrent ones on
    // side streams joined back to it): for a single launch a graph saves
    // nothing, and its replay leaves the GPU idle for several microseconds.
    return launch_groups(p, st, solve);
  }
  if (!p->gexec) {
    // One graph: one persistent launch per group, as parallel branches
    // (each launch finds its queue counters at zero and leaves them so).
    HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    const fpssft_status r = launch_groups(p, p->cap_stream, solve);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(p->cap_stream, &graph);
    if (r != FPSSFT_OK) {
      if (graph) hipGraphDestroy(graph);
      return r;
    }
    if (e2 != hipSuccess) return hip_status(e2);
    p->graph = graph;
    HIP_TRY(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
  }
  HIP_TRY(hipGraphLaunch(p->gexec, st));
  return FPSSFT_OK;
}

fpssft_status fpssft_lines_fft(fpssft_plan_t p, int32_t cube, const void* x, int32_t t0, int32_t count,
                               void* spectra, void* stream) {
  if (!p || cube < 0 || cube >= p->B || !x || !spectra) return FPSSFT_ERR_INVALID_ARG;
  if (!on_plan_device(p)) return FPSSFT_ERR_INVALID_ARG;
  const CubeDesc& cd = p->descs[cube];
  if (t0 < 0 || count < 0 || (int64_t)t0 + count > cd.T) return FPSSFT_ERR_INVALID_ARG;
  if (lines_single_lds_bytes(cd) > p->lds_max) return FPSSFT_ERR_UNSUPPORTED;  // two lines in LDS
  if (count == 0) return FPSSFT_OK;
  HIP_TRY(fpssft::launch_lines_single(p->ctx, key_of(p, cube), cube, (const float2*)x, t0, count,
                                      (float2*)spectra, cd.L, lines_single_lds_bytes(cd), p->clthreads[cube],
                                      (hipStream_t)stream));
  return FPSSFT_OK;
}

fpssft_status fpssft_lines_fft_all(fpssft_plan_t p, const void* const* xs, void* spectra, void* stream) {
  if (!p || !xs || !spectra) return FPSSFT_ERR_INVALID_ARG;
  if (!on_plan_device(p)) return FPSSFT_ERR_INVALID_ARG;
  for (int c = 0; c < p->B; ++c)
    if (!xs[c]) return FPSSFT_ERR_INVALID_ARG;
  if (p->lines_too_long) return FPSSFT_ERR_UNSUPPORTED;  // the line kernel keeps two lines in LDS
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(p->xs_tab.update(xs, st));
  HIP_TRY(fpssft::launch_reset(p->d_lqueue, 8 * (int)p->groups.size(), st));
  return launch_groups(p, st, [&](int gi, hipStream_t s) {
    const Group& g = p->groups[gi];
    if (g.item_count == 0) return hipSuccess;
    return fpssft::launch_lines_items(p->ctx, g.key, p->d_items + g.item_first, p->d_ranges + 16 * gi,
                                      p->d_lqueue + 8 * gi, g.lines_grid, (const float2* const*)p->xs_tab.dev,
                                      (float2*)spectra, g.maxL, g.lds_lines, g.lines_threads, s);
  });
}

fpssft_status fpssft_amp_backward(fpssft_plan_t p, int32_t cube, const fpssft_out* fwd, const void* grad_amps,
                                  void* grad_x, void* stream) {
  if (!p || cube < 0 || cube >= p->B || !check_out(fwd) || !grad_amps || !grad_x) return FPSSFT_ERR_INVALID_ARG;
  if (!on_plan_device(p)) return FPSSFT_ERR_INVALID_ARG;
  const CubeDesc& cd = p->descs[cube];
  // the adjoint follows the line-0 amplitude of Eq. decoding
  if (bwd_lds_bytes(cd) > p->lds_max || (cd.flags & FPS_AMP_AVERAGE)) return FPSSFT_ERR_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(fpssft::launch_zero_single((float2*)grad_x, cd.N, st));
  HIP_TRY(fpssft::launch_backward_single(p->ctx, key_of(p, cube), cube, to_ptrs(*fwd), (const float2*)grad_amps,
                                         (float2*)grad_x, bwd_lds_bytes(cd), p->tune.block_threads, st));
  return FPSSFT_OK;
}

fpssft_status fpssft_amp_backward_batched(fpssft_plan_t p, const fpssft_out* fwds, const void* const* grad_amps,
                                          void* const* grad_xs, void* stream) {
  if (!p || !fwds || !grad_amps || !grad_xs) return FPSSFT_ERR_INVALID_ARG;
  if (!on_plan_device(p)) return FPSSFT_ERR_INVALID_ARG;
  std::vector<OutPtrs> op(p->B);
  std::vector<int64_t> lens(p->B);
  for (int c = 0; c < p->B; ++c) {
    if (!check_out(&fwds[c]) || !grad_amps[c] || !grad_xs[c]) return FPSSFT_ERR_INVALID_ARG;
    if (bwd_lds_bytes(p->descs[c]) > p->lds_max || (p->descs[c].flags & FPS_AMP_AVERAGE))
      return FPSSFT_ERR_UNSUPPORTED;
    op[c] = to_ptrs(fwds[c]);
    lens[c] = p->descs[c].N;
  }
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(p->outs_tab.update(op.data(), st));
  HIP_TRY(p->ga_tab.update(grad_amps, st));
  HIP_TRY(p->gx_tab.update(grad_xs, st));
  HIP_TRY(p->len_tab.update(lens.data(), st));
  HIP_TRY(fpssft::launch_zero_multi((float2* const*)p->gx_tab.dev, (const int64_t*)p->len_tab.dev, p->B,
                                    p->max_N, st));
  for (const Group& g : p->groups) {
    HIP_TRY(fpssft::launch_backward_batched(p->ctx, g.key, p->d_order + g.first, g.count,
                                            (const OutPtrs*)p->outs_tab.dev, (const float2* const*)p->ga_tab.dev,
                                            (float2* const*)p->gx_tab.dev, g.lds_bwd, p->tune.block_threads, st));
  }
  return FPSSFT_OK;
}

}  // extern "C"
