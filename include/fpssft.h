/*
 * fpssft.h — C ABI of the MI355X (gfx950) FPS-SFT hot path.
 *
 * FPS-SFT (Wang, Patel, Petropulu, arXiv 1711.11407) recovers the K on-grid
 * sinusoids (a, w) of a D-dimensional cube x from samples taken along
 * discrete lines (Sec. 2, problem statement after Eq. sigModel2). Every
 * iteration gathers D+1 lines of length L = LCM(N_0..N_{D-1}) with one random
 * slope alpha and offsets tau, tau + e_0, ..., tau + e_{D-1} (Eq. sample_slice;
 * Multi-dimensional extension), takes their 1/L-normalised L-point DFTs
 * (Eq. hs), subtracts the projections of the sinusoids recovered so far
 * (construction-subtraction, Sec. 2.2), tests each bin for 1-sparsity and
 * decodes frequency and amplitude from the phase differences between the
 * shifted lines (Eq. decoding).
 *
 * Conventions shared by every entry point
 *  - Cube layout: complex64 (interleaved float re, im), row-major, the last
 *    dimension contiguous: flat(n) = sum_k n_k * prod_{j>k} N_j.
 *  - Device pointers are HIP device addresses on the device that was
 *    current when the plan was created; they stay owned by the caller.
 *  - `stream` is a hipStream_t (NULL = the default stream). Device work is
 *    stream-ordered and asynchronous; the host never waits unless stated.
 *  - Nothing throws. Argument errors are returned synchronously and no
 *    device work is enqueued. The algorithm's outcome (OK, INCOMPLETE,
 *    CAPACITY) is written to device memory (fpssft_out.info).
 *  - A plan owns device workspace: at most one call per plan may be in
 *    flight at a time (calls on one stream are naturally serialised).
 *  - The input cube is never modified.
 */
#ifndef FPSSFT_H
#define FPSSFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FPSSFT_MAX_D 4
#define FPSSFT_ABI_VERSION 3
/* Words of fpssft_out.info. */
#define FPSSFT_INFO_LEN 8

/* Return codes (negative) and device-side outcomes (non-negative). */
typedef enum {
  FPSSFT_OK = 0,              /* device outcome: an empty residual was seen  */
  FPSSFT_INCOMPLETE = 1,      /* device outcome: T_max reached, residual != 0 */
  FPSSFT_CAPACITY = 2,        /* device outcome: max_k records, more found    */
  FPSSFT_ERR_INVALID_ARG = -1,
  FPSSFT_ERR_UNSUPPORTED = -2, /* valid, but beyond the library (LDS, 32-bit) */
  FPSSFT_ERR_HIP = -3,         /* a HIP runtime call failed                   */
  FPSSFT_ERR_NOMEM = -4,
  FPSSFT_ERR_NO_DEVICE = -5
} fpssft_status;

/* One cube's problem description (host struct, copied by the plan).
 *  ndim, dims   D in [1, FPSSFT_MAX_D] and N_k >= 1 (Sec. 2: x is defined on
 *               [N_0] x ... x [N_{D-1}]). L = LCM(N_k) (Lemma 1).
 *  max_iters    T_max; 0 selects floor(N / ((D+1) L)) but at least 1, the
 *               paper's budget of about 100% of the samples (Sec. 3).
 *  max_k        capacity of the record list, 1 .. 2^26.
 *  seed         seed of the SplitMix64 line schedule (below).
 *  zero_thresh  theta0: a bin is nonzero iff |r| > theta0 (Sec. 2.2: a
 *               nonzero bin is 1-sparse with high probability).
 *  mag_rel_tol  rho: 1-sparse needs | |r_i(m)| - |r_0(m)| | <= rho |r_0(m)|
 *               for every shifted line i (the magnitude test of Sec. 2.1).
 *  grid_tol     gamma: the decoded u_k = N_k phi / (2 pi) must be within
 *               gamma of an integer; gamma < 0 disables the check.
 *  flags        FPSSFT_FLAG_* below, OR-ed; 0 is the paper's method with
 *               the frequency-domain peel.
 *  schedule     optional host array int32 [max_iters][2][ndim]: per
 *               iteration the slope alpha then the offset tau, entries in
 *               [0, N_k). NULL: drawn from `seed` (fpssft_schedule_generate).
 *               When given, max_iters must be > 0; slopes outside Lemma 2's
 *               set are accepted (e.g. axis-only schedules). */
typedef struct {
  int32_t ndim;
  int32_t dims[FPSSFT_MAX_D];
  int32_t max_iters;
  int32_t max_k;
  uint64_t seed;
  float zero_thresh;
  float mag_rel_tol;
  float grid_tol;
  uint32_t flags;
  const int32_t* schedule;
} fpssft_desc;

/* Variants of the method (fpssft_desc.flags).
 *  AXIS_SCHEDULE  generated schedule with axis-aligned slopes: iteration t
 *                 uses alpha = e_{t mod D} (the row/column lines of the
 *                 earlier 2-D sparse FFT that Sec. 2.1 reviews, and whose
 *                 deadlock on grid-shaped supports Sec. 2.2 describes); the
 *                 offsets are drawn as in the default schedule, D draws per
 *                 iteration from the same SplitMix64 stream, and no slope is
 *                 drawn. Ignored when `schedule` is given.
 *  AMP_AVERAGE    amplitude of a decoded bin averaged over the D+1 lines,
 *                 a = (1/(D+1)) sum_i r_i(m) W_L^{q_i}, q_i = [sum_k c_k m_k
 *                 tau_k^{(i)}]_L, instead of line 0 alone (Eq. decoding uses
 *                 line 0; for noisy data the average has 1/(D+1) of the
 *                 variance). fpssft_amp_backward returns UNSUPPORTED.
 *  LITERAL_PEEL   construction-subtraction as the paper states it (Sec. 2.2):
 *                 the recovered sinusoids' line spectra are inverse
 *                 transformed and subtracted from the gathered samples
 *                 before the line DFT, instead of being subtracted from the
 *                 line spectra. Equal up to rounding; slower (two more
 *                 transforms per line). UNSUPPORTED together with lines too
 *                 long for LDS.
 *  DETERMINISTIC  bit-reproducible results. Every plan has them: the
 *                 construction-subtraction sums each bin's contributions in
 *                 64-bit fixed point, exact and independent of the order in
 *                 which the work-group's threads meet them (no float
 *                 atomics), so repeated calls on the same input give
 *                 identical bits. The flag is accepted and changes nothing. */
#define FPSSFT_FLAG_AXIS_SCHEDULE 0x1u
#define FPSSFT_FLAG_AMP_AVERAGE 0x2u
#define FPSSFT_FLAG_LITERAL_PEEL 0x4u
#define FPSSFT_FLAG_DETERMINISTIC 0x8u

/* Per-cube outputs: all DEVICE pointers, caller-owned.
 *
 * The result is the recovered set of Sec. 2.2, i.e. the set S of Eq.
 * sigModel2: distinct frequencies with nonzero amplitudes. Each iteration
 * decodes some bins; every such decoding is a detection. A frequency
 * detected again in a later iteration (a false detection in an earlier
 * iteration leaves such a residue behind) is merged into its first record:
 * its amplitude is the sum of its detections' amplitudes. A merged frequency
 * whose sum has |a| <= theta0 is not part of the set; it is listed after the
 * set (positions k .. k+kd-1) so that the detection trace stays complete.
 *  freqs     int32 [max_k][ndim]  frequency indices m_k in [0, N_k): the
 *                                 set (0..k-1) in the order of first
 *                                 detection, then the merged frequencies
 *                                 left out of it (k..k+kd-1), same order
 *  amps      complex64 [max_k]    amplitudes a of the same entries
 *                                 (Eq. decoding; sums of detections)
 *  rec_iter  int32 [max_k]        detection i: iteration
 *  rec_bin   int32 [max_k]        detection i: its bin m in that
 *                                 iteration's lines
 *  rec_sin   int32 [max_k]        detection i: index of its frequency in
 *                                 freqs / amps (< k + kd)
 *  info      int32 [FPSSFT_INFO_LEN]  k (set size), iterations executed,
 *                                 outcome, n (detections), kd (merged
 *                                 frequencies left out of the set), 0, 0, 0
 * Detections are in canonical order: iteration ascending, bin ascending;
 * max_k bounds the number of detections n (CAPACITY when more are found),
 * hence also k + kd <= n. Entries past those counts are left unchanged. */
typedef struct {
  int32_t* freqs;
  void* amps;
  int32_t* rec_iter;
  int32_t* rec_bin;
  int32_t* rec_sin;
  int32_t* info;
} fpssft_out;

/* Launch shapes for the cubes of one (D, L) class, chosen by the autotuner
 * per class; 0 in a field keeps the plan-wide value of fpssft_tuning.
 *  ndim, line_length  the class: cubes with D = ndim and L = line_length
 *  block_threads      threads per work-group of the solve kernels
 *  lines_samples      samples per work item of the line gather + FFT kernel */
typedef struct {
  int32_t ndim;
  int32_t line_length;
  int32_t block_threads;
  int32_t lines_samples;
} fpssft_shape_tuning;

/* Launch-shape choices of the autotuner (0 = library default; chunk_iters
 * is taken as given when >= 0, so pass -1 for its default).
 *  block_threads  threads per work-group of the solve and adjoint kernels
 *                 (64..512, multiple of 64); for D >= 3 the solve kernels
 *                 use at least 64 (D+3), room for two linking waves
 *  max_radix      largest FFT radix of the block (LDS) transforms: the line
 *                 gather + FFT kernel, and the solve kernels' lines that
 *                 are not power-of-two lines of 64..512 points (2, 4, 8)
 *  chunk_iters    iterations the plain path gathers and transforms ahead
 *                 in parallel before its sequential decode (>= 0)
 *  lines_wg       consecutive iterations per work item of the persistent
 *                 line gather + FFT kernel (>= 1) when lines_samples < 0
 *  lines_threads  threads per work-group of that kernel (64..1024)
 *  direct_launch  fpssft_execute_batched: 0 replays one HIP graph holding
 *                 the persistent solve launches (default), 1 launches them
 *                 on the stream directly (no graph; the launches may then be
 *                 captured into the caller's own graph)
 *  lines_samples  > 0: a work item of the line kernel takes
 *                 max(1, lines_samples / ((D+1) L)) consecutive iterations
 *                 of its cube (about that many samples, whatever the line
 *                 length); < 0: lines_wg iterations; 0: default 3072
 *  group_by_length  1: one persistent launch per kernel instantiation and
 *                 line length (and launch shape); the launches of a call
 *                 run concurrently (parallel branches of the graph, or
 *                 side streams joined back to the caller's stream);
 *                 0: one per kernel instantiation and launch shape
 *  nshapes, shapes  per-(D, L) overrides (host array, copied by the plan;
 *                 may be NULL when nshapes is 0) */
typedef struct {
  int32_t block_threads;
  int32_t max_radix;
  int32_t chunk_iters;
  int32_t lines_wg;
  int32_t lines_threads;
  int32_t direct_launch;
  int32_t lines_samples;
  int32_t group_by_length;
  int32_t nshapes;
  const fpssft_shape_tuning* shapes;
} fpssft_tuning;

typedef struct fpssft_plan_st* fpssft_plan_t;

/* ---- host-only calls (no device needed) ------------------------------- */

/* Text for a status code. Static storage; never NULL. */
const char* fpssft_strerror(int32_t status);

/* FPSSFT_ABI_VERSION of the loaded library. */
int32_t fpssft_abi_version(void);

/* Check a description. On success writes L (Lemma 1) and the effective
 * T_max to the optional outputs. INVALID_ARG for out-of-range fields;
 * UNSUPPORTED when N_k * L >= 2^31 or N >= 2^40 (index arithmetic is exact
 * 32-bit per dimension) or L > 65536. */
fpssft_status fpssft_validate(const fpssft_desc* desc, int32_t* line_length,
                              int32_t* max_iters);

/* The line schedule that `desc` (with schedule == NULL) produces: host
 * array int32 [T][2][ndim], iterations 0..T-1 (Sec. 2.2: a random slope in
 * Lemma 2's set and a random offset each iteration; with
 * FPSSFT_FLAG_AXIS_SCHEDULE, axis slopes and random offsets). One SplitMix64 stream
 * (Steele, Lea, Flood 2014) per cube, output i = mix(seed + (i+1) * 0x9E37...).
 * A draw on [0, n) is floor(z * n / 2^64). Per iteration: draw alpha_0..
 * alpha_{D-1}, redraw all D until gcd(c_0 alpha_0, ..., c_{D-1} alpha_{D-1})
 * = 1 (c_k = L / N_k; Lemma 2's set in 2-D), then draw tau_0..tau_{D-1}. */
fpssft_status fpssft_schedule_generate(const fpssft_desc* desc, int32_t T,
                                       int32_t* alpha_tau);

/* ---- plans ------------------------------------------------------------- */

/* Build a plan for `batch` cubes on the current HIP device: validates every
 * description, draws or copies the schedules, builds twiddle tables
 * W_L^k = exp(-j 2 pi k / L) (fp64 on the host, rounded to fp32) and FFT
 * factorisations, and uploads them. `tuning` may be NULL.
 * Lines whose D+1 spectra, a second buffer and the twiddles do not fit in
 * LDS (160 KB) are transformed one line at a time, with the twiddles read
 * from device memory. When even the D+1 spectra plus one line of scratch do
 * not fit ((D+2) L * 8 bytes > 160 KB, e.g. L > 6800 for D = 2), those
 * buffers move to a device workspace of the plan ((D+2) L * 8 bytes per
 * cube) and the radix passes of each line run through it.
 * fpssft_lines_fft and fpssft_lines_fft_all keep two lines in LDS
 * (2 L * 8 bytes) and return UNSUPPORTED for longer ones (L > 10240);
 * fpssft_amp_backward puts its two line buffers in the same workspace.
 * Lines are at most 65536 points (L = LCM(N_k)), and N_k L < 2^31.
 * A cube's record store (max_k slots of 16 + 4 D bytes, one per set entry,
 * and a hash of the set's frequencies, 4 bytes a slot for the smallest
 * power of two of at least 2 max_k and 64 slots) stays in LDS when it fits
 * beside the spectra, else the plan allocates it in device memory. */
fpssft_status fpssft_plan_create(const fpssft_desc* descs, int32_t batch,
                                 const fpssft_tuning* tuning, fpssft_plan_t* plan);

/* The plan of the problem statement (Sec. 2; the line design of Lemmas 1
 * and 2): fpssft_plan_create with the library's default launch shapes. */
fpssft_status fpssft_plan(const fpssft_desc* descs, int32_t batch, fpssft_plan_t* plan);

/* Release the plan and its device memory (waits for the plan's device; the
 * caller's current device is left as it was). */
fpssft_status fpssft_plan_destroy(fpssft_plan_t plan);

/* Host copy of cube `cube`'s schedule, int32 [T_max][2][ndim]. */
fpssft_status fpssft_plan_get_schedule(fpssft_plan_t plan, int32_t cube,
                                       int32_t* alpha_tau);

/* L, T_max and the element offset of cube `cube`'s block in the packed
 * spectra buffer of fpssft_lines_fft_all (any output may be NULL). */
fpssft_status fpssft_plan_cube_info(fpssft_plan_t plan, int32_t cube,
                                    int32_t* line_length, int32_t* max_iters,
                                    int64_t* spectra_offset);

/* Total complex64 elements of the packed spectra buffer: sum over cubes of
 * T_max * (D+1) * L. */
int64_t fpssft_plan_spectra_elems(fpssft_plan_t plan);

/* ---- the hot path ------------------------------------------------------ */

/* Errors of the calls below, returned before anything is enqueued:
 * INVALID_ARG for a NULL plan, input, output or gradient pointer (every
 * pointer field of an fpssft_out included), a cube index outside
 * [0, batch), an iteration range outside [0, T_max), or a current HIP
 * device other than the plan's (the calls enqueue on the current device,
 * and the plan's buffers live on its own); UNSUPPORTED as
 * stated per call. HIP errors while enqueueing return FPSSFT_ERR_HIP.
 * Algorithmic outcomes (OK, INCOMPLETE, CAPACITY) are not errors: they go
 * to info[2] on the device. The calls do not synchronize the stream. */

/* Plain per-cube FPS-SFT on cube `cube` of the plan: the method of Sec.
 * 2.2 with the Multi-dimensional extension, iteration by iteration until an
 * empty residual or T_max (Sec. 3): gather the D+1 lines (Eq.
 * sample_slice), take their 1/L DFTs (Eq. hs), subtract the recovered set
 * (construction-subtraction, Eq. freqSum), test every bin for 1-sparsity,
 * decode frequency and amplitude (Eq. decoding) and record. The line gather
 * + FFT kernel transforms the first chunk of iterations in parallel, then
 * one work-group runs the sequential part, gathering and transforming
 * further lines itself when the chunk runs out.
 * x: device complex64 cube, read only; out: device outputs (fpssft_out),
 * written by the call. */
fpssft_status fpssft_execute(fpssft_plan_t plan, int32_t cube, const void* x,
                             const fpssft_out* out, void* stream);

/* fpssft_execute for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same launches with the same results, bit for bit, but the
 * pre-chunk spectra and a record store that does not fit in LDS come from a
 * static device array of 4 MiB (one per GPU, held until the process ends)
 * instead of the plan's workspace. The call allocates nothing. Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (concurrent
 * streams, other threads) race and must be ordered by the caller. Nothing in
 * the array needs to start at zero. UNSUPPORTED when the cube needs more
 * than 4 MiB: chunk_iters (D+1) L * 8 bytes rounded up to 256, plus the
 * record store (above) when it exceeds LDS, plus the line workspace (above)
 * of lines that exceed LDS. Argument errors as for
 * fpssft_execute. */
fpssft_status fpssft_execute_noalloc(fpssft_plan_t plan, int32_t cube, const void* x,
                                     const fpssft_out* out, void* stream);

/* The same method (Sec. 2.2) for all cubes of the plan in one persistent
 * launch per kernel instantiation (each work-group solves the cube of its
 * index in an order of shortest lines first, smallest cubes first within a
 * line length, then takes the next ones from
 * a device queue), replayed from a HIP graph or launched
 * directly (fpssft_tuning). xs: host array of `batch` device cube pointers;
 * outs: host array of `batch` output structs (device pointers inside).
 * Results equal fpssft_execute's cube by cube, bit for bit. */
fpssft_status fpssft_execute_batched(fpssft_plan_t plan, const void* const* xs,
                                     const fpssft_out* outs, void* stream);

/* Line gather + L-point DFT (Eq. sample_slice, Eq. hs) of iterations
 * t0..t0+count-1 of cube `cube`: spectra (device complex64, caller-owned)
 * receives [count][D+1][L], s_hat(alpha, tau^{(t,i)}, m) with the 1/L
 * factor. */
fpssft_status fpssft_lines_fft(fpssft_plan_t plan, int32_t cube, const void* x,
                               int32_t t0, int32_t count, void* spectra,
                               void* stream);

/* The same for every cube over its whole budget t = 0..T_max-1, in one
 * launch, into the packed buffer (see fpssft_plan_cube_info). xs: host
 * array of `batch` device cube pointers. */
fpssft_status fpssft_lines_fft_all(fpssft_plan_t plan, const void* const* xs,
                                   void* spectra, void* stream);

/* Adjoint of the set amplitudes of Eq. decoding with the decisions of a
 * forward run held fixed (frequencies, iterations, bins, merges: not
 * differentiated). This form is not in the paper; it is built on its
 * amplitude estimate and construction-subtraction (Sec. 2.2), which make
 * the amplitudes linear in x, a = M x. It writes grad_x = M^H grad_a
 * (PyTorch's complex convention: for real l, grad = dl/dRe + j dl/dIm).
 * fwd: the forward outputs of cube `cube` (records and info on device);
 * grad_amps: device complex64 [max_k], the cotangents of the entries
 * 0..k+kd-1 of freqs/amps (the set and the merged frequencies left out of
 * it, all sums of detections; later entries ignored); grad_x: device
 * complex64 cube,
 * overwritten (zero off the sampled lines). UNSUPPORTED for
 * FPSSFT_FLAG_AMP_AVERAGE plans, and when a cube's LDS share exceeds
 * 160 KB: per detection its cotangent, iteration, frequency indices and
 * bin ((16 + 4 D) max_k bytes), 4 min(T, max_k) bytes of per-iteration
 * indices, plus,
 * unless its lines live in the plan's device workspace (above), the line
 * cotangent and the FFT's second buffer (16 L bytes) and, for lines short
 * enough to be transformed with all D+1 in LDS, the twiddles (8 L
 * bytes). */
fpssft_status fpssft_amp_backward(fpssft_plan_t plan, int32_t cube,
                                  const fpssft_out* fwd, const void* grad_amps,
                                  void* grad_x, void* stream);

/* The adjoint for every cube of the plan in one launch: host arrays of
 * `batch` forward outputs, cotangent pointers and gradient-cube pointers. */
fpssft_status fpssft_amp_backward_batched(fpssft_plan_t plan,
                                          const fpssft_out* fwds,
                                          const void* const* grad_amps,
                                          void* const* grad_xs, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FPSSFT_H */
