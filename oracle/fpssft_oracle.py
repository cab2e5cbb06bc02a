"""FP64 reference oracle for FPS-SFT (Wang, Patel, Petropulu, arXiv 1711.11407).

TEST INFRASTRUCTURE ONLY. This module is the slow, plain, obviously-correct
CPU statement of what the GPU path computes. Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import it; the product path never
does. It shares no code with the HIP implementation (no tables, no helpers,
no constants) and imports nothing from the package.

Everything is numpy, complex128 / exact Python or int64 integers, and follows
the paper in its own order and notation:

  * line length L = LCM(N_0..N_{D-1}), c_k = L / N_k       (Lemma 1; Sec. 2.3)
  * slope set A: gcd(c_0 a_0, ..., c_{D-1} a_{D-1}) = 1   (Lemma 2; D > 2 is
    a reading of the Multi-dimensional extension paragraph)
  * per-iteration random slope and offset                  (Sec. 2.2)
  * D+1 lines: offset tau, and tau + e_{i-1} for line i    (Sec. 2.2, Eq.
    decoding, and the Multi-dimensional extension)
  * line samples s(l) = x([alpha l + tau] mod N)           (Eq. sample_slice)
  * construction-subtraction done literally in the time domain: build the
    recovered sinusoids' line spectrum, IDFT it, subtract from the samples
                                                           (Sec. 2.2, after
                                                            Eq. decoding)
  * L-point line DFT with 1/L normalisation                (Eq. hs)
  * 1-sparsity: nonzero test and magnitude equality across the shifted lines
                                                           (Sec. 2.1 and 2.2)
  * frequency decode from phase differences, amplitude with the unshifted
    offset's phase removed                                 (Eq. decoding)
  * iteration cap T_max = floor(N / ((D+1) L))             (Sec. 3)
  * the recovered set: distinct frequencies with nonzero amplitudes (the
    set S of Eq. sigModel2); a frequency detected again later is merged into
    its first record by summing amplitudes                 (Sec. 2.2)

Readings taken where the paper is silent (thresholds, rounding, stopping,
re-detection) are listed in the repository's design notes and in the
docstrings below. All arithmetic is fp64, the decisions included (threshold
tests, the phase, rint of the decoded phase). The thresholds are the float32
values the GPU plan receives, widened exactly to fp64. A float32 decision
step (`Params.decision = "float32"`) exists only as a diagnostic, to measure
how far the precision of the decisions matters on a workload.
"""
from __future__ import annotations

import dataclasses
import math
from fractions import Fraction
from functools import reduce
from typing import Sequence

import numpy as np

STATUS_OK = 0          # an empty residual was observed: all recovered
STATUS_INCOMPLETE = 1  # iteration cap reached with a nonzero residual
STATUS_CAPACITY = 2    # the record list reached its capacity

# ---------------------------------------------------------------------------
# Line design (Lemma 1, Lemma 2)
# ---------------------------------------------------------------------------


def line_length(dims: Sequence[int]) -> int:
    """L = LCM(N_0, ..., N_{D-1}) (Lemma 1; Multi-dimensional extension)."""
    return reduce(lambda a, b: a * b // math.gcd(a, b), [int(d) for d in dims], 1)


def c_factors(dims: Sequence[int]) -> list[int]:
    """c_k = L / N_k (Lemma 2)."""
    L = line_length(dims)
    return [L // int(d) for d in dims]


def default_max_iters(dims: Sequence[int]) -> int:
    """T_max = floor(N / ((D+1) L)), the paper's budget of about 100% of the
    samples (Sec. 3: 85 for 256x256), at least 1."""
    N = int(np.prod(dims))
    return max(1, N // ((len(dims) + 1) * line_length(dims)))


def samples_used(dims: Sequence[int], iterations: int) -> int:
    """Samples consumed: (D+1) lines of L samples per iteration, counted with
    multiplicity (complexity analysis, Sec. 2.3)."""
    return (len(dims) + 1) * line_length(dims) * int(iterations)


def in_slope_set(alpha: Sequence[int], dims: Sequence[int]) -> bool:
    """Membership in the slope set A of Lemma 2.

    In 2-D the paper's set is {a0 coprime a1, a0 coprime c1, a1 coprime c0};
    with c0 coprime c1 (L is the LCM) that is gcd(c0 a0, c1 a1) = 1. For any
    D the set used here is gcd(c_0 a_0, ..., c_{D-1} a_{D-1}) = 1.
    """
    c = c_factors(dims)
    g = 0
    for ck, ak in zip(c, alpha):
        g = math.gcd(g, int(ck) * int(ak))
    return g == 1


# ---------------------------------------------------------------------------
# Counter-based generator for the line schedule (SplitMix64)
# ---------------------------------------------------------------------------

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(seed: int, counter: int) -> int:
    """Output number `counter` (0-based) of SplitMix64 started at `seed`
    (Steele, Lea and Flood, OOPSLA 2014): the state after counter+1 steps is
    seed + (counter+1) * golden-gamma, passed through the published mix."""
    z = (int(seed) + (int(counter) + 1) * _GOLDEN) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def _below(z: int, n: int) -> int:
    """Map a 64-bit word to [0, n): floor(z * n / 2^64)."""
    return (z * int(n)) >> 64


def schedule(dims: Sequence[int], T: int, seed: int, axis: bool = False):
    """Per-iteration slope and offset (Sec. 2.2: a random slope from Lemma 2's
    set and a random offset each iteration; D-D: both from X_D).

    Draw order, one counter stream per cube: for each iteration, draw the D
    slope components (uniform on [N_k]) and redraw all D until the slope is
    in A; then draw the D offset components (uniform on [N_k]).

    axis=True: the slopes of the row/column method reviewed in Sec. 2.1 and
    shown to deadlock in Sec. 2.2, alpha = e_{t mod D} (the unit vector,
    reduced mod N_k), with no slope drawn; offsets as above.
    Returns int64 arrays alpha [T, D] and tau [T, D].
    """
    dims = [int(d) for d in dims]
    D = len(dims)
    alpha = np.zeros((T, D), dtype=np.int64)
    tau = np.zeros((T, D), dtype=np.int64)
    ctr = 0
    for t in range(T):
        while not axis:
            a = []
            for k in range(D):
                a.append(_below(splitmix64(seed, ctr), dims[k]))
                ctr += 1
            if in_slope_set(a, dims):
                break
        if axis:
            a = [(1 if k == t % D else 0) % dims[k] for k in range(D)]
        alpha[t] = a
        for k in range(D):
            tau[t, k] = _below(splitmix64(seed, ctr), dims[k])
            ctr += 1
    return alpha, tau


# ---------------------------------------------------------------------------
# Lines and their DFTs (Eq. sample_slice, Eq. hs)
# ---------------------------------------------------------------------------


def line_offsets(dims: Sequence[int], tau: Sequence[int]) -> list[list[int]]:
    """The D+1 offsets of one iteration: tau, then tau with coordinate i-1
    advanced by one (mod N_{i-1}) for line i = 1..D."""
    dims = [int(d) for d in dims]
    offs = [[int(v) for v in tau]]
    for k in range(len(dims)):
        o = [int(v) for v in tau]
        o[k] = (o[k] + 1) % dims[k]
        offs.append(o)
    return offs


def line_positions(dims: Sequence[int], alpha: Sequence[int],
                   offset: Sequence[int], L: int) -> np.ndarray:
    """n_k(l) = [alpha_k l + tau_k]_{N_k} for l in [L], exact int64 [L, D]."""
    l = np.arange(L, dtype=np.int64)
    cols = [(int(a) * l + int(o)) % int(n) for a, o, n in zip(alpha, offset, dims)]
    return np.stack(cols, axis=1)


def gather_line(x: np.ndarray, alpha, offset, L: int) -> np.ndarray:
    pos = line_positions(x.shape, alpha, offset, L)
    return x[tuple(pos.T)]


def line_dft(s: np.ndarray) -> np.ndarray:
    """s_hat(m) = (1/L) sum_l s(l) exp(-j 2 pi l m / L) (Eq. hs). An explicit
    DFT matrix for L <= 64, numpy's FFT above."""
    L = s.shape[-1]
    if L <= 64:
        lm = np.outer(np.arange(L), np.arange(L)) % L
        F = np.exp(-2j * np.pi * lm / L)
        return (F @ s) / L
    return np.fft.fft(s) / L


def line_idft_unnormalised(sh: np.ndarray) -> np.ndarray:
    """s(l) = sum_m s_hat(m) exp(+j 2 pi l m / L): the inverse of line_dft."""
    L = sh.shape[-1]
    return np.fft.ifft(sh) * L


def projection_bin(freqs: np.ndarray, alpha: Sequence[int], dims: Sequence[int]) -> np.ndarray:
    """The bin m of an L-point line DFT that frequency index vectors project
    onto: [sum_k (L/N_k) m_k alpha_k]_L (Eq. orthogonality, the integer form
    of Eq. lines)."""
    L = line_length(dims)
    c = c_factors(dims)
    f = np.asarray(freqs, dtype=np.int64).reshape(-1, len(dims))
    acc = np.zeros(len(f), dtype=np.int64)
    for k in range(len(dims)):
        acc = (acc + (c[k] * int(alpha[k]) % L) * f[:, k]) % L
    return acc


def offset_phase(freqs: np.ndarray, offset: Sequence[int], dims: Sequence[int]) -> np.ndarray:
    """exp(j 2 pi sum_k m_k tau_k / N_k) per frequency (Eq. freqSum), with
    each m_k tau_k reduced mod N_k first so the fp64 angle stays small."""
    f = np.asarray(freqs, dtype=np.int64).reshape(-1, len(dims))
    frac = np.zeros(len(f))
    for k, n in enumerate(dims):
        frac = frac + ((f[:, k] * int(offset[k])) % int(n)) / float(n)
    return np.exp(2j * np.pi * frac)


# ---------------------------------------------------------------------------
# The FPS-SFT iteration
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Params:
    zero_thresh: float = 1e-3   # theta0: a bin is nonzero iff |r| > theta0
    mag_rel_tol: float = 1e-3   # rho: | |r_i| - |r_0| | <= rho |r_0|, i = 1..D
    grid_tol: float = 1e-2      # gamma: |u - rint(u)| <= gamma (< 0: off)
    max_iters: int = 0          # 0: floor(N / ((D+1) L))
    max_k: int = 4096           # capacity of the record list
    amp_average: bool = False   # amplitude: mean over the D+1 lines of
                                # r_i(m) exp(-j 2 pi sum m_k tau_k^(i) / N_k)
                                # instead of line 0 alone (Eq. decoding)
    decision: str = "float64"   # precision of the decisions; "float32" is a
                                # diagnostic only (see decide_bins)


@dataclasses.dataclass
class Result:
    """The recovered set and the trace of the detections that produced it.

    freqs/amps: the recovered set, distinct frequencies in the order of
    their first detection; a frequency detected several times carries the
    sum of its detections' amplitudes; a merged frequency whose amplitude
    sum has |a| <= theta0 is not in the set (Eq. sigModel2 has a != 0) but in
    dropped_freqs/dropped_amps. rec_*: one entry per detection, canonical
    (iteration, bin) order; rec_sin[i] indexes concat(freqs, dropped_freqs).
    """
    freqs: np.ndarray          # int64 [k, D]
    amps: np.ndarray           # complex128 [k]
    rec_freqs: np.ndarray      # int64 [n, D]: decoded frequency of each detection
    rec_amps: np.ndarray       # complex128 [n]: amplitude decoded at that detection
    rec_iter: np.ndarray       # int64 [n]: iteration of the detection
    rec_bin: np.ndarray        # int64 [n]: its bin in that iteration's lines
    rec_sin: np.ndarray        # int64 [n]: index of its frequency in the set
    dropped_freqs: np.ndarray  # int64 [kd, D]
    dropped_amps: np.ndarray   # complex128 [kd]
    iters: int                 # iterations executed (lines gathered)
    status: int

    @property
    def k(self) -> int:
        return len(self.amps)

    @property
    def n(self) -> int:
        return len(self.rec_amps)


def _threshold(v: float) -> float:
    """A threshold as the plan's kernels receive it: rounded to float32."""
    return float(np.float32(v))


def decide_bins(r: np.ndarray, dims: Sequence[int], params: Params):
    """Per-bin 1-sparsity test and phase decode on one iteration's residual
    line spectra r [D+1, L] (Eq. decoding; magnitude equality as in Sec. 2.1).

    fp64 throughout: magnitudes of the complex128 residuals, phi = atan2 of
    r_{k+1}(m) conj(r_0(m)) in (-pi, pi], u_k = N_k phi / (2 pi), m_k =
    rint(u_k) (round half to even) mod N_k, on-grid check |u_k - rint(u_k)|
    <= gamma. The thresholds are the plan's float32 values.

    params.decision == "float32" takes the same steps on the residuals
    rounded to complex64 in float32 arithmetic; it is a diagnostic that
    shows how close a workload's decisions are to the precision boundary,
    not the reference.
    Returns (any_nonzero, candidate mask [L], decoded frequencies [L, D]).
    """
    D = len(dims)
    if params.decision == "float32":
        rr = r.astype(np.complex64)
        ft = np.float32
    elif params.decision == "float64":
        rr = np.asarray(r, dtype=np.complex128)
        ft = np.float64
    else:
        raise ValueError("decision must be 'float64' or 'float32'")
    mag = np.abs(rr).astype(ft)
    th0 = ft(_threshold(params.zero_thresh))
    rho = ft(_threshold(params.mag_rel_tol))
    gtol = ft(_threshold(params.grid_tol))
    inv2pi = ft(1.0 / (2.0 * np.pi))
    any_nonzero = bool((mag > th0).any())
    cand = mag[0] > th0
    for i in range(1, D + 1):
        cand &= np.abs(mag[i] - mag[0]) <= rho * mag[0]
    dec = np.zeros((r.shape[1], D), dtype=np.int64)
    for k in range(D):
        z = rr[k + 1] * np.conj(rr[0])
        phi = np.arctan2(z.imag, z.real).astype(ft)            # (-pi, pi]
        u = (ft(dims[k]) * phi) * inv2pi
        v = np.rint(u)
        if params.grid_tol >= 0:
            cand &= np.abs(u - v) <= gtol
        dec[:, k] = np.mod(v.astype(np.int64), int(dims[k]))
    return any_nonzero, cand, dec


def merge_detections(rec_freqs: np.ndarray, rec_amps: np.ndarray, zero_thresh: float):
    """The recovered set from the detection list (Sec. 2.2: the set of
    recovered sinusoids; Eq. sigModel2: distinct frequencies, a != 0).

    Frequencies in the order of their first detection; the amplitude of a
    frequency is the sum of its detections' amplitudes, added in detection
    order. A frequency detected more than once whose sum has |a| <= theta0
    is dropped from the set. Returns (freqs, amps, dropped_freqs,
    dropped_amps, rec_sin) with rec_sin indexing concat(freqs, dropped).
    """
    rec_freqs = np.asarray(rec_freqs, dtype=np.int64)
    D = rec_freqs.shape[1] if rec_freqs.ndim == 2 else 0
    first: dict = {}
    order: list = []
    sums: list = []
    count: list = []
    grp = np.zeros(len(rec_amps), dtype=np.int64)
    for i, (f, a) in enumerate(zip(rec_freqs.tolist(), rec_amps)):
        key = tuple(f)
        if key not in first:
            first[key] = len(order)
            order.append(key)
            sums.append(complex(a))
            count.append(1)
        else:
            g = first[key]
            sums[g] += complex(a)
            count[g] += 1
        grp[i] = first[key]
    th0 = _threshold(zero_thresh)
    keep = [count[g] == 1 or abs(sums[g]) > th0 for g in range(len(order))]
    index = np.zeros(len(order), dtype=np.int64)
    kept = [g for g in range(len(order)) if keep[g]]
    dropped = [g for g in range(len(order)) if not keep[g]]
    for i, g in enumerate(kept + dropped):
        index[g] = i

    def pack(gs):
        return (np.array([order[g] for g in gs], dtype=np.int64).reshape(-1, D),
                np.array([sums[g] for g in gs], dtype=np.complex128))

    fk, ak = pack(kept)
    fd, ad = pack(dropped)
    return fk, ak, fd, ad, index[grp]


def run(x: np.ndarray, alpha: np.ndarray, tau: np.ndarray,
        params: Params = Params()) -> Result:
    """FPS-SFT on cube x with the given per-iteration slopes and offsets.

    Per iteration t (Sec. 2.2):
      1. gather the D+1 lines (Eq. sample_slice);
      2. construction-subtraction: project the recovered list onto the L
         bins of each line with its offset phase (Eq. freqSum), IDFT, and
         subtract the constructed samples from the gathered ones;
      3. L-point DFT of each line (Eq. hs);
      4. stop if every bin of every line has |r| <= theta0 (empty residual);
      5. for each bin independently, against this iteration's residual:
         nonzero + magnitude equality, phase decode, optional on-grid check,
         projection consistency (the decoded frequency must project onto
         this bin), amplitude a = r_0(m) exp(-j 2 pi sum m_k tau_k / N_k)
         (or its mean over the D+1 lines, params.amp_average);
         append in bin order.
    Every detection is a further record of the list (a frequency found
    again is one more term), and the construction-subtraction sums every
    record; the output merges the list into the recovered set
    (merge_detections). A full list (max_k detections) stops the run with
    STATUS_CAPACITY after appending the candidates that fit, in bin order.
    """
    dims = [int(d) for d in x.shape]
    D = len(dims)
    L = line_length(dims)
    T = params.max_iters if params.max_iters > 0 else default_max_iters(dims)
    x64 = np.asarray(x).astype(np.complex128)

    rf: list[np.ndarray] = []
    ra: list[complex] = []
    rt: list[int] = []
    rm: list[int] = []
    status, iters = STATUS_INCOMPLETE, T
    for t in range(T):
        a_vec = [int(v) for v in alpha[t]]
        offs = line_offsets(dims, tau[t])
        rec_f = np.array(rf, dtype=np.int64).reshape(-1, D)
        rec_a = np.array(ra, dtype=np.complex128)
        bins = projection_bin(rec_f, a_vec, dims)
        r = np.zeros((D + 1, L), dtype=np.complex128)
        for i, off in enumerate(offs):
            s = gather_line(x64, a_vec, off, L)
            sh_r = np.zeros(L, dtype=np.complex128)
            if len(rec_a):
                np.add.at(sh_r, bins, rec_a * offset_phase(rec_f, off, dims))
            s = s - line_idft_unnormalised(sh_r)
            r[i] = line_dft(s)
        any_nonzero, cand, dec = decide_bins(r, dims, params)
        if not any_nonzero:
            status, iters = STATUS_OK, t + 1
            break
        full = False
        for m in np.nonzero(cand)[0]:
            f = dec[m]
            if projection_bin(f, a_vec, dims)[0] != m:
                continue
            if len(ra) >= params.max_k:
                full = True
                break
            if params.amp_average:
                # each line's bin value carries its own offset's phase
                amp = np.mean([r[i, m] * np.conj(offset_phase(f, offs[i], dims)[0])
                               for i in range(D + 1)])
            else:
                amp = r[0, m] * np.conj(offset_phase(f, offs[0], dims)[0])
            rf.append(f.copy())
            ra.append(amp)
            rt.append(t)
            rm.append(int(m))
        if full:
            status, iters = STATUS_CAPACITY, t + 1
            break
    rec_f = np.array(rf, dtype=np.int64).reshape(-1, D)
    rec_a = np.array(ra, dtype=np.complex128)
    fk, ak, fd, ad, rec_sin = merge_detections(rec_f, rec_a, params.zero_thresh)
    return Result(freqs=fk, amps=ak, rec_freqs=rec_f, rec_amps=rec_a,
                  rec_iter=np.array(rt, dtype=np.int64),
                  rec_bin=np.array(rm, dtype=np.int64), rec_sin=rec_sin,
                  dropped_freqs=fd, dropped_amps=ad, iters=iters, status=status)


# ---------------------------------------------------------------------------
# Amplitudes as a linear function of the samples (support held fixed)
# ---------------------------------------------------------------------------


def replay_amplitudes(x: np.ndarray, rec_freqs: np.ndarray, rec_iter: np.ndarray,
                      rec_bin: np.ndarray, alpha: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Recompute every detection's amplitude from samples x with the
    decisions (frequency, iteration, bin of each detection) of a previous run
    held fixed.

    For each iteration that produced detections, in order: gather line 0,
    subtract the time-domain construction of the detections of earlier
    iterations (with their replayed amplitudes), take the line DFT and read
    each detection's bin, removing the unshifted offset's phase (Eq.
    decoding). The map x -> amplitudes is linear, so its gradient is exact.
    """
    dims = [int(d) for d in x.shape]
    D = len(dims)
    L = line_length(dims)
    x64 = np.asarray(x).astype(np.complex128)
    freqs = np.asarray(rec_freqs, dtype=np.int64).reshape(-1, D)
    out = np.zeros(len(freqs), dtype=np.complex128)
    for t in sorted(set(int(v) for v in rec_iter)):
        a_vec = [int(v) for v in alpha[t]]
        off0 = line_offsets(dims, tau[t])[0]
        prev = np.nonzero(np.asarray(rec_iter) < t)[0]
        s = gather_line(x64, a_vec, off0, L)
        sh_r = np.zeros(L, dtype=np.complex128)
        if len(prev):
            np.add.at(sh_r, projection_bin(freqs[prev], a_vec, dims),
                      out[prev] * offset_phase(freqs[prev], off0, dims))
        r0 = line_dft(s - line_idft_unnormalised(sh_r))
        cur = np.nonzero(np.asarray(rec_iter) == t)[0]
        for i in cur:
            out[i] = r0[int(rec_bin[i])] * np.conj(offset_phase(freqs[i], off0, dims)[0])
    return out


def set_amplitudes(rec_amps: np.ndarray, rec_sin: np.ndarray, k: int) -> np.ndarray:
    """Amplitudes of the k frequencies of the recovered set from the
    detections' amplitudes: the sum over each frequency's detections, in
    detection order (the merge of merge_detections, decisions fixed)."""
    out = np.zeros(k, dtype=np.complex128)
    for a, g in zip(rec_amps, np.asarray(rec_sin, dtype=np.int64)):
        if g < k:
            out[g] += a
    return out


def replay_set(x: np.ndarray, res: Result, alpha, tau) -> np.ndarray:
    """The recovered set's amplitudes as a function of x, decisions fixed."""
    a = replay_amplitudes(x, res.rec_freqs, res.rec_iter, res.rec_bin, alpha, tau)
    return set_amplitudes(a, res.rec_sin, res.k)


def touched_positions(dims, rec_iter, alpha, tau) -> np.ndarray:
    """Flat indices of the line-0 samples of every iteration that produced a
    detection: the only samples the amplitudes depend on."""
    dims = [int(d) for d in dims]
    L = line_length(dims)
    pos = []
    for t in sorted(set(int(v) for v in rec_iter)):
        p = line_positions(dims, alpha[t], line_offsets(dims, tau[t])[0], L)
        pos.append(np.ravel_multi_index(tuple(p.T), dims))
    if not pos:
        return np.zeros(0, dtype=np.int64)
    return np.unique(np.concatenate(pos))


def grad_sum_abs2_fd(x: np.ndarray, res: Result, alpha, tau, positions=None,
                     h: float = 1.0) -> np.ndarray:
    """Gradient of l(x) = sum_i |a_i(x)|^2 over the recovered set (amplitudes
    replayed with the decisions of `res` fixed) by central finite
    differences in fp64, in PyTorch's convention dl/dRe + j dl/dIm. l is
    quadratic in (Re x, Im x), so central differences are exact up to
    rounding for any h. Only `positions` (default: the touched line samples)
    are probed; every other sample has zero gradient because no amplitude
    reads it."""
    dims = x.shape
    x64 = np.asarray(x).astype(np.complex128)
    if positions is None:
        positions = touched_positions(dims, res.rec_iter, alpha, tau)
    g = np.zeros(int(np.prod(dims)), dtype=np.complex128)

    def loss(xx):
        return float(np.sum(np.abs(replay_set(xx, res, alpha, tau)) ** 2))

    flat = x64.reshape(-1)
    for n in positions:
        parts = []
        for step in (h, 1j * h):
            xp = flat.copy(); xp[n] += step
            xm = flat.copy(); xm[n] -= step
            parts.append((loss(xp.reshape(dims)) - loss(xm.reshape(dims))) / (2 * h))
        g[n] = parts[0] + 1j * parts[1]
    return g.reshape(dims)


def amp_matrix(x_shape, res: Result, alpha, tau, positions) -> np.ndarray:
    """Columns of the linear map M (set amplitudes = M x) at the given flat
    positions, by replaying unit impulses: M[:, j] = replay(e_{positions[j]})."""
    N = int(np.prod(x_shape))
    cols = []
    for n in positions:
        e = np.zeros(N, dtype=np.complex128); e[n] = 1.0
        cols.append(replay_set(e.reshape(x_shape), res, alpha, tau))
    return np.stack(cols, axis=1) if cols else np.zeros((res.k, 0), np.complex128)


# ---------------------------------------------------------------------------
# Brute-force references for pins
# ---------------------------------------------------------------------------


def dft_nd_direct(x: np.ndarray) -> np.ndarray:
    """X(m) = (1/N) sum_n x(n) exp(-j 2 pi sum_k m_k n_k / N_k), by the
    definition (O(N^2)); for tiny cubes only."""
    dims = x.shape
    N = int(np.prod(dims))
    grids = np.stack(np.unravel_index(np.arange(N), dims), axis=1)
    ang = np.zeros((N, N))
    for k, n in enumerate(dims):
        ang = ang + np.outer(grids[:, k], grids[:, k]) / float(n)
    return (np.exp(-2j * np.pi * ang) @ x.reshape(-1)).reshape(dims) / N


def projection_set(m: int, alpha: Sequence[int], dims: Sequence[int]) -> list[tuple]:
    """P_m: all grid frequencies with frac(sum_k m_k alpha_k / N_k - m / L) = 0
    (Eq. lines), enumerated with exact rationals; tiny cubes only."""
    L = line_length(dims)
    out = []
    for f in np.ndindex(*[int(d) for d in dims]):
        v = sum(Fraction(int(fk) * int(ak), int(n)) for fk, ak, n in zip(f, alpha, dims))
        v -= Fraction(int(m), L)
        if v.denominator == 1:
            out.append(tuple(int(q) for q in f))
    return out
