"""Seeded synthetic inputs for FPS-SFT: K-sparse on-grid sinusoid cubes.

This module is shared by the tests, the benchmark and the smoke check. It
draws signals of the model of Section 2 (Eq. sigModel2): a superposition of
K complex sinusoids whose frequencies lie on the D-D DFT grid,

    x(n) = sum_{(a, w) in S} a * exp(j n^T w),  w_k = 2 pi m_k / N_k.

It holds none of the transform's arithmetic: no line sampling, no line DFT,
no decoding. The cube is synthesised exactly as N * ifftn(X) with X the sparse
D-D spectrum (X[m] = a), which realises the model above under the 1/N DFT
normalisation the paper uses for its column DFTs (Section 2.1).

Layout: complex64, row-major, last index contiguous (the C-ABI's layout).
"""
from __future__ import annotations

import dataclasses
from typing import Sequence

import numpy as np

# Default noiseless thresholds (theta0, rho, gamma) and the noisy-case ones.
# They are plan inputs shared by the oracle and the GPU path; the reasoning
# for the values is the margin analysis of the decision steps.
NOISELESS_THRESH = dict(zero_thresh=1e-3, mag_rel_tol=1e-3, grid_tol=1e-2)


@dataclasses.dataclass
class Cube:
    """One synthetic cube with its planted ground truth."""

    x: np.ndarray            # complex64, shape dims
    freqs: np.ndarray        # int64 [K, D], planted frequency indices m
    amps: np.ndarray         # complex128 [K], planted amplitudes a
    seed: int                # data seed (the line-schedule seed is seed + 1)
    noise_sigma: float = 0.0 # per-sample complex noise std (0 = noiseless)

    @property
    def dims(self):
        return tuple(self.x.shape)

    @property
    def schedule_seed(self) -> int:
        return self.seed + 1


def _draw(rng: np.random.Generator, dims: Sequence[int], K: int, mag,
          cluster: int = 0):
    dims = tuple(int(d) for d in dims)
    N = int(np.prod(dims))
    if K > N:
        raise ValueError("K exceeds the number of grid frequencies")
    if cluster:
        # One contiguous (wrapping) block of side s (s^D = cluster frequencies
        # in 2-D) at a uniform position, plus K - cluster distinct others.
        side = int(round(cluster ** (1.0 / len(dims))))
        if side ** len(dims) != cluster:
            raise ValueError("cluster must be a perfect D-th power")
        corner = [int(rng.integers(0, d)) for d in dims]
        grids = np.meshgrid(*[np.arange(side)] * len(dims), indexing="ij")
        block = np.stack([(g.ravel() + c) % d for g, c, d in
                          zip(grids, corner, dims)], axis=1)
        flat_block = np.ravel_multi_index(tuple(block.T), dims)
        rest = np.setdiff1d(np.arange(N), flat_block)
        others = rng.choice(rest, K - cluster, replace=False)
        flat = np.concatenate([flat_block, others])
    else:
        flat = rng.choice(N, K, replace=False)
    freqs = np.stack(np.unravel_index(flat, dims), axis=1).astype(np.int64)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=K)
    if mag == "unit":
        absval = np.ones(K)
    else:
        lo, hi = mag
        absval = rng.uniform(lo, hi, size=K)
    amps = absval * np.exp(1j * phase)
    return freqs, amps


def synthesize(dims: Sequence[int], freqs: np.ndarray, amps: np.ndarray) -> np.ndarray:
    """x = N * ifftn(X) with X[freqs] = amps; returns complex128."""
    dims = tuple(int(d) for d in dims)
    X = np.zeros(dims, dtype=np.complex128)
    if len(amps):
        np.add.at(X, tuple(np.asarray(freqs).T), amps)
    return np.fft.ifftn(X) * float(np.prod(dims))


def plant(dims: Sequence[int], K: int, seed: int, mag="unit",
          snr_db: float | None = None, cluster: int = 0,
          rng: np.random.Generator | None = None) -> Cube:
    """A K-sparse cube: distinct uniform frequencies, phase U[0, 2pi).

    mag: "unit" or (lo, hi) for |a| ~ U[lo, hi].
    snr_db: additive circular complex Gaussian noise with per-sample variance
    sigma^2 = sum |a|^2 / 10^(snr_db/10) (the mean sample power of the
    noiseless cube is sum |a|^2 for distinct on-grid frequencies).
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    freqs, amps = _draw(rng, dims, K, mag, cluster)
    x = synthesize(dims, freqs, amps)
    sigma = 0.0
    if snr_db is not None:
        sigma = float(np.sqrt(np.sum(np.abs(amps) ** 2) / 10.0 ** (snr_db / 10.0)))
        noise = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
        x = x + noise * (sigma / np.sqrt(2.0))
    return Cube(x=x.astype(np.complex64), freqs=freqs, amps=amps, seed=int(seed),
                noise_sigma=sigma)


def image_like(dims: Sequence[int], K: int, seed: int) -> Cube:
    """A pixel-sparse 2-D "image" with clustered support, used through
    duality: the image is the sparse spectrum, x = N IDFT(image). Blobs are
    axis-aligned rectangles of 1..12 x 1..12 pixels at uniform positions
    (wrapping), added until the support holds exactly K pixels (the last
    blob is trimmed). Intensities are real, U[0.5, 1.5], as in a magnitude
    image. Stands in for the image experiment of Sec. 3, whose image is not
    available."""
    if len(dims) != 2:
        raise ValueError("image_like is 2-D")
    rng = np.random.default_rng(seed)
    n0, n1 = (int(d) for d in dims)
    mask = np.zeros((n0, n1), dtype=bool)
    order = []
    while len(order) < K:
        h, w = (int(v) for v in rng.integers(1, 13, size=2))
        r0, c0 = int(rng.integers(0, n0)), int(rng.integers(0, n1))
        for i in range(h):
            for j in range(w):
                p = ((r0 + i) % n0, (c0 + j) % n1)
                if not mask[p] and len(order) < K:
                    mask[p] = True
                    order.append(p)
    freqs = np.array(sorted(order), dtype=np.int64)
    amps = rng.uniform(0.5, 1.5, size=K).astype(np.complex128)
    x = synthesize(dims, freqs, amps)
    return Cube(x=x.astype(np.complex64), freqs=freqs, amps=amps, seed=int(seed))


def random_dense(dims: Sequence[int], seed: int) -> np.ndarray:
    """A dense random complex cube (not sparse), for identity checks."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(dims) + 1j * rng.standard_normal(dims))


# ---------------------------------------------------------------------------
# The five workloads (2-D/3-D shapes, sparsity, magnitudes, noise, seeds).
# ---------------------------------------------------------------------------

def cfg1() -> Cube:
    """2-D 64x64, K=8, unit magnitude, noiseless, seed 0."""
    return plant((64, 64), 8, seed=0)


def cfg2() -> Cube:
    """2-D 256x256, K=100, |a|~U[0.5,1.5], 20 dB per-sample SNR, seed 2."""
    return plant((256, 256), 100, seed=2, mag=(0.5, 1.5), snr_db=20.0)


def cfg2_thresh(cube: Cube, L: int) -> dict:
    """Thresholds for the noisy workload: theta0 = 4 sigma / sqrt(L) is four
    standard deviations of a noise-only line bin; the magnitude test is loose
    and the on-grid check is off."""
    return dict(zero_thresh=4.0 * cube.noise_sigma / np.sqrt(L), mag_rel_tol=0.5,
                grid_tol=-1.0)


def cfg3() -> Cube:
    """3-D 128^3, K=500, |a|~U[0.5,1.5], noiseless, seed 3."""
    return plant((128, 128, 128), 500, seed=3, mag=(0.5, 1.5))


SIDES_CFG4 = (64, 128, 256, 512)


def cfg4_shapes(B: int = 1024, seed: int = 4):
    """Per-cube (dims, K, child seed) of the batched workload: N0 and N1 drawn
    independently and uniformly from {64,128,256,512}, K ~ U{10..300}."""
    rng = np.random.default_rng(seed)
    n0 = rng.choice(SIDES_CFG4, size=B)
    n1 = rng.choice(SIDES_CFG4, size=B)
    ks = rng.integers(10, 301, size=B)
    children = np.random.SeedSequence(seed).spawn(B)
    out = []
    for b in range(B):
        child_seed = int(children[b].generate_state(1, dtype=np.uint32)[0])
        out.append(((int(n0[b]), int(n1[b])), int(ks[b]), child_seed))
    return out


def cfg4(B: int = 1024, seed: int = 4, only=None):
    """The batched workload: B independent 2-D cubes of uneven sides and K.
    `only` restricts generation to a subset of cube indices (the shapes and
    seeds of the others are unchanged)."""
    shapes = cfg4_shapes(B, seed)
    idx = range(B) if only is None else only
    return [plant(shapes[b][0], shapes[b][1], seed=shapes[b][2]) for b in idx]


def cfg5(B: int = 64, seed: int = 5):
    """Differentiation workload: B cubes of 256x256, K=50, unit magnitude."""
    children = np.random.SeedSequence(seed).spawn(B)
    return [plant((256, 256), 50,
                  seed=int(children[b].generate_state(1, dtype=np.uint32)[0]))
            for b in range(B)]
