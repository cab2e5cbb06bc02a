"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these re-type the oracle's formulas: they check it against brute
force on tiny cubes (the D-D DFT by its definition, exhaustive enumeration of
projection sets with exact rationals), library routines in special cases
(numpy FFT along an axis, a 1-D full DFT), published test vectors, planted
ground truth, the paper's printed numbers and closed forms of the adjoint.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TH = O.Params(**W.NOISELESS_THRESH)


# --------------------------------------------------------------------------
# The generator (SplitMix64) against its published test vector
# --------------------------------------------------------------------------

def test_splitmix64_known_answer():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.json")) as f:
        g = json.load(f)
    got = [O.splitmix64(g["seed"], i) for i in range(len(g["outputs"]))]
    assert got == g["outputs"]


def test_schedule_draws_from_slope_set_and_grid():
    for dims in [(8, 8), (16, 24), (64, 128), (6, 10, 4), (128, 128, 128)]:
        al, ta = O.schedule(dims, 50, seed=11)
        L = O.line_length(dims)
        c = [L // d for d in dims]
        for a, t in zip(al, ta):
            assert all(0 <= a[k] < dims[k] and 0 <= t[k] < dims[k] for k in range(len(dims)))
            g = 0
            for ck, ak in zip(c, a):
                g = math.gcd(g, int(ck * ak))
            assert g == 1
        al2, ta2 = O.schedule(dims, 50, seed=11)
        assert (al == al2).all() and (ta == ta2).all()
        al3, _ = O.schedule(dims, 50, seed=12)
        assert not (al == al3).all()


# --------------------------------------------------------------------------
# Line DFT = projection of the D-D DFT (Eq. hs -> Eq. freqSum), any x
# --------------------------------------------------------------------------

def test_direct_dft_matches_numpy_fftn():
    for dims in [(4, 6), (3, 5), (2, 3, 4)]:
        x = W.random_dense(dims, 1)
        np.testing.assert_allclose(O.dft_nd_direct(x), np.fft.fftn(x) / x.size,
                                   atol=1e-13)


@pytest.mark.parametrize("dims", [(4, 6), (6, 10), (8, 8), (3, 5), (4, 4, 6), (2, 3, 5)])
def test_projection_slice_identity(dims):
    """For ANY cube, the 1/L line DFT at bin m equals the sum of the D-D DFT
    (1/N) over the frequencies of P_m, each rotated by the offset phase."""
    x = W.random_dense(dims, 7)
    X = O.dft_nd_direct(x)
    L = O.line_length(dims)
    rng = np.random.default_rng(3)
    slopes = list(itertools.product(*[range(d) for d in dims]))
    for trial in range(12):
        alpha = slopes[rng.integers(len(slopes))]
        tau = [int(rng.integers(d)) for d in dims]
        got = O.line_dft(O.gather_line(x, alpha, tau, L))
        want = np.zeros(L, dtype=np.complex128)
        for m in range(L):
            for f in O.projection_set(m, alpha, dims):
                ph = sum(f[k] * tau[k] / dims[k] for k in range(len(dims)))
                want[m] += X[f] * np.exp(2j * np.pi * ph)
        np.testing.assert_allclose(got, want, atol=1e-12)


def test_projection_bin_matches_rational_enumeration():
    for dims in [(4, 6), (6, 10), (2, 3, 4)]:
        L = O.line_length(dims)
        for alpha in itertools.product(*[range(d) for d in dims]):
            owner = {}
            for m in range(L):
                for f in O.projection_set(m, alpha, dims):
                    owner[f] = m
            fs = np.array(sorted(owner))
            np.testing.assert_array_equal(O.projection_bin(fs, alpha, dims),
                                          [owner[tuple(f)] for f in fs])


def test_axis_lines_are_numpy_fft_along_axis():
    """A slope e_k in a cube with N_k = L is a row/column: its line DFT is
    numpy's FFT along axis k, scaled by 1/N_k (Sec. 2.1's column DFT)."""
    dims = (16, 16, 16)
    x = W.random_dense(dims, 5)
    L = O.line_length(dims)
    for k in range(3):
        alpha = [0, 0, 0]; alpha[k] = 1
        tau = [3, 7, 11]
        got = O.line_dft(O.gather_line(x, alpha, tau, L))
        idx = list(tau); idx[k] = slice(None)
        # the line starts at tau_k: sample l is column entry (l + tau_k) mod N_k
        want = np.fft.fft(np.roll(x[tuple(idx)], -tau[k])) / dims[k]
        np.testing.assert_allclose(got, want, atol=1e-12)


def test_wrapping_axis_line_repeats_the_column():
    """N_0 = 4, N_1 = 8: L = 8, the slope (1, 0) visits the column twice, so
    only even bins are nonzero and bin 2q is the 4-point DFT's bin q."""
    dims = (4, 8)
    x = W.random_dense(dims, 6)
    got = O.line_dft(O.gather_line(x, (1, 0), (1, 5), 8))
    col = np.fft.fft(x[[1, 2, 3, 0], 5]) / 4
    np.testing.assert_allclose(got[0::2], col, atol=1e-12)
    np.testing.assert_allclose(got[1::2], 0, atol=1e-12)


# --------------------------------------------------------------------------
# Lemma 1 (line length) and Lemma 2 (slope set), by exhaustive enumeration
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [(2, 3), (4, 6), (6, 4), (2, 2, 3), (3, 5)])
def test_lemma1_lcm_is_minimal_orthogonal_length(dims):
    """With L = LCM every frequency, for every slope, lands exactly on a bin
    (Eq. gline has a solution m, and Eq. orthogonal's f(m) is 0 or 1 for all
    m); for every shorter length some slope and frequency fall between bins."""
    from fractions import Fraction
    grid = list(itertools.product(*[range(d) for d in dims]))

    def on_bin_grid(Lp):
        for alpha in grid:
            for f in grid:
                v = sum(Fraction(f[k] * alpha[k], dims[k]) for k in range(len(dims)))
                if (v * Lp).denominator != 1:
                    return False
        return True

    L = O.line_length(dims)
    assert L == math.lcm(*dims)
    assert on_bin_grid(L)
    assert not any(on_bin_grid(Lp) for Lp in range(1, L))
    for alpha in grid:
        for f in grid:
            v = sum(f[k] * alpha[k] / dims[k] for k in range(len(dims)))
            fh = np.array([np.mean(np.exp(2j * np.pi * np.arange(L) * (v - m / L)))
                           for m in range(L)])
            assert np.all(np.minimum(abs(fh), abs(fh - 1)) < 1e-9)
            assert np.sum(abs(fh - 1) < 1e-9) == 1


def paper_slope_set_2d(alpha, dims):
    """Lemma 2's set, written as the paper states it."""
    L = math.lcm(*dims)
    c0, c1 = L // dims[0], L // dims[1]
    a0, a1 = alpha
    return math.gcd(a0, a1) == 1 and math.gcd(a0, c1) == 1 and math.gcd(a1, c0) == 1


@pytest.mark.parametrize("dims", [(4, 6), (6, 10), (8, 8), (4, 12), (9, 6)])
def test_lemma2_uniform_disjoint_projection_2d(dims):
    L = O.line_length(dims)
    N = dims[0] * dims[1]
    n_in = 0
    for alpha in itertools.product(range(dims[0]), range(dims[1])):
        assert O.in_slope_set(alpha, dims) == paper_slope_set_2d(alpha, dims)
        if not O.in_slope_set(alpha, dims):
            continue
        n_in += 1
        sets = [O.projection_set(m, alpha, dims) for m in range(L)]
        assert all(len(s) == N // L for s in sets)
        assert len(set().union(*map(set, sets))) == N   # disjoint cover
    assert n_in > 0


@pytest.mark.parametrize("dims", [(2, 3, 4), (4, 4, 6), (3, 3, 3)])
def test_slope_set_gives_uniform_projection_3d(dims):
    L = O.line_length(dims)
    N = int(np.prod(dims))
    for alpha in itertools.product(*[range(d) for d in dims]):
        if O.in_slope_set(alpha, dims):
            sizes = [len(O.projection_set(m, alpha, dims)) for m in range(L)]
            assert sizes == [N // L] * L


# --------------------------------------------------------------------------
# Exact recovery of planted on-grid sinusoids (noiseless, fp64 input)
# --------------------------------------------------------------------------

def _recover(dims, K, seed, mag="unit", params=TH, cluster=0):
    cube = W.plant(dims, K, seed=seed, mag=mag, cluster=cluster)
    x = W.synthesize(dims, cube.freqs, cube.amps)      # complex128, exact model
    T = params.max_iters or O.default_max_iters(dims)
    al, ta = O.schedule(dims, T, seed + 1)
    return cube, O.run(x, al, ta, params)


@pytest.mark.parametrize("dims,K", [((64, 64), 8), ((16, 24), 12), ((32, 32), 40),
                                    ((8, 8, 12), 20), ((128, 64), 100),
                                    ((6, 10), 3), ((4, 6, 10, 2), 6)])
def test_planted_exact_recovery(dims, K):
    # Small cubes get more than the paper's budget of about N samples.
    T = max(O.default_max_iters(dims), 30)
    cube, res = _recover(dims, K, seed=sum(dims) + K, mag=(0.5, 1.5),
                         params=O.Params(**W.NOISELESS_THRESH, max_iters=T))
    assert res.status == O.STATUS_OK
    got = {tuple(f): a for f, a in zip(res.freqs.tolist(), res.amps)}
    want = {tuple(f): a for f, a in zip(cube.freqs.tolist(), cube.amps)}
    assert set(got) == set(want)
    assert max(abs(got[f] - want[f]) for f in want) < 1e-12
    # Canonical record order: iteration ascending, bin ascending.
    key = list(zip(res.rec_iter.tolist(), res.rec_bin.tolist()))
    assert key == sorted(key) and len(set(key)) == len(key)


def test_support_equals_brute_force_dft_nonzeros():
    for dims, K, seed in [((8, 8), 3, 1), ((6, 10), 4, 2), ((4, 4, 6), 5, 3)]:
        cube, res = _recover(dims, K, seed, params=O.Params(**W.NOISELESS_THRESH, max_iters=30))
        assert res.status == O.STATUS_OK
        X = O.dft_nd_direct(W.synthesize(dims, cube.freqs, cube.amps))
        nz = {tuple(int(v) for v in f) for f in np.argwhere(np.abs(X) > 1e-9)}
        assert {tuple(f) for f in res.freqs.tolist()} == nz
        for f, a in zip(res.freqs.tolist(), res.amps):
            assert abs(X[tuple(f)] - a) < 1e-12


def test_one_dimensional_case_is_the_full_dft():
    """D = 1: L = N and the only slope in A is 1, so every bin holds one
    frequency; even a dense spectrum comes out as numpy's FFT / N."""
    N = 32
    x = W.random_dense((N,), 9)
    al, ta = O.schedule((N,), 4, 1)
    assert (al == 1).all()
    res = O.run(x, al, ta, O.Params(**W.NOISELESS_THRESH, max_iters=4))
    assert res.status == O.STATUS_OK and res.iters == 2 and res.k == N
    X = np.fft.fft(x) / N
    np.testing.assert_allclose(res.amps[np.argsort(res.freqs[:, 0])], X, atol=1e-12)


def test_zero_input_stops_at_first_iteration():
    x = np.zeros((32, 48), dtype=np.complex64)
    al, ta = O.schedule(x.shape, 5, 1)
    res = O.run(x, al, ta, TH)
    assert res.status == O.STATUS_OK and res.iters == 1 and res.k == 0


def test_iteration_cap_and_capacity():
    dims = (64, 64)
    cube = W.plant(dims, 300, seed=5)
    al, ta = O.schedule(dims, 1, 6)
    res = O.run(cube.x, al, ta, O.Params(**W.NOISELESS_THRESH, max_iters=1))
    assert res.status == O.STATUS_INCOMPLETE and res.iters == 1 and 0 < res.k < 300
    al, ta = O.schedule(dims, 21, 6)
    res = O.run(cube.x, al, ta, O.Params(**W.NOISELESS_THRESH, max_k=10))
    assert res.status == O.STATUS_CAPACITY and res.k == 10


# --------------------------------------------------------------------------
# Deadlock (Sec. 2.1-2.2, Fig. 1's situation)
# --------------------------------------------------------------------------

def test_deadlock_axis_schedule_fails_random_slope_succeeds():
    dims = (8, 8)
    freqs = np.array([[0, 0], [0, 3], [2, 0], [2, 3]])
    amps = np.exp(2j * np.pi * np.array([0.1, 0.35, 0.6, 0.85]))
    x = W.synthesize(dims, freqs, amps)
    T = 6
    al = np.array([[1, 0], [0, 1]] * (T // 2))
    ta = np.array([[t % 8, (3 * t) % 8] for t in range(T)])
    res = O.run(x, al, ta, O.Params(**W.NOISELESS_THRESH, max_iters=T))
    assert res.status == O.STATUS_INCOMPLETE and res.k == 0
    # The diagonal projects the four corners to four distinct bins.
    assert sorted(O.projection_bin(freqs, (1, 1), dims).tolist()) == [0, 2, 3, 5]
    res = O.run(x, np.array([[1, 1], [1, 1]]), np.array([[0, 0], [5, 2]]),
                O.Params(**W.NOISELESS_THRESH, max_iters=2))
    assert res.status == O.STATUS_OK and res.k == 4 and res.iters == 2


# --------------------------------------------------------------------------
# The paper's printed numbers (Sec. 3), as cited fixtures
# --------------------------------------------------------------------------

def test_paper_sample_accounting():
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as f:
        g = json.load(f)
    assert O.default_max_iters((256, 256)) == g["tmax_256x256"]
    img = g["image_experiment"]
    dims = tuple(img["dims"])
    assert O.line_length(dims) == img["line_length"]
    N = dims[0] * dims[1]
    for pct, iters in zip(img["percent_samples"], img["iterations"]):
        # The printed percentages are the exact ratios cut to one decimal
        # (14.0625 -> 14.0, 23.4375 -> 23.4, 70.3125 -> 70.3).
        assert math.floor(1000.0 * O.samples_used(dims, iters) / N) / 10.0 == pct
    k256 = g["k_equals_n0_256x256"]
    frac = 100.0 * O.samples_used((256, 256), k256["iterations"]) / 65536
    assert abs(frac - k256["percent_samples"]) < 0.1


@pytest.mark.slow
def test_statistics_match_the_paper_at_256x256():
    """Fig. 2's regime at reduced Monte-Carlo size: K = N0 recovers with
    about 5.9% of samples; K = 5 N0 recovers almost always within T_max = 85
    (the paper: about 96%); K = 6 N0 never does."""
    dims = (256, 256)
    iters = []
    for s in range(8):
        cube, res = _recover(dims, 256, seed=1000 + s)
        assert res.status == O.STATUS_OK
        assert {tuple(f) for f in res.freqs.tolist()} == {tuple(f) for f in cube.freqs.tolist()}
        iters.append(res.iters - 1)           # decoding iterations
    pct = 100.0 * np.mean([O.samples_used(dims, i) for i in iters]) / 65536
    assert 3.5 < pct < 8.5
    ok = sum(_recover(dims, 1280, seed=2000 + s)[1].status == O.STATUS_OK for s in range(6))
    assert ok >= 4
    ok6 = sum(_recover(dims, 1536, seed=3000 + s)[1].status == O.STATUS_OK for s in range(3))
    assert ok6 == 0


@pytest.mark.slow
def test_clustered_supports_recover():
    for cl in (9, 25):
        for s in range(2):
            cube, res = _recover((256, 256), 256, seed=4000 + 10 * cl + s, cluster=cl)
            assert res.status == O.STATUS_OK
            assert {tuple(f) for f in res.freqs.tolist()} == {tuple(f) for f in cube.freqs.tolist()}


# --------------------------------------------------------------------------
# The 1-sparsity test and decode on hand-built residuals
# --------------------------------------------------------------------------

def test_decide_bins_on_constructed_residuals():
    dims = (16, 24)
    L = 48
    r = np.zeros((3, L), dtype=np.complex128)
    a = 0.7 * np.exp(0.4j)
    m0, m1 = 5, 17
    r[0, 3] = a
    r[1, 3] = a * np.exp(2j * np.pi * m0 / 16)
    r[2, 3] = a * np.exp(2j * np.pi * m1 / 24)
    b1, b2 = 0.9, 0.6 * np.exp(1.1j)   # two frequencies in bin 9
    r[0, 9] = b1 + b2
    r[1, 9] = b1 * np.exp(2j * np.pi * 2 / 16) + b2 * np.exp(2j * np.pi * 7 / 16)
    r[2, 9] = b1 * np.exp(2j * np.pi * 4 / 24) + b2 * np.exp(2j * np.pi * 1 / 24)
    r[:, 20] = 1e-5                    # below theta0
    anyz, cand, dec = O.decide_bins(r, dims, TH)
    assert anyz
    assert np.nonzero(cand)[0].tolist() == [3]
    assert dec[3].tolist() == [m0, m1]
    anyz, cand, _ = O.decide_bins(np.full((3, L), 1e-5 + 0j), dims, TH)
    assert not anyz and not cand.any()


# --------------------------------------------------------------------------
# Amplitudes as a linear map of the samples (support fixed)
# --------------------------------------------------------------------------

def _fixed_run(dims, K, seed):
    cube = W.plant(dims, K, seed=seed)
    x = W.synthesize(dims, cube.freqs, cube.amps)
    al, ta = O.schedule(dims, 30, seed + 1)
    return x, al, ta, O.run(x, al, ta, O.Params(**W.NOISELESS_THRESH, max_iters=30))


def test_replay_reproduces_the_run_and_is_linear():
    x, al, ta, res = _fixed_run((32, 48), 60, 21)
    assert len(set(res.rec_iter.tolist())) >= 2
    rep = O.replay_amplitudes(x, res.rec_freqs, res.rec_iter, res.rec_bin, al, ta)
    np.testing.assert_allclose(rep, res.rec_amps, atol=1e-12)
    np.testing.assert_allclose(O.replay_set(x, res, al, ta), res.amps, atol=1e-12)
    rng = np.random.default_rng(0)
    y = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
    z = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
    f = lambda v: O.replay_amplitudes(v, res.rec_freqs, res.rec_iter, res.rec_bin, al, ta)
    np.testing.assert_allclose(f(2.5 * y - 1j * z), 2.5 * f(y) - 1j * f(z), atol=1e-11)


def test_single_iteration_amplitude_map_closed_form():
    """If every record comes from one iteration, a_i = exp(-j theta_i) *
    (1/L) sum_l x[n(l)] exp(-j 2 pi l m_i / L): row i of M holds exactly
    those L coefficients on the line-0 positions (Eq. hs, Eq. decoding)."""
    dims = (16, 16)
    freqs = np.array([[1, 2], [5, 9], [0, 7]])       # bins 3, 14, 7 under (1, 1)
    x = W.synthesize(dims, freqs, np.exp(1j * np.array([0.3, 1.7, 4.0])))
    al, ta = np.array([[1, 1], [1, 3]]), np.array([[2, 5], [7, 1]])
    res = O.run(x, al, ta, O.Params(**W.NOISELESS_THRESH, max_iters=2))
    assert res.status == O.STATUS_OK and set(res.rec_iter.tolist()) == {0}
    L = 16
    pos = O.line_positions(dims, al[0], ta[0], L)
    flat = np.ravel_multi_index(tuple(pos.T), dims)
    M = O.amp_matrix(dims, res, al, ta, np.arange(256))
    for i in range(res.k):
        th = 2 * np.pi * sum(res.freqs[i, k] * ta[0, k] / dims[k] for k in range(2))
        row = np.zeros(256, dtype=np.complex128)
        row[flat] = np.exp(-1j * th) * np.exp(-2j * np.pi * np.arange(L) * res.rec_bin[i] / L) / L
        np.testing.assert_allclose(M[i], row, atol=1e-13)


def test_fd_gradient_equals_conjugate_transpose_map():
    """grad of sum |a|^2 = 2 M^H a (PyTorch's complex convention); central
    differences of the quadratic loss are exact, and no sample off the
    touched lines has a gradient."""
    x, al, ta, res = _fixed_run((16, 24), 30, 31)
    assert len(set(res.rec_iter.tolist())) >= 2
    allpos = np.arange(16 * 24)
    g = O.grad_sum_abs2_fd(x, res, al, ta, positions=allpos)
    M = O.amp_matrix(x.shape, res, al, ta, allpos)
    np.testing.assert_allclose(g.reshape(-1), 2 * M.conj().T @ res.amps, atol=1e-9)
    touched = O.touched_positions(x.shape, res.rec_iter, al, ta)
    off = np.setdiff1d(allpos, touched)
    assert np.all(g.reshape(-1)[off] == 0)


# --------------------------------------------------------------------------
# The recovered set: distinct frequencies, nonzero amplitudes (Eq. sigModel2)
# --------------------------------------------------------------------------

def test_merge_detections_by_hand():
    """A frequency detected twice is one element of the set with the sum of
    the amplitudes, at the position of its first detection; a sum at or
    below theta0 leaves the set (a != 0) and is reported as dropped."""
    a, b, c = 0.5 + 0.2j, -0.3 + 0.9j, 0.25 - 0.1j
    f = np.array([[1, 2], [3, 4], [1, 2]])
    fk, ak, fd, ad, sin = O.merge_detections(f, np.array([a, b, c]), 1e-3)
    assert fk.tolist() == [[1, 2], [3, 4]] and len(fd) == 0
    np.testing.assert_allclose(ak, [a + c, b], rtol=0, atol=1e-15)
    assert sin.tolist() == [0, 1, 0]
    f = np.array([[1, 2], [3, 4], [1, 2], [1, 2], [5, 6]])
    fk, ak, fd, ad, sin = O.merge_detections(f, np.array([a, b, c, -(a + c) + 1e-6, 2.0]), 1e-3)
    assert fk.tolist() == [[3, 4], [5, 6]] and fd.tolist() == [[1, 2]]
    np.testing.assert_allclose(ak, [b, 2.0], rtol=0, atol=1e-15)
    assert abs(ad[0] - 1e-6) < 1e-15
    assert sin.tolist() == [2, 0, 2, 2, 1]       # the dropped frequency follows the set
    # a single detection stays, whatever its amplitude
    fk, ak, fd, ad, sin = O.merge_detections(np.array([[0, 1]]), np.array([1e-9]), 1e-3)
    assert fk.tolist() == [[0, 1]] and len(fd) == 0


def test_redetection_in_the_batched_workload_is_merged():
    """Cube 148 of the batched workload (128 x 64, K = 275): a false
    detection at iteration 5 is found again at iteration 6 with the opposite
    amplitude. The set keeps the 275 planted frequencies; the false one
    leaves it with an amplitude sum of rounding size. The detections' sum
    per frequency equals the set's amplitudes (construction-subtraction of
    the list and of the set agree: linearity)."""
    cube = W.cfg4(only=[148])[0]
    assert cube.dims == (128, 64) and len(cube.amps) == 275
    al, ta = O.schedule(cube.dims, O.default_max_iters(cube.dims), cube.schedule_seed)
    res = O.run(cube.x, al, ta, O.Params(**W.NOISELESS_THRESH, max_k=512))
    assert res.status == O.STATUS_OK and res.n == 277 and res.k == 275
    assert {tuple(f) for f in res.freqs.tolist()} == {tuple(f) for f in cube.freqs.tolist()}
    assert res.dropped_freqs.tolist() == [[83, 46]] and abs(res.dropped_amps[0]) < 1e-5
    twice = [i for i in range(res.n) if res.rec_freqs[i].tolist() == [83, 46]]
    assert [int(res.rec_iter[i]) for i in twice] == [5, 6]
    assert abs(res.rec_amps[twice[0]]) > 1.0
    assert all(res.rec_sin[i] == res.k for i in twice)
    total = np.zeros(res.k + 1, dtype=np.complex128)
    np.add.at(total, res.rec_sin, res.rec_amps)
    np.testing.assert_allclose(total[:res.k], res.amps, atol=1e-15)
    want = {tuple(f): a for f, a in zip(cube.freqs.tolist(), cube.amps)}
    assert max(abs(want[tuple(f)] - a) for f, a in zip(res.freqs.tolist(), res.amps)) < 1e-5
    # replay reproduces the merged set (decisions fixed) and stays linear
    x = cube.x.astype(np.complex128)
    np.testing.assert_allclose(O.replay_set(x, res, al, ta), res.amps, atol=1e-12)


def test_noisy_set_is_a_set():
    """Under noise (20 dB) frequencies are found again; the output is still
    a set of distinct frequencies with |a| > theta0 in the order of first
    detection, and the detection amplitudes sum to it."""
    cube = W.plant((128, 128), 60, seed=42, mag=(0.5, 1.5), snr_db=20.0)
    th = W.cfg2_thresh(cube, 128)
    al, ta = O.schedule(cube.dims, 42, cube.schedule_seed)
    res = O.run(cube.x, al, ta, O.Params(**th, max_k=4096))
    assert res.n > res.k + len(res.dropped_amps)           # some frequency found twice
    keys = [tuple(f) for f in res.freqs.tolist()]
    assert len(set(keys)) == len(keys)
    assert np.all(np.abs(res.amps) > np.float32(th["zero_thresh"]))
    first = {}
    for i, f in enumerate(res.rec_freqs.tolist()):
        first.setdefault(tuple(f), i)
    pos = [first[k] for k in keys]
    assert pos == sorted(pos)
    total = np.zeros(res.k + len(res.dropped_amps), dtype=np.complex128)
    np.add.at(total, res.rec_sin, res.rec_amps)
    np.testing.assert_allclose(total[:res.k], res.amps, atol=1e-12)


@pytest.mark.parametrize("case", ["cfg1", "cfg4_sample", "odd_shapes"])
def test_float32_decisions_agree_on_the_workloads(case):
    """The reference decides in fp64; the kernels decide in float32. On
    these workloads a float32 decision step gives the same decisions, i.e.
    no decision lies within float32 rounding of its threshold (the margins
    of the default thresholds are 20x or more)."""
    if case == "cfg1":
        cubes = [W.cfg1()]
    elif case == "cfg4_sample":
        cubes = W.cfg4(only=range(0, 1024, 64))
    else:
        cubes = [W.plant(d, k, seed=s, mag=(0.5, 1.5)) for d, k, s in
                 [((16, 24), 12, 1), ((6, 10), 3, 2), ((8, 8, 12), 20, 3), ((7, 9), 4, 4)]]
    for c in cubes:
        T = max(O.default_max_iters(c.dims), 30) if np.prod(c.dims) < 4096 else 0
        T = T or O.default_max_iters(c.dims)
        al, ta = O.schedule(c.dims, T, c.schedule_seed)
        r64 = O.run(c.x, al, ta, O.Params(**W.NOISELESS_THRESH, max_iters=T, max_k=512))
        r32 = O.run(c.x, al, ta, O.Params(**W.NOISELESS_THRESH, max_iters=T, max_k=512, decision="float32"))
        assert (r64.status, r64.iters, r64.n) == (r32.status, r32.iters, r32.n)
        np.testing.assert_array_equal(r64.rec_freqs, r32.rec_freqs)
        np.testing.assert_array_equal(r64.rec_bin, r32.rec_bin)
