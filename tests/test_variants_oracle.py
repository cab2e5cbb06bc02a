"""Pins of the oracle's method variants: the axis-aligned schedule (the
row/column lines of the method reviewed in Sec. 2.1) and line-averaged
amplitudes. The checks use library routines, planted ground truth, the
deadlock construction of Sec. 2.2 and a closed-form variance ratio; none
re-types the oracle's formulas."""
import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.mark.parametrize("dims", [(8, 8), (16, 24), (4, 6, 10), (32,)])
def test_axis_schedule_cycles_unit_slopes(dims):
    T = 9
    al, ta = O.schedule(dims, T, seed=5, axis=True)
    D = len(dims)
    for t in range(T):
        want = [(1 if k == t % D else 0) % dims[k] for k in range(D)]
        assert al[t].tolist() == want
    assert ((ta >= 0) & (ta < np.array(dims))).all()
    # no slope is drawn: the offsets are the stream's consecutive draws
    z = [(O.splitmix64(5, i) * dims[i % D]) >> 64 for i in range(T * D)]
    assert ta.ravel().tolist() == z


def test_axis_schedule_lines_are_numpy_fft_along_the_axes():
    """With alpha = e_0 a line of a square cube is a column from offset tau_0,
    with alpha = e_1 a row: the line DFT is numpy's FFT of that column or
    row, divided by N (projection-slice, axis case)."""
    dims = (16, 16)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(dims) + 1j * rng.standard_normal(dims)
    al, ta = O.schedule(dims, 4, seed=11, axis=True)
    L = O.line_length(dims)
    for t in range(4):
        got = O.line_dft(O.gather_line(x, al[t], ta[t], L))
        t0, t1 = (int(v) for v in ta[t])
        seq = np.roll(x[:, t1], -t0) if t % 2 == 0 else np.roll(x[t0, :], -t1)
        np.testing.assert_allclose(got, np.fft.fft(seq) / 16, atol=1e-13)


def test_axis_schedule_deadlocks_where_random_slopes_recover():
    """Sec. 2.2: frequencies on the corners of a rectangle share a bin on
    every row and every column, so the axis-aligned lines never see a
    1-sparse bin; the random slopes of FPS-SFT recover all four."""
    dims = (16, 16)
    freqs = np.array([[1, 2], [1, 9], [12, 2], [12, 9]])
    amps = np.exp(2j * np.pi * np.array([0.05, 0.3, 0.55, 0.8]))
    x = W.synthesize(dims, freqs, amps)
    T = 20
    params = O.Params(**W.NOISELESS_THRESH, max_iters=T)
    al, ta = O.schedule(dims, T, seed=21, axis=True)
    res = O.run(x, al, ta, params)
    assert res.status == O.STATUS_INCOMPLETE and res.k == 0 and res.iters == T
    al, ta = O.schedule(dims, T, seed=21)
    res = O.run(x, al, ta, params)
    assert res.status == O.STATUS_OK
    assert {tuple(f) for f in res.freqs.tolist()} == {tuple(f) for f in freqs.tolist()}


@pytest.mark.parametrize("dims,K", [((64, 64), 8), ((16, 24), 12), ((8, 8, 12), 20), ((6, 10), 3)])
def test_line_averaged_amplitudes_recover_planted_truth(dims, K):
    cube = W.plant(dims, K, seed=sum(dims) + 7 * K, mag=(0.5, 1.5))
    x = W.synthesize(dims, cube.freqs, cube.amps)          # complex128, exact to rounding
    T = max(O.default_max_iters(dims), 30)
    al, ta = O.schedule(dims, T, cube.schedule_seed)
    base = O.run(x, al, ta, O.Params(**W.NOISELESS_THRESH, max_iters=T))
    avg = O.run(x, al, ta, O.Params(**W.NOISELESS_THRESH, max_iters=T, amp_average=True))
    assert avg.status == O.STATUS_OK
    np.testing.assert_array_equal(avg.freqs, base.freqs)
    np.testing.assert_array_equal(avg.rec_iter, base.rec_iter)
    want = {tuple(f): a for f, a in zip(cube.freqs.tolist(), cube.amps)}
    got = {tuple(f): a for f, a in zip(avg.freqs.tolist(), avg.amps)}
    assert set(got) == set(want)
    assert max(abs(got[f] - want[f]) for f in want) < 1e-12


def test_line_averaged_amplitude_has_a_third_of_the_variance():
    """One sinusoid plus white noise, 2-D: the D+1 = 3 lines hold disjoint
    samples, so each line's bin value carries independent noise of the same
    variance; their phase-aligned mean has 1/3 of the squared error of line
    0 alone (binomial-scale tolerance over 600 trials)."""
    dims = (32, 32)
    L = 32
    sigma = 0.02                     # per sample; per bin sigma / sqrt(L)
    params = dict(zero_thresh=0.2, mag_rel_tol=0.2, grid_tol=0.25, max_iters=3)
    e0, e1 = [], []
    rng = np.random.default_rng(9)
    for trial in range(600):
        f = rng.integers(0, 32, size=2)
        a = np.exp(2j * np.pi * rng.random())
        x = W.synthesize(dims, f[None, :], np.array([a]))
        x = x + sigma / np.sqrt(2) * (rng.standard_normal(dims) + 1j * rng.standard_normal(dims))
        al, ta = O.schedule(dims, 3, seed=trial)
        r0 = O.run(x, al, ta, O.Params(**params))
        r1 = O.run(x, al, ta, O.Params(**params, amp_average=True))
        assert r0.k >= 1 and r1.k >= 1 and r0.freqs[0].tolist() == f.tolist()
        e0.append(abs(r0.amps[0] - a) ** 2)
        e1.append(abs(r1.amps[0] - a) ** 2)
    ratio = np.mean(e1) / np.mean(e0)
    assert abs(np.mean(e0) / (sigma ** 2 / L) - 1) < 0.2     # line 0: sigma^2 / L
    assert 0.27 < ratio < 0.40, ratio
