"""Host logic of the Fig. 2 sweep (no GPU): planting, cluster structure,
determinism, and the perfect-recovery criterion on oracle results."""
import numpy as np

import fig2
import oracle as O
import workloads as W


def test_plant_sweep_is_deterministic_and_labelled():
    a, la = fig2.plant_sweep((16, 64), 3, (0, 9), seed=5)
    b, lb = fig2.plant_sweep((16, 64), 3, (0, 9), seed=5)
    assert la == lb == [(cl, K, r) for cl in (0, 9) for K in (16, 64) for r in range(3)]
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x.freqs, y.freqs)
        assert x.schedule_seed == y.schedule_seed
    seeds = {c.schedule_seed for c in a}
    assert len(seeds) == len(a)


def test_clustered_supports_hold_a_wrapping_block():
    cubes, labels = fig2.plant_sweep((64,), 4, (25,), seed=3)
    for c in cubes:
        f = {tuple(v) for v in c.freqs.tolist()}
        assert len(f) == 64
        # some 5x5 block (wrapping at 256) is fully contained in the support
        hit = False
        for r0, c0 in f:
            if all(((r0 + i) % 256, (c0 + j) % 256) in f for i in range(5) for j in range(5)):
                hit = True
                break
        assert hit


def test_perfect_criterion_on_oracle_results():
    cubes, _ = fig2.plant_sweep((64,), 2, (0,), seed=7)
    for c in cubes:
        al, ta = O.schedule(c.dims, O.default_max_iters(c.dims), c.schedule_seed)
        r = O.run(c.x, al, ta, O.Params(**W.NOISELESS_THRESH, max_k=128))
        host = dict(status=r.status, k=r.k, freqs=r.freqs, amps=r.amps)
        assert fig2.perfect(host, c)
        bad = dict(host, amps=r.amps * 1.01)
        assert not fig2.perfect(bad, c)
        short = dict(host, k=r.k - 1, freqs=r.freqs[:-1], amps=r.amps[:-1])
        assert not fig2.perfect(short, c)


def test_image_like_support_is_clustered_and_exact():
    c = W.image_like((64, 72), 300, seed=5)
    f = {tuple(v) for v in c.freqs.tolist()}
    assert len(f) == 300 and len(c.amps) == 300
    assert np.all(np.isreal(c.amps)) and c.amps.real.min() >= 0.5 and c.amps.real.max() <= 1.5
    # clustered: most pixels have a 4-neighbour in the support (uniform: ~26%)
    nb = sum(any(((a + da) % 64, (b + db) % 72) in f for da, db in ((1, 0), (-1, 0), (0, 1), (0, -1)))
             for a, b in f)
    assert nb / len(f) > 0.8
    # duality: the DFT of x is the image
    X = np.fft.fftn(c.x.astype(np.complex128)) / c.x.size
    img = np.zeros((64, 72), dtype=np.complex128)
    img[tuple(c.freqs.T)] = c.amps
    assert np.abs(X - img).max() < 1e-5
