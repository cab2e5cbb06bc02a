"""Host logic of the noise study (no GPU): planting and scoring."""
import numpy as np

import noise_study as N


def test_plant_sweep_is_deterministic_with_requested_snr():
    a, la = N.plant_sweep((20.0, 40.0), 2, seed=3)
    b, lb = N.plant_sweep((20.0, 40.0), 2, seed=3)
    assert la == lb == [(20.0, 0), (20.0, 1), (40.0, 0), (40.0, 1)]
    for x, y, (snr, _) in zip(a, b, la):
        np.testing.assert_array_equal(x.x, y.x)
        want = np.sqrt(np.sum(np.abs(x.amps) ** 2) / 10 ** (snr / 10))
        assert abs(x.noise_sigma - want) < 1e-12
        # the sample noise power is the requested one within sampling error
        clean = np.fft.ifftn(_dense(x)) * x.x.size
        assert abs(np.std(x.x - clean) / want - 1) < 0.02


def _dense(cube):
    X = np.zeros(cube.dims, dtype=np.complex128)
    X[tuple(cube.freqs.T)] = cube.amps
    return X


def test_score_counts_hits_and_sums_repeated_records():
    cubes, _ = N.plant_sweep((60.0,), 1, seed=4)
    c = cubes[0]
    f = c.freqs
    host = dict(k=len(f) + 2, freqs=np.concatenate([f, f[:1], [[0, 0]]]) if (0, 0) not in set(map(tuple, f.tolist()))
                else np.concatenate([f, f[:1], [[1, 1]]]),
                amps=np.concatenate([c.amps * 0.5, [0.5 * c.amps[0]], [1.0]]))
    s = N.score(host, c)
    assert s["recall"] == 1.0
    assert abs(s["precision"] - len(f) / (len(f) + 1)) < 1e-12
    # every amplitude halved except the first, restored by its repeated record
    want = np.linalg.norm(0.5 * c.amps[1:]) / np.linalg.norm(c.amps)
    assert abs(s["amp_err"] - want) < 1e-12
