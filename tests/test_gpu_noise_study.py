"""The noise study of the amplitude variants on the batched GPU path:
statistics at high SNR (exact support; the line average cuts the amplitude
error by about sqrt(D+1) = sqrt(3)), sampled cubes against the FP64 oracle
at 60 dB, and the oracle agreement at 20 dB reported (parity unpinned there:
near-threshold decisions flip between fp32 and fp64)."""
import numpy as np
import pytest

import oracle as O
from gpu_common import compare, log, oracle_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def study():
    import noise_study
    return noise_study.sweep(snrs=(20.0, 60.0), runs=16, seed=5, log=log)


def _row(res, variant, snr):
    return next(r for r in res["table"] if r["variant"] == variant and r["snr_db"] == snr)


def test_noise_study_statistics(study):
    for r in study["table"]:
        log(f"{r['variant']:>8} {r['snr_db']:4.0f} dB: recall {r['recall']:.3f} precision {r['precision']:.3f} "
            f"amp_err {r['amp_err']} ok {r['ok']:.2f} iters {r['iters']:.1f}")
    for v in ("line0", "average"):
        r = _row(study, v, 60.0)
        assert r["recall"] == 1.0 and r["precision"] == 1.0 and r["ok"] == 1.0
    ratio = _row(study, "average", 60.0)["amp_err"] / _row(study, "line0", 60.0)["amp_err"]
    log(f"60 dB amplitude error, average / line 0: {ratio:.3f} (1/sqrt(3) = 0.577)")
    assert 0.45 < ratio < 0.75


def test_noise_study_sampled_cubes_match_the_oracle(study):
    plan, specs, cubes, labels = study["plan"], study["specs"], study["cubes"], study["labels"]
    n = len(cubes)
    agree = []
    for vi in range(2):
        for i, (snr, r) in enumerate(labels):
            if r >= 2:
                continue
            j = vi * n + i
            ref, _, _ = oracle_for(plan, j, cubes[i].x, specs[j])
            got = study["hosts"][j]
            if snr >= 60.0:
                compare(got, ref, f"{snr} dB run {r} variant {vi}", amp_tol=1e-4)
            else:
                g = {tuple(f) for f in got["freqs"][:got["k"]].tolist()}
                o = {tuple(f) for f in ref.freqs.tolist()}
                agree.append(len(g & o) / max(1, len(g | o)))
    log(f"20 dB record-set agreement with the oracle (Jaccard): {np.round(agree, 2).tolist()}")
