"""The method variants on the GPU against the FP64 oracle with the same
options: the time-domain construction-subtraction of Sec. 2.2 (the oracle's
own form), line-averaged amplitudes, and the axis-aligned schedule with its
deadlock. Plain and batched paths; mixed plans where variant cubes and
default cubes run in different kernel instantiations of one launch."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import compare, log, oracle_for, spec_for, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_1711_11407_amd as F
    return F


def run_both(F, cubes, specs, tuning=None):
    """Plain and batched results of every cube, each checked against the
    oracle; returns the plain host results."""
    torch, dev = torch_dev()
    plan = F.Plan(specs, tuning=tuning)
    xs = [torch.from_numpy(c.x).to(dev) for c in cubes]
    plain = [plan.execute(i, xs[i]).host() for i in range(len(cubes))]
    batched = [o.host() for o in plan.execute_batched(xs)]
    for i, c in enumerate(cubes):
        ref, _, _ = oracle_for(plan, i, c.x, specs[i])
        compare(plain[i], ref, f"plain {c.dims} K={len(c.amps)}")
        compare(batched[i], ref, f"batched {c.dims} K={len(c.amps)}")
    return plain


LITERAL = [((64, 64), 8, 0), ((256, 256), 100, 0), ((128, 64), 274, 0), ((16, 24), 12, 30),
           ((6, 10), 3, 30), ((512, 512), 300, 0), ((128, 128, 128), 200, 40), ((2048,), 30, 3)]


@pytest.mark.parametrize("dims,K,T", LITERAL)
def test_literal_peel_matches_oracle(F, dims, K, T):
    cube = W.plant(dims, K, seed=700 + K, mag=(0.5, 1.5))
    spec = spec_for(F, dims, 701 + K, max_iters=T, max_k=max(64, 2 * K), literal_peel=True)
    log(f"literal peel dims={dims} K={K}")
    got = run_both(F, [cube], [spec])[0]
    # the same decisions as the frequency-domain peel
    dflt = run_both(F, [cube], [spec_for(F, dims, 701 + K, max_iters=T, max_k=max(64, 2 * K))])[0]
    for key in ("freqs", "rec_iter", "rec_bin"):
        np.testing.assert_array_equal(got[key], dflt[key])


def test_literal_peel_records_in_global_memory(F):
    cube = W.plant((256, 256), 600, seed=5, mag=(0.5, 1.5))
    run_both(F, [cube], [spec_for(F, cube.dims, 6, max_k=30000, literal_peel=True)])


AVG = [((64, 64), 8, 0), ((256, 256), 100, 0), ((16, 24), 12, 30), ((512, 576), 300, 0),
       ((128, 128, 128), 200, 40), ((64, 512), 150, 0)]


@pytest.mark.parametrize("dims,K,T", AVG)
def test_line_averaged_amplitudes_match_oracle(F, dims, K, T):
    cube = W.plant(dims, K, seed=800 + K, mag=(0.5, 1.5))
    spec = spec_for(F, dims, 801 + K, max_iters=T, max_k=max(64, 2 * K), amp_average=True)
    log(f"line-averaged amplitudes dims={dims} K={K}")
    got = run_both(F, [cube], [spec])[0]
    want = {tuple(f): a for f, a in zip(cube.freqs.tolist(), cube.amps)}
    if got["status"] == O.STATUS_OK:
        err = max(abs(a - want[tuple(f)]) for f, a in zip(got["freqs"].tolist(), got["amps"]))
        assert err < 1e-4, err


def test_axis_schedule_deadlock_and_recovery(F):
    """Rectangle corners: the axis-aligned lines never isolate them (Sec.
    2.2); the default schedule recovers them. Both as the oracle."""
    dims = (16, 16)
    freqs = np.array([[1, 2], [1, 9], [12, 2], [12, 9]])
    amps = np.exp(2j * np.pi * np.array([0.05, 0.3, 0.55, 0.8]))
    x = W.synthesize(dims, freqs, amps).astype(np.complex64)
    cube = W.Cube(x=x, freqs=freqs, amps=amps, seed=20)
    specs = [spec_for(F, dims, 21, max_iters=20, axis_schedule=True), spec_for(F, dims, 21, max_iters=20)]
    got = run_both(F, [cube, cube], specs)
    assert got[0]["status"] == O.STATUS_INCOMPLETE and got[0]["k"] == 0 and got[0]["iters"] == 20
    assert got[1]["status"] == O.STATUS_OK and got[1]["k"] == 4


def test_axis_schedule_recovers_separable_support(F):
    cube = W.plant((64, 64), 6, seed=901, mag=(0.5, 1.5))
    spec = spec_for(F, cube.dims, 902, max_iters=40, axis_schedule=True)
    got = run_both(F, [cube], [spec])[0]
    log(f"axis schedule, K=6 at 64x64: status {got['status']} after {got['iters']} iterations")


@pytest.mark.parametrize("direct", [0, 1])
def test_mixed_variants_in_one_batched_launch(F, direct):
    """Default, literal, averaged and axis cubes of several shapes in one
    plan: the batched launch (one persistent kernel per instantiation) gives
    every cube the oracle's result."""
    shapes = [(64, 64), (128, 256), (16, 24), (256, 256), (64, 128), (512, 512)]
    cubes, specs = [], []
    for i, d in enumerate(shapes * 2):
        c = W.plant(d, 20 + 13 * i, seed=950 + i, mag=(0.5, 1.5))
        opt = [dict(), dict(literal_peel=True), dict(amp_average=True),
               dict(literal_peel=True, amp_average=True)][i % 4]
        T = 30 if d == (16, 24) else 0
        cubes.append(c)
        specs.append(spec_for(F, d, 960 + i, max_iters=T, max_k=256, **opt))
    run_both(F, cubes, specs, tuning=dict(direct_launch=direct))


def test_variant_limits(F):
    torch, dev = torch_dev()
    # the adjoint follows the line-0 amplitude only
    cube = W.plant((64, 64), 8, seed=3)
    plan = F.Plan([spec_for(F, cube.dims, 4, amp_average=True)])
    x = torch.from_numpy(cube.x).to(dev)
    res = plan.execute(0, x)
    with pytest.raises(F.FpsSftError) as e:
        plan.amp_backward(0, res, 2 * res.amps)
    assert e.value.status == -2
    # the time-domain construction-subtraction needs the lines in LDS
    with pytest.raises(F.FpsSftError) as e:
        F.Plan([spec_for(F, (512, 576), 4, literal_peel=True)])
    assert e.value.status == -2
