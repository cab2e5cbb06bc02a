"""The allocation-free plain entry point (fpssft_execute_noalloc) through
the C ABI against fpssft_execute: two calls in a row, the second on a
smaller cube, each bit-identical to the allocating entry point and equal to
the FP64 oracle; one cube with its record store in device memory (the
static scratch array); a cube needing more than the array is rejected."""
import numpy as np
import pytest

import workloads as W
from gpu_common import compare, log, oracle_for, spec_for, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_1711_11407_amd as F
    return F


KEYS = ("freqs", "amps", "dropped_freqs", "dropped_amps", "rec_iter", "rec_bin", "rec_sin")


def check_same(a, b, what):
    for key in ("k", "n", "kd", "iters", "status"):
        assert a[key] == b[key], (what, key)
    for key in KEYS:
        np.testing.assert_array_equal(a[key], b[key], err_msg=f"{what} {key}")


def test_noalloc_equals_execute_two_calls_shrinking(F):
    torch, dev = torch_dev()
    # large cube first (pre-chunk of 8 iterations of 3 x 512 values), then a
    # smaller one, then a cube whose records live in the scratch array
    cubes = [W.plant((512, 256), 280, seed=91, mag=(0.5, 1.5)),
             W.plant((64, 128), 60, seed=92, mag=(0.5, 1.5)),
             W.plant((256, 256), 600, seed=93, mag=(0.5, 1.5))]
    specs = [spec_for(F, cubes[0].dims, 191, max_k=512), spec_for(F, cubes[1].dims, 192, max_k=128),
             spec_for(F, cubes[2].dims, 193, max_k=20000)]
    plan = F.Plan(specs, tuning=dict(chunk_iters=8))
    for c in range(len(cubes)):
        log(f"no-alloc cube {c} {cubes[c].dims}")
        x = torch.from_numpy(cubes[c].x).to(dev)
        want = plan.execute(c, x).host()
        out = plan.alloc_result(c, dev)
        got = plan.execute_noalloc(c, x, out).host()
        check_same(got, want, f"cube {c}")
        ref, _, _ = oracle_for(plan, c, cubes[c].x, specs[c])
        compare(got, ref, f"no-alloc cube {c}")
        # the same call again into the same outputs
        got2 = plan.execute_noalloc(c, x, out).host()
        check_same(got2, want, f"cube {c} again")


def test_noalloc_rejects_more_than_the_array(F):
    torch, dev = torch_dev()
    cube = W.plant((256, 256), 40, seed=94)
    # records in device memory: 200000 slots of 24 bytes and their hash exceed 4 MiB
    spec = spec_for(F, cube.dims, 195, max_k=200000)
    plan = F.Plan([spec])
    x = torch.from_numpy(cube.x).to(dev)
    out = plan.alloc_result(0, dev)
    with pytest.raises(F.FpsSftError) as e:
        plan.execute_noalloc(0, x, out)
    assert e.value.status == -2
    # the plan still works through the allocating entry point
    assert plan.execute(0, x).host()["status"] == 0
