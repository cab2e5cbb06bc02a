"""Seeded random sweep of valid problems against the FP64 oracle: random
dimension count, side lengths with mixed prime factors (radix 2/3/5/7
stages, power-of-two and other line lengths), sparsity, capacity and
iteration limits (OK, INCOMPLETE and CAPACITY outcomes) and method flags.
Every cube runs on the plain path and, all together in one plan (several
kernel instantiations), on the batched path in both launch forms."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import compare, log, oracle_for, spec_for, torch_dev

pytestmark = pytest.mark.gpu

SIDES = {1: (30, 64, 96, 105, 128, 256, 448),
         2: (4, 6, 8, 10, 12, 14, 16, 20, 24, 32, 48, 64),
         3: (4, 6, 8, 10, 12, 16),
         4: (2, 3, 4, 6)}


def draw_cases(n, seed):
    rng = np.random.default_rng(seed)
    cases = []
    while len(cases) < n:
        D = int(rng.choice([1, 2, 2, 2, 3, 3, 4]))
        dims = tuple(int(rng.choice(SIDES[D])) for _ in range(D))
        N = int(np.prod(dims))
        K = int(rng.integers(1, max(2, N // 6)))
        T = int(rng.choice([0, 0, 2, 5, 40]))
        max_k = int(rng.choice([K + 64, K + 64, max(1, K // 2)]))   # sometimes too small: CAPACITY
        flags = dict(literal_peel=bool(rng.random() < 0.25), amp_average=bool(rng.random() < 0.25),
                     axis_schedule=bool(rng.random() < 0.1))
        cases.append((dims, K, T, max_k, flags, int(rng.integers(1, 1 << 30))))
    return cases


@pytest.fixture(scope="module")
def F():
    import paper_1711_11407_amd as F
    return F


@pytest.mark.parametrize("seed", [11, 12, 13, 14, 15, 16])
def test_random_problems_match_the_oracle(F, seed):
    torch, dev = torch_dev()
    cases = draw_cases(40, seed)
    cubes, specs = [], []
    for dims, K, T, max_k, flags, s in cases:
        cube = W.plant(dims, K, seed=s, mag=(0.5, 1.5))
        cubes.append(cube)
        specs.append(spec_for(F, dims, s + 1, max_iters=T, max_k=max_k, **flags))
    outcomes = {}
    for direct in (0, 1):
        plan = F.Plan(specs, tuning=dict(direct_launch=direct))
        xs = [torch.from_numpy(c.x).to(dev) for c in cubes]
        batched = [o.host() for o in plan.execute_batched(xs)]
        for i, c in enumerate(cubes):
            ref, _, _ = oracle_for(plan, i, c.x, specs[i])
            what = f"seed {seed} case {i} {cases[i][:4]} {cases[i][4]}"
            compare(batched[i], ref, "batched " + what)
            if direct == 0:
                compare(plan.execute(i, xs[i]).host(), ref, "plain " + what)
                outcomes[ref.status] = outcomes.get(ref.status, 0) + 1
    log(f"seed {seed}: outcomes {outcomes}")
    assert len(outcomes) >= 2
