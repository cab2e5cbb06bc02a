"""Adjoint of the amplitude estimates (decisions fixed) on the GPU against
the FP64 finite-difference gradient of the oracle's replayed amplitudes."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import compare, log, oracle_for, oracle_pool, spec_for, torch_dev

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def F():
    import paper_1711_11407_amd as F
    return F


def fd_reference(cube_x, ref, al, ta):
    x64 = cube_x.astype(np.complex128)
    pos = O.touched_positions(cube_x.shape, ref.rec_iter, al, ta)
    g = O.grad_sum_abs2_fd(x64, ref, al, ta, positions=pos)
    return g, pos


@pytest.mark.parametrize("dims,K,seed,T", [((64, 64), 40, 3, 30), ((16, 24), 20, 4, 30),
                                           ((8, 8, 12), 30, 5, 40), ((256, 256), 50, 6, 0),
                                           # register line transforms of 512 points (2-D and
                                           # 1-D) and a 3-D cube with 64-point lines
                                           ((512, 64), 60, 7, 0), ((512,), 12, 8, 6),
                                           ((16, 16, 64), 30, 9, 0)])
def test_amp_backward_matches_fd(F, dims, K, seed, T):
    torch, dev = torch_dev()
    cube = W.plant(dims, K, seed=seed)
    spec = spec_for(F, dims, seed + 1, max_iters=T, max_k=256)
    plan = F.Plan([spec])
    x = torch.from_numpy(cube.x).to(dev).requires_grad_(True)
    amps, freqs, info = F.sft_amplitudes(plan, 0, x)
    loss = (amps.abs() ** 2).sum()
    loss.backward()
    g = x.grad.cpu().numpy().astype(np.complex128)
    ref, al, ta = oracle_for(plan, 0, cube.x, spec)
    k = int(info[0].item())
    assert k == ref.k
    gref, pos = fd_reference(cube.x, ref, al, ta)
    err = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    log(f"adjoint {dims} K={K}: k={k}, {len(pos)} touched samples, grad rel L2 err={err:.2e}")
    assert err <= GRAD_TOL
    mask = np.ones(g.size, bool)
    mask[pos] = False
    assert np.all(g.reshape(-1)[mask] == 0)


def test_dot_product_identity(F):
    """<M x, y> = <x, M^H y> with M applied by the GPU forward (decisions of
    one run held: x is a small perturbation-free scaling of the input) and
    M^H by the adjoint kernel."""
    torch, dev = torch_dev()
    dims = (128, 128)
    cube = W.plant(dims, 60, seed=8)
    spec = spec_for(F, dims, 9, max_k=128)
    plan = F.Plan([spec])
    x = torch.from_numpy(cube.x).to(dev)
    res = plan.execute(0, x)
    h = res.host()
    rng = np.random.default_rng(1)
    y = (rng.standard_normal(spec.max_k) + 1j * rng.standard_normal(spec.max_k)).astype(np.complex64)
    y[h["k"]:] = 0
    xt = plan.amp_backward(0, res, torch.from_numpy(y).to(dev)).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(y[:h["k"]].astype(np.complex128), h["amps"].astype(np.complex128))   # <y, Mx>
    rhs = np.vdot(xt.reshape(-1), cube.x.reshape(-1).astype(np.complex128))            # <M^H y, x>
    assert abs(lhs - rhs) / abs(lhs) < 1e-5


def test_cfg5_batched_backward(F):
    """Differentiation workload: 64 cubes of 256x256, K=50; batched forward
    and backward. Every cube's records equal the oracle's, every cube's
    gradient equals the FP64 reference gradient 2 M^H a (M: the oracle's
    linear map from samples to set amplitudes with its decisions fixed) and
    is zero off the touched line samples; two cubes are also checked against
    FP64 finite differences, and each gradient equals the single-cube
    adjoint's."""
    torch, dev = torch_dev()
    cubes = W.cfg5()
    specs = [spec_for(F, c.dims, c.schedule_seed, max_k=128) for c in cubes]
    plan = F.Plan(specs)
    log("oracle and reference gradients over 64 cubes (process pool)")
    refs = oracle_pool([("cfg5", c, plan.max_iters(c), 128, True) for c in range(len(cubes))])
    xs = [torch.from_numpy(c.x).to(dev).requires_grad_(True) for c in cubes]
    outs = F.sft_amplitudes_batched(plan, xs)
    loss = sum((a.abs() ** 2).sum() for a, _, _ in outs)
    loss.backward()
    res = plan.execute_batched([x.detach() for x in xs])
    worst = 0.0
    for c in range(len(cubes)):
        ref, (pos, gpos) = refs[c]
        compare(res[c].host(), ref, f"cfg5 cube {c}")
        g = xs[c].grad.cpu().numpy().astype(np.complex128).reshape(-1)
        gref = np.zeros_like(g)
        gref[pos] = gpos
        err = np.linalg.norm(g - gref) / np.linalg.norm(gref)
        assert err <= GRAD_TOL, (c, err)
        worst = max(worst, err)
        mask = np.ones(g.size, bool)
        mask[pos] = False
        assert np.all(g[mask] == 0), c
    log(f"cfg5: 64 gradients, worst rel L2 against 2 M^H a {worst:.1e}")
    for c in (0, 63):
        ref, al, ta = oracle_for(plan, c, cubes[c].x, specs[c])
        gfd, _ = fd_reference(cubes[c].x, ref, al, ta)
        g = xs[c].grad.cpu().numpy().astype(np.complex128)
        assert np.linalg.norm(g - gfd) / np.linalg.norm(gfd) <= GRAD_TOL, c
        single = plan.execute(c, xs[c].detach())
        g1 = plan.amp_backward(c, single, 2 * single.amps).cpu().numpy()
        np.testing.assert_allclose(g1, g, rtol=0, atol=1e-5 * np.abs(g).max())


def test_bound_backward_equals_plan_backward(F):
    """The pre-marshalled batched adjoint (Bound.run_backward) gives the same
    gradients as Plan.amp_backward_batched, over repeated calls."""
    import torch
    dev = torch.device("cuda", 0)
    cubes = [W.plant((64, 64), 10 + 5 * i, seed=70 + i) for i in range(6)]
    specs = [spec_for(F, c.dims, c.schedule_seed, max_k=64) for c in cubes]
    plan = F.Plan(specs)
    xs = [torch.from_numpy(c.x).to(dev) for c in cubes]
    bound = plan.bind(xs)
    outs = bound.run_batched()
    gas = [(2 * o.amps).contiguous() for o in outs]
    ref = [g.cpu().numpy() for g in plan.amp_backward_batched(outs, gas)]
    bound.bind_backward(gas)
    for _ in range(3):
        got = [g.cpu().numpy() for g in bound.run_backward()]
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)


def test_amp_backward_with_redetection(F):
    """Cube 148 of the batched workload holds a frequency detected twice
    (its two detections cancel and it leaves the set): the gradient of
    sum |a|^2 over the set equals the FP64 reference 2 M^H a, where M is the
    oracle's map from samples to the merged set amplitudes."""
    torch, dev = torch_dev()
    cube = W.cfg4(only=[148])[0]
    spec = spec_for(F, cube.dims, cube.schedule_seed, max_k=512)
    plan = F.Plan([spec])
    x = torch.from_numpy(cube.x).to(dev).requires_grad_(True)
    amps, freqs, info = F.sft_amplitudes(plan, 0, x)
    assert int(info[3]) == int(info[0]) + 2 and int(info[4]) == 1
    (amps.abs() ** 2).sum().backward()
    g = x.grad.cpu().numpy().astype(np.complex128).reshape(-1)
    ref, al, ta = oracle_for(plan, 0, cube.x, spec)
    pos = O.touched_positions(cube.dims, ref.rec_iter, al, ta)
    M = O.amp_matrix(cube.dims, ref, al, ta, pos)
    gref = np.zeros_like(g)
    gref[pos] = 2.0 * (M.conj().T @ ref.amps)
    err = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    log(f"re-detection cube: {len(pos)} touched samples, grad rel L2 err={err:.2e}")
    assert err <= GRAD_TOL


@pytest.mark.parametrize("dims,K", [((512, 576), 40), ((64, 8192), 30), ((64, 16384), 30)])
def test_amp_backward_long_lines(F, dims, K):
    """The adjoint on long lines: 512 x 576 (L = 4608: lines in LDS,
    twiddles from device memory) and 64 x 8192, 64 x 16384 (lines in the
    cube's device workspace). Checked by the dot-product identity
    <y, M x> = <M^H y, x>, against the FP64 finite-difference gradient of
    sum |a|^2 at 24 sampled touched positions, and zero off them."""
    torch, dev = torch_dev()
    cube = W.plant(dims, K, seed=700 + K)
    spec = spec_for(F, dims, 701, max_k=128)
    plan = F.Plan([spec])
    log(f"adjoint long lines {dims} L={O.line_length(dims)}")
    x = torch.from_numpy(cube.x).to(dev)
    res = plan.execute(0, x)
    h = res.host()
    ref, al, ta = oracle_for(plan, 0, cube.x, spec)
    compare(h, ref, f"forward {dims}")
    rng = np.random.default_rng(2)
    y = (rng.standard_normal(spec.max_k) + 1j * rng.standard_normal(spec.max_k)).astype(np.complex64)
    y[h["k"]:] = 0
    xt = plan.amp_backward(0, res, torch.from_numpy(y).to(dev)).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(y[:h["k"]].astype(np.complex128), h["amps"].astype(np.complex128))
    rhs = np.vdot(xt.reshape(-1), cube.x.reshape(-1).astype(np.complex128))
    assert abs(lhs - rhs) / abs(lhs) < 1e-5
    # gradient of sum |a|^2 through autograd, against finite differences
    xg = torch.from_numpy(cube.x).to(dev).requires_grad_(True)
    amps, _, _ = F.sft_amplitudes(plan, 0, xg)
    (amps.abs() ** 2).sum().backward()
    g = xg.grad.cpu().numpy().astype(np.complex128).reshape(-1)
    pos = O.touched_positions(cube.x.shape, ref.rec_iter, al, ta)
    sample = rng.choice(pos, size=min(24, len(pos)), replace=False)
    gref = O.grad_sum_abs2_fd(cube.x.astype(np.complex128), ref, al, ta, positions=sample).reshape(-1)
    err = np.linalg.norm(g[sample] - gref[sample]) / np.linalg.norm(gref[sample])
    assert err <= GRAD_TOL, err
    mask = np.ones(g.size, bool)
    mask[pos] = False
    assert np.all(g[mask] == 0)
