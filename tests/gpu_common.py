"""Helpers shared by the GPU parity tests: run the HIP path and the FP64
oracle on the same seeded input and compare them."""
import sys

import numpy as np

import oracle as O
import workloads as W

AMP_TOL = 1e-4   # relative L2 on complex amplitudes (FP32 vs FP64, noiseless)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    return torch, torch.device("cuda", 0)


def spec_for(F, dims, seed, **kw):
    args = dict(W.NOISELESS_THRESH)
    args.update(kw)
    return F.CubeSpec(tuple(dims), seed=seed, **args)


def oracle_for(plan, cube_idx, x, spec):
    """Oracle run with the plan's schedule (checked equal to the oracle's own
    generator unless the schedule was given explicitly)."""
    sched = plan.schedule(cube_idx)
    if spec.schedule is None:
        al, ta = O.schedule(spec.dims, plan.max_iters(cube_idx), spec.seed, axis=spec.axis_schedule)
        assert (sched[:, 0] == al).all() and (sched[:, 1] == ta).all()
    else:
        al, ta = sched[:, 0].astype(np.int64), sched[:, 1].astype(np.int64)
    params = O.Params(zero_thresh=spec.zero_thresh, mag_rel_tol=spec.mag_rel_tol,
                      grid_tol=spec.grid_tol, max_iters=plan.max_iters(cube_idx),
                      max_k=spec.max_k, amp_average=spec.amp_average)
    return O.run(x, al, ta, params), al, ta


def compare(got: dict, ref, what="", amp_tol=AMP_TOL):
    """Bit-exact decisions, amplitudes within amp_tol relative L2."""
    assert got["status"] == ref.status, (what, "status", got["status"], ref.status)
    assert got["iters"] == ref.iters, (what, "iters", got["iters"], ref.iters)
    assert got["k"] == ref.k, (what, "k", got["k"], ref.k)
    np.testing.assert_array_equal(got["freqs"], ref.freqs, err_msg=f"{what}: freqs")
    np.testing.assert_array_equal(got["rec_iter"], ref.rec_iter, err_msg=f"{what}: rec_iter")
    np.testing.assert_array_equal(got["rec_bin"], ref.rec_bin, err_msg=f"{what}: rec_bin")
    if ref.k:
        err = np.linalg.norm(got["amps"] - ref.amps) / np.linalg.norm(ref.amps)
        assert err <= amp_tol, (what, "amp rel L2", err)
        return err
    return 0.0
