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
    """The GPU result against the oracle's: the same outcome, iteration
    count, recovered set (frequencies in first-detection order), merged
    frequencies left out of the set, and detection trace (iteration, bin and
    set index of every detection), all bit-exact; amplitudes of the set
    within amp_tol relative L2 and each within amp_tol of its own magnitude.
    Returns the relative L2 error."""
    assert got["status"] == ref.status, (what, "status", got["status"], ref.status)
    assert got["iters"] == ref.iters, (what, "iters", got["iters"], ref.iters)
    assert got["k"] == ref.k, (what, "k", got["k"], ref.k)
    assert got["n"] == ref.n, (what, "detections", got["n"], ref.n)
    np.testing.assert_array_equal(got["freqs"], ref.freqs, err_msg=f"{what}: freqs")
    np.testing.assert_array_equal(got["dropped_freqs"], ref.dropped_freqs, err_msg=f"{what}: dropped freqs")
    np.testing.assert_array_equal(got["rec_iter"], ref.rec_iter, err_msg=f"{what}: rec_iter")
    np.testing.assert_array_equal(got["rec_bin"], ref.rec_bin, err_msg=f"{what}: rec_bin")
    np.testing.assert_array_equal(got["rec_sin"], ref.rec_sin, err_msg=f"{what}: rec_sin")
    if ref.k:
        err = np.linalg.norm(got["amps"] - ref.amps) / np.linalg.norm(ref.amps)
        assert err <= amp_tol, (what, "amp rel L2", err)
        per = np.abs(got["amps"] - ref.amps) / np.abs(ref.amps)
        assert per.max() <= amp_tol, (what, "worst record", int(per.argmax()), float(per.max()))
        return err
    return 0.0


def max_record_error(got: dict, ref) -> float:
    """Largest relative error of one set amplitude (0 for an empty set)."""
    if not ref.k:
        return 0.0
    return float((np.abs(got["amps"] - ref.amps) / np.abs(ref.amps)).max())


# ---------------------------------------------------------------------------
# The oracle over whole workloads, one single-threaded process per core
# ---------------------------------------------------------------------------

def _oracle_task(task):
    """One oracle run in a worker. task: (kind, key, T, max_k, want_grad)
    with kind "cfg4" (key: cube index of the batched workload) or "cfg5"
    (key: cube index of the differentiation workload). Returns the oracle's
    Result and, when asked, the FP64 reference gradient of l = sum |a|^2 over
    the recovered set, 2 M^H a, at the touched positions (M: the oracle's
    linear map from samples to set amplitudes, decisions fixed)."""
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    kind, key, T, max_k, want_grad = task
    cube = W.cfg4(only=[key])[0] if kind == "cfg4" else W.cfg5()[key]
    al, ta = O.schedule(cube.dims, T, cube.schedule_seed)
    res = O.run(cube.x, al, ta, O.Params(**W.NOISELESS_THRESH, max_iters=T, max_k=max_k))
    grad = None
    if want_grad:
        pos = O.touched_positions(cube.dims, res.rec_iter, al, ta)
        M = O.amp_matrix(cube.dims, res, al, ta, pos)
        grad = (pos, 2.0 * (M.conj().T @ res.amps))
    return res, grad


def oracle_pool(tasks):
    """Run _oracle_task over `tasks` in a spawn pool (at most 16 processes,
    one thread each); results in task order."""
    import multiprocessing as mp
    import os
    n = max(1, min(len(os.sched_getaffinity(0)), 16, len(tasks)))
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    os.environ.update({k: "1" for k in saved})
    try:
        with mp.get_context("spawn").Pool(n) as pool:
            return pool.map(_oracle_task, tasks, chunksize=max(1, len(tasks) // (4 * n)))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
