"""Batched persistent path (one persistent launch per kernel instantiation
for many uneven cubes, replayed from a HIP graph or launched directly)
against the plain path and the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import compare, log, max_record_error, oracle_for, oracle_pool, spec_for, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_1711_11407_amd as F
    return F


def batched_setup(F, cubes, max_k=512, tuning=None):
    torch, dev = torch_dev()
    specs = [spec_for(F, c.dims, c.schedule_seed, max_k=max_k) for c in cubes]
    plan = F.Plan(specs, tuning=tuning)
    xs = [torch.from_numpy(c.x).to(dev) for c in cubes]
    return plan, specs, xs


@pytest.mark.parametrize("direct", [0, 1])
def test_batched_small_mixed_equals_oracle(F, direct):
    """Mixed dimensions and line lengths: several kernel instantiations in
    one call, as one graph or as direct launches in sequence."""
    cubes = [W.plant(d, k, seed=s, mag=(0.5, 1.5)) for d, k, s in
             [((64, 64), 30, 1), ((16, 24), 10, 2), ((128, 128, 128), 200, 3), ((6, 10), 2, 4),
              ((512, 64), 120, 5), ((8, 8, 12), 15, 6), ((256, 256), 1000, 7)]]
    specs = []
    for c in cubes:
        T = max(O.default_max_iters(c.dims), 30) if np.prod(c.dims) < 4096 else 0
        specs.append(spec_for(F, c.dims, c.schedule_seed, max_k=2048, max_iters=T))
    torch, dev = torch_dev()
    plan = F.Plan(specs, tuning=dict(direct_launch=direct))
    xs = [torch.from_numpy(c.x).to(dev) for c in cubes]
    outs = plan.execute_batched(xs)
    outs = plan.execute_batched(xs, outs)   # second call: queue counters reset by the last launch
    for i, (c, o) in enumerate(zip(cubes, outs)):
        ref, _, _ = oracle_for(plan, i, c.x, specs[i])
        compare(o.host(), ref, f"cube {i} {c.dims}")


def test_batched_graph_replays_are_stable(F):
    """Repeated graph replays into the same outputs, with eager work between
    them, give bit-identical results (the construction-subtraction sums are
    exact, hence independent of thread timing)."""
    cubes = W.cfg4(B=48, seed=4)
    plan, specs, xs = batched_setup(F, cubes)
    torch, _ = torch_dev()
    outs = plan.execute_batched(xs)
    first = [o.host() for o in outs]
    for rep in range(3):
        # eager work between replays, then replay into the same outputs
        for o in outs:
            o.info.zero_()
            o.freqs.fill_(-1)
            o.amps.zero_()
        torch.cuda.synchronize()
        plan.execute_batched(xs, outs)
        for a, o in zip(first, outs):
            b = o.host()
            for key in ("k", "n", "kd", "iters", "status"):
                assert a[key] == b[key], key
            for key in ("freqs", "amps", "dropped_freqs", "dropped_amps", "rec_iter", "rec_bin", "rec_sin"):
                np.testing.assert_array_equal(a[key], b[key], err_msg=key)
    # new output buffers re-upload the pointer table
    outs2 = plan.execute_batched(xs)
    for a, o in zip(first, outs2):
        np.testing.assert_array_equal(a["freqs"], o.host()["freqs"])
        np.testing.assert_array_equal(a["amps"], o.host()["amps"])


def bench_tuning():
    from paper_1711_11407_amd import tune
    return tune.load(tune._arch(), "batched")


def test_cfg4_full_batch_parity(F):
    """The full 1024-cube workload in the launch shape the benchmark times:
    every cube against the FP64 oracle (records, trace, outcome, amplitudes
    per record), and batched equal to plain (bit for bit unless the plain
    path transforms its first iterations ahead with the line kernel)."""
    log("generating cfg4 (1024 cubes)")
    cubes = W.cfg4()
    tuning = bench_tuning()
    pre_chunk = (tuning or {}).get("chunk_iters", 8) > 0
    plan, specs, xs = batched_setup(F, cubes, tuning=tuning)
    torch, dev = torch_dev()
    log("oracle over 1024 cubes (process pool)")
    refs = oracle_pool([("cfg4", c, plan.max_iters(c), 512, False) for c in range(len(cubes))])
    log("batched execute")
    bout = plan.execute_batched(xs)
    torch.cuda.synchronize()
    log("plain execute x1024")
    pouts = [plan.execute(c, xs[c]) for c in range(len(cubes))]
    torch.cuda.synchronize()
    n_ok = n_exact = n_merged = 0
    worst = 0.0
    for c in range(len(cubes)):
        sched = plan.schedule(c)
        al, ta = O.schedule(cubes[c].dims, plan.max_iters(c), specs[c].seed)
        assert (sched[:, 0] == al).all() and (sched[:, 1] == ta).all(), c
        b, p = bout[c].host(), pouts[c].host()
        ref = refs[c][0]
        compare(b, ref, f"cfg4 cube {c} {cubes[c].dims} batched")
        for key in ("k", "n", "kd", "iters", "status"):
            assert b[key] == p[key], (c, key)
        for key in ("freqs", "rec_iter", "rec_bin", "rec_sin", "dropped_freqs"):
            np.testing.assert_array_equal(b[key], p[key], err_msg=f"cube {c} {key}")
        if pre_chunk:
            # the plain path's first iterations come from the block FFT of
            # the line kernel: other rounding of the same spectra
            np.testing.assert_allclose(b["amps"], p["amps"], rtol=1e-5, atol=0, err_msg=f"cube {c}")
        else:
            np.testing.assert_array_equal(b["amps"], p["amps"], err_msg=f"cube {c} amps")
        worst = max(worst, max_record_error(b, ref))
        n_ok += ref.status == O.STATUS_OK
        n_merged += ref.n != ref.k
        if ref.status == O.STATUS_OK:
            n_exact += {tuple(f) for f in ref.freqs.tolist()} == {tuple(f) for f in cubes[c].freqs.tolist()}
    log(f"cfg4: {n_ok}/1024 empty residual, {n_exact} exact support, {n_merged} with re-detections; "
        f"worst per-record amplitude error {worst:.1e}")


def test_redetection_merged_like_the_oracle(F):
    """Cube 148 of the batched workload (128 x 64, K = 275): a false
    detection of (83, 46) at iteration 5 is detected again with the opposite
    amplitude at iteration 6; the merged frequency has a zero sum and leaves
    the set, which is then exactly the planted one. Plain and batched paths,
    both launch forms."""
    shapes = W.cfg4_shapes()
    assert shapes[148][0] == (128, 64) and shapes[148][1] == 275
    cube = W.cfg4(only=[148])[0]
    for direct in (0, 1):
        plan, specs, xs = batched_setup(F, [cube, W.cfg4(only=[0])[0]], tuning=dict(direct_launch=direct))
        ref, _, _ = oracle_for(plan, 0, cube.x, specs[0])
        assert ref.n == ref.k + 2 and len(ref.dropped_freqs) == 1
        assert ref.status == O.STATUS_OK
        assert {tuple(f) for f in ref.freqs.tolist()} == {tuple(f) for f in cube.freqs.tolist()}
        got_b = plan.execute_batched(xs)[0].host()
        got_p = plan.execute(0, xs[0]).host()
        compare(got_b, ref, f"cube 148 batched direct={direct}")
        compare(got_p, ref, f"cube 148 plain direct={direct}")
        assert np.abs(got_b["dropped_amps"]).max() <= specs[0].zero_thresh


@pytest.mark.parametrize("max_k", [512, 20000])
@pytest.mark.parametrize("threads", [256, 192, 128])
def test_redetection_merged_every_path(F, threads, max_k):
    """The merge of cube 148 on every solve path: spare waves linking beside
    the transforms (256 threads), the wave path with links after the
    transforms (192 = D+1 waves), the block path (128), each with the record
    store and its frequency hash in LDS (max_k 512) or in device memory
    (max_k 20000: 20000 x 24 bytes of slots exceed LDS)."""
    cube = W.cfg4(only=[148])[0]
    log(f"cube 148 threads={threads} max_k={max_k}")
    plan, specs, xs = batched_setup(F, [cube], max_k=max_k, tuning=dict(block_threads=threads))
    ref, _, _ = oracle_for(plan, 0, cube.x, specs[0])
    assert ref.n == ref.k + 2 and len(ref.dropped_freqs) == 1
    compare(plan.execute_batched(xs)[0].host(), ref, f"cube 148 batched threads={threads} max_k={max_k}")
    compare(plan.execute(0, xs[0]).host(), ref, f"cube 148 plain threads={threads} max_k={max_k}")


SHAPES = [dict(ndim=2, line_length=64, block_threads=192), dict(ndim=2, line_length=128, block_threads=320),
          dict(ndim=2, line_length=512, block_threads=512, lines_samples=1536)]


@pytest.mark.parametrize("tuning", [dict(block_threads=128), dict(block_threads=512, max_radix=4),
                                    dict(direct_launch=1), dict(direct_launch=0),
                                    dict(group_by_length=1, direct_launch=1),
                                    dict(group_by_length=1, direct_launch=0),
                                    dict(shapes=SHAPES, direct_launch=1),
                                    dict(shapes=SHAPES, group_by_length=1, direct_launch=0)])
def test_batched_launch_shapes_agree(F, tuning):
    """Every launch shape, grouping and launch form gives the oracle's
    records, and (construction-subtraction sums being exact) the same bits
    as the default shapes whenever the FFT radices agree."""
    cubes = W.cfg4(B=40, seed=9)
    plan, specs, xs = batched_setup(F, cubes, tuning=tuning)
    outs = plan.execute_batched(xs)
    outs = plan.execute_batched(xs, outs)
    for c in range(0, 40, 5):
        ref, _, _ = oracle_for(plan, c, cubes[c].x, specs[c])
        compare(outs[c].host(), ref, f"{tuning} cube {c}")
    if tuning.get("block_threads", 256) < 192:
        return  # fewer waves than lines: the block FFT path, other rounding
    base, _, _ = batched_setup(F, cubes)
    bouts = base.execute_batched(xs)
    for c in range(40):
        a, b = outs[c].host(), bouts[c].host()
        for key in ("freqs", "rec_iter", "rec_bin", "rec_sin"):
            np.testing.assert_array_equal(a[key], b[key], err_msg=f"{tuning} cube {c} {key}")
        np.testing.assert_array_equal(a["amps"], b["amps"], err_msg=f"{tuning} cube {c} amps")


def test_grouped_line_fft_equals_single(F):
    """The whole-budget line FFT with one concurrent launch per line length
    and per-(D, L) item sizes equals the per-cube line FFT."""
    torch, dev = torch_dev()
    cubes = W.cfg4(B=24, seed=10)
    plan, specs, xs = batched_setup(F, cubes, tuning=dict(shapes=SHAPES, group_by_length=1))
    spec_all = plan.lines_fft_all(xs)
    torch.cuda.synchronize()
    for c in range(len(cubes)):
        L, T, off = plan.info[c]
        one = plan.lines_fft(c, xs[c], 0, T).cpu().numpy().reshape(-1)
        blk = spec_all[off:off + T * 3 * L].cpu().numpy()
        np.testing.assert_array_equal(blk, one, err_msg=f"cube {c}")
