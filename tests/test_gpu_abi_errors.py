"""Error behaviour of the hot-path calls through the C ABI: argument errors
come back synchronously as FPSSFT_ERR_INVALID_ARG (nothing is enqueued),
limits as FPSSFT_ERR_UNSUPPORTED, and a failed call leaves the plan usable."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import compare, oracle_for, spec_for, torch_dev

pytestmark = pytest.mark.gpu

INVALID, UNSUPPORTED = -1, -2


@pytest.fixture(scope="module")
def setup():
    import paper_1711_11407_amd as F
    from paper_1711_11407_amd import _binding as B
    torch, dev = torch_dev()
    cubes = [W.plant((64, 64), 8, seed=31), W.plant((32, 48), 6, seed=32)]
    specs = [spec_for(F, c.dims, c.schedule_seed, max_k=64) for c in cubes]
    plan = F.Plan(specs)
    xs = [torch.from_numpy(c.x).to(dev) for c in cubes]
    outs = [plan.alloc_result(i, dev) for i in range(2)]
    return F, B, plan, cubes, specs, xs, outs


def test_execute_argument_errors(setup):
    F, B, plan, cubes, specs, xs, outs = setup
    lib = B.lib()
    o = outs[0].c_out()
    x = C.c_void_p(xs[0].data_ptr())
    assert lib.fpssft_execute(None, 0, x, C.byref(o), None) == INVALID
    assert lib.fpssft_execute(plan._h, 2, x, C.byref(o), None) == INVALID
    assert lib.fpssft_execute(plan._h, -1, x, C.byref(o), None) == INVALID
    assert lib.fpssft_execute(plan._h, 0, None, C.byref(o), None) == INVALID
    assert lib.fpssft_execute(plan._h, 0, x, None, None) == INVALID
    for field in ("freqs", "amps", "rec_iter", "rec_bin", "rec_sin", "info"):
        bad = outs[0].c_out()
        setattr(bad, field, None)
        assert lib.fpssft_execute(plan._h, 0, x, C.byref(bad), None) == INVALID, field


def test_batched_and_lines_argument_errors(setup):
    F, B, plan, cubes, specs, xs, outs = setup
    lib = B.lib()
    xp = (C.c_void_p * 2)(xs[0].data_ptr(), None)
    op = (B.Out * 2)(outs[0].c_out(), outs[1].c_out())
    assert lib.fpssft_execute_batched(plan._h, xp, op, None) == INVALID
    xp = (C.c_void_p * 2)(xs[0].data_ptr(), xs[1].data_ptr())
    assert lib.fpssft_execute_batched(plan._h, None, op, None) == INVALID
    assert lib.fpssft_execute_batched(plan._h, xp, None, None) == INVALID
    torch, dev = torch_dev()
    T = plan.max_iters(0)
    buf = torch.empty(T * 3 * plan.line_length(0), dtype=torch.complex64, device=dev)
    sp = C.c_void_p(buf.data_ptr())
    x = C.c_void_p(xs[0].data_ptr())
    assert lib.fpssft_lines_fft(plan._h, 0, x, -1, 1, sp, None) == INVALID
    assert lib.fpssft_lines_fft(plan._h, 0, x, 0, -1, sp, None) == INVALID
    assert lib.fpssft_lines_fft(plan._h, 0, x, T - 1, 2, sp, None) == INVALID
    assert lib.fpssft_lines_fft(plan._h, 5, x, 0, 1, sp, None) == INVALID
    assert lib.fpssft_lines_fft(plan._h, 0, x, 0, 0, sp, None) == 0     # empty range: nothing to do
    assert lib.fpssft_lines_fft_all(plan._h, xp, None, None) == INVALID


def test_backward_argument_errors(setup):
    F, B, plan, cubes, specs, xs, outs = setup
    torch, dev = torch_dev()
    lib = B.lib()
    res = plan.execute(0, xs[0], outs[0])
    o = res.c_out()
    ga = C.c_void_p(res.amps.data_ptr())
    gx = torch.empty_like(xs[0])
    assert lib.fpssft_amp_backward(plan._h, 0, C.byref(o), None, C.c_void_p(gx.data_ptr()), None) == INVALID
    assert lib.fpssft_amp_backward(plan._h, 0, C.byref(o), ga, None, None) == INVALID
    assert lib.fpssft_amp_backward(plan._h, 3, C.byref(o), ga, C.c_void_p(gx.data_ptr()), None) == INVALID


def test_plan_is_usable_after_failed_calls(setup):
    """The rejected calls above enqueued nothing: the plan still gives the
    oracle's result on both paths."""
    F, B, plan, cubes, specs, xs, outs = setup
    for i in range(2):
        ref, _, _ = oracle_for(plan, i, cubes[i].x, specs[i])
        compare(plan.execute(i, xs[i], outs[i]).host(), ref, f"plain {i}")
    for i, o in enumerate(plan.execute_batched(xs)):
        ref, _, _ = oracle_for(plan, i, cubes[i].x, specs[i])
        compare(o.host(), ref, f"batched {i}")


def test_plan_limits(setup):
    F, B, plan, cubes, specs, xs, outs = setup
    # lines longer than 65536 points
    with pytest.raises(F.FpsSftError) as e:
        F.Plan([spec_for(F, (65537, 2), 1)])
    assert e.value.status == UNSUPPORTED
    # lines too long for LDS even one at a time: planned with a device
    # workspace (8192 x 8192, L = 8192; 3 x 16384, L = 49152); the line-FFT
    # entry points keep two lines in LDS and refuse L = 49152
    F.Plan([spec_for(F, (8192, 8192), 1)])
    big = F.Plan([spec_for(F, (3, 16384), 1)])
    torch, dev = torch_dev()
    xbig = torch.zeros((3, 16384), dtype=torch.complex64, device=dev)
    small_out = torch.empty(4, dtype=torch.complex64, device=dev)
    with pytest.raises(F.FpsSftError) as e:
        big.lines_fft(0, xbig, 0, 1, out=small_out)
    assert e.value.status == UNSUPPORTED
    with pytest.raises(F.FpsSftError) as e:
        big.lines_fft_all([xbig], out=small_out)
    assert e.value.status == UNSUPPORTED
    # bad tuning values
    for tn in (dict(block_threads=96), dict(block_threads=1024), dict(max_radix=3), dict(lines_threads=32)):
        with pytest.raises(F.FpsSftError) as e:
            F.Plan([spec_for(F, (64, 64), 1)], tuning=tn)
        assert e.value.status == INVALID, tn


def test_plan_alive_at_interpreter_exit_is_destroyed_cleanly():
    """A plan still referenced when the interpreter exits is destroyed
    without an error from its destructor (one child process)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1711_11407_amd as F\n"
            "keep = F.Plan([F.CubeSpec((64, 64), seed=1)])\n"
            "print('plan ok', flush=True)\n" % root)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=100)
    assert r.returncode == 0 and "plan ok" in r.stdout, r.stderr
    assert "Exception ignored" not in r.stderr, r.stderr
