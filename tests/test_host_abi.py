"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/fpssft.h declares, validates descriptions, and draws the
same line schedule as the oracle's independent SplitMix64 generator."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fpssft.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fpssft_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def F():
    import paper_1711_11407_amd as F
    from paper_1711_11407_amd import _binding
    _binding.lib()
    return F


def test_library_exports_every_declared_symbol(F):
    from paper_1711_11407_amd import _binding
    names = header_functions()
    assert len(names) >= 15
    lib = C.CDLL(_binding.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert {s[0] for s in _binding.SIGNATURES} == set(names)
    assert lib.fpssft_abi_version() == 3
    # the calls the problem statement's boundary names
    for n in ("fpssft_plan", "fpssft_execute", "fpssft_execute_batched", "fpssft_amp_backward"):
        assert n in names, n


def test_validate_line_length_and_budget(F):
    assert F.validate(F.CubeSpec((256, 256))) == (256, 85)
    assert F.validate(F.CubeSpec((512, 576))) == (4608, 21)
    assert F.validate(F.CubeSpec((128, 128, 128))) == (128, 4096)
    assert F.validate(F.CubeSpec((6, 10), max_iters=7)) == (30, 7)
    assert F.validate(F.CubeSpec((32,))) == (32, 1)
    for dims in [(64, 64), (64, 512), (16, 24), (4, 4, 6), (7, 9, 2, 5)]:
        L, T = F.validate(F.CubeSpec(dims))
        assert L == O.line_length(dims) and T == O.default_max_iters(dims)


@pytest.mark.parametrize("kw,code", [
    (dict(dims=(0, 4)), -1), (dict(dims=(4, 4), max_k=0), -1), (dict(dims=(4, 4), max_iters=-1), -1),
    (dict(dims=(4, 4), zero_thresh=-1.0), -1), (dict(dims=(4, 4), mag_rel_tol=float("nan")), -1),
    (dict(dims=(65537, 3)), -2), (dict(dims=(50000, 50000)), -2),
    (dict(dims=(4, 4), schedule=np.zeros((2, 2, 2), np.int32)), -1),
    (dict(dims=(4, 4), max_iters=1, schedule=np.array([[[4, 0], [0, 0]]], np.int32)), -1),
])
def test_validate_rejects(F, kw, code):
    with pytest.raises(F.FpsSftError) as e:
        F.validate(F.CubeSpec(**kw))
    assert e.value.status == code


def test_five_dimensions_rejected(F):
    with pytest.raises(ValueError):
        F.CubeSpec((2, 2, 2, 2, 2)).to_c()


@pytest.mark.parametrize("dims,seed", [((64, 64), 1), ((16, 24), 7), ((128, 128, 128), 4),
                                       ((512, 576), 99), ((6, 10, 4), 2 ** 63 + 5), ((32,), 3),
                                       ((3, 5, 7, 2), 12)])
def test_schedule_matches_oracle_generator(F, dims, seed):
    T = 60
    got = F.schedule_generate(F.CubeSpec(dims, seed=seed), T)
    al, ta = O.schedule(dims, T, seed)
    np.testing.assert_array_equal(got[:, 0, :], al)
    np.testing.assert_array_equal(got[:, 1, :], ta)


@pytest.mark.parametrize("dims", [(64, 64), (16, 24), (4, 6, 10), (32,), (1, 8), (3, 5, 7, 2)])
def test_axis_schedule_matches_oracle_generator(F, dims):
    got = F.schedule_generate(F.CubeSpec(dims, seed=3, axis_schedule=True), 30)
    al, ta = O.schedule(dims, 30, 3, axis=True)
    np.testing.assert_array_equal(got[:, 0, :], al)
    np.testing.assert_array_equal(got[:, 1, :], ta)


def test_unknown_flag_rejected(F):
    import ctypes as C
    from paper_1711_11407_amd import _binding as B
    d, _keep = F.CubeSpec((8, 8), amp_average=True, literal_peel=True, axis_schedule=True,
                          deterministic=True).to_c()
    assert d.flags == 0xF and B.lib().fpssft_validate(C.byref(d), None, None) == 0
    for bad in (0x10, 0x80000000):
        d.flags = bad
        assert B.lib().fpssft_validate(C.byref(d), None, None) == -1


def test_workload_schedules_match(F):
    for cube in [W.cfg1()]:
        T = O.default_max_iters(cube.dims)
        got = F.schedule_generate(F.CubeSpec(cube.dims, seed=cube.schedule_seed), T)
        al, ta = O.schedule(cube.dims, T, cube.schedule_seed)
        assert (got[:, 0] == al).all() and (got[:, 1] == ta).all()
    for dims, K, seed in W.cfg4_shapes(64):
        T = O.default_max_iters(dims)
        got = F.schedule_generate(F.CubeSpec(dims, seed=seed + 1), T)
        al, ta = O.schedule(dims, T, seed + 1)
        assert (got[:, 0] == al).all() and (got[:, 1] == ta).all()


def test_plan_without_device_reports_no_device(F):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(F.FpsSftError) as e:
        F.Plan([F.CubeSpec((8, 8))])
    assert e.value.status == -5


def test_tuning_cache_roundtrip(tmp_path):
    from paper_1711_11407_amd import tune
    path = str(tmp_path / "t.json")
    assert tune.load("gfx950", "batched", path) is None
    out = dict(tuning=dict(block_threads=128, max_radix=4, chunk_iters=2, lines_wg=4, lines_threads=256,
                           direct_launch=1),
               results={"solve": []})
    tune.save("gfx950", "batched", out, path)
    tune.save("gfx942", "batched", dict(out, tuning=dict(block_threads=64)), path)
    assert tune.load("gfx950", "batched", path) == out["tuning"]
    assert tune.load("gfx942", "batched", path) == dict(block_threads=64)
    assert tune.load("gfx950", "other", path) is None

