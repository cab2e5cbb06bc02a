"""GPU parity of the plain per-cube path and the line gather + FFT kernel
against the FP64 oracle, through the C ABI."""
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


def run_plain(F, cube_x, spec, tuning=None):
    torch, dev = torch_dev()
    plan = F.Plan([spec], tuning=tuning)
    x = torch.from_numpy(np.ascontiguousarray(cube_x)).to(dev)
    got = plan.execute(0, x).host()
    return plan, got


def test_smoke_cfg1(F):
    import __graft_entry__ as g
    g.smoke()


@pytest.mark.parametrize("name", ["cfg1", "cfg3"])
def test_plain_configs(F, name):
    cube = getattr(W, name)()
    spec = spec_for(F, cube.dims, cube.schedule_seed, max_k=1024)
    log(f"plain {name} dims={cube.dims} K={len(cube.amps)}")
    plan, got = run_plain(F, cube.x, spec)
    ref, _, _ = oracle_for(plan, 0, cube.x, spec)
    err = compare(got, ref, name)
    assert ref.status == O.STATUS_OK
    assert {tuple(f) for f in got["freqs"].tolist()} == {tuple(f) for f in cube.freqs.tolist()}
    log(f"  k={got['k']} iters={got['iters']} amp err={err:.2e}")


SHAPES = [
    ((16, 24), 12, 30),        # L = 48, c = (3, 2), radix 8 + 2 + 3
    ((6, 10), 3, 30),          # L = 30: generic radix 3 and 5
    ((64, 512), 150, 0),       # c = (8, 1)
    ((512, 64), 150, 0),
    ((4, 6, 10, 2), 6, 40),    # D = 4, L = 60
    ((8, 8, 12), 20, 40),      # D = 3, L = 24
    ((30,), 30, 3),            # D = 1: every bin 1-sparse, dense spectrum
    ((128, 128), 300, 0),
    ((256, 256), 1280, 0),     # the paper's K = 5 N0 regime
    ((7, 9), 4, 40),           # L = 63 = 7 * 9
    ((384, 96), 200, 0),       # L = 384: a two-bin decode pass with a ragged second bin set
    ((640, 128), 250, 0),      # L = 640: two decode passes, the second ragged
    ((96, 96, 96), 300, 40),   # D = 3, L = 96 on the block path
]


@pytest.mark.parametrize("dims,K,T", SHAPES)
def test_plain_shapes(F, dims, K, T):
    seed = 100 + sum(dims) + K
    cube = W.plant(dims, K, seed=seed, mag=(0.5, 1.5))
    spec = spec_for(F, dims, seed + 1, max_iters=T, max_k=max(64, 2 * K))
    log(f"plain shape dims={dims} K={K} T={T}")
    plan, got = run_plain(F, cube.x, spec)
    ref, _, _ = oracle_for(plan, 0, cube.x, spec)
    compare(got, ref, str(dims))


@pytest.mark.parametrize("tuning", [
    dict(block_threads=64), dict(block_threads=512), dict(block_threads=128), dict(max_radix=2), dict(max_radix=4),
    dict(chunk_iters=0), dict(chunk_iters=1), dict(chunk_iters=64), dict(lines_wg=3),
    dict(lines_wg=64, block_threads=512),
])
def test_plain_launch_shapes_agree(F, tuning):
    cube = W.plant((128, 256), 200, seed=77, mag=(0.5, 1.5))
    spec = spec_for(F, cube.dims, 78, max_k=512)
    log(f"tuning {tuning}")
    plan, got = run_plain(F, cube.x, spec, tuning)
    ref, _, _ = oracle_for(plan, 0, cube.x, spec)
    compare(got, ref, str(tuning))


def test_records_in_global_memory(F):
    """A capacity too large for LDS keeps the record list in the outputs."""
    cube = W.plant((256, 256), 600, seed=5, mag=(0.5, 1.5))
    spec = spec_for(F, cube.dims, 6, max_k=30000)
    plan, got = run_plain(F, cube.x, spec)
    ref, _, _ = oracle_for(plan, 0, cube.x, spec)
    compare(got, ref, "global records")


def test_zero_input(F):
    x = np.zeros((64, 128), dtype=np.complex64)
    spec = spec_for(F, x.shape, 3)
    plan, got = run_plain(F, x, spec)
    assert got["status"] == 0 and got["iters"] == 1 and got["k"] == 0


def test_iteration_cap_and_capacity(F):
    cube = W.plant((64, 64), 300, seed=5)
    spec = spec_for(F, cube.dims, 6, max_iters=1, max_k=512)
    plan, got = run_plain(F, cube.x, spec)
    ref, _, _ = oracle_for(plan, 0, cube.x, spec)
    compare(got, ref, "T=1")
    assert got["status"] == O.STATUS_INCOMPLETE
    spec = spec_for(F, cube.dims, 6, max_k=10)
    plan, got = run_plain(F, cube.x, spec)
    ref, _, _ = oracle_for(plan, 0, cube.x, spec)
    compare(got, ref, "capacity")
    assert got["status"] == O.STATUS_CAPACITY and got["n"] == 10


def test_deadlock_axis_schedule(F):
    dims = (8, 8)
    freqs = np.array([[0, 0], [0, 3], [2, 0], [2, 3]])
    x = W.synthesize(dims, freqs, np.exp(2j * np.pi * np.array([0.1, 0.35, 0.6, 0.85]))).astype(np.complex64)
    T = 6
    sched = np.zeros((T, 2, 2), np.int32)
    sched[:, 0] = [[1, 0], [0, 1]] * (T // 2)
    sched[:, 1] = [[t % 8, (3 * t) % 8] for t in range(T)]
    spec = spec_for(F, dims, 0, max_iters=T, schedule=sched)
    plan, got = run_plain(F, x, spec)
    assert got["status"] == O.STATUS_INCOMPLETE and got["k"] == 0
    ref, _, _ = oracle_for(plan, 0, x, spec)
    compare(got, ref, "deadlock")
    sched2 = np.array([[[1, 1], [0, 0]], [[1, 1], [5, 2]]], np.int32)
    spec = spec_for(F, dims, 0, max_iters=2, schedule=sched2)
    plan, got = run_plain(F, x, spec)
    assert got["status"] == O.STATUS_OK and got["k"] == 4


@pytest.mark.parametrize("dims", [(64, 64), (16, 24), (128, 128, 128), (6, 10), (4, 6, 10, 2), (256, 512),
                                  (15, 21), (3, 5, 7, 3)])
def test_lines_fft_matches_oracle_line_dft(F, dims):
    """Eq. sample_slice + Eq. hs: every gathered line's 1/L DFT, fp32 vs fp64
    on the same complex64 cube, relative max error <= 1e-5 of the line's
    spectrum norm. (15, 21) and (3, 5, 7, 3) give an odd number (D+1) L of
    spectrum values per iteration."""
    torch, dev = torch_dev()
    x = W.random_dense(dims, 11).astype(np.complex64)
    spec = spec_for(F, dims, 5, max_iters=12)
    plan = F.Plan([spec])
    xt = torch.from_numpy(x).to(dev)
    sp = plan.lines_fft(0, xt, 0, 12).cpu().numpy()
    sched = plan.schedule(0)
    L = O.line_length(dims)
    for t in range(12):
        for i, off in enumerate(O.line_offsets(dims, sched[t, 1])):
            want = O.line_dft(O.gather_line(x.astype(np.complex128), sched[t, 0], off, L))
            err = np.abs(sp[t, i] - want).max() / max(np.linalg.norm(want), 1e-30)
            assert err < 1e-5, (t, i, err)


def test_lines_fft_all_packed_layout(F):
    torch, dev = torch_dev()
    shapes = [(64, 128), (32, 32), (16, 24), (15, 21)]
    specs = [spec_for(F, d, 3 + i, max_iters=[20, 5, 9, 7][i]) for i, d in enumerate(shapes)]
    plan = F.Plan(specs)
    xs = [torch.from_numpy(W.random_dense(d, i).astype(np.complex64)).to(dev) for i, d in enumerate(shapes)]
    allsp = plan.lines_fft_all(xs).cpu().numpy()
    for c, d in enumerate(shapes):
        L, T, off = plan.info[c]
        blk = allsp[off:off + T * (len(d) + 1) * L].reshape(T, len(d) + 1, L)
        one = plan.lines_fft(c, xs[c], 0, T).cpu().numpy()
        # whole-batch and single-cube calls may use different FFT kernels:
        # equal up to fp32 rounding
        np.testing.assert_allclose(blk, one, rtol=0, atol=1e-6 * np.abs(one).max())


def test_noisy_cfg2_reports_agreement(F):
    """20 dB per-sample noise: the noiseless decoder's decisions are not
    stable (parity unpinned); the run must complete and its records must be
    valid frequencies. The agreement with the oracle is reported."""
    cube = W.cfg2()
    L = 256
    th = W.cfg2_thresh(cube, L)
    spec = F.CubeSpec(cube.dims, seed=cube.schedule_seed, max_k=8192, **th)
    plan, got = run_plain(F, cube.x, spec)
    ref, _, _ = oracle_for(plan, 0, cube.x, spec)
    assert got["k"] > 0 and (got["freqs"] >= 0).all() and (got["freqs"] < 256).all()
    truth = {tuple(f) for f in cube.freqs.tolist()}
    g = {tuple(f) for f in got["freqs"].tolist()}
    o = {tuple(f) for f in ref.freqs.tolist()}
    log(f"cfg2: gpu k={got['k']} iters={got['iters']} recall={len(g & truth)/len(truth):.2f} "
        f"oracle k={ref.k} recall={len(o & truth)/len(truth):.2f} jaccard(gpu,oracle)="
        f"{len(g & o)/max(1, len(g | o)):.2f}")


@pytest.mark.parametrize("tuning", [None, dict(lines_samples=512), dict(lines_samples=20000),
                                    dict(lines_wg=3)])
def test_lines_fft_all_mixed_lengths_matches_single(F, tuning):
    """The persistent whole-budget line FFT over a group of cubes of mixed
    line lengths (and a 3-D group), for several work-item sizes: every
    packed block equals the single-cube line FFT of the same iterations."""
    torch, dev = torch_dev()
    shapes = [(64, 64), (128, 64), (512, 512), (64, 512), (256, 256), (128, 128, 128), (64, 128, 64)]
    T = [21, 21, 40, 21, 85, 30, 12]
    specs = [spec_for(F, d, 50 + i, max_iters=T[i]) for i, d in enumerate(shapes)]
    plan = F.Plan(specs, tuning=tuning)
    xs = [torch.from_numpy(W.random_dense(d, 60 + i).astype(np.complex64)).to(dev) for i, d in enumerate(shapes)]
    allsp = plan.lines_fft_all(xs).cpu().numpy()
    for c, d in enumerate(shapes):
        L, Tc, off = plan.info[c]
        blk = allsp[off:off + Tc * (len(d) + 1) * L].reshape(Tc, len(d) + 1, L)
        one = plan.lines_fft(c, xs[c], 0, Tc).cpu().numpy()
        np.testing.assert_allclose(blk, one, rtol=0, atol=1e-6 * np.abs(one).max())
        # and the whole-batch path itself against the FP64 line DFT
        x64 = xs[c].cpu().numpy().astype(np.complex128)
        sched = plan.schedule(c)
        for t in sorted({0, Tc // 2, Tc - 1}):
            for i, offs in enumerate(O.line_offsets(d, sched[t, 1])):
                want = O.line_dft(O.gather_line(x64, sched[t, 0], offs, L))
                err = np.abs(blk[t, i] - want).max() / max(np.linalg.norm(want), 1e-30)
                assert err < 1e-5, (d, t, i, err)


# Long lines (L = LCM too long for the D+1 spectra, a second buffer and the
# twiddles in LDS): transformed one line at a time. 512 x 576 is the shape of
# the paper's image experiment (Sec. 3), L = 4608 = 2^9 3^2; 2048 x 4096 is a
# power-of-two line length past the in-LDS limit.
LONG = [((512, 576), 300, 0), ((6000,), 40, 3), ((2048, 4096), 200, 0)]


@pytest.mark.parametrize("dims,K,T", LONG)
def test_long_lines_plain_and_batched(F, dims, K, T):
    torch, dev = torch_dev()
    cube = W.plant(dims, K, seed=400 + K, mag=(0.5, 1.5))
    short = W.plant((64, 128), 30, seed=401)
    specs = [spec_for(F, dims, 402, max_iters=T, max_k=512), spec_for(F, short.dims, 403, max_k=64)]
    log(f"long lines dims={dims} K={K} L={O.line_length(dims)}")
    plan = F.Plan(specs)
    xs = [torch.from_numpy(cube.x).to(dev), torch.from_numpy(short.x).to(dev)]
    plain = [plan.execute(c, xs[c]).host() for c in range(2)]
    batched = [o.host() for o in plan.execute_batched(xs)]
    for c, x in enumerate((cube.x, short.x)):
        ref, _, _ = oracle_for(plan, c, x, specs[c])
        compare(plain[c], ref, f"plain {c}")
        compare(batched[c], ref, f"batched {c}")
    assert plain[0]["status"] == O.STATUS_OK
    assert {tuple(f) for f in plain[0]["freqs"].tolist()} == {tuple(f) for f in cube.freqs.tolist()}


# Lines too long for LDS even one at a time ((D+2) L * 8 bytes > 160 KB):
# the D+1 spectra and the scratch line live in a device workspace of the
# plan. Power-of-two and mixed-radix (3 * 2^14) lengths, 1-D to 3-D, records
# in LDS and in device memory.
LONGER = [((64, 16384), 100, 0, 512), ((32768,), 30, 3, 512), ((3, 16384), 40, 3, 512),
          ((4, 4, 8192), 20, 0, 512), ((64, 16384), 100, 0, 20000)]


@pytest.mark.parametrize("dims,K,T,max_k", LONGER)
def test_lines_in_device_memory_plain_batched_noalloc(F, dims, K, T, max_k):
    torch, dev = torch_dev()
    cube = W.plant(dims, K, seed=500 + K, mag=(0.5, 1.5))
    short = W.plant((64, 128), 30, seed=501)
    specs = [spec_for(F, dims, 502, max_iters=T, max_k=max_k), spec_for(F, short.dims, 503, max_k=64)]
    log(f"lines in device memory dims={dims} K={K} L={O.line_length(dims)} max_k={max_k}")
    plan = F.Plan(specs)
    xs = [torch.from_numpy(cube.x).to(dev), torch.from_numpy(short.x).to(dev)]
    plain = [plan.execute(c, xs[c]).host() for c in range(2)]
    batched = [o.host() for o in plan.execute_batched(xs)]
    for c, x in enumerate((cube.x, short.x)):
        ref, _, _ = oracle_for(plan, c, x, specs[c])
        compare(plain[c], ref, f"plain {c}")
        compare(batched[c], ref, f"batched {c}")
    assert plain[0]["status"] == O.STATUS_OK
    assert {tuple(f) for f in plain[0]["freqs"].tolist()} == {tuple(f) for f in cube.freqs.tolist()}
    # the allocation-free entry point takes the workspace from its scratch
    if max_k <= 512:
        out = plan.alloc_result(0, dev)
        got = plan.execute_noalloc(0, xs[0], out).host()
        for k in ("k", "n", "iters", "status"):
            assert got[k] == plain[0][k], k
        np.testing.assert_array_equal(got["freqs"], plain[0]["freqs"])
        np.testing.assert_array_equal(got["amps"], plain[0]["amps"])


@pytest.mark.parametrize("dims", [(512, 576), (64, 8192)])
def test_long_lines_fft_matches_oracle_line_dft(F, dims):
    """Line spectra of long lines against the FP64 line DFT: 512 x 576 (the
    solve keeps its spectra in LDS) and 64 x 8192 (the solve keeps them in
    device memory; the line kernel still holds its two lines in LDS)."""
    torch, dev = torch_dev()
    x = W.random_dense(dims, 17).astype(np.complex64)
    spec = spec_for(F, dims, 9, max_iters=4)
    plan = F.Plan([spec, spec_for(F, (64, 64), 10, max_iters=3)])
    xt = torch.from_numpy(x).to(dev)
    one = plan.lines_fft(0, xt, 0, 4).cpu().numpy()
    allsp = plan.lines_fft_all([xt, torch.from_numpy(W.random_dense((64, 64), 3).astype(np.complex64)).to(dev)])
    L, T, off = plan.info[0]
    blk = allsp.cpu().numpy()[off:off + T * 3 * L].reshape(T, 3, L)
    sched = plan.schedule(0)
    for t in range(4):
        for i, offs in enumerate(O.line_offsets(dims, sched[t, 1])):
            want = O.line_dft(O.gather_line(x.astype(np.complex128), sched[t, 0], offs, L))
            for got in (one[t, i], blk[t, i]):
                err = np.abs(got - want).max() / max(np.linalg.norm(want), 1e-30)
                assert err < 1e-5, (t, i, err)


def test_image_scale_sparsity(F):
    """K = 8411 on 512 x 576 (the sparsity of the paper's first image, 2.85%
    nonzero): same records as the oracle; the paper needs 14.0% of the
    samples (3 iterations) for its image, the iteration count here is logged."""
    torch, dev = torch_dev()
    cube = W.plant((512, 576), 8411, seed=8411)
    spec = spec_for(F, cube.dims, 8412, max_k=16384)
    plan, got = run_plain(F, cube.x, spec)
    ref, _, _ = oracle_for(plan, 0, cube.x, spec)
    compare(got, ref, "image scale")
    log(f"K=8411 on 512x576: status {got['status']} after {got['iters']} iterations "
        f"({100.0 * got['iters'] * 3 * 4608 / (512 * 576):.1f}% of the samples)")
    assert got["status"] == O.STATUS_OK


def test_clustered_image_512x576(F):
    """A pixel-sparse clustered image (rectangular blobs, 2.85% of the
    pixels, real intensities) through duality, at the image experiment's
    shape: plain and batched equal the oracle record by record."""
    torch, dev = torch_dev()
    cube = W.image_like((512, 576), 8411, seed=2017)
    spec = spec_for(F, cube.dims, cube.schedule_seed, max_k=16384)
    plan = F.Plan([spec])
    x = torch.from_numpy(cube.x).to(dev)
    got = plan.execute(0, x).host()
    bat = plan.execute_batched([x])[0].host()
    ref, _, _ = oracle_for(plan, 0, cube.x, spec)
    compare(got, ref, "clustered image, plain")
    compare(bat, ref, "clustered image, batched")
    assert got["status"] == O.STATUS_OK
    assert {tuple(f) for f in got["freqs"].tolist()} == {tuple(f) for f in cube.freqs.tolist()}
    log(f"clustered image: {got['iters']} iterations ({100.0 * got['iters'] * 3 * 4608 / (512 * 576):.1f}% "
        f"of the samples)")
