"""Autotuner for the launch shapes of the FPS-SFT kernels.

Launch shapes are chosen per (D, L) class of the caller's workload: each
class's cubes are planned on their own and timed with HIP events around
repeated launches.

  solve    block_threads                -> persistent batched solve of the
           class (wave mapping: one wave per line when there are at least
           D+1 waves, the block FFT in LDS otherwise)
  lines    lines_samples                 -> line gather + FFT of the class
           over its whole iteration budget
  radix    max_radix x lines_threads     -> the block (LDS) FFTs and the
           work-group size of the line kernel over the whole workload
  launch   per-class solve shapes or one block size for all, x
           group_by_length x direct_launch -> one persistent launch per line
           length or solve shape, run concurrently (parallel graph branches
           or side streams), or one queue per kernel instantiation; graph
           replay or direct launches
  plain    chunk_iters                   -> plain per-cube path on a subset

Every solve candidate's outputs are compared with the class's first
candidate (identical frequencies, bins, iteration counts and outcomes) and
every line-FFT candidate's spectra with its class's first candidate (the
same bits; the radix candidates within 1e-5 of the spectra's peak): a
candidate that changes a result is rejected. The result is stored as JSON
keyed by GPU architecture and workload, with one entry per (D, L) class,
and read back with `load`.

    python -m paper_1711_11407_amd.tune            # the batched workload
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")

SOLVE_THREADS = (128, 192, 256, 320, 384, 512)
LINES_SAMPLES = (1536, 3072, 6144)
LINES_THREADS = (128, 256, 512)
RADIX = (4, 8)
PLAIN_GRID = dict(chunk_iters=(0, 2, 4, 8, 16))


def _arch() -> str:
    import torch
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


def _time_ms(torch, fn, reps: int, warmup: int = 2) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _decisions(outs):
    import torch
    info = torch.stack([o.info for o in outs]).cpu()
    sig = [tuple(info[c, :5].tolist()) for c in range(len(outs))]
    freqs = [o.freqs[: int(info[c, 0]) + int(info[c, 4])].cpu() for c, o in enumerate(outs)]
    bins = [o.rec_bin[: int(info[c, 3])].cpu() for c, o in enumerate(outs)]
    return sig, freqs, bins


def _same(a, b) -> bool:
    if a[0] != b[0]:
        return False
    return all((x == y).all() for x, y in zip(a[1], b[1])) and all((x == y).all() for x, y in zip(a[2], b[2]))


def _classes(specs):
    """Cube indices per (D, L) class, classes in order of first appearance."""
    import math
    out = {}
    for c, s in enumerate(specs):
        dims = [int(v) for v in s.dims]
        L = 1
        for d in dims:
            L = L * d // math.gcd(L, d)
        out.setdefault((len(dims), L), []).append(c)
    return out


def _spectra_close(a, b, tol: float) -> bool:
    import torch
    if tol == 0:
        return bool(torch.equal(a, b))
    return bool(((a - b).abs().max() <= tol * b.abs().max()).item())


def tune(specs, xs, reps: int = 10, plain_cubes: int = 128, log=print) -> dict:
    """Best launch shapes for the workload (specs, device inputs xs)."""
    import torch
    from . import Plan

    results = {"shapes": [], "radix": [], "launch": [], "plain": []}
    shapes = []
    for (D, L), idx in _classes(specs).items():
        sub_s = [specs[c] for c in idx]
        sub_x = [xs[c] for c in idx]
        entry = {"ndim": D, "line_length": L, "cubes": len(idx), "solve": [], "lines": []}
        # persistent solve of the class
        ref = best_ms = None
        best_bt = None
        for bt in SOLVE_THREADS:
            plan = Plan(sub_s, tuning=dict(block_threads=bt, direct_launch=1))
            bound = plan.bind(sub_x)
            ms = _time_ms(torch, bound.run_batched, reps)
            dec = _decisions(bound.outs)
            ok = ref is None or _same(ref, dec)
            ref = ref or dec
            entry["solve"].append(dict(block_threads=bt, ms=round(ms, 4), same_decisions=ok))
            log(f"D={D} L={L} ({len(idx)} cubes) solve block_threads={bt}: {ms * 1e3:.1f} us"
                f"{'' if ok else '  (decisions differ: rejected)'}")
            if ok and (best_ms is None or ms < best_ms):
                best_ms, best_bt = ms, bt
            del plan, bound
        # line gather + FFT of the class over its whole budget
        sref = None
        best_ms = None
        best_lines = None
        for ns in LINES_SAMPLES:
            plan = Plan(sub_s, tuning=dict(lines_samples=ns))
            bound = plan.bind(sub_x)
            ms = _time_ms(torch, bound.run_lines_all, reps)
            spec = bound.spectra
            ok = sref is None or _spectra_close(spec, sref, 0.0)
            sref = spec.clone() if sref is None else sref
            entry["lines"].append(dict(lines_samples=ns, ms=round(ms, 4), same_spectra=ok))
            log(f"D={D} L={L} lines lines_samples={ns}: {ms * 1e3:.1f} us"
                f"{'' if ok else '  (spectra differ: rejected)'}")
            if ok and (best_ms is None or ms < best_ms):
                best_ms, best_lines = ms, dict(lines_samples=ns)
            del plan, bound
        shapes.append(dict(ndim=D, line_length=L, block_threads=best_bt, **best_lines))
        results["shapes"].append(entry)
        del sref

    # radix of the block FFTs and work-group size of the line kernel over
    # the whole workload
    best = dict(shapes=shapes)
    sref = None
    best_ms = None
    for mr, lt in itertools.product(RADIX, LINES_THREADS):
        plan = Plan(specs, tuning=dict(best, max_radix=mr, lines_threads=lt))
        bound = plan.bind(xs)
        ms = _time_ms(torch, bound.run_lines_all, reps)
        ok = sref is None or _spectra_close(bound.spectra, sref, 1e-5)
        sref = bound.spectra.clone() if sref is None else sref
        results["radix"].append(dict(max_radix=mr, lines_threads=lt, ms=round(ms, 4), close_spectra=ok))
        log(f"lines max_radix={mr} lines_threads={lt}: {ms * 1e3:.1f} us"
            f"{'' if ok else '  (spectra differ: rejected)'}")
        if ok and (best_ms is None or ms < best_ms):
            best_ms = ms
            best.update(max_radix=mr, lines_threads=lt)
        del plan, bound
    del sref

    # grouping and launch form of the persistent solve on the whole
    # workload: the per-class solve shapes (one launch per shape, run
    # concurrently) against one block size for every class (one queue)
    uniform = sorted({sh["block_threads"] for sh in shapes} | {256})
    cands = [("per-class", None, gbl, dl) for gbl in (0, 1) for dl in (0, 1)]
    cands += [("uniform", bt, 0, dl) for bt in uniform for dl in (0, 1)]
    ref = best_ms = None
    best_launch = None
    for kind, bt, gbl, dl in cands:
        if kind == "per-class":
            sh = shapes
        else:
            sh = [{k: v for k, v in e.items() if k != "block_threads"} for e in shapes]
        tn = dict(best, shapes=sh, group_by_length=gbl, direct_launch=dl)
        if bt:
            tn["block_threads"] = bt
        plan = Plan(specs, tuning=tn)
        bound = plan.bind(xs)
        ms = _time_ms(torch, bound.run_batched, reps)
        dec = _decisions(bound.outs)
        ok = ref is None or _same(ref, dec)
        ref = ref or dec
        results["launch"].append(dict(solve_shapes=kind, block_threads=bt, group_by_length=gbl, direct_launch=dl,
                                      ms=round(ms, 4), same_decisions=ok))
        log(f"solve {kind}{'' if bt is None else f' block_threads={bt}'} group_by_length={gbl} "
            f"direct_launch={dl}: {ms * 1e3:.1f} us{'' if ok else '  (decisions differ: rejected)'}")
        if ok and (best_ms is None or ms < best_ms):
            best_ms = ms
            best_launch = dict(shapes=sh, group_by_length=gbl, direct_launch=dl)
            if bt:
                best_launch["block_threads"] = bt
        del plan, bound
    best.update(best_launch)

    # plain per-cube path on a subset
    sub = list(range(min(plain_cubes, len(specs))))
    best_ms = None
    pref = None
    for ch in PLAIN_GRID["chunk_iters"]:
        tn = dict(best, chunk_iters=ch)
        plan = Plan([specs[c] for c in sub], tuning=tn)
        bound = plan.bind([xs[c] for c in sub])
        ms = _time_ms(torch, bound.run_plain_all, max(1, reps // 5), warmup=1)
        dec = _decisions(bound.outs)
        ok = pref is None or _same(pref, dec)
        pref = pref or dec
        results["plain"].append(dict(chunk_iters=ch, ms=round(ms, 4), same_decisions=ok))
        log(f"plain chunk_iters={ch}: {ms * 1e3:.1f} us for {len(sub)} cubes{'' if ok else ' (rejected)'}")
        # transforming ahead costs one more launch per call: it must win by 2%
        if ok and (best_ms is None or ms < 0.98 * best_ms):
            best_ms, best["chunk_iters"] = ms, ch
        del plan, bound
    return dict(tuning=best, results=results)


def save(arch: str, workload: str, out: dict, path: str = DEFAULT_PATH) -> None:
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.setdefault(arch, {})[workload] = dict(out["tuning"], measured=out["results"],
                                               date=time.strftime("%Y-%m-%d"))
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def load(arch: str, workload: str, path: str = DEFAULT_PATH):
    """Tuned shapes for (arch, workload) as a Plan tuning dict, or None."""
    try:
        with open(path) as f:
            ent = json.load(f).get(arch, {}).get(workload)
    except FileNotFoundError:
        return None
    if not ent:
        return None
    keys = ("block_threads", "max_radix", "chunk_iters", "lines_wg", "lines_threads", "direct_launch",
            "lines_samples", "group_by_length", "shapes")
    return {k: ent[k] for k in keys if k in ent}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default=DEFAULT_PATH)
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import torch
    import workloads as W
    from . import CubeSpec

    dev = torch.device("cuda", 0)
    cubes = W.cfg4()
    specs = [CubeSpec(c.dims, seed=c.schedule_seed, max_k=512, **W.NOISELESS_THRESH) for c in cubes]
    xs = [torch.from_numpy(c.x).to(dev) for c in cubes]
    out = tune(specs, xs, reps=args.reps, log=lambda m: print(m, flush=True))
    arch = _arch()
    save(arch, "batched", out, args.out)
    print(json.dumps({"arch": arch, "tuning": out["tuning"]}), flush=True)


if __name__ == "__main__":
    main()
