"""Monte-Carlo reproduction of the FPS-SFT half of Fig. 2 (Sec. 3) on the
batched GPU path.

Setting of Sec. 3: 256 x 256 cubes, L = 256, three lines of 256 samples per
iteration, T_max = floor(N / (3 L)) = 85 (about 100% of the samples). For
each sparsity K and support type (uniform; one cluster of 9 or 25
frequencies plus uniform others), `runs` independent cubes are planted with
unit magnitudes and random phases and all of them are solved in ONE
persistent launch. Reported per point:

  p_perfect   fraction of runs with perfect recovery: an empty residual
              (outcome OK), the recovered frequency set equal to the planted
              one, and the amplitudes within 1e-3 relative L2 (Fig. 2(a))
  pct_samples mean percentage of the N samples used by the perfect runs,
              iterations x (D+1) L / N (Fig. 2(b))

The paper prints three of the curves' values: about 96% success at
K = 5 N0 (uniform; clustered cases similar), 0% at K = 6 N0 with
T_max = 85, and 5.9% of the samples at K = N0. Inputs are synthetic (the
paper's are too); no dataset is used.

--schedule axis runs the same sweep on the axis-aligned lines of the
row/column method that Sec. 2.1 reviews and Sec. 2.2 shows to deadlock
(iteration t samples along e_{t mod 2}); --schedule both prints the two
curves side by side. Only the line set changes: decode, thresholds and
budget are FPS-SFT's, so the comparison isolates the effect of random
slopes.

    python fig2.py --runs 100 [--schedule random|axis|both] [--out results.json]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

import workloads as W

DIMS = (256, 256)
N0 = 256
K_GRID = (128, 256, 512, 768, 1024, 1280, 1408, 1536)   # N0/2 .. 6 N0
SCENARIOS = (0, 9, 25)                                  # cluster size, 0 = uniform
PERFECT_AMP_TOL = 1e-3


def plant_sweep(Ks, runs: int, clusters, seed: int = 2017):
    """The planted cubes, in (cluster, K, run) order, with their labels."""
    cubes, labels = [], []
    root = np.random.SeedSequence(seed)
    points = [(cl, K) for cl in clusters for K in Ks]
    for (cl, K), child in zip(points, root.spawn(len(points))):
        for r, cs in enumerate(child.spawn(runs)):
            rng = np.random.default_rng(cs)
            cube_seed = int(cs.generate_state(1, dtype=np.uint64)[0] >> np.uint64(1))
            cubes.append(W.plant(DIMS, K, seed=cube_seed, cluster=cl, rng=rng))
            labels.append((cl, K, r))
    return cubes, labels


def perfect(host: dict, cube) -> bool:
    if host["status"] != 0 or host["k"] != len(cube.amps):
        return False
    got = {tuple(f): a for f, a in zip(host["freqs"].tolist(), host["amps"].tolist())}
    if set(got) != {tuple(f) for f in cube.freqs.tolist()}:
        return False
    want = np.asarray(cube.amps)
    have = np.array([got[tuple(f)] for f in cube.freqs.tolist()])
    return float(np.linalg.norm(have - want) / np.linalg.norm(want)) <= PERFECT_AMP_TOL


def sweep(Ks=K_GRID, runs: int = 100, clusters=SCENARIOS, seed: int = 2017, tuning=None,
          reps: int = 3, log=print, axis: bool = False):
    """Plant, solve in one batched launch, and summarise. Returns a dict with
    the per-point table, the per-cube host results and the launch time."""
    import torch
    import paper_1711_11407_amd as F

    t0 = time.perf_counter()
    cubes, labels = plant_sweep(Ks, runs, clusters, seed)
    log(f"planted {len(cubes)} cubes of {DIMS} in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda", 0)
    max_k = int(2 ** np.ceil(np.log2(max(Ks) + 1)))
    specs = [F.CubeSpec(DIMS, seed=c.schedule_seed, max_k=max_k, axis_schedule=axis, **W.NOISELESS_THRESH)
             for c in cubes]
    plan = F.Plan(specs, tuning=tuning)
    xs = [torch.from_numpy(c.x).to(dev) for c in cubes]
    bound = plan.bind(xs)
    bound.run_batched()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        bound.run_batched()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    hosts = [o.host() for o in bound.outs]
    L = 256
    table = []
    for cl in clusters:
        for K in Ks:
            idx = [i for i, (c, k, _) in enumerate(labels) if c == cl and k == K]
            ok = [i for i in idx if perfect(hosts[i], cubes[i])]
            pct = [100.0 * hosts[i]["iters"] * 3 * L / (DIMS[0] * DIMS[1]) for i in ok]
            table.append({"cluster": cl, "K": K, "K_over_N0": K / N0, "runs": len(idx),
                          "p_perfect": len(ok) / len(idx),
                          "pct_samples": float(np.mean(pct)) if pct else None})
    log(f"one batched launch over {len(cubes)} cubes: {ms:.3f} ms "
        f"({len(cubes) / (ms * 1e-3):.0f} transforms/s)")
    return {"table": table, "ms_per_launch": ms, "cubes": len(cubes), "hosts": hosts,
            "labels": labels, "planted": cubes, "plan": plan}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--runs", type=int, default=100)
    ap.add_argument("--seed", type=int, default=2017)
    ap.add_argument("--schedule", choices=["random", "axis", "both"], default="random",
                    help="line slopes: FPS-SFT's random ones, axis-aligned ones, or both sweeps")
    ap.add_argument("--out", default=None, help="write the table(s) as JSON")
    args = ap.parse_args(argv)
    kinds = ["random", "axis"] if args.schedule == "both" else [args.schedule]
    results = {}
    for kind in kinds:
        results[kind] = sweep(runs=args.runs, seed=args.seed, axis=(kind == "axis"),
                              log=lambda m: print(m, flush=True))
    head = f"{'support':>10} {'K/N0':>6}"
    for kind in kinds:
        head += f" {kind + ' P':>10} {kind + ' %smp':>12}"
    print(head)
    rows = zip(*[results[k]["table"] for k in kinds])
    for row in rows:
        sup = "uniform" if row[0]["cluster"] == 0 else f"cluster {row[0]['cluster']}"
        line = f"{sup:>10} {row[0]['K_over_N0']:>6.2f}"
        for r in row:
            pct = "-" if r["pct_samples"] is None else f"{r['pct_samples']:.2f}"
            line += f" {r['p_perfect']:>10.2f} {pct:>12}"
        print(line)
    summary = {"dims": DIMS, "T_max": 85, "runs": args.runs, "seed": args.seed}
    for kind in kinds:
        summary[kind] = {"table": results[kind]["table"], "cubes": results[kind]["cubes"],
                         "ms_per_launch": round(results[kind]["ms_per_launch"], 3)}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(summary, f, indent=1)
    print(json.dumps({k: {kk: vv for kk, vv in v.items() if kk != "table"} if isinstance(v, dict) else v
                      for k, v in summary.items()}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
