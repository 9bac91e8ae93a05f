"""Batched sweep: many seeds of uneven grid sizes in one graph-replayed
launch per kernel class, with the project's autotuner.

    python -m paper_2209_01444_amd.sweep --count 256 --steps 1000
    python -m paper_2209_01444_amd.sweep --count 256 --steps 10000 --snapshots out/ --every 100

Reports aggregate MLUPS (all members' nodes x main steps / s); can check
members bit for bit against single-solver runs and write (phi, C, theta,
ux, uy) snapshots for the surrogate's training set.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from paper_2209_01444_amd import dlb, workloads

TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "batch_tuning.json")


def signature(cfgs) -> str:
    sizes = sorted(f"{c['nx']}x{c['ny']}" for c in cfgs)
    hist = {s: sizes.count(s) for s in set(sizes)}
    c0 = cfgs[0]
    return json.dumps({"precision": c0["precision"], "use_ns": c0["use_ns"], "walls": c0["walls"],
                       "n_sub": c0["n_sub"], "sizes": dict(sorted(hist.items()))}, sort_keys=True)


def tuned(batch: dlb.Batch, cases, trial_steps: int = 5) -> dict:
    """Autotune once per batch signature; cache the choice in a JSON file."""
    key = signature(batch.cfgs)
    cache = {}
    if os.path.exists(TUNE_CACHE):
        with open(TUNE_CACHE) as fh:
            cache = json.load(fh)
    if key in cache and "node_tile" in cache[key]:
        batch.set_config(*cache[key]["config"])
        batch.set_node_tile(cache[key]["node_tile"])
        return cache[key]
    for m, (_, noise) in zip(batch.members, cases):
        m.init_seed(noise)
    ms = batch.autotune(trial_steps)
    rec = {"config": list(batch.config()), "node_tile": batch.node_tile, "ms_per_step": ms}
    cache[key] = rec
    os.makedirs(os.path.dirname(TUNE_CACHE), exist_ok=True)
    with open(TUNE_CACHE, "w") as fh:
        json.dump(cache, fh, indent=1)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--check", type=int, default=0, help="members checked bit for bit against single runs")
    ap.add_argument("--check-steps", type=int, default=200)
    ap.add_argument("--snapshots", default="")
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--max-size", type=int, default=1024)
    ap.add_argument("--sizes", default="128,256,512,1024", help="grid sizes the seeds draw from")
    args = ap.parse_args()

    sizes = tuple(int(v) for v in args.sizes.split(","))
    cases = [c for c in workloads.batched_sweep(args.count, args.seed, sizes)
             if c[0]["nx"] <= args.max_size]
    for c, _ in cases:
        c["precision"] = args.precision
    b = dlb.Batch([c for c, _ in cases])
    tune = tuned(b, cases)
    for m, (_, noise) in zip(b.members, cases):
        m.init_seed(noise)
    nodes = b.nodes
    print(json.dumps({"members": len(cases), "nodes": nodes, "config": tune}), flush=True)

    snaps = []
    b.step(1)
    b.sync()
    t0 = time.perf_counter()
    done = 0
    while done < args.steps - 1:
        k = min(args.every if args.snapshots else args.steps, args.steps - 1 - done)
        b.step(k)
        done += k
        if args.snapshots:
            b.sync()
            snaps.append(done + 1)
            os.makedirs(args.snapshots, exist_ok=True)
            for i, m in enumerate(b.members):
                f = m.fields(("phi", "C", "theta", "ux", "uy"))
                np.save(os.path.join(args.snapshots, f"m{i:03d}_t{done + 1:06d}.npy"),
                        np.stack([f[k] for k in ("phi", "C", "theta", "ux", "uy")]).astype(np.float32))
    b.sync()
    el = time.perf_counter() - t0
    out = {"members": len(cases), "nodes": nodes, "steps": args.steps - 1, "seconds": el,
           "aggregate_MLUPS": nodes * (args.steps - 1) / el / 1e6, "config": b.config(),
           "node_tile": b.node_tile,
           "precision": args.precision}
    if args.snapshots:
        out["note"] = "timing includes snapshot transfers"
    if args.check:
        # fresh batch, short run, bitwise comparison with single solvers
        b.close()
        del b
        idx = np.random.default_rng(0).choice(len(cases), size=min(args.check, len(cases)), replace=False)
        b2 = dlb.Batch([c for c, _ in cases])
        b2.set_config(*tune["config"])
        b2.set_node_tile(tune["node_tile"])
        for m, (_, noise) in zip(b2.members, cases):
            m.init_seed(noise)
        b2.step(args.check_steps)
        ok = []
        for i in idx:
            cfg, noise = cases[i]
            s = dlb.Solver(dict(cfg, flow_fuse=tune["config"][0])).init_seed(noise).step(args.check_steps)
            fa, fb = b2.members[i].fields(), s.fields()
            ok.append(bool(all(np.array_equal(fa[k], fb[k]) for k in dlb.FIELDS)))
            s.close()
        out["bitwise_checked"] = [int(i) for i in idx]
        out["bitwise_equal"] = ok
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
