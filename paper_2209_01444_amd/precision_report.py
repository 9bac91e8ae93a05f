"""Error of the reduced-precision storage modes against the FP64 GPU run.

Runs the thermosolutal-with-flow workload (orientation fixed at 0 so grid
sizes compare cleanly) in FP64 and in the FP32 / FP16-shift / BF16-shift
storage modes, and reports for each mode after `steps` main steps:
relative L-inf and L2 errors of phi, C, theta, ux, uy against FP64, and the
errors of the tip velocity (last 100 steps), tip radius and solid fraction.
The FP64 GPU path is itself checked against the CPU oracle by the parity
tests.

    python -m paper_2209_01444_amd.precision_report --size 1024 --steps 20000
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from paper_2209_01444_amd import dlb, workloads

FIELDS = ("phi", "C", "theta", "ux", "uy")


def run(size: int, steps: int, precision: str, seed: int = 2) -> dict:
    cfg, noise = workloads.thermosolutal_flow(size, size, seed=seed, precision=precision, orient=0.0)
    s = dlb.Solver(cfg).init_seed(noise)
    t0 = time.perf_counter()
    s.step(steps - 100)
    r1 = s.reduce(allow_nonfinite=True)
    s.step(100)
    r2 = s.reduce(allow_nonfinite=True)
    el = time.perf_counter() - t0
    f = s.fields(FIELDS)
    out = {"fields": f, "tip_v": (r2["tip_s"] - r1["tip_s"]) / 100.0, "tip_rho": r2["tip_rho"],
           "solid_fraction": r2["solid_fraction"], "nonfinite": r2["nonfinite"], "seconds": el}
    s.close()
    return out


def compare(ref: dict, other: dict) -> dict:
    res = {}
    for k in FIELDS:
        a, b = other["fields"][k], ref["fields"][k]
        scale = max(np.abs(b).max(), 1e-300)
        res[f"{k}_linf_rel"] = float(np.abs(a - b).max() / scale)
        res[f"{k}_l2_rel"] = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    with np.errstate(invalid="ignore", divide="ignore"):
        res["tip_v_rel_max"] = float(np.nanmax(np.abs(other["tip_v"] / ref["tip_v"] - 1)))
        res["tip_rho_rel_max"] = float(np.nanmax(np.abs(other["tip_rho"] / ref["tip_rho"] - 1)))
    res["solid_fraction_rel"] = float(abs(other["solid_fraction"] / ref["solid_fraction"] - 1))
    res["nonfinite"] = other["nonfinite"]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--modes", default="f32,f32m,f16s,bf16s")
    args = ap.parse_args()
    ref = run(args.size, args.steps, "f64")
    print(json.dumps({"size": args.size, "steps": args.steps, "mode": "f64",
                      "tip_v": ref["tip_v"].tolist(), "tip_rho": ref["tip_rho"].tolist(),
                      "solid_fraction": ref["solid_fraction"], "seconds": ref["seconds"]}), flush=True)
    for m in args.modes.split(","):
        o = run(args.size, args.steps, m)
        print(json.dumps({"size": args.size, "steps": args.steps, "mode": m, "seconds": o["seconds"],
                          **compare(ref, o)}), flush=True)


if __name__ == "__main__":
    main()
