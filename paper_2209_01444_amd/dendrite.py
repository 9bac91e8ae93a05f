"""Thermal dendrite at the paper's resolution (Sec. 4.2): tip velocity and
radius against the steady value the paper reports (V d0 / alpha = 0.0166;
0.017 from the Green's-function solution it cites).

    python -m paper_2209_01444_amd.dendrite

Each record gives, every `every` main steps, t/tau0, the dimensionless tip
velocity V d0/alpha of arm 0 over the last window, and rho_tip/d0.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from paper_2209_01444_amd import dlb, workloads

PAPER_V = 0.0166  # steady V d0 / alpha of Sec. 4.2
D0_OVER_W0 = 0.1385


def run(steps: int = 16000, every: int = 500, precision: str = "f32", L: int = 512) -> dict:
    import torch

    cfg = workloads.thermal_dendrite(precision, L)
    d0 = D0_OVER_W0 * cfg["W0"]
    s = dlb.Solver(cfg).init_seed(None)
    torch.cuda.synchronize()
    prev = s.reduce()["tip_s"]
    series, el, t = [], 0.0, 0
    while t < steps:
        n = min(every, steps - t)
        t0 = time.perf_counter()
        s.step(n)
        torch.cuda.synchronize()
        el += time.perf_counter() - t0
        t += n
        r = s.reduce()
        v = (r["tip_s"] - prev) / n
        prev = r["tip_s"]
        series.append({"t_tau0": t / cfg["tau0"], "V": (v * d0 / cfg["alpha"]).round(5).tolist(),
                       "rho_d0": (r["tip_rho"] / d0).round(3).tolist()})
    return {"workload": cfg["name"], "precision": precision, "steps": steps, "seconds": el,
            "MLUPS": L * L * steps / el / 1e6, "V_final": float(np.mean(series[-1]["V"])),
            "paper_V": PAPER_V, "series": series}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=16000)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--precision", default="f32")
    args = ap.parse_args()
    print(json.dumps(run(args.steps, args.every, args.precision)), flush=True)


if __name__ == "__main__":
    main()
