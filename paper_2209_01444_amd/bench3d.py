"""Throughput of the 3-D path (D3Q7 phase field, solute and heat; include/
dlb3.h) on one GPU: a centred thermosolutal seed on an n^3 grid, main steps
timed with HIP events on the solver's stream, MLUPS and the algorithmic HBM
rate of k3_step (each population and history word read and written once per
node and step: 2 x (21 + 2) words).

With --flow: the same seed in a periodic box with D3Q19 melt flow (15 sub-steps
per main step, Pr = nu/alpha = 23.1, initial flow 0.01 lu per main step along x);
the dominant kernel is then k3_flow, one sub-step reading and writing 19
populations and reading phi: 156 B per node and sub-step in FP32.

    python -m paper_2209_01444_amd.bench3d [--n 256] [--precision f32] [--steps 200] [--flow]
"""
from __future__ import annotations

import argparse
import json

from paper_2209_01444_amd import dlb3


def workload(n: int, precision: str, flow: bool = False) -> dict:
    """Thermosolutal set of the 2-D benchmark in 3-D: W0 = 1, tau0 = 20,
    eps4 = 0.05, lambda = 3.1913, Mc_inf = 0.5325, k = 0.15, D = alpha = 0.1,
    theta0 = -0.55, U0 = 0, seed of radius 10 at the centre, walls."""
    c = (n - 1) / 2.0
    cfg = dict(nx=n, ny=n, nz=n, walls=1, precision=precision, W0=1.0, tau0=20.0, eps4=0.05, lambda_=3.1913,
               Mcinf=0.5325, k=0.15, D=0.1, alpha=0.1, theta0=-0.55, U0=0.0, c_init_U=1, seed_R=10.0,
               seed_x=c, seed_y=c, seed_z=c)
    if flow:
        cfg.update(walls=0, use_ns=1, n_sub=15, nu=2.31, u0x=0.01)
    return cfg


def run(n: int = 256, precision: str = "f32", steps: int = 200, warmup: int = 20, flow: bool = False) -> dict:
    import torch

    cfg = workload(n, precision, flow)
    s = dlb3.Solver3(cfg).init_seed()
    s.step(warmup)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(s.stream)
    s.step(steps)
    ev[1].record(s.stream)
    ev[1].synchronize()
    ms = ev[0].elapsed_time(ev[1])
    nodes = n ** 3
    sp = {"f64": 8, "f32": 4}.get(precision, 2)  # population word
    hw = 8 if precision == "f64" else 4  # history word (the arithmetic type)
    if flow:  # k3_step also reads the 19 flow populations and 6 more history words each way
        bytes_per_node = (2 * 21 + 19) * sp + 2 * 8 * hw + 15 * (2 * 19 * sp + hw)
    else:
        bytes_per_node = 2 * 21 * sp + 2 * 2 * hw
    r = s.reduce()
    return {"metric": "3-D coupled-lattice MLUPS", "value": round(nodes * steps / (ms * 1e-3) / 1e6, 1),
            "unit": "MLUPS", "precision": precision, "grid": [n, n, n], "steps": steps, "melt_flow": flow,
            "ms_per_step": round(ms / steps, 5),
            "roofline": {"bound": "hbm", "kernel": "k3_step + 15 k3_flow" if flow else "k3_step",
                         "bytes_per_node_step": bytes_per_node,
                         "achieved_GBps": round(nodes * bytes_per_node * steps / (ms * 1e-3) / 1e9, 1),
                         "peak_GBps": 8000.0,
                         "frac": round(nodes * bytes_per_node * steps / (ms * 1e-3) / 8e12, 4)},
            "tips_lu": [round(float(t), 3) for t in r["tip_s"]], "nonfinite": int(r["nonfinite"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--flow", action="store_true")
    args = ap.parse_args()
    print(json.dumps(run(args.n, args.precision, args.steps, flow=args.flow)), flush=True)


if __name__ == "__main__":
    main()
