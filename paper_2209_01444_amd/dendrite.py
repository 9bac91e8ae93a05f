"""Dendrites at the paper's resolution.

Thermal (Sec. 4.2): tip velocity and radius against the steady value the
paper reports (V d0 / alpha = 0.0166; 0.017 from the Green's-function
solution it cites).  Each record gives, every `every` main steps, t/tau0,
the dimensionless tip velocity V d0/alpha of each arm over the last window,
and rho_tip/d0.

Solutal, isothermal (Sec. 4.3): the concentration frozen into the solid on
the central dendrite axis against the Gibbs-Thomson relation the paper
checks, c_s/c_l^0 = k [1 - (1 - k) d0/r_tip], with r_tip the tip radius when
the tip passed that point.  In the model's variables c_s/c_l^0 is C in the
solid (C = k (1 + (1 - k) U) at phi = 1) and U = -d0 kappa at a curved
interface of an isothermal alloy.

Thermal with melt flow (Sec. 4.2): inflow W0/tau0 from the west; the
paper describes the upstream arm outgrowing the others, the vertical arms
settling at the pure-diffusion velocity and the downstream arm slowing to
a lower constant velocity.

Solutal with melt flow (Sec. 4.3): the same comparison of the arms; the
section gives no inflow or viscosity for it (workloads.solutal_dendrite).

Thermosolutal with pure diffusion (Sec. 4.4): 2400^2 with far-field walls to
t D/d0^2 = 470000; the tip velocity V d0/D and radius of the four arms, the
selection parameter 2 D d0/(rho^2 V), and phi, U, theta along the central
axis at the end (the section compares these with other authors' curves,
which the text does not reproduce).  With melt flow, to t D/d0^2 = 150000:
the section describes a fast upstream arm, clearly growing arms across the
flow and a suppressed downstream arm.

    python -m paper_2209_01444_amd.dendrite [--solutal] [--thermosolutal] [--flow] [--stencil]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from paper_2209_01444_amd import dlb, workloads

PAPER_V = 0.0166  # steady V d0 / alpha of Sec. 4.2
D0_OVER_W0 = 0.1385
# Sec. 4.3 prints d0 = 0.2762 W0 next to lambda = 3.191; a1 W0 / lambda gives 0.2770 W0
D0_SOLUTAL = 0.8839 / 3.191
D0_THERMOSOLUTAL = 0.8839 / 3.1913  # 0.2770 W0, as Sec. 4.4 prints


def run(steps: int = 16000, every: int = 500, precision: str = "f32", L: int = 512, flow: bool = False,
        grad_stencil: int = 0) -> dict:
    """Thermal dendrite; with flow=True the melt-flow case (inflow along +x):
    arm 0 (+x) grows downstream, arm 2 (-x) upstream, arms 1 and 3 across
    the flow.  grad_stencil=1: the stencil-gradient ablation of the local
    scheme."""
    import torch

    cfg = dict(workloads.thermal_dendrite(precision, L, flow=flow), grad_stencil=grad_stencil)
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
    out = {"workload": cfg["name"], "precision": precision, "steps": steps, "seconds": el,
           "MLUPS": L * L * steps / el / 1e6, "V_final": float(np.mean(series[-1]["V"])),
           "paper_V": PAPER_V, "series": series}
    if flow:
        v = series[-1]["V"]
        out.update(V_downstream=v[0], V_upstream=v[2], V_vertical=0.5 * (v[1] + v[3]))
    return out


def run_solutal_flow(steps: int = 30000, every: int = 3000, precision: str = "f32", L: int = 1000) -> dict:
    """Solutal dendrite with melt flow (Sec. 4.3): tip velocity V d0/D and
    radius of the four arms; arm 0 downstream (+x), arm 2 upstream."""
    import torch

    cfg = workloads.solutal_dendrite(precision, L, flow=True)
    d0 = D0_SOLUTAL * cfg["W0"]
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
        series.append({"t_tau0": t / cfg["tau0"], "V": (v * d0 / cfg["D"]).round(5).tolist(),
                       "rho_d0": (r["tip_rho"] / d0).round(3).tolist()})
    v = series[-1]["V"]
    return {"workload": cfg["name"], "precision": precision, "steps": steps, "seconds": el,
            "MLUPS": L * L * steps / el / 1e6, "V_downstream": v[0], "V_upstream": v[2],
            "V_vertical": 0.5 * (v[1] + v[3]), "series": series}


def run_solutal(steps: int = 40000, every: int = 200, precision: str = "f32", L: int = 1000,
                skip_w0: float = 8.0) -> dict:
    """Grow the isothermal alloy dendrite, recording arm 0's tip position and
    radius every `every` steps; then compare C on the central axis, from
    skip_w0 W0 outside the initial seed to skip_w0 W0 behind the final tip,
    with the Gibbs-Thomson value at the tip radius of the passage time."""
    import torch

    cfg = workloads.solutal_dendrite(precision, L)
    W0, k = cfg["W0"], cfg["k"]
    d0 = D0_SOLUTAL * W0
    s = dlb.Solver(cfg).init_seed(None)
    torch.cuda.synchronize()
    t_hist, s_hist, r_hist = [], [], []
    el, t = 0.0, 0
    while t < steps:
        n = min(every, steps - t)
        t0 = time.perf_counter()
        s.step(n)
        torch.cuda.synchronize()
        el += time.perf_counter() - t0
        t += n
        r = s.reduce()
        t_hist.append(t)
        s_hist.append(float(r["tip_s"][0]))
        r_hist.append(float(r["tip_rho"][0]))
    f = s.fields()
    yc, xc = int(round(cfg["seed_y"])), cfg["seed_x"]
    row = f["C"][yc]
    s_arr, r_arr = np.array(s_hist), np.array(r_hist)
    x0 = int(np.ceil(xc + cfg["seed_R"] + skip_w0 * W0))
    x1 = int(np.floor(xc + s_arr[-1] - skip_w0 * W0))
    xs = np.arange(x0, x1 + 1)
    # tip radius when the tip passed each x (the tip position grows monotonically)
    rho = np.interp(xs - xc, s_arr, r_arr)
    pred = k * (1.0 - (1.0 - k) * d0 / rho)
    meas = row[xs]
    err = meas / pred - 1.0
    return {"workload": cfg["name"], "precision": precision, "steps": steps, "seconds": el,
            "MLUPS": L * L * steps / el / 1e6, "t_tau0": steps / cfg["tau0"], "tip_s": s_arr[-1],
            "rho_final_d0": r_arr[-1] / d0, "axis_range_lu": [int(x0 - xc), int(x1 - xc)],
            "Cs_measured_mean": float(meas.mean()), "Cs_gibbs_thomson_mean": float(pred.mean()),
            "max_rel_err": float(np.abs(err).max()), "mean_rel_err": float(err.mean()),
            "trapping_free_value_k": k,
            "profile": [[int(x - xc), round(float(m), 5), round(float(q), 5)]
                        for x, m, q in zip(xs[::10], meas[::10], pred[::10])]}


def run_thermosolutal(t_end: float = 470000.0, records: int = 20, precision: str = "f32", L: int = 2400,
                      profile_step: int = 4, verbose: bool = True, flow: bool = False) -> dict:
    """Thermosolutal dendrite with pure diffusion (Sec. 4.4) to t D/d0^2 =
    t_end, recorded `records` times: per arm the tip velocity V d0/D over the
    last window, rho_tip/d0 and the selection parameter 2 D d0/(rho^2 V);
    at the end phi, U and theta along the +x axis from the seed centre to the
    wall (every profile_step nodes), with x measured from the tip.
    flow=True: the melt-flow run (inflow along +x: arm 0 downstream, arm 2
    upstream, arms 1 and 3 across the flow)."""
    import sys

    import torch

    cfg = workloads.thermosolutal_dendrite(precision, L, flow=flow)
    d0 = D0_THERMOSOLUTAL * cfg["W0"]
    D = cfg["D"]
    steps = int(round(t_end * d0 * d0 / D))
    s = dlb.Solver(cfg).init_seed(None)
    torch.cuda.synchronize()
    prev = s.reduce()["tip_s"]
    series, el, t = [], 0.0, 0
    for j in range(records):
        n = (steps * (j + 1)) // records - t
        t0 = time.perf_counter()
        s.step(n)
        torch.cuda.synchronize()
        el += time.perf_counter() - t0
        t += n
        r = s.reduce()
        v = (r["tip_s"] - prev) / n
        prev = r["tip_s"]
        rho = r["tip_rho"]
        series.append({"tD_d0sq": round(t * D / (d0 * d0)), "V": (v * d0 / D).round(8).tolist(),
                       "rho_d0": (rho / d0).round(3).tolist(),
                       "sigma": (2.0 * D * d0 / (rho * rho * v)).round(4).tolist(),
                       "tip_lu": r["tip_s"].round(2).tolist(), "nonfinite": int(r["nonfinite"])})
        if verbose:
            print(f"[thermosolutal] step {t}/{steps}: {json.dumps(series[-1])}", file=sys.stderr, flush=True)
    f = s.fields()
    yc, xc = int(round(cfg["seed_y"])), int(round(cfg["seed_x"]))
    tip = xc + float(series[-1]["tip_lu"][0])
    xs = np.arange(xc, L, profile_step)
    prof = [[round((x - tip) / d0, 2), round(float(f["phi"][yc, x]), 5), round(float(f["U"][yc, x]), 5),
             round(float(f["theta"][yc, x]), 5)] for x in xs]
    ring = np.ones((L, L), bool)
    ring[1:-1, 1:-1] = False
    last = series[-1]
    out = {"workload": cfg["name"], "precision": precision, "steps": steps, "t_end_tD_d0sq": t_end,
           "seconds": el, "MLUPS": L * L * steps / el / 1e6, "d0_lu": d0,
           "V_final": float(np.mean(last["V"])), "rho_final_d0": float(np.mean(last["rho_d0"])),
           "sigma_final": float(np.mean(last["sigma"])),
           "wall_max_dev": {"phi": float(np.abs(f["phi"][ring] + 1.0).max()),
                            "U": float(np.abs(f["U"][ring] - cfg["U0"]).max()),
                            "theta": float(np.abs(f["theta"][ring] - cfg["theta0"]).max())},
           "series": series, "axis_profile_x_d0_phi_U_theta": prof}
    if flow:
        v = last["V"]
        out.update(V_downstream=v[0], V_upstream=v[2], V_vertical=0.5 * (v[1] + v[3]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--every", type=int, default=None)
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--solutal", action="store_true")
    ap.add_argument("--thermosolutal", action="store_true", help="Sec. 4.4 pure diffusion, far-field walls")
    ap.add_argument("--t-end", type=float, default=None,
                    help="thermosolutal: final t D/d0^2 (470000; 150000 with --flow)")
    ap.add_argument("--flow", action="store_true", help="thermal dendrite with melt flow")
    ap.add_argument("--stencil", action="store_true", help="stencil-gradient ablation of the local scheme")
    args = ap.parse_args()
    if args.thermosolutal:
        t_end = args.t_end if args.t_end is not None else (150000.0 if args.flow else 470000.0)
        print(json.dumps(run_thermosolutal(t_end, 20, args.precision, flow=args.flow)), flush=True)
    elif args.solutal and args.flow:
        print(json.dumps(run_solutal_flow(args.steps or 30000, args.every or 3000, args.precision)), flush=True)
    elif args.solutal:
        print(json.dumps(run_solutal(args.steps or 40000, args.every or 200, args.precision)), flush=True)
    else:
        print(json.dumps(run(args.steps or 16000, args.every or 500, args.precision, flow=args.flow,
                             grad_stencil=int(args.stencil))), flush=True)


if __name__ == "__main__":
    main()
