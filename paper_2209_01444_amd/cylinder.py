"""Flow past a stationary diffuse cylinder (Sec. 4.1): drag coefficient and
recirculation length of the diffuse-interface flow model, against the values
the paper lists for Re = 20 and 40 (table of Sec. 4.1).

    python -m paper_2209_01444_amd.cylinder --Re 20,40

The solid is the frozen phase field of a diffuse circle (dlb_params.phi_static);
each main step runs n_sub flow sub-steps (workloads.cylinder_flow).  The
hydrodynamic force F_f = -sum [1 - q(phi)] f comes from dlb_reduce in
sub-step units; C_d = F_fx / (rho0 R u0^2) with u0 the inflow speed per
sub-step, and L_W = L / R with L the distance from the rear of the cylinder
(x_c + R) to the point on the centre line where u_x changes sign.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from paper_2209_01444_amd import dlb, workloads

# the paper's table of Sec. 4.1 ("present" rows): Re -> (C_d, L_W)
PAPER = {20: (2.153, 1.853), 40: (1.598, 4.491)}


def drag_coefficient(red: dict, cfg: dict, key: str = "Fx") -> float:
    """C_d from the applied force ("Fx", reading of the passage on the
    hydrodynamic force) or from its literal form, f summed over the nodes
    covered by the solid ("Fx_solid")."""
    u0 = cfg["u_in"][0] / cfg["n_sub"]
    return float(red[key]) / (cfg["rho0"] * cfg["seed_R"] * u0 * u0)


def recirculation_length(ux: np.ndarray, cfg: dict) -> float:
    """L / R from u_x on the node row through the centre: the first sign
    change from backward to forward flow behind x_c + R, interpolated
    linearly; 0 if there is no backward flow."""
    R, xc = cfg["seed_R"], cfg["seed_x"]
    row = ux[int(round(cfg["seed_y"]))]
    x0 = int(np.ceil(xc + R))
    if row[x0] >= 0.0:
        return 0.0
    for x in range(x0, len(row) - 1):
        if row[x] < 0.0 <= row[x + 1]:
            xs = x + row[x] / (row[x] - row[x + 1])
            return (xs - (xc + R)) / R
    return float("nan")


def run(Re: float, R: int = 20, precision: str = "f32", max_substeps: int = 200000,
        check_substeps: int = 3000, tol: float = 1e-5, n_sub: int = 15, width: float | None = None,
        length: int = 70, height: int = 40) -> dict:
    """Run to steady drag (relative change below tol over check_substeps).
    width: tanh width of the diffuse cylinder in lu (default sqrt(2) W0);
    length, height: the domain in units of R."""
    import torch

    cfg = workloads.cylinder_flow(Re, R, precision, n_sub, length, height)
    if width is not None:
        cfg["W0"] = width / np.sqrt(2.0)
    s = dlb.Solver(cfg).init_seed(None)
    torch.cuda.synchronize()
    every = max(1, check_substeps // n_sub)
    cd_prev, cd, hist = None, None, []
    el = 0.0
    while s.step_count * n_sub < max_substeps:
        t0 = time.perf_counter()
        s.step(every)
        torch.cuda.synchronize()
        el += time.perf_counter() - t0
        red = s.reduce()
        cd = drag_coefficient(red, cfg)
        cd_solid = drag_coefficient(red, cfg, "Fx_solid")
        hist.append((s.step_count * n_sub, cd))
        if cd_prev is not None and abs(cd - cd_prev) <= tol * abs(cd):
            break
        cd_prev = cd
    f = s.fields()
    lw = recirculation_length(f["ux"], cfg)
    subs = s.step_count * n_sub
    return {"Re": Re, "R": R, "precision": precision, "nx": cfg["nx"], "ny": cfg["ny"],
            "width": float(np.sqrt(2.0) * cfg["W0"]), "Cd": cd,
            "Cd_solid_nodes": cd_solid, "L_W": lw, "length": length, "height": height,
            "substeps": subs, "seconds": el, "flow_MLUPS": cfg["nx"] * cfg["ny"] * subs / el / 1e6,
            "paper": PAPER.get(int(Re)), "Cd_history": hist[-5:]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--Re", default="20,40")
    ap.add_argument("--R", type=int, default=20)
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--max-substeps", type=int, default=200000)
    ap.add_argument("--width", type=float, default=None, help="tanh width of the cylinder's interface (lu)")
    ap.add_argument("--length", type=int, default=70, help="domain length in units of R")
    ap.add_argument("--height", type=int, default=40, help="domain height in units of R")
    args = ap.parse_args()
    for Re in (float(v) for v in args.Re.split(",")):
        r = run(Re, args.R, args.precision, args.max_substeps, width=args.width, length=args.length,
                height=args.height)
        if r["paper"]:
            r["Cd_rel_err"] = r["Cd"] / r["paper"][0] - 1
            r["Cd_solid_nodes_rel_err"] = r["Cd_solid_nodes"] / r["paper"][0] - 1
            r["L_W_rel_err"] = r["L_W"] / r["paper"][1] - 1
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
